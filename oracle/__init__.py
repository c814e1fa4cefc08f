"""CPU oracle for the DPR1 eigensolver (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library never uses it.
"""
