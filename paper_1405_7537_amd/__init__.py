"""Forward-stable eigensolver for diagonal-plus-rank-one matrices on MI355X.

``dpr1.py`` holds the thin binding over the HIP C-ABI library (``libdpr1.so``);
``workloads.py`` holds the seeded synthetic inputs.  Nothing is imported here
eagerly, so the workload generators can be used without loading the library.
"""
__all__ = ["dpr1", "workloads"]
