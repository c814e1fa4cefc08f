"""High-precision reference eigenpairs of D + rho z z^T (mpmath), used to pin the oracle.

This is independent of both the oracle and the GPU path: it solves the plain
definition -- the eigenvalues are the zeros of the secular function
f(lambda) = 1 + rho sum zeta_j^2/(d_j - lambda) (eq. Pick) and v = x/||x|| with
x = (D - lambda I)^{-1} z (eq. Aeigenvec) -- in 256-bit arithmetic, each root
parametrised from its nearest pole so that lambda - d_i keeps full relative
precision.  A second, fully independent check (``dense``) runs mpmath's
symmetric eigensolver on the explicit matrix for tiny n.
"""
from __future__ import annotations

import mpmath as mp

PREC = 256


def _mp(x):
    return mp.mpf(float(x))


def _solve_increasing(psi, dpsi, hi):
    """Root of an increasing psi on (0, hi] with psi(0+) = -inf.  Returns t (mpf)."""
    lo = hi * mp.mpf(2) ** -3000
    if psi(hi) <= 0:
        return hi
    # geometric halving while the bracket spans a large ratio
    for _ in range(200):
        if hi <= 4 * lo:
            break
        m = mp.sqrt(lo * hi)
        if psi(m) < 0:
            lo = m
        else:
            hi = m
    t = (lo + hi) / 2
    for _ in range(400):
        p = psi(t)
        if p < 0:
            lo = t
        else:
            hi = t
        dp = dpsi(t)
        nt = t - p / dp if dp != 0 else (lo + hi) / 2
        if not (lo < nt < hi):
            nt = (lo + hi) / 2
        if abs(nt - t) <= abs(t) * mp.mpf(2) ** (-PREC + 24) or hi - lo <= abs(t) * mp.mpf(2) ** (-PREC + 24):
            t = nt
            break
        t = nt
    return t


def eig(d, z, rho, vectors=True, ks=None):
    """Reference eigenpairs for rho > 0 and strictly decreasing d.

    Returns a list of dicts (one per requested k, 0-based) with keys
    ``i`` (nearest pole), ``mu`` (lambda - d_i, mpf), ``lam`` (mpf) and ``v``
    (list of mpf, sign as in eq. Aeigenvec) when ``vectors``.
    """
    with mp.workprec(PREC):
        n = len(d)
        D = [_mp(x) for x in d]
        Z = [_mp(x) for x in z]
        R = _mp(rho)
        Z2 = [x * x for x in Z]
        out = []
        ks = range(n) if ks is None else ks
        for k in ks:
            if k == 0:
                i, s = 0, 1
                half = R * mp.fsum(Z2) * 2           # lambda_1 <= d_1 + rho ||z||^2
            else:
                gap = D[k - 1] - D[k]
                mid = D[k] + gap / 2
                F = 1 + R * mp.fsum(Z2[j] / (D[j] - mid) for j in range(n))
                if F > 0:
                    i, s = k, 1                      # root below the midpoint
                else:
                    i, s = k - 1, -1
                half = gap / 2
            sig = D[i]
            dl = [D[j] - sig for j in range(n)]      # exact at this precision

            def psi(t):
                return s * (1 + R * mp.fsum(Z2[j] / (dl[j] - s * t) for j in range(n)))

            def dpsi(t):
                return R * mp.fsum(Z2[j] / (dl[j] - s * t) ** 2 for j in range(n))

            if k == 0:
                t = _solve_increasing(psi, dpsi, half)
            else:
                # the root lies within the half gap of its nearest pole; allow the
                # full gap to be safe when it sits exactly at the midpoint
                t = _solve_increasing(psi, dpsi, 2 * half * (1 - mp.mpf(2) ** -200))
            mu = s * t
            rec = {"i": i, "mu": mu, "lam": sig + mu}
            if vectors:
                x = [Z[j] / (dl[j] - mu) for j in range(n)]
                nrm = mp.sqrt(mp.fsum(xx * xx for xx in x))
                rec["v"] = [xx / nrm for xx in x]
                rec["xnorm"] = nrm
            out.append(rec)
        return out


def dense(d, z, rho, dps=60):
    """Eigenvalues (descending) and eigenvectors of the explicit matrix via mp.eigsy.

    Eigenvector signs are normalised to the convention of eq. (Aeigenvec):
    v_k has the sign of (D - lambda_k I)^{-1} z in its largest component.
    """
    with mp.workdps(dps):
        n = len(d)
        A = mp.matrix(n, n)
        for r in range(n):
            for c in range(n):
                A[r, c] = _mp(rho) * _mp(z[r]) * _mp(z[c]) + (_mp(d[r]) if r == c else 0)
        E, Q = mp.eigsy(A)
        order = sorted(range(n), key=lambda t: -E[t])
        lams, vecs = [], []
        for t in order:
            lam = E[t]
            v = [Q[r, t] for r in range(n)]
            x = [_mp(z[r]) / (_mp(d[r]) - lam) for r in range(n)]
            jm = max(range(n), key=lambda r: abs(x[r]))
            if v[jm] * x[jm] < 0:
                v = [-a for a in v]
            lams.append(lam)
            vecs.append(v)
        return lams, vecs


def rel(a, b):
    """|a - b| / |b| as a float (b exact reference)."""
    with mp.workprec(PREC):
        a, b = mp.mpf(a), mp.mpf(b)
        if b == 0:
            return float(abs(a))
        return float(abs(a - b) / abs(b))


def dense_values(d, z, rho, dps=60):
    """Eigenvalues (descending) of the explicit matrix via mp.eigsy, for any d and z (reducible
    inputs included: no eigenvector normalisation, which needs d_j != lambda)."""
    with mp.workdps(dps):
        n = len(d)
        A = mp.matrix(n, n)
        for r in range(n):
            for c in range(n):
                A[r, c] = _mp(rho) * _mp(z[r]) * _mp(z[c]) + (_mp(d[r]) if r == c else 0)
        E = mp.eigsy(A, eigvals_only=True)
        return sorted([E[t] for t in range(n)], key=lambda x: -x)


def dense_values_hermitian(d, z, rho, dps=60):
    """Eigenvalues (descending) of the explicit Hermitian matrix D + rho z z^H (complex z) via
    mp.eighe, formed from the complex entries directly (no use of |z|)."""
    with mp.workdps(dps):
        n = len(d)
        A = mp.matrix(n, n)
        zc = [mp.mpc(_mp(complex(x).real), _mp(complex(x).imag)) for x in z]
        for r in range(n):
            for c in range(n):
                A[r, c] = _mp(rho) * zc[r] * mp.conj(zc[c]) + (_mp(d[r]) if r == c else 0)
        E = mp.eighe(A, eigvals_only=True)
        return sorted([mp.re(E[t]) for t in range(n)], key=lambda x: -x)
