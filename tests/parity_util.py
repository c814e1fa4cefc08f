"""Helpers of the GPU parity tests (no GPU needed to import).

* ``rel``: elementwise relative difference.
* ``check_repr``: the shifted representation of every eigenpair -- the index i of the pole used
  as shift, mu = lambda - d_i and ||x|| of eq. (eigenvecAi) -- against the oracle's.  Indices must
  be equal except where the shift test of Algorithm 1 is a tie: F, the secular function at the
  midpoint of the eigenvalue's gap, zero to rounding, so that the eigenvalue sits at the midpoint
  and either neighbouring pole is nearest.  Such a tie is confirmed with F evaluated in 100-digit
  arithmetic; mu and ||x|| are then not comparable (they belong to different poles) and are
  skipped, while lambda and v are still compared by the caller.
* ``range_cause``: why a problem may be reported with DPR1_INFO_RANGE (its input outside the
  binary64 range of the method, or an eigenpair whose shifted representation does not fit in
  binary64, as the oracle finds it); None when the library must solve it.
"""
import mpmath as mp
import numpy as np

DBL_MIN = 2.2250738585072014e-308
MU_TOL = 1e-13
XN_TOL = 1e-13
TIE_TOL = 1e-11


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b)
    return np.abs(a - b) / np.where(den == 0, 1.0, den)


def midpoint_F(d, z, rho, k):
    """F = 1 + rho sum zeta_j^2 / ((d_j - d_k) - tau), tau = (d_{k-1} - d_k)/2, in 100 digits,
    with the midpoint rounded as binary64 computes it, and the scale 1 + |rho| sum |terms|."""
    tau = (d[k - 1] - d[k]) / 2
    with mp.workdps(100):
        s = mp.mpf(0)
        sa = mp.mpf(0)
        for j in range(len(d)):
            den = mp.mpf(float(d[j] - d[k])) - mp.mpf(float(tau))
            t = mp.mpf(float(z[j])) ** 2 / den
            s += t
            sa += abs(t)
        r = mp.mpf(float(rho))
        return float(1 + r * s), float(1 + abs(r) * sa)


def check_repr(d, z, rho, idx, mu, xn, diags, ks=None, mu_tol=MU_TOL, xn_tol=XN_TOL):
    """Assert the shifted representation of the library (idx, mu, xn: arrays over the caller's
    eigenvalue indices ks, default all) against the oracle's diags (same order).  Returns
    (ties, max rel error of mu, max rel error of ||x||)."""
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = d.size
    ks = np.arange(n) if ks is None else np.asarray(ks)
    neg = rho < 0
    # the problem Algorithm 1 solves: rho > 0 (Sec. 1 reduction for rho < 0)
    ds, zs, rs = (-d[::-1], z[::-1], -rho) if neg else (d, z, rho)
    ties = 0
    wm = wx = 0.0
    for m, k in enumerate(ks):
        g = diags[m]
        oi = (n - 1 - g["i"]) if neg else g["i"]
        omu = -g["mu"] if neg else g["mu"]
        if int(idx[m]) != oi:
            ksol = (n - 1 - k) if neg else k           # index in the solved problem
            gi = (n - 1 - int(idx[m])) if neg else int(idx[m])
            assert ksol >= 1 and {gi, g["i"]} == {ksol - 1, ksol}, (k, idx[m], oi)
            F, scale = midpoint_F(ds, zs, rs, ksol)
            assert abs(F) <= TIE_TOL * scale, (k, idx[m], oi, F, scale)
            ties += 1
            continue
        em = float(rel(mu[m], omu))
        ex = float(rel(xn[m], g["xnorm"]))
        assert em <= mu_tol, (k, mu[m], omu, em)
        assert ex <= xn_tol, (k, xn[m], g["xnorm"], ex)
        wm, wx = max(wm, em), max(wx, ex)
    return ties, wm, wx


def range_cause(d, z, diags):
    """None, or a short text naming why the problem lies outside the binary64 range."""
    d = np.asarray(d, dtype=np.float64)
    az = np.abs(np.asarray(z, dtype=np.float64))
    if np.any((az > 0) & (az < 2.0 ** -511)):
        return "input: |z_j| < 2^-511"
    if d.size > 1 and np.any(np.abs(np.diff(d)) < 2.0 ** -1000):
        return "input: poles closer than 2^-1000"
    for k, g in enumerate(diags):
        mu, xn, b = g["mu"], g["xnorm"], g["b"]
        if not (abs(mu) >= DBL_MIN and abs(mu) < np.inf):
            return f"pair {k}: mu = {mu:.3g} not a normal number"
        if not np.isfinite(abs(mu) * xn):
            return f"pair {k}: |mu| ||x|| not finite"
        if not np.isfinite(b):
            return f"pair {k}: tip b beyond binary64"
    return None
