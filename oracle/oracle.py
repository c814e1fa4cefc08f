"""ctypes front end of the CPU oracle (``dpr1_oracle.c``).

TEST INFRASTRUCTURE ONLY: a plain, slow implementation of Algorithm 1 of
Jakovcevic Stor, Slapnicar and Barlow (forward-stable eigendecomposition of
D + rho z z^T), in binary64 with binary128 where the paper asks for double the
working precision.  Imported only by ``tests/``, ``__graft_entry__.smoke`` and
the ``cpu_baseline`` leg of ``bench.py``.  It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpr1_oracle.c")
_LIB = os.path.join(_HERE, "libdpr1_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction, OpenMP, libquadmath)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
            "-shared", "-Wall", "-o", tmp, _SRC, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Opts(C.Structure):
    _fields_ = [("mode_b", C.c_int32), ("polish", C.c_int32),
                ("kappa_polish", C.c_double), ("nearzero", C.c_double),
                ("remedy", C.c_int32), ("pad", C.c_int32), ("knu_thr", C.c_double)]


class EigDiag(C.Structure):
    _fields_ = [("i", C.c_int32), ("side", C.c_int32), ("used_ext_b", C.c_int32),
                ("polished", C.c_int32), ("nearzero", C.c_int32), ("singular", C.c_int32),
                ("bisect_iters", C.c_int32), ("polish_iters", C.c_int32),
                ("sigma", C.c_double), ("mu", C.c_double), ("nu", C.c_double),
                ("lam", C.c_double), ("b", C.c_double), ("Kb", C.c_double),
                ("Kz", C.c_double), ("kappa_nu_bound", C.c_double), ("kappa_g", C.c_double),
                ("xnorm", C.c_double), ("Knu", C.c_double), ("remedied", C.c_int32), ("pad2", C.c_int32)]


DIAG_FIELDS = [f for f, _ in EigDiag._fields_]
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.oracle_dpr1eig.argtypes = [dp, dp, C.c_double, C.c_int64, C.c_int64,
                                     C.POINTER(Opts), dp, dp, C.POINTER(EigDiag)]
        L.oracle_dpr1eig_all.argtypes = [dp, dp, C.c_double, C.c_int64, C.POINTER(Opts),
                                         dp, dp, C.c_int64, C.POINTER(EigDiag), C.c_int]
        L.oracle_dpr1eig_some.argtypes = [dp, dp, C.c_double, C.c_int64, C.POINTER(C.c_int64),
                                          C.c_int64, C.POINTER(Opts), dp, dp, C.c_int64,
                                          C.POINTER(EigDiag), C.c_int]
        L.oracle_dpr1_backward.argtypes = [dp, dp, C.c_double, C.c_int64, dp, dp, dp, dp, dp,
                                           dp, dp, dp, C.c_int]
        L.oracle_check.argtypes = [dp, dp, C.c_double, C.c_int64]
        L.oracle_max_threads.restype = C.c_int
        L.oracle_tip.argtypes = [dp, dp, C.c_double, C.c_int64, C.c_int64, C.c_int32, dp, dp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def make_opts(mode_b=0, polish=1, kappa_polish=16.0, nearzero=10.0, remedy=0, knu_thr=32.0) -> Opts:
    return Opts(mode_b, polish, kappa_polish, nearzero, remedy, 0, knu_thr)


def diag_to_dict(dg: np.ndarray | EigDiag):
    return {f: getattr(dg, f) for f in DIAG_FIELDS}


def eig(d, z, rho, vectors=True, opts: Opts | None = None, nthreads=0, diags=False):
    """All eigenpairs.  Returns (lam[n], V[n,n] column k = v_k or None[, diag list])."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = d.size
    lam = np.empty(n)
    # V stored column-major: column k contiguous -> use a (n, n) array indexed [k, j]
    Vt = np.empty((n, n)) if vectors else None
    dg = (EigDiag * n)() if diags else None
    rc = lib().oracle_dpr1eig_all(_p(d), _p(z), float(rho), n,
                                  C.byref(opts) if opts is not None else None,
                                  _p(lam), _p(Vt), n, dg, int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_dpr1eig_all failed with code {rc}")
    V = Vt.T if vectors else None
    if diags:
        return lam, V, [diag_to_dict(x) for x in dg]
    return lam, V


def eig_one(d, z, rho, k, vectors=True, opts: Opts | None = None):
    """One eigenpair (0-based k); rho must be positive.  Returns (lam, v, diag)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = d.size
    lam = C.c_double()
    v = np.empty(n) if vectors else None
    dg = EigDiag()
    rc = lib().oracle_dpr1eig(_p(d), _p(z), float(rho), n, int(k),
                              C.byref(opts) if opts is not None else None,
                              C.byref(lam), _p(v), C.byref(dg))
    if rc != 0:
        raise ValueError(f"oracle_dpr1eig failed with code {rc}")
    return lam.value, v, diag_to_dict(dg)


def eig_some(d, z, rho, ks, vectors=False, opts: Opts | None = None, nthreads=0):
    """Eigenpairs for the listed 0-based indices only (rho > 0)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    n, nk = d.size, ks.size
    lam = np.empty(nk)
    Vt = np.empty((nk, n)) if vectors else None
    dg = (EigDiag * nk)()
    rc = lib().oracle_dpr1eig_some(_p(d), _p(z), float(rho), n,
                                   ks.ctypes.data_as(C.POINTER(C.c_int64)), nk,
                                   C.byref(opts) if opts is not None else None,
                                   _p(lam), _p(Vt), n, dg, int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_dpr1eig_some failed with code {rc}")
    return lam, (Vt.T if vectors else None), [diag_to_dict(x) for x in dg]


def check(d, z, rho) -> int:
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    return lib().oracle_check(_p(d), _p(z), float(rho), d.size)


def backward(d, z, rho, sigma, mu, V, lam_bar=None, V_bar=None, nthreads=0):
    """Dense reverse-mode derivative (explicit Abar = V X V^T).  V[j, k] = v_k[j]."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    n = d.size
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    Vc = np.asfortranarray(V, dtype=np.float64)
    Vbc = np.asfortranarray(V_bar, dtype=np.float64) if V_bar is not None else None
    lb = np.ascontiguousarray(lam_bar, dtype=np.float64) if lam_bar is not None else None
    db, zb = np.empty(n), np.empty(n)
    rb = C.c_double()
    fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None
    rc = lib().oracle_dpr1_backward(_p(d), _p(z), float(rho), n, _p(sigma), _p(mu),
                                    fp(Vc), _p(lb), fp(Vbc), _p(db), _p(zb), C.byref(rb),
                                    int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_dpr1_backward failed with code {rc}")
    return db, zb, rb.value


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def tip(d, z, rho, i, mode=0):
    """(b, K_b) of A_i^{-1} for shift index i (0-based); mode 0 binary128, 2 binary64."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    b, kb = C.c_double(), C.c_double()
    rc = lib().oracle_tip(_p(d), _p(z), float(rho), d.size, int(i), int(mode),
                          C.byref(b), C.byref(kb))
    if rc != 0:
        raise ValueError(f"oracle_tip failed with code {rc}")
    return b.value, kb.value


def eig_general(d, z, rho, vectors=True, tol=0.0):
    """All eigenpairs of D + rho z z^T for any finite d (any order, repeated values) and any finite
    z (zeros allowed), by the reduction of Sec. 1 of the paper: sort the poles decreasingly (the
    same permutation applied to z), deflate a pole whose z_j is zero (eigenpair (d_j, e_j)), and
    merge a group of equal poles by an orthogonal transformation of its block that maps its part
    w of z onto ||w|| e_first (a Householder reflection): the pole then appears once in the reduced
    problem, with z = ||w||, and the other vectors of the reflection give ||w||-orthogonal
    eigenvectors for the same eigenvalue.  The reduced problem (strictly decreasing poles, no zero
    z) is solved by Algorithm 1 (``eig``).  A z_j with |z_j| < 2^-511, whose square is not a normal
    binary64 number, is deflated like a zero.  With tol > 0 (the divide-and-conquer driver), poles
    within tol of a group's largest join that group and take its value.  Returns (lam decreasing,
    V with V[:, k] = v_k).
    Ties between equal eigenvalues are in no particular order."""
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    # |z_j| < 2^-511 counts as zero: its square is not a normal binary64 number
    z = np.where(np.abs(z) < 2.0 ** -511, 0.0, z)
    n = d.size
    order = np.argsort(-d, kind="stable")            # sorted position s -> original row order[s]
    ds, zs = d[order], z[order]
    red_d, red_z = [], []
    cols = []          # (value, kind, payload): kind 0 reduced k; 1 unit vector at s; 2 reflection column
    members = []       # per reduced entry: list of (s, scale) rows it spreads to
    s = 0
    while s < n:
        e = s + 1
        while e < n and ds[s] - ds[e] <= tol:     # tol = 0: equal poles (Sec. 1)
            e += 1
        w = zs[s:e]
        nw = float(np.sqrt(np.sum(w * w)))
        if nw == 0.0:
            for t in range(s, e):
                cols.append((ds[s], 1, t))
        elif e - s == 1:
            members.append([(s, 1.0)])
            red_d.append(ds[s])
            red_z.append(zs[s])
        else:
            members.append([(t, zs[t] / nw) for t in range(s, e)])
            red_d.append(ds[s])
            red_z.append(nw)
            u = w / nw
            u[0] += 1.0 if u[0] >= 0 else -1.0
            H = np.eye(e - s) - (2.0 / float(u @ u)) * np.outer(u, u)
            for t in range(1, e - s):
                cols.append((ds[s], 2, (s, H[:, t])))
        s = e
    m = len(red_d)
    lam_r, V_r = (np.empty(0), np.empty((0, 0)))
    if m:
        lam_r, V_r = eig(np.array(red_d), np.array(red_z), rho, vectors=True)
    for k in range(m):
        cols.append((lam_r[k], 0, k))
    cols.sort(key=lambda c: -c[0])
    lam = np.array([c[0] for c in cols])
    if not vectors:
        return lam, None
    U = np.zeros((n, n))                              # rows in sorted positions
    for c, (_, kind, pay) in enumerate(cols):
        if kind == 0:
            for r, mem in enumerate(members):
                for (t, sc) in mem:
                    U[t, c] = V_r[r, pay] * sc
        elif kind == 1:
            U[pay, c] = 1.0
        else:
            s0, h = pay
            U[s0:s0 + h.size, c] = h
    V = np.empty((n, n))
    V[order, :] = U
    return lam, V


def eig_hermitian(d, z, rho, vectors=True):
    """All eigenpairs of D + rho z z^H with real d and complex z, the extension of Algorithm 1 to the
    Hermitian case that the paper states after Algorithm 1 (and in the abstract).  Phi = diag(z_j/|z_j|)
    (1 where z_j = 0) is unitary with Phi D Phi^H = D and z = Phi |z|, so
    D + rho z z^H = Phi (D + rho |z||z|^T) Phi^H: the eigenvalues are those of the real problem with
    |z| (eig_general), and v_k = Phi v_k^real.  Returns (lam decreasing, V complex, V[:, k] = v_k)."""
    d = np.asarray(d, dtype=np.float64)
    z = np.asarray(z, dtype=np.complex128)
    a = np.abs(z)
    safe = np.where(a > 0, a, 1.0)
    # the phase componentwise (real over real), so that a real z_j gives exactly +-1
    ph = np.where(a > 0, z.real / safe + 1j * (z.imag / safe), 1.0 + 0.0j)
    lam, Vr = eig_general(d, a, rho, vectors=vectors)
    if not vectors:
        return lam, None
    return lam, ph[:, None] * Vr


def tridiag_eig(a, b):
    """All eigenpairs of the symmetric tridiagonal T (diagonal a [n], off-diagonal b [n-1]) by
    divide and conquer with rank-one merges, the application the paper gives for DPR1 problems
    (Sec. 1): split at m = n // 2 with beta = b[m-1],
        T = diag(T1 - beta e_m e_m^T, T2 - beta e_1 e_1^T) + beta u u^T,  u = e_m + e_{m+1},
    solve the halves, and with T_h = Q_h Lambda_h Q_h^T merge through the DPR1 problem
        D = diag(Lambda1, Lambda2),  z = Q^T u = [last row of Q1, first row of Q2],  rho = beta
    (eig_general: unsorted poles, equal poles and zero z_j handled as in Sec. 1); the eigenvectors
    of T are diag(Q1, Q2) V.  |beta| <= 8 eps max|d| decouples the halves (every z_j treated as 0);
    a z_j below 2^-300 max|z| is treated as 0 (far below the accuracy of the children's
    eigenvectors); poles within 8 eps max|d| are merged like equal ones.
    Returns (lam decreasing, Q with Q[:, k] = q_k)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = a.size
    if n == 1:
        return a.copy(), np.ones((1, 1))
    m = n // 2
    beta = float(b[m - 1])
    a1 = a[:m].copy()
    a1[-1] -= beta
    a2 = a[m:].copy()
    a2[0] -= beta
    l1, Q1 = tridiag_eig(a1, b[:m - 1])
    l2, Q2 = tridiag_eig(a2, b[m:])
    d = np.concatenate([l1, l2])
    z = np.concatenate([Q1[-1, :], Q2[0, :]])
    # a component below 2^-300 of the largest is taken as 0: it lies far below the absolute
    # accuracy of the children's eigenvectors it comes from, and kept it would put an eigenvalue
    # within ~rho z_j^2 (below 1e-180) of its pole, where binary64 loses the shifted representation
    # and so is a component whose share of the rank-one term is negligible, |beta z_j| <= 2 eps
    # max|d| (zeroing it changes T by at most 2 sqrt(2) |beta z_j|), as divide and conquer deflates
    dmax = np.max(np.abs(d))
    ztiny = max(np.ldexp(np.max(np.abs(z)), -300), 2.0 * np.finfo(float).eps * dmax / abs(beta) if beta else np.inf)
    z = np.where(np.abs(z) < ztiny, 0.0, z)
    # poles within 8 eps max|d| are merged like equal ones: the perturbation is within the
    # accuracy of the children's eigenvalues (divide and conquer deflation)
    tol = 8.0 * np.finfo(float).eps * np.max(np.abs(d))
    if abs(beta) <= tol:          # a negligible coupling decouples the halves
        lam, V = eig_general(d, np.zeros(n), 1.0, tol=tol)
    else:
        lam, V = eig_general(d, z, beta, tol=tol)
    Q = np.zeros((n, n))
    Q[:m, :] = Q1 @ V[:m, :]
    Q[m:, :] = Q2 @ V[m:, :]
    return lam, Q
