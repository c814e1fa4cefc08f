"""Python binding of libdpr1.so (argument marshalling only).

Device memory and streams come from PyTorch; every step of the eigensolver
runs in the HIP kernels behind the C ABI declared in include/dpr1.h.  There is
no CPU fallback: the calls raise if the library is not built or no GPU is
present.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdpr1.so")

INFO_TEXT = {0: "ok", 1: "d is not strictly decreasing", 2: "some z_j is zero (reducible)",
             3: "non-finite input", 4: "rho is zero or not finite",
             5: "a shifted representation left the binary64 range"}
NSTATS = 12
STAT_NAMES = ["kb_gt_100", "polished", "nearzero", "singular", "iters_max", "iters_sum", "continued",
              "polish_steps_max", "knu_gt", "remedy_r1", "remedy_r2", "ext_b"]


class Opts(C.Structure):
    _fields_ = [("mode_b", C.c_int32), ("root", C.c_int32), ("polish", C.c_int32),
                ("split", C.c_int32), ("kappa_polish", C.c_double), ("nearzero", C.c_double),
                ("main_passes", C.c_int32), ("waves_per_simd", C.c_int32), ("events", C.c_void_p),
                ("vwrite", C.c_int32), ("remedy", C.c_int32), ("knu_thr", C.c_double), ("knu", C.c_void_p)]


class Plan(C.Structure):
    _fields_ = [("nprob", C.c_int64), ("ntotal", C.c_int64), ("nitems", C.c_int64),
                ("nmax", C.c_int64), ("ngroups", C.c_int64), ("split", C.c_int32), ("grid", C.c_int32),
                ("opts", Opts)]


_lib = None
vp = C.c_void_p
i64 = C.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        L.dpr1_default_opts.argtypes = [C.POINTER(Opts)]
        L.dpr1_workspace_size.argtypes = [i64]
        L.dpr1_workspace_size.restype = C.c_size_t
        L.dpr1_eig.argtypes = [vp, vp, C.c_double, i64, vp, vp, i64, vp, vp, vp, vp, vp,
                               C.POINTER(Opts), vp, C.c_size_t, vp]
        L.dpr1_noalloc_scratch_bytes.argtypes = []
        L.dpr1_noalloc_scratch_bytes.restype = C.c_size_t
        L.dpr1_eig_noalloc.argtypes = [vp, vp, C.c_double, i64, vp, vp, i64, vp, vp, vp, vp, vp,
                                       C.POINTER(Opts), vp]
        L.dpr1_batched_workspace_size.argtypes = [i64, C.POINTER(C.c_int64)]
        L.dpr1_batched_workspace_size.restype = C.c_size_t
        L.dpr1_batched_plan.argtypes = [i64, C.POINTER(C.c_int64), C.POINTER(Opts), C.POINTER(Plan),
                                        vp, C.c_size_t, vp]
        L.dpr1_eig_batched.argtypes = [C.POINTER(Plan), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp, C.c_size_t, vp]
        L.dpr1_autotune.argtypes = [vp, vp, C.c_double, i64, vp, vp, i64, vp, vp, vp, vp, C.POINTER(Opts),
                                    C.c_int32, C.POINTER(C.c_double), vp, C.c_size_t, vp]
        L.dpr1_batched_autotune.argtypes = [C.POINTER(Plan), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                            C.c_int32, C.POINTER(C.c_double), vp, C.c_size_t, vp]
        if hasattr(L, "dpr1_backward_workspace_size"):
            L.dpr1_backward_workspace_size.argtypes = [i64, i64]
            L.dpr1_backward_workspace_size.restype = C.c_size_t
            L.dpr1_eig_backward_batched.argtypes = [i64, i64] + [vp] * 12 + [vp, C.c_size_t, vp]
            L.dpr1_eig_backward.argtypes = [vp, vp, C.c_double, i64, vp, vp, vp, vp, i64, vp, vp, i64, vp, vp,
                                            vp, vp, C.c_size_t, vp]
        L.dpr1_general_workspace_size.argtypes = [i64]
        L.dpr1_general_workspace_size.restype = C.c_size_t
        L.dpr1_eig_general.argtypes = [vp, vp, C.c_double, i64, vp, vp, i64, vp, C.POINTER(Opts), vp,
                                       C.c_size_t, vp]
        L.dpr1_eig_hermitian.argtypes = [vp, vp, C.c_double, i64, vp, vp, i64, vp, C.POINTER(Opts), vp,
                                         C.c_size_t, vp]
        L.dpr1_tridiag_workspace_size.argtypes = [i64]
        L.dpr1_tridiag_workspace_size.restype = C.c_size_t
        L.dpr1_tridiag_eig.argtypes = [vp, vp, i64, vp, vp, i64, vp, C.POINTER(Opts), vp, C.c_size_t, vp]
        L.dpr1_strerror.argtypes = [C.c_int]
        L.dpr1_strerror.restype = C.c_char_p
        _lib = L
    return _lib


def opts(mode_b=0, root=1, polish=1, split=0, kappa_polish=16.0, nearzero=10.0, main_passes=0,
         events=None, waves_per_simd=0, vwrite=0, remedy=0, knu_thr=32.0) -> Opts:
    return Opts(mode_b, root, polish, split, kappa_polish, nearzero, main_passes, waves_per_simd, events, vwrite,
                remedy, knu_thr, None)


class HipEvents:
    """Four hipEvent_t handles for the solve's profiling hook (opts.events)."""

    def __init__(self):
        self.rt = C.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.rt.hipEventSynchronize.argtypes = [C.c_void_p]
        self.rt.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.rt.hipEventDestroy.argtypes = [C.c_void_p]
        self.arr = (C.c_void_p * 4)()
        for t in range(4):
            h = C.c_void_p()
            if self.rt.hipEventCreate(C.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.arr[t] = h

    @property
    def ptr(self):
        return C.cast(self.arr, C.c_void_p)

    def ms(self, a, b):
        self.rt.hipEventSynchronize(self.arr[b])
        out = C.c_float()
        if self.rt.hipEventElapsedTime(C.byref(out), self.arr[a], self.arr[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def eig_ms(self):
        return self.ms(0, 1)

    def vec_ms(self):
        return self.ms(2, 3)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(x, device, dtype=torch.float64):
    if isinstance(x, np.ndarray):
        x = np.ascontiguousarray(x)   # torch refuses negative strides (e.g. d[::-1])
    t = torch.as_tensor(x, dtype=dtype)
    return t.to(device).contiguous()


def _rc(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed: {rc} ({lib().dpr1_strerror(rc).decode()})")


class Result:
    """Outputs of one solve; V[:, k] is the eigenvector of lam[k]."""

    def __init__(self, **kw):
        self.__dict__.update(kw)

    def stats_dict(self):
        s = self.stats.cpu().tolist()
        return dict(zip(STAT_NAMES, s))


def workspace_bytes(n):
    return int(lib().dpr1_workspace_size(int(n)))


def eig(d, z, rho, vectors=True, opts: Opts | None = None, check=True, want_stats=False,
        work=None, out=None, device="cuda", ldv=None, want_knu=False):
    """All eigenpairs of D + rho z z^T.  d, z: 1-D float64 (device tensors or host data).

    Returns a Result with lam [n], V [n, n] (V[:, k] = v_k, column-major storage with leading
    dimension ldv >= n, default n), shift_idx, mu, xnorm, info and (optionally) stats.  With
    `out`, its V slot may be an [n, n] view with unit column stride (a slice of a wider buffer)."""
    d = _dev(d, device)
    z = _dev(z, device)
    n = d.numel()
    dev = d.device
    if out is None:
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        ld = n if ldv is None else int(ldv)
        if ld < max(n, 1):
            raise ValueError("ldv must be >= n")
        Vt = torch.empty((n, ld), dtype=torch.float64, device=dev)[:, :n] if vectors else None
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        mu = torch.empty(n, dtype=torch.float64, device=dev)
        xn = torch.empty(n, dtype=torch.float64, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
    else:
        lam, Vt, idx, mu, xn, info = out
    stats = torch.empty(NSTATS, dtype=torch.int32, device=dev) if want_stats else None
    wb = workspace_bytes(n)
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
    if Vt is not None and (tuple(Vt.shape) != (n, n) or (n > 1 and Vt.stride(1) != 1)):
        raise ValueError("V storage must be an [n, n] view with unit column stride")
    ld = max(n, 1) if Vt is None or n <= 1 else Vt.stride(0)
    knu = None
    if want_knu:
        knu = torch.empty(n, dtype=torch.float64, device=dev)
        o = Opts()
        if opts is not None:
            C.memmove(C.byref(o), C.byref(opts), C.sizeof(Opts))
        else:
            lib().dpr1_default_opts(C.byref(o))
        o.knu = knu.data_ptr()
        opts = o
    rc = lib().dpr1_eig(_ptr(d), _ptr(z), float(rho), n, _ptr(lam), _ptr(Vt), ld, _ptr(idx), _ptr(mu),
                        _ptr(xn), _ptr(info), _ptr(stats), C.byref(opts) if opts is not None else None,
                        _ptr(work), wb, _stream())
    _rc(rc, "dpr1_eig")
    r = Result(lam=lam, V=Vt.t() if Vt is not None else None, shift_idx=idx, mu=mu, xnorm=xn,
               info=info, stats=stats, work=work, knu=knu)
    if check:
        code = int(info.item())
        if code != 0:
            raise ValueError(f"dpr1_eig: info = {code} ({INFO_TEXT.get(code, '?')})")
    return r


NOALLOC_MAX_N = 32768


def eig_noalloc(d, z, rho, vectors=True, opts: Opts | None = None, check=True, out=None, device="cuda"):
    """dpr1_eig_noalloc: as eig(), with the library's static device scratch as workspace (n <=
    NOALLOC_MAX_N).  With `out` = (lam, Vt, shift_idx, mu, xnorm, info) preallocated, the call
    itself allocates nothing."""
    d = _dev(d, device)
    z = _dev(z, device)
    n = d.numel()
    dev = d.device
    if out is None:
        lam = torch.empty(n, dtype=torch.float64, device=dev)
        Vt = torch.empty((n, n), dtype=torch.float64, device=dev) if vectors else None
        idx = torch.empty(n, dtype=torch.int32, device=dev)
        mu = torch.empty(n, dtype=torch.float64, device=dev)
        xn = torch.empty(n, dtype=torch.float64, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
    else:
        lam, Vt, idx, mu, xn, info = out
    ld = max(n, 1) if Vt is None or n <= 1 else Vt.stride(0)
    rc = lib().dpr1_eig_noalloc(_ptr(d), _ptr(z), float(rho), n, _ptr(lam), _ptr(Vt), ld, _ptr(idx), _ptr(mu),
                                _ptr(xn), _ptr(info), None, C.byref(opts) if opts is not None else None,
                                _stream())
    _rc(rc, "dpr1_eig_noalloc")
    r = Result(lam=lam, V=Vt.t() if Vt is not None else None, shift_idx=idx, mu=mu, xnorm=xn, info=info)
    if check:
        code = int(info.item())
        if code != 0:
            raise ValueError(f"dpr1_eig_noalloc: info = {code} ({INFO_TEXT.get(code, '?')})")
    return r


def eig_general(d, z, rho, vectors=True, opts: Opts | None = None, check=True, device="cuda"):
    """All eigenpairs of D + rho z z^T for any finite d (any order, repeated values) and z (zeros
    allowed): dpr1_eig_general sorts, deflates zero z_j, merges equal poles and solves the reduced
    problem on the device.  Synchronises the stream.  Returns a Result with lam [n] decreasing,
    V [n, n] (rows in the input order; equal eigenvalues get an orthonormal basis of their
    eigenspace) and info."""
    d = _dev(d, device)
    z = _dev(z, device)
    n = d.numel()
    dev = d.device
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.float64, device=dev) if vectors else None
    info = torch.empty(1, dtype=torch.int32, device=dev)
    wb = int(lib().dpr1_general_workspace_size(n))
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
    rc = lib().dpr1_eig_general(_ptr(d), _ptr(z), float(rho), n, _ptr(lam), _ptr(Vt), max(n, 1), _ptr(info),
                                C.byref(opts) if opts is not None else None, _ptr(work), wb, _stream())
    _rc(rc, "dpr1_eig_general")
    r = Result(lam=lam, V=Vt.t() if Vt is not None else None, info=info)
    if check:
        code = int(info.item())
        if code != 0:
            raise ValueError(f"dpr1_eig_general: info = {code} ({INFO_TEXT.get(code, '?')})")
    return r


def eig_hermitian(d, z, rho, vectors=True, opts: Opts | None = None, check=True, device="cuda"):
    """All eigenpairs of D + rho z z^H with real d and complex z (dpr1_eig_hermitian): the real
    problem with |z| through the front end, then v = diag(z_j/|z_j|) v_real.  Synchronises the
    stream.  Returns a Result with lam [n] float64 decreasing, V [n, n] complex128 (V[:, k] = v_k,
    rows in the input order) and info."""
    d = _dev(d, device)
    z = _dev(z, device, dtype=torch.complex128)
    n = d.numel()
    if z.numel() != n:
        raise ValueError("z must have n entries")
    dev = d.device
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.complex128, device=dev) if vectors else None
    info = torch.empty(1, dtype=torch.int32, device=dev)
    wb = int(lib().dpr1_general_workspace_size(n))
    work = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev)
    rc = lib().dpr1_eig_hermitian(_ptr(d), _ptr(z), float(rho), n, _ptr(lam), _ptr(Vt), max(n, 1), _ptr(info),
                                  C.byref(opts) if opts is not None else None, _ptr(work), wb, _stream())
    _rc(rc, "dpr1_eig_hermitian")
    r = Result(lam=lam, V=Vt.t() if Vt is not None else None, info=info)
    if check:
        code = int(info.item())
        if code != 0:
            raise ValueError(f"dpr1_eig_hermitian: info = {code} ({INFO_TEXT.get(code, '?')})")
    return r


def tridiag_eig(a, b, opts: Opts | None = None, check=True, device="cuda", work=None):
    """All eigenpairs of the symmetric tridiagonal matrix with diagonal a [n] and off-diagonal b [n-1]
    by divide and conquer over DPR1 merges (dpr1_tridiag_eig).  Synchronises the stream.
    Returns a Result with lam [n] decreasing, Q [n, n] (Q[:, k] = q_k) and info."""
    a = _dev(a, device)
    n = a.numel()
    b = _dev(b, device) if n > 1 else torch.zeros(1, dtype=torch.float64, device=a.device)
    if b.numel() < n - 1:
        raise ValueError("b must have n - 1 entries")
    dev = a.device
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Qt = torch.empty((n, n), dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    wb = int(lib().dpr1_tridiag_workspace_size(n))
    if wb == 0:
        raise ValueError("n must be in [1, 65536]")
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
    rc = lib().dpr1_tridiag_eig(_ptr(a), _ptr(b), n, _ptr(lam), _ptr(Qt), n, _ptr(info),
                                C.byref(opts) if opts is not None else None, _ptr(work), wb, _stream())
    _rc(rc, "dpr1_tridiag_eig")
    r = Result(lam=lam, Q=Qt.t(), info=info, work=work)
    if check:
        code = int(info.item())
        if code != 0:
            raise ValueError(f"dpr1_tridiag_eig: info = {code} ({INFO_TEXT.get(code, '?')})")
    return r


def autotune(d, z, rho, vectors=True, opts: Opts | None = None, reps=3, device="cuda"):
    """Time every (split, pass budget) candidate on this problem (dpr1_autotune) and return
    (the options with the fastest split and main_passes, its mean ms).  Synchronises the stream."""
    d = _dev(d, device)
    z = _dev(z, device)
    n = d.numel()
    dev = d.device
    o = Opts()
    if opts is not None:
        C.memmove(C.byref(o), C.byref(opts), C.sizeof(Opts))
    else:
        lib().dpr1_default_opts(C.byref(o))
    lam = torch.empty(n, dtype=torch.float64, device=dev)
    Vt = torch.empty((n, n), dtype=torch.float64, device=dev) if vectors else None
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    mu = torch.empty(n, dtype=torch.float64, device=dev)
    xn = torch.empty(n, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    wb = workspace_bytes(n)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    best = C.c_double()
    rc = lib().dpr1_autotune(_ptr(d), _ptr(z), float(rho), n, _ptr(lam), _ptr(Vt), max(n, 1), _ptr(idx), _ptr(mu),
                             _ptr(xn), _ptr(info), C.byref(o), int(reps), C.byref(best), _ptr(work), wb,
                             _stream())
    _rc(rc, "dpr1_autotune")
    return o, float(best.value)


class Batch:
    """A planned ragged batch (sizes fixed); solve() can be called repeatedly."""

    def __init__(self, offs, opts: Opts | None = None, vectors=True, device="cuda"):
        offs = np.ascontiguousarray(offs, dtype=np.int64)
        self.offs_host = offs
        self.nprob = offs.size - 1
        self.ntotal = int(offs[-1])
        sizes = np.diff(offs)
        self.sizes = sizes
        self.vectors = vectors
        voffs = np.zeros(self.nprob, dtype=np.int64)
        voffs[1:] = np.cumsum(sizes[:-1] ** 2)
        self.voffs_host = voffs
        self.vtotal = int(np.sum(sizes ** 2))
        self.dev = torch.device(device)
        self.offs = torch.as_tensor(offs).to(self.dev)
        self.voffs = torch.as_tensor(voffs).to(self.dev)
        self.wb = int(lib().dpr1_batched_workspace_size(self.nprob, offs.ctypes.data_as(C.POINTER(C.c_int64))))
        if self.wb == 0:
            raise ValueError("invalid batch offsets")
        self.work = torch.empty(self.wb, dtype=torch.uint8, device=self.dev)
        self.plan = Plan()
        rc = lib().dpr1_batched_plan(self.nprob, offs.ctypes.data_as(C.POINTER(C.c_int64)),
                                     C.byref(opts) if opts is not None else None, C.byref(self.plan),
                                     _ptr(self.work), self.wb, _stream())
        _rc(rc, "dpr1_batched_plan")
        N = self.ntotal
        self.lam = torch.empty(N, dtype=torch.float64, device=self.dev)
        self.V = torch.empty(self.vtotal, dtype=torch.float64, device=self.dev) if vectors else None
        self.shift_idx = torch.empty(N, dtype=torch.int32, device=self.dev)
        self.mu = torch.empty(N, dtype=torch.float64, device=self.dev)
        self.xnorm = torch.empty(N, dtype=torch.float64, device=self.dev)
        self.info = torch.empty(self.nprob, dtype=torch.int32, device=self.dev)
        self.stats = torch.empty(NSTATS, dtype=torch.int32, device=self.dev)

    def solve(self, d, z, rho, want_stats=False):
        """Enqueue the solve on the current stream (no synchronisation)."""
        rc = lib().dpr1_eig_batched(C.byref(self.plan), _ptr(self.offs), _ptr(d), _ptr(z), _ptr(rho),
                                    _ptr(self.lam), _ptr(self.V), _ptr(self.voffs) if self.V is not None else None,
                                    _ptr(self.shift_idx), _ptr(self.mu), _ptr(self.xnorm), _ptr(self.info),
                                    _ptr(self.stats) if want_stats else None, _ptr(self.work), self.wb,
                                    _stream())
        _rc(rc, "dpr1_eig_batched")
        return self

    def autotune(self, d, z, rho, reps=3):
        """Time every (split, pass budget) candidate on this batch (dpr1_batched_autotune) and keep
        the fastest in the plan; returns its mean ms.  Synchronises the stream."""
        best = C.c_double()
        rc = lib().dpr1_batched_autotune(C.byref(self.plan), _ptr(self.offs), _ptr(d), _ptr(z), _ptr(rho),
                                         _ptr(self.lam), _ptr(self.V),
                                         _ptr(self.voffs) if self.V is not None else None, _ptr(self.shift_idx),
                                         _ptr(self.mu), _ptr(self.xnorm), _ptr(self.info), int(reps),
                                         C.byref(best), _ptr(self.work), self.wb, _stream())
        _rc(rc, "dpr1_batched_autotune")
        return float(best.value)

    def vblock(self, p):
        """V of problem p as an [n_p, n_p] view (V[:, k] = v_k)."""
        n = int(self.sizes[p])
        o = int(self.voffs_host[p])
        return self.V[o:o + n * n].view(n, n).t()

    def check(self):
        info = self.info.cpu().numpy()
        bad = np.nonzero(info)[0]
        if bad.size:
            raise ValueError(f"dpr1_eig_batched: problem {bad[0]} info = {info[bad[0]]}")


def eig_batched(d, z, rho, offs, vectors=True, opts: Opts | None = None, check=True, want_stats=False,
                device="cuda"):
    b = Batch(offs, opts=opts, vectors=vectors, device=device)
    b.solve(_dev(d, device), _dev(z, device), _dev(rho, device), want_stats=want_stats)
    if check:
        b.check()
    return b


# --------------------------------------------------------------- backward
def backward_batched(d, z, rho, shift_idx, mu, xnorm, V, lam_bar=None, V_bar=None, work=None):
    """Reverse mode for nb problems of equal size n.

    d, z, shift_idx, mu, xnorm, lam_bar: [nb, n]; rho: [nb]; V, V_bar: column-major storage of
    [nb] n x n matrices (tensors whose memory is V[b] with element (j, k) at j + k n).  V may be
    None: the kernels then recompute its elements from z and (shift_idx, mu, xnorm).
    Returns (d_bar [nb, n], z_bar [nb, n], rho_bar [nb])."""
    nb, n = d.shape
    dev = d.device
    d_bar = torch.empty((nb, n), dtype=torch.float64, device=dev)
    z_bar = torch.empty((nb, n), dtype=torch.float64, device=dev)
    rho_bar = torch.empty(nb, dtype=torch.float64, device=dev)
    wb = int(lib().dpr1_backward_workspace_size(n, nb))
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=dev)
    for t in (d, z, rho, shift_idx, mu, xnorm, V, lam_bar, V_bar):
        if t is not None:
            assert t.is_contiguous() and t.device == dev
    rc = lib().dpr1_eig_backward_batched(nb, n, _ptr(d), _ptr(z), _ptr(rho), _ptr(shift_idx), _ptr(mu),
                                         _ptr(xnorm), _ptr(V), _ptr(lam_bar), _ptr(V_bar), _ptr(d_bar),
                                         _ptr(z_bar), _ptr(rho_bar), _ptr(work), wb, _stream())
    _rc(rc, "dpr1_eig_backward_batched")
    return d_bar, z_bar, rho_bar


def backward(d, z, rho, shift_idx, mu, xnorm, V=None, lam_bar=None, V_bar=None, work=None):
    """Reverse mode for one problem (dpr1_eig_backward): d, z, shift_idx, mu, xnorm, lam_bar [n],
    rho a number; V as returned by eig() (V[:, k] = v_k, column-major storage with any leading
    dimension) or None (recomputed from z and the shifted representation); V_bar [n, n] in either
    layout.  Returns (d_bar [n], z_bar [n], rho_bar [1])."""
    n = d.numel()
    dev = d.device
    d_bar = torch.empty(n, dtype=torch.float64, device=dev)
    z_bar = torch.empty(n, dtype=torch.float64, device=dev)
    rho_bar = torch.empty(1, dtype=torch.float64, device=dev)
    wb = int(lib().dpr1_backward_workspace_size(n, 1))
    if work is None or work.numel() < wb:
        work = torch.empty(wb, dtype=torch.uint8, device=dev)

    def colmajor(M):
        if M is None:
            return None, n
        if M.stride(0) == 1 and M.stride(1) >= n:
            return M, M.stride(1)
        return M.t().contiguous().t(), n
    Vc, ldv = colmajor(V)
    Vbc, ldvb = colmajor(V_bar)
    for t in (d, z, shift_idx, mu, xnorm, lam_bar):
        if t is not None:
            assert t.is_contiguous() and t.device == dev
    rc = lib().dpr1_eig_backward(_ptr(d), _ptr(z), float(rho), n, _ptr(shift_idx), _ptr(mu), _ptr(xnorm), _ptr(Vc),
                                 ldv, _ptr(lam_bar), _ptr(Vbc), ldvb, _ptr(d_bar), _ptr(z_bar), _ptr(rho_bar),
                                 _ptr(work), wb, _stream())
    _rc(rc, "dpr1_eig_backward")
    return d_bar, z_bar, rho_bar


def _rho_like(rho):
    """(device, shape) of a tensor rho, None for a Python number (which gets no gradient)."""
    return (rho.device, rho.shape) if torch.is_tensor(rho) else None


def _rho_grad(ctx, rb):
    """rho's gradient on rho's own device and shape; None when rho was a Python number or does not
    need a gradient."""
    if ctx.rho_like is None or not ctx.needs_input_grad[2]:
        return None
    dev, shape = ctx.rho_like
    return rb.reshape(shape).to(dev)


class DPR1Eig(torch.autograd.Function):
    """(lam, V) = eig(D + rho z z^T) with a hand-written adjoint.

    Forward: dpr1_eig.  Backward: dpr1_eig_backward, which needs only V and the shifted
    representation (shift_idx, mu, ||x||) saved by the forward."""

    @staticmethod
    def forward(ctx, d, z, rho):
        rho_v = float(rho)
        r = eig(d.detach(), z.detach(), rho_v, vectors=True)
        ctx.rho_like = _rho_like(rho)
        ctx.rho_v = rho_v
        ctx.save_for_backward(d.detach(), z.detach(), r.shift_idx, r.mu, r.xnorm, r.V)
        return r.lam, r.V

    @staticmethod
    def backward(ctx, lam_bar, V_bar):
        d, z, idx, mu, xn, V = ctx.saved_tensors
        lb = lam_bar.contiguous() if lam_bar is not None else None
        db, zb, rb = backward(d.contiguous(), z.contiguous(), ctx.rho_v, idx, mu, xn, V, lb, V_bar)
        return db, zb, _rho_grad(ctx, rb)


class DPR1EigValues(torch.autograd.Function):
    """lam = eigenvalues of D + rho z z^T, differentiable without ever storing V.

    Forward: dpr1_eig without eigenvectors.  Backward: dpr1_eig_backward_batched with V = NULL,
    whose GEMM tile loads recompute v_k[j] from the saved (shift_idx, mu, ||x||)."""

    @staticmethod
    def forward(ctx, d, z, rho):
        rho_t = rho if torch.is_tensor(rho) else torch.tensor(float(rho), dtype=torch.float64, device=d.device)
        r = eig(d.detach(), z.detach(), float(rho_t), vectors=False)
        ctx.rho_like = _rho_like(rho)
        ctx.save_for_backward(d.detach(), z.detach(), rho_t.detach().reshape(1).to(d.device), r.shift_idx, r.mu,
                              r.xnorm)
        return r.lam

    @staticmethod
    def backward(ctx, lam_bar):
        d, z, rho, idx, mu, xn = ctx.saved_tensors
        n = d.numel()
        db, zb, rb = backward_batched(d.contiguous().view(1, n), z.contiguous().view(1, n), rho, idx.view(1, n),
                                      mu.view(1, n), xn.view(1, n), None, lam_bar.contiguous().view(1, n), None)
        return db.view(n), zb.view(n), _rho_grad(ctx, rb)


class DPR1EigBatched(torch.autograd.Function):
    """Uniform batch: d, z [nb, n], rho [nb] -> lam [nb, n], V [nb, n, n] (V[b][:, k] = v_k)."""

    @staticmethod
    def forward(ctx, d, z, rho):
        nb, n = d.shape
        offs = np.arange(nb + 1, dtype=np.int64) * n
        b = Batch(offs, device=d.device)
        b.solve(d.detach().contiguous(), z.detach().contiguous(), rho.detach().contiguous())
        # a rejected problem (info != 0) has undefined eigenpairs: refuse it rather than hand its
        # unwritten V block to the caller and to the backward
        b.check()
        Vst = b.V.view(nb, n, n)          # [b, k, j] = v_k[j] (column-major blocks)
        ctx.save_for_backward(d.detach(), z.detach(), rho.detach(), b.shift_idx.view(nb, n), b.mu.view(nb, n),
                              b.xnorm.view(nb, n), Vst)
        return b.lam.view(nb, n), Vst.transpose(1, 2)

    @staticmethod
    def backward(ctx, lam_bar, V_bar):
        d, z, rho, idx, mu, xn, Vst = ctx.saved_tensors
        lb = lam_bar.contiguous() if lam_bar is not None else None
        Vb = V_bar.transpose(1, 2).contiguous() if V_bar is not None else None
        return backward_batched(d.contiguous(), z.contiguous(), rho.contiguous(), idx, mu, xn, Vst, lb, Vb)
