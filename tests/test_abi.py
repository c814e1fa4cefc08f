"""The C-ABI library builds for gfx950, loads, and exports every declared entry point (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "dpr1.h")
LIB = os.path.join(ROOT, "paper_1405_7537_amd", "libdpr1.so")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(dpr1_[a-z_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["dpr1_eig", "dpr1_eig_batched", "dpr1_batched_plan", "dpr1_workspace_size",
                 "dpr1_batched_workspace_size", "dpr1_eig_backward_batched",
                 "dpr1_backward_workspace_size", "dpr1_default_opts", "dpr1_strerror",
                 "dpr1_eig_general", "dpr1_general_workspace_size", "dpr1_eig_hermitian"]:
        assert must in names, must


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdpr1.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_has_gfx950_code_object():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data


def test_host_side_queries(lib):
    lib.dpr1_workspace_size.argtypes = [ctypes.c_int64]
    lib.dpr1_workspace_size.restype = ctypes.c_size_t
    assert lib.dpr1_workspace_size(0) == 0
    a = lib.dpr1_workspace_size(1000)
    b = lib.dpr1_workspace_size(2000)
    assert 0 < a < b
    lib.dpr1_strerror.argtypes = [ctypes.c_int]
    lib.dpr1_strerror.restype = ctypes.c_char_p
    assert lib.dpr1_strerror(0) == b"ok"


def test_argument_errors_need_no_gpu(lib):
    """Synchronous argument checks return -p before anything touches the device."""
    vp = ctypes.c_void_p
    lib.dpr1_eig.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int64, vp, vp, vp,
                             vp, vp, vp, vp, ctypes.c_size_t, vp]
    fake = vp(0x1000)
    assert lib.dpr1_eig(None, fake, 1.0, 4, fake, None, 4, None, None, None, fake, None, None, fake, 1 << 20, None) == -1
    assert lib.dpr1_eig(fake, fake, 0.0, 4, fake, None, 4, None, None, None, fake, None, None, fake, 1 << 20, None) == -3
    assert lib.dpr1_eig(fake, fake, float("nan"), 4, fake, None, 4, None, None, None, fake, None, None, fake, 1 << 20, None) == -3
    assert lib.dpr1_eig(fake, fake, 1.0, 0, fake, None, 4, None, None, None, fake, None, None, fake, 1 << 20, None) == -4
    assert lib.dpr1_eig(fake, fake, 1.0, 8, fake, fake, 4, None, None, None, fake, None, None, fake, 1 << 20, None) == -7
    assert lib.dpr1_eig(fake, fake, 1.0, 8, fake, None, 8, None, None, None, fake, None, None, fake, 16, None) == -15


def test_invalid_register_budget_is_rejected_before_launch(lib):
    """opts.waves_per_simd other than 0, 4, 6, 8 is argument 13 (dpr1_eig) / 3 (dpr1_batched_plan)."""
    from paper_1405_7537_amd.dpr1 import Opts, Plan
    vp = ctypes.c_void_p
    lib.dpr1_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.dpr1_eig.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int64, vp, vp, vp,
                             vp, vp, ctypes.POINTER(Opts), vp, ctypes.c_size_t, vp]
    o = Opts()
    lib.dpr1_default_opts(ctypes.byref(o))
    assert o.waves_per_simd == 0
    o.waves_per_simd = 5
    fake = vp(0x1000)
    assert lib.dpr1_eig(fake, fake, 1.0, 8, fake, None, 8, None, None, None, fake, None, ctypes.byref(o),
                        fake, 1 << 20, None) == -13
    lib.dpr1_batched_plan.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(Opts),
                                      ctypes.POINTER(Plan), vp, ctypes.c_size_t, vp]
    offs = (ctypes.c_int64 * 3)(0, 5, 9)
    plan = Plan()
    assert lib.dpr1_batched_plan(2, offs, ctypes.byref(o), ctypes.byref(plan), fake, 1 << 24, None) == -3
    # opts.mode_b: 0 .. 3, anything else is argument 13 (dpr1_eig) / 3 (dpr1_batched_plan)
    for bad in (-1, 4):
        o.mode_b = bad
        assert lib.dpr1_eig(fake, fake, 1.0, 8, fake, None, 8, None, None, None, fake, None, ctypes.byref(o),
                            fake, 1 << 20, None) == -13
        assert lib.dpr1_batched_plan(2, offs, ctypes.byref(o), ctypes.byref(plan), fake, 1 << 24, None) == -3
    o.mode_b = 0
    # opts.vwrite: 0 .. 8 (chunks of the overlapped write), anything else is argument 13 as well
    o.waves_per_simd = 0
    for bad in (-1, 9):
        o.vwrite = bad
        assert lib.dpr1_eig(fake, fake, 1.0, 8, fake, None, 8, None, None, None, fake, None, ctypes.byref(o),
                            fake, 1 << 20, None) == -13


def test_general_front_end_argument_errors_need_no_gpu(lib):
    """dpr1_eig_general checks its arguments before its first device-to-host copy."""
    from paper_1405_7537_amd.dpr1 import Opts
    vp = ctypes.c_void_p
    lib.dpr1_general_workspace_size.argtypes = [ctypes.c_int64]
    lib.dpr1_general_workspace_size.restype = ctypes.c_size_t
    assert lib.dpr1_general_workspace_size(0) == 0
    a, b = lib.dpr1_general_workspace_size(1000), lib.dpr1_general_workspace_size(2000)
    assert 0 < a < b < 2000 * 1000   # O(n): no n x n scratch
    lib.dpr1_eig_general.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int64, vp,
                                     ctypes.POINTER(Opts), vp, ctypes.c_size_t, vp]
    fake = vp(0x1000)
    big = 1 << 30
    assert lib.dpr1_eig_general(None, fake, 1.0, 4, fake, None, 4, fake, None, fake, big, None) == -1
    assert lib.dpr1_eig_general(fake, None, 1.0, 4, fake, None, 4, fake, None, fake, big, None) == -2
    assert lib.dpr1_eig_general(fake, fake, 0.0, 4, fake, None, 4, fake, None, fake, big, None) == -3
    assert lib.dpr1_eig_general(fake, fake, float("inf"), 4, fake, None, 4, fake, None, fake, big, None) == -3
    assert lib.dpr1_eig_general(fake, fake, 1.0, 0, fake, None, 4, fake, None, fake, big, None) == -4
    assert lib.dpr1_eig_general(fake, fake, 1.0, 4, None, None, 4, fake, None, fake, big, None) == -5
    assert lib.dpr1_eig_general(fake, fake, 1.0, 8, fake, fake, 4, fake, None, fake, big, None) == -7
    assert lib.dpr1_eig_general(fake, fake, 1.0, 4, fake, None, 4, None, None, fake, big, None) == -8
    o = Opts()
    lib.dpr1_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.dpr1_default_opts(ctypes.byref(o))
    o.waves_per_simd = 3
    assert lib.dpr1_eig_general(fake, fake, 1.0, 4, fake, None, 4, fake, ctypes.byref(o), fake, big, None) == -9
    assert lib.dpr1_eig_general(fake, fake, 1.0, 4, fake, None, 4, fake, None, None, big, None) == -10
    assert lib.dpr1_eig_general(fake, fake, 1.0, 4, fake, None, 4, fake, None, fake, 16, None) == -11

    lib.dpr1_eig_hermitian.argtypes = lib.dpr1_eig_general.argtypes
    assert lib.dpr1_eig_hermitian(None, fake, 1.0, 4, fake, None, 4, fake, None, fake, big, None) == -1
    assert lib.dpr1_eig_hermitian(fake, fake, float("nan"), 4, fake, None, 4, fake, None, fake, big, None) == -3
    assert lib.dpr1_eig_hermitian(fake, fake, 1.0, 4, fake, None, 4, fake, None, fake, 16, None) == -11


def test_noalloc_limits_need_no_gpu(lib):
    """dpr1_eig_noalloc: its scratch holds the workspace of the largest accepted n, and larger
    problems are refused (DPR1_ETOOBIG) before any device work."""
    lib.dpr1_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.dpr1_workspace_size.argtypes = [ctypes.c_int64]
    lib.dpr1_workspace_size.restype = ctypes.c_size_t
    src = open(HDR).read()
    nmax = int(re.search(r"#define DPR1_NOALLOC_MAX_N (\d+)", src).group(1))
    assert lib.dpr1_noalloc_scratch_bytes() == lib.dpr1_workspace_size(nmax)
    assert lib.dpr1_noalloc_scratch_bytes() < 16 << 20
    vp = ctypes.c_void_p
    lib.dpr1_eig_noalloc.argtypes = [vp, vp, ctypes.c_double, ctypes.c_int64, vp, vp, ctypes.c_int64,
                                     vp, vp, vp, vp, vp, vp, vp]
    fake = vp(16)
    assert lib.dpr1_eig_noalloc(fake, fake, 1.0, nmax + 1, fake, None, 0, None, None, None, fake,
                                None, None, None) == -1001
    assert lib.dpr1_eig_noalloc(fake, fake, 1.0, 0, fake, None, 0, None, None, None, fake,
                                None, None, None) == -4
    assert lib.dpr1_eig_noalloc(None, fake, 1.0, 5, fake, None, 0, None, None, None, fake,
                                None, None, None) == -1


def test_single_backward_argument_errors_need_no_gpu(lib):
    """dpr1_eig_backward checks its arguments before any launch (-p as the parameter list orders them)."""
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.dpr1_eig_backward.argtypes = [vp, vp, ctypes.c_double, i64, vp, vp, vp, vp, i64, vp, vp, i64, vp, vp, vp, vp,
                                      ctypes.c_size_t, vp]
    f = vp(0x1000)
    ok = dict(d=f, z=f, rho=1.0, n=8, si=f, mu=f, xn=f, V=f, ldv=8, lb=None, Vb=f, ldvb=8, db=f, zb=f, rb=f, w=f,
              wb=1 << 24)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return lib.dpr1_eig_backward(a["d"], a["z"], a["rho"], a["n"], a["si"], a["mu"], a["xn"], a["V"], a["ldv"],
                                     a["lb"], a["Vb"], a["ldvb"], a["db"], a["zb"], a["rb"], a["w"], a["wb"], None)
    assert call(d=None) == -1
    assert call(z=None, V=None) == -2
    assert call(rho=0.0) == -3 and call(rho=float("nan")) == -3
    assert call(n=0) == -4
    assert call(si=None) == -5
    assert call(ldv=7) == -9
    assert call(ldvb=7) == -12
    assert call(rb=None) == -15
    assert call(w=None) == -16
    assert call(wb=16) == -17
