"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bar (from the design): eigenvalue relative error <= 1e-13 and eigenvector componentwise
relative error <= 1e-12, element by element.
"""
import math

import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W
from parity_util import check_repr, range_cause

pytestmark = pytest.mark.gpu

LAM_TOL = 1e-13
VEC_TOL = 1e-12


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_7537_amd.dpr1 as D
    D.lib()
    return D


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b)
    out = np.abs(a - b) / np.where(den == 0, 1.0, den)
    return out


def compare(D, orc, d, z, rho, opts=None, oopts=None, tag=""):
    print(f"[parity] {tag} n={len(d)} rho={rho}", flush=True)
    r = D.eig(d, z, rho, opts=opts, want_stats=True)
    lam = r.lam.cpu().numpy()
    V = r.V.cpu().numpy()
    lo, Vo, dg = orc.eig(d, z, rho, opts=oopts, diags=True)
    el = rel(lam, lo)
    ev = rel(V, Vo)
    print(f"[parity] {tag}: max rel lam {el.max():.3e} V {ev.max():.3e} stats {r.stats_dict()}", flush=True)
    assert el.max() <= LAM_TOL, (np.argmax(el), el.max())
    assert ev.max() <= VEC_TOL, (np.unravel_index(np.argmax(ev), ev.shape), ev.max())
    ties, em, ex = check_repr(d, z, rho, r.shift_idx.cpu().numpy(), r.mu.cpu().numpy(), r.xnorm.cpu().numpy(), dg)
    print(f"[parity] {tag}: shifted representation: {ties} ties, max rel mu {em:.3e} ||x|| {ex:.3e}", flush=True)
    return r, lo, Vo, dg


def test_examples(D, orc):
    for tag, (d, z, rho) in [("ex1", W.example1()), ("ex2", W.example2()), ("ex3", W.example3())]:
        compare(D, orc, d, z, rho, tag=tag)


def test_example2_shifted_representation_32_digits(D, orc):
    """Example 2 (Sec. 3): the GPU's pair (d_i, mu) represents lambda_2..lambda_4 to 32 digits,
    against the printed 32-digit eigenvalues (golden fixture), and lambda itself is within one
    unit in the last place of them."""
    import mpmath as mp
    from golden.load import load
    g = load("example2.txt")
    d, z, rho = W.example2()
    r = D.eig(d, z, rho)
    lam, idx, mu = r.lam.cpu().numpy(), r.shift_idx.cpu().numpy(), r.mu.cpu().numpy()
    with mp.workdps(40):
        ref = [mp.mpf(x[0]) for x in g["lambda32"]]
        for k in range(4):
            assert abs(lam[k] - float(ref[k])) <= math.ulp(float(ref[k])), k
        for k in (1, 2, 3):
            s = mp.mpf(float(d[idx[k]])) + mp.mpf(float(mu[k]))
            assert abs(s - ref[k]) <= mp.mpf("1e-31"), (k, s, ref[k])


def test_config_small_uniform(D, orc):
    compare(D, orc, *W.uniform(256, 0), tag="n256")


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 64, 65, 127, 129, 300])
def test_ragged_sizes(D, orc, n):
    compare(D, orc, *W.uniform(n, 40 + n), tag=f"ragged{n}")


def test_bisection_root(D, orc):
    compare(D, orc, *W.uniform(200, 3), opts=D.opts(root=0), tag="bisect")


def test_negative_rho(D, orc):
    d, z, _ = W.uniform(150, 8)
    compare(D, orc, d, z, -0.8, tag="negrho")


def test_large_rho_exterior(D, orc):
    compare(D, orc, *W.uniform(512, 11, rho=10.0), tag="rho10")


def test_graded_clustered(D, orc):
    r, *_ = compare(D, orc, *W.graded(1024, 1, pair_every=64), tag="graded1024")
    assert r.stats_dict()["polished"] >= 1


def test_example4_kb_counts(D, orc):
    for beta, count in [(1e-3, 25), (1e-8, 201), (1e-15, 201)]:
        d, z, rho = W.example4(beta)
        r, *_ = compare(D, orc, d, z, rho, opts=D.opts(mode_b=1), oopts=orc.make_opts(mode_b=1),
                        tag=f"ex4 beta={beta}")
        assert r.stats_dict()["kb_gt_100"] == count


@pytest.mark.parametrize("n,ldv,rho", [(2001, 2002, -0.8), (2048, 2050, 1.3), (1537, 1538, 0.6)])
def test_address_ordered_writer_edges(D, orc, n, ldv, rho):
    """The address-ordered eigenvector writer (columns 16-byte aligned: even ldv) with an odd n
    (the last position of every column stored alone), a padded leading dimension and rho < 0
    (positions and columns reversed): every eigenpair against the oracle, the padding untouched."""
    import torch
    d, z, _ = W.uniform(n, 41)
    Vt = torch.full((n, ldv), 7.0, dtype=torch.float64, device="cuda")
    out = (torch.empty(n, dtype=torch.float64, device="cuda"), Vt[:, :n],
           torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    print(f"[parity] writer edges n={n} ldv={ldv} rho={rho}", flush=True)
    r = D.eig(d, z, rho, opts=D.opts(vwrite=1), out=out)
    torch.cuda.synchronize()
    assert int(r.info.item()) == 0
    lo, Vo = orc.eig(d, z, rho)
    assert rel(r.lam.cpu().numpy(), lo).max() <= LAM_TOL
    assert rel(r.V.cpu().numpy(), Vo).max() <= VEC_TOL
    assert torch.all(Vt[:, n:] == 7.0)


def test_knu2_gate(D, orc):
    """Algorithm 1's gate on the bound of eq. (knu2) (mode_b = 3): Example 4's printed counts of
    double-precision tips (25, 201, 201), Example 3's k = 2, 3, 4, and Example 1's none, each with
    parity against the oracle under the same gate.  On the C2-like graded matrix the gate leaves b
    in standard precision for eigenvalues whose result is sensitive to it, where the two sides'
    binary64 tips (summed in different orders) legitimately differ beyond the parity bar (the
    reason the default forms b in double-double always): there the GPU takes the oracle's
    decisions eigenvalue by eigenvalue, the count of double-precision tips among them."""
    cases = [(W.example4(b), c, f"ex4 beta={b}") for b, c in [(1e-3, 25), (1e-8, 201), (1e-15, 201)]]
    cases += [(W.example3(), 3, "ex3"), (W.example1(), 0, "ex1")]
    for (d, z, rho), count, tag in cases:
        r, *_ = compare(D, orc, d, z, rho, opts=D.opts(mode_b=3), oopts=orc.make_opts(mode_b=3), tag=tag + " knu2")
        assert r.stats_dict()["ext_b"] == count, (tag, r.stats_dict())
    d, z, rho = W.graded(1024, 2, pair_every=64)
    r = D.eig(d, z, rho, opts=D.opts(mode_b=3), want_stats=True)
    _, _, dg = orc.eig(d, z, rho, opts=orc.make_opts(mode_b=3), diags=True)
    n_orc = sum(x["used_ext_b"] for x in dg)
    print(f"[parity] graded1024 knu2: double-precision tips GPU {r.stats_dict()['ext_b']}, oracle {n_orc}",
          flush=True)
    assert r.stats_dict()["ext_b"] == n_orc


def test_example4_orthogonality_without_extended_b(D):
    """Table 1's pattern on the GPU: with the tip b in standard precision only (mode_b = 2, the
    paper's dpr1eig_nd) the eigenvectors of Example 4 lose orthogonality as beta falls (O of
    order 1e4 at beta = 1e-8 and beyond 1e6 at 1e-15), while b in double-double keeps O < 1."""
    import torch
    for beta, lo_nd in [(1e-3, None), (1e-8, 1e2), (1e-15, 1e6)]:
        d, z, rho = W.example4(beta)
        n = d.size
        out = {}
        for mb in (0, 2):
            r = D.eig(d, z, rho, opts=D.opts(mode_b=mb, polish=0 if mb == 2 else 1))
            torch.cuda.synchronize()
            V = r.V.cpu().numpy()
            G = V.T @ V - np.eye(n)
            out[mb] = np.max(np.linalg.norm(G, axis=0)) / (n * np.finfo(float).eps)
        print(f"[parity] Table 1 beta={beta}: O(nd) {out[2]:.3g}, O(dd) {out[0]:.3g}", flush=True)
        assert out[0] < 1.0
        if lo_nd is not None:
            assert out[2] > lo_nd


def test_near_zero_and_singular(D, orc):
    d = np.array([2.0, 1.0, -1.0, -2.0])
    z = np.array([0.7, -1.1, 0.9, 0.0])
    rho = 1.3
    s = 1 + rho * sum(z[j] ** 2 / d[j] for j in range(3))
    z[3] = math.sqrt(s * 2.0 / rho)
    r, *_ = compare(D, orc, d, z, rho, tag="nearzero")
    assert r.stats_dict()["nearzero"] == 1
    r = D.eig([1.0, -1.0], [0.75, 1.25], 1.0, want_stats=True)
    assert r.lam.cpu().numpy()[1] == 0.0


def test_info_codes(D):
    d, z, rho = W.uniform(16, 2)
    assert int(D.eig(d[::-1].copy(), z, rho, check=False).info.item()) == 1
    z0 = z.copy()
    z0[5] = 0.0
    assert int(D.eig(d, z0, rho, check=False).info.item()) == 2
    dn = d.copy()
    dn[3] = np.inf
    assert int(D.eig(dn, z, rho, check=False).info.item()) == 3
    with pytest.raises(RuntimeError):
        D.eig(d, z, 0.0)


@pytest.mark.parametrize("n,pad,rho", [(700, 5, 1.0), (2500, 3, -0.7), (4100, 64, 2.0)])
def test_strided_v(D, orc, n, pad, rho):
    """V written into a wider column-major buffer (ldv = n + pad): the columns match the
    oracle, and the padding rows between columns are left untouched."""
    import torch
    d, z, _ = W.uniform(n, 11)
    ld = n + pad
    print(f"[parity] strided n={n} ldv={ld} rho={rho}", flush=True)
    buf = torch.full((n, ld), float("nan"), dtype=torch.float64, device="cuda")
    out = (torch.empty(n, dtype=torch.float64, device="cuda"), buf[:, :n],
           torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))
    r = D.eig(d, z, rho, out=out)
    lo, Vo = orc.eig(d, z, rho)
    el = rel(r.lam.cpu().numpy(), lo)
    b = buf.cpu().numpy()
    ev = rel(b[:, :n].T, Vo)
    print(f"[parity] strided: max rel lam {el.max():.3e} V {ev.max():.3e}", flush=True)
    assert el.max() <= LAM_TOL
    assert ev.max() <= VEC_TOL
    assert np.isnan(b[:, n:]).all()


@pytest.mark.parametrize("case", range(3))
def test_tiny_zeta_shift(D, orc, case):
    """3x3 problems whose middle pole has z_i ~ 1e-9 next to heavy neighbours: the
    tip b is ~1e15 times the root of eq. (secAi)."""
    from test_oracle_pins import TINY_ZETA
    d, z, rho = TINY_ZETA[case]
    compare(D, orc, np.array(d), np.array(z), rho, tag=f"tinyzeta{case}")


def test_huge_tip_between_tiny_zetas(D, orc):
    """An eigenvalue between two poles with zeta 1e-100 and 1e-120, far from both: the arrowhead
    inverse at either pole has |b| ~ 1e200-1e240 (the case that once broke the oracle's interval)."""
    d = np.array([2.0, 1.0, 0.5, 0.0, -1.0])
    z = np.array([1.0, 1e-100, 1e-120, 1.0, 0.7])
    compare(D, orc, d, z, 1.0, tag="huge tip rho>0")
    compare(D, orc, d, z, -1.0, tag="huge tip rho<0")


@pytest.mark.parametrize("n,seed,rho", [(300, 50, 1.0), (777, 51, -2.0)])
def test_zeta_spanning_150_decades(D, orc, n, seed, rho):
    """|z_j| = 10^U(-150, 0) with random signs, as the merges of a divide and conquer produce:
    many eigenvalues within 1e-300 of their poles, and shift poles whose zeta is tiny."""
    rng = np.random.default_rng(seed)
    d, _, _ = W.uniform(n, seed)
    z = 10.0 ** rng.uniform(-150, 0, n) * rng.choice([-1.0, 1.0], n)
    compare(D, orc, d, z, rho, tag=f"zeta 1e-150..1 seed {seed}")


def test_config_graded_4096(D, orc):
    """Graded/clustered matrix at its full size (n = 4096, every 64th pair of poles at a
    relative gap of 1e-10): every eigenpair against the oracle, element by element."""
    r, *_ = compare(D, orc, *W.graded(4096, 1), tag="graded4096")
    assert r.stats_dict()["polished"] >= 1


def test_config_n32768_sampled(D, orc):
    """n = 32768 with the full V (8.6 GB), solved as the benchmark solves it (default options,
    one launch sequence).  Sampled eigenpairs against the oracle to the parity bar; for every
    eigenpair: strict ordering and interlacing (eq. interlace), unit norm, and the residual
    (D - lambda I) v + rho z (z^T v) = 0 relative to ||A||."""
    import torch
    n = 32768
    d, z, rho = W.uniform(n, 2, zscale=1.0 / math.sqrt(n))
    print(f"[parity] n32768 full V", flush=True)
    r = D.eig(d, z, rho, opts=D.opts(root=1), want_stats=True)
    lam = r.lam.cpu().numpy()
    st = r.stats_dict()
    print(f"[parity] n32768 stats {st}", flush=True)
    assert np.all(np.diff(lam) < 0)
    assert lam[0] > d[0] and np.all(lam[1:] >= d[1:]) and np.all(lam[1:] <= d[:-1])

    # sample: the ends, the middle, the smallest relative gaps, the smallest |lambda|, random
    gap = np.minimum(np.abs(np.diff(lam, prepend=np.inf)), np.abs(np.diff(lam, append=-np.inf)))
    rng = np.random.default_rng(77)
    ks = np.unique(np.concatenate([
        [0, 1, 2, n // 2, n - 2, n - 1],
        np.argsort(gap / np.abs(lam))[:16],
        np.argsort(np.abs(lam))[:8],
        rng.choice(n, 40, replace=False)])).astype(np.int64)
    lo, Vo, dgs = orc.eig_some(d, z, rho, ks, vectors=True)
    ties, em, ex = check_repr(d, z, rho, r.shift_idx.cpu().numpy()[ks], r.mu.cpu().numpy()[ks],
                              r.xnorm.cpu().numpy()[ks], dgs, ks=ks)
    print(f"[parity] n32768 sample: {ties} ties, max rel mu {em:.3e} ||x|| {ex:.3e}", flush=True)
    Vt = r.V.t()                                          # rows = eigenvectors
    Vs = Vt[torch.as_tensor(ks, device=Vt.device)].cpu().numpy().T
    el = rel(lam[ks], lo)
    ev = rel(Vs, Vo)
    print(f"[parity] n32768 sample {ks.size}: max rel lam {el.max():.3e} V {ev.max():.3e}", flush=True)
    assert el.max() <= LAM_TOL, (ks[np.argmax(el)], el.max())
    assert ev.max() <= VEC_TOL, (np.unravel_index(np.argmax(ev), ev.shape), ev.max())

    # properties of every eigenpair, checked on the device in column chunks
    dd = torch.as_tensor(d, device=Vt.device)
    zz = torch.as_tensor(z, device=Vt.device)
    anorm = float(np.max(np.abs(d)) + abs(rho) * np.dot(z, z))
    worst_norm = 0.0
    worst_res = 0.0
    for k0 in range(0, n, 4096):
        blk = Vt[k0:k0 + 4096]
        lb = r.lam[k0:k0 + 4096]
        worst_norm = max(worst_norm, float((torch.linalg.vector_norm(blk, dim=1) - 1.0).abs().max()))
        res = blk * (dd[None, :] - lb[:, None]) + rho * (blk @ zz)[:, None] * zz[None, :]
        worst_res = max(worst_res, float(res.abs().max()) / anorm)
        del res
    print(f"[parity] n32768 all pairs: max | ||v|| - 1 | {worst_norm:.3e} max residual {worst_res:.3e}",
          flush=True)
    assert worst_norm <= 1e-13
    # the residual's own rounding: the length-n product z^T v alone may round by n*u*||z||*||v||
    assert worst_res <= 1e-12


@pytest.mark.parametrize("split,wps,mp", [(1, 0, 0), (3, 6, 2), (5, 8, 3), (16, 8, 2), (12, 4, 4), (8, 6, 1)])
def test_launch_shapes_keep_parity(D, orc, split, wps, mp):
    """Every split W (waves per 64-eigenvalue block, powers of two or not), register budget and
    pass budget (1: every root continues in k_fix) gives the oracle's eigenpairs."""
    r, *_ = compare(D, orc, *W.uniform(1000, 7), opts=D.opts(split=split, waves_per_simd=wps, main_passes=mp),
                    tag=f"W{split}/occ{wps}/mp{mp}")
    if mp == 1:
        assert r.stats_dict()["continued"] > 500


@pytest.mark.parametrize("n", [3000, 9000])
def test_single_solve_graph_capture(D, n):
    """dpr1_eig enqueues kernels only (no host sync, no memset): captured in a HIP graph, every
    replay reproduces the eager solve bit for bit, with other eager solves in between.  At
    n = 9000 the solve forks the first half's eigenvector write to the library's second stream
    and joins it back, so the graph holds the fork and the join."""
    import torch
    d, z, rho = W.uniform(n, 33)
    dd = torch.as_tensor(d, device="cuda")
    zz = torch.as_tensor(z, device="cuda")

    def buffers():
        return (torch.empty(n, dtype=torch.float64, device="cuda"),
                torch.empty((n, n), dtype=torch.float64, device="cuda")[:, :n],
                torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
                torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(1, dtype=torch.int32, device="cuda"))

    out, out2 = buffers(), buffers()
    work = torch.empty(D.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    work2 = torch.empty_like(work)
    D.eig(dd, zz, rho, out=out, work=work, check=False)
    torch.cuda.synchronize()
    ref = [t.clone() for t in out]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            D.eig(dd, zz, rho, out=out, work=work, check=False)
    for rep in range(3):
        for t in out:
            t.zero_()
        D.eig(dd, zz, 0.5 * rho, out=out2, work=work2, check=False)     # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert torch.equal(a, b), rep
        assert int(out[5].item()) == 0


def test_extreme_range_is_exact_or_reported(D, orc):
    """300 problems at the edges of the range (workloads.extreme: poles over 20 decades or 1e-14
    apart, |z_j| = 10^U(-150, 0), |rho| 1e-8..1e8): each is within the parity bar of the oracle
    element by element (eigenvalues, eigenvectors, shifted representation), or reported with
    DPR1_INFO_RANGE for a cause the oracle confirms (parity_util.range_cause); never NaN with
    info 0, never a report without a cause, never a missed report."""
    ok = reported = 0
    for seed in range(300):
        d, z, rho = W.extreme(seed)
        r = D.eig(d, z, rho, check=False)
        info = int(r.info.item())
        lo, Vo, dg = orc.eig(d, z, rho, diags=True)
        cause = range_cause(d, z, dg)
        if info == 5:
            assert cause is not None, (seed, "reported without a cause")
            reported += 1
            continue
        assert info == 0, (seed, info)
        assert cause is None or cause.endswith("tip b beyond binary64"), (seed, cause)
        lam = r.lam.cpu().numpy()
        V = r.V.cpu().numpy()
        assert np.max(rel(lam, lo)) <= LAM_TOL, seed
        assert np.max(rel(V, Vo)) <= VEC_TOL, (seed, np.max(rel(V, Vo)))
        check_repr(d, z, rho, r.shift_idx.cpu().numpy(), r.mu.cpu().numpy(), r.xnorm.cpu().numpy(), dg)
        ok += 1
    print(f"[parity] extreme range: {ok} within the bar, {reported} reported", flush=True)


def test_overlapped_write_matches_sequential(D):
    """The overlapped eigenvector write (vwrite = 2, 3 and 8: that many chunks, n >= 8192) and the
    sequential one (vwrite = 1 and the default 0) give the same outputs bit for bit, also with
    rho < 0 and a padded leading dimension."""
    import torch
    for n, rho, pad in ((8192, 1.0, 0), (10000, -0.5, 3)):
        d, z, _ = W.uniform(n, 61)
        print(f"[parity] overlap vs sequential n={n} rho={rho} pad={pad}", flush=True)
        outs = []
        for vw in (1, 0, 2, 3, 8):
            # outputs poisoned first: a fresh allocation may hold the previous solve's results
            o = (torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                 torch.full((n, n + pad), float("nan"), dtype=torch.float64, device="cuda")[:, :n],
                 torch.full((n,), -1, dtype=torch.int32, device="cuda"),
                 torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                 torch.full((n,), float("nan"), dtype=torch.float64, device="cuda"),
                 torch.full((1,), -1, dtype=torch.int32, device="cuda"))
            r = D.eig(d, z, rho, opts=D.opts(vwrite=vw), out=o)
            torch.cuda.synchronize()
            assert not torch.isnan(r.V).any() and not torch.isnan(r.lam).any()
            outs.append([r.lam.cpu(), r.V.cpu(), r.shift_idx.cpu(), r.mu.cpu(), r.xnorm.cpu()])
        for o in outs[1:]:
            for a, b in zip(outs[0], o):
                assert torch.equal(a, b)


def _sampled_columns(D, V_t, ks):
    """Columns ks of a [n, n] column-major V (given as V.t(), rows = eigenvectors) on the host."""
    import torch
    return V_t[torch.as_tensor(ks, device=V_t.device)].cpu().numpy().T


def test_index_range_beyond_2_32(D, orc):
    """n = 70000 with the full V (39 GB): element indices k ldv + j pass 2^31 from column 30679 on
    and 2^32 from column 61356 on, so every V address must be formed in 64 bits.  Sampled eigenpairs
    (the first and last columns, both sides of each boundary, random ones) against the oracle to
    the parity bar, for rho > 0 and for rho < 0 (reversed positions and columns)."""
    import torch
    n = 70000
    d, z, rho = W.uniform(n, 23, zscale=1.0 / math.sqrt(n))
    rng = np.random.default_rng(5)
    ks = np.unique(np.concatenate([[0, 1, 30678, 30679, 61355, 61356, n - 2, n - 1],
                                   rng.choice(n, 12, replace=False)])).astype(np.int64)
    for sgn in (1.0, -1.0):
        print(f"[parity] n={n} full V, rho sign {sgn:+.0f}", flush=True)
        r = D.eig(d, z, sgn * rho)
        lam = r.lam.cpu().numpy()
        if sgn > 0:
            lo, Vo, _ = orc.eig_some(d, z, rho, ks, vectors=True)
        else:
            # Sec. 1: D + rho z z^T with rho < 0 is minus the problem (-d reversed, z reversed, -rho);
            # its eigenpair n-1-k gives lambda_k negated and v_k reversed and negated (the oracle's
            # own convention for rho < 0)
            lm, Vm, _ = orc.eig_some(-d[::-1], z[::-1], rho, n - 1 - ks, vectors=True)
            lo, Vo = -lm, -Vm[::-1, :]
        Vs = _sampled_columns(D, r.V.t(), ks)
        el, ev = rel(lam[ks], lo), rel(Vs, Vo)
        print(f"[parity] n={n} rho sign {sgn:+.0f}: max rel lam {el.max():.3e} V {ev.max():.3e}", flush=True)
        assert el.max() <= LAM_TOL, (ks[np.argmax(el)], el.max())
        assert ev.max() <= VEC_TOL, (np.unravel_index(np.argmax(ev), ev.shape), ev.max())
        del r
        torch.cuda.empty_cache()


def test_batched_offsets_beyond_2_32(D, orc):
    """A batch of 16 problems of order 17000: the packed V holds 4.6e9 elements (37 GB), so the
    later problems' blocks start past 2^32.  The last eigenpairs of the first, a middle and the
    last problem, and a few random ones of each, against the oracle element by element."""
    import torch
    nb, n = 16, 17000
    d2, z2, rho2 = W.uniform_batch(nb, n, 29)
    z2 = z2 / math.sqrt(n)
    offs = np.arange(nb + 1, dtype=np.int64) * n
    print(f"[parity] batch {nb} x n={n}: V {nb * n * n * 8 / 1e9:.1f} GB", flush=True)
    b = D.eig_batched(d2.reshape(-1), z2.reshape(-1), rho2, offs)
    lam_all = b.lam.cpu().numpy()
    rng = np.random.default_rng(9)
    for p in (0, nb // 2, nb - 1):
        ks = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 6, replace=False)])).astype(np.int64)
        lo, Vo, _ = orc.eig_some(d2[p], z2[p], rho2[p], ks, vectors=True)
        Vs = _sampled_columns(D, b.vblock(p).t(), ks)
        el, ev = rel(lam_all[p * n + ks], lo), rel(Vs, Vo)
        print(f"[parity] batch problem {p} (V offset {p * n * n}): max rel lam {el.max():.3e} V {ev.max():.3e}",
              flush=True)
        assert el.max() <= LAM_TOL and ev.max() <= VEC_TOL, (p, el.max(), ev.max())
    del b
    torch.cuda.empty_cache()
