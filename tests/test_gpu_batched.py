"""GPU parity of the persistent batched solver (ragged problem sizes) against the CPU oracle."""
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


def check_problem(b, orc, d, z, rho, offs, p, vectors=True):
    """Problem p of a solved batch against the oracle: returns the largest relative errors of its
    eigenvalues and eigenvector components, after asserting its shifted representation
    (shift index, mu, ||x||: parity_util.check_repr)."""
    a, e = offs[p], offs[p + 1]
    lo, Vo, dg = orc.eig(d[a:e], z[a:e], rho[p], vectors=vectors, diags=True)
    lam = b.lam[a:e].cpu().numpy()
    el = np.max(np.abs(lam - lo) / np.abs(lo))
    ev = 0.0
    if vectors:
        V = b.vblock(p).cpu().numpy()
        ev = np.max(np.abs(V - Vo) / np.abs(Vo))
    check_repr(d[a:e], z[a:e], rho[p], b.shift_idx[a:e].cpu().numpy(), b.mu[a:e].cpu().numpy(),
               b.xnorm[a:e].cpu().numpy(), dg)
    return el, ev


def test_small_mix_every_problem(D, orc):
    d, z, rho, offs = W.batched(48, 3, nmin=1, nmax=300)
    rho[::5] *= -1.0                    # some problems with rho < 0
    print(f"[batched] small mix sizes {np.diff(offs).min()}..{np.diff(offs).max()} total {offs[-1]}", flush=True)
    b = D.eig_batched(d, z, rho, offs, want_stats=True)
    worst = (0.0, 0.0)
    for p in range(48):
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        worst = (max(worst[0], el), max(worst[1], ev))
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, el, ev)
    print(f"[batched] small mix worst lam {worst[0]:.2e} V {worst[1]:.2e}", flush=True)


def test_bad_problem_is_isolated(D, orc):
    d, z, rho, offs = W.batched(6, 4, nmin=20, nmax=80)
    d[offs[2] + 3] = d[offs[2] + 4] - 1.0   # unsorted
    z[offs[4] + 1] = 0.0                     # reducible
    rho[5] = 0.0
    b = D.eig_batched(d, z, rho, offs, check=False)
    info = b.info.cpu().numpy().tolist()
    assert info == [0, 0, 1, 0, 2, 4]
    # rejected problems get defined outputs: NaN eigenvalues, in-range shift indices
    lam = b.lam.cpu().numpy()
    idx = b.shift_idx.cpu().numpy()
    for p in (2, 4, 5):
        a, e = offs[p], offs[p + 1]
        assert np.all(np.isnan(lam[a:e]))
        assert np.array_equal(idx[a:e], np.arange(e - a))
    for p in (0, 1, 3):
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL


def test_eigenvalues_only_matches_vectors_run(D):
    """Skipping V changes no other output: eigenvalues, shift indices, mu and ||x|| (also of
    polished and continued roots) are bit for bit those of the run with vectors."""
    d, z, rho, offs = W.batched(32, 6, nmin=16, nmax=600)
    o = D.opts(main_passes=2)  # leaves some roots to the cooperative kernel at these sizes
    b1 = D.eig_batched(d, z, rho, offs, vectors=True, want_stats=True, opts=o)
    b2 = D.eig_batched(d, z, rho, offs, vectors=False, opts=o)
    st = b1.stats.cpu().numpy()
    print(f"[batched] polished {st[1]} continued {st[6]}", flush=True)
    assert st[1] > 0 and st[6] > 0
    for name in ("lam", "shift_idx", "mu", "xnorm"):
        assert np.array_equal(getattr(b1, name).cpu().numpy(), getattr(b2, name).cpu().numpy()), name


def test_repeat_solve_and_graph_capture(D):
    """The planned solve is launch-only: repeat it and replay it from a HIP graph."""
    import torch
    d, z, rho, offs = W.batched(40, 7, nmin=16, nmax=400)
    b = D.Batch(offs)
    dd = torch.as_tensor(d, device="cuda")
    zz = torch.as_tensor(z, device="cuda")
    rr = torch.as_tensor(rho, device="cuda")
    b.solve(dd, zz, rr)
    torch.cuda.synchronize()
    lam0 = b.lam.clone()
    V0 = b.V.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.lam.zero_()
        with torch.cuda.graph(g, stream=s):
            b.solve(dd, zz, rr)
    for rep in range(3):
        b.lam.fill_(0.0)
        b.V.fill_(0.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.lam, lam0), rep
        assert torch.equal(b.V, V0), rep


def test_config_batched_mix_sampled(D, orc):
    """The full 2048-problem mix (sizes log-uniform in [16, 2048]): over 300 problems checked in
    full against the oracle (every 8th, the 64 largest and the 16 smallest), every eigenvalue for
    interlacing."""
    d, z, rho, offs = W.batched(2048, 3)
    print(f"[batched] mix: total n {offs[-1]}, sum n^2 {int(np.sum(np.diff(offs) ** 2))}", flush=True)
    b = D.eig_batched(d, z, rho, offs, want_stats=True)
    print(f"[batched] stats {b.stats_dict() if hasattr(b, 'stats_dict') else b.stats.cpu().tolist()}", flush=True)
    sizes = np.diff(offs)
    pick = sorted(set(range(0, 2048, 8)) | set(np.argsort(-sizes)[:64].tolist()) | set(np.argsort(sizes)[:16].tolist()))
    assert len(pick) >= 256
    worst = (0.0, 0.0)
    for p in pick:
        el, ev = check_problem(b, orc, d, z, rho, offs, int(p))
        worst = (max(worst[0], el), max(worst[1], ev))
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, sizes[p], el, ev)
    print(f"[batched] mix: {len(pick)} problems, worst lam {worst[0]:.2e} V {worst[1]:.2e}", flush=True)
    # every eigenvalue: strict interlacing with its problem's poles
    lam = b.lam.cpu().numpy()
    for p in range(2048):
        a, e = offs[p], offs[p + 1]
        inter = np.empty(2 * (e - a))
        inter[0::2], inter[1::2] = lam[a:e], d[a:e]
        assert np.all(inter[:-1] > inter[1:]), p


def test_large_and_odd_sizes(D, orc):
    """Problems above one eigenvector row tile (2048 positions) and odd sizes whose V columns
    start at every offset modulo a cache line, with both signs of rho."""
    sizes = [2100, 3000, 17, 64, 65, 2049, 1, 2, 4100, 333]
    d, z, rho, offs = W.batched(len(sizes), 8, sizes=sizes)
    rho[1::2] *= -1.0
    print(f"[batched] large/odd sizes {sizes}", flush=True)
    b = D.eig_batched(d, z, rho, offs)
    for p in range(len(sizes)):
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, sizes[p], el, ev)


def test_more_problems_than_a_grid_row(D, orc):
    """70000 tiny problems: more than 65535, the largest second grid dimension, so every
    per-problem launch must index problems along the first one."""
    rng = np.random.default_rng(21)
    sizes = rng.integers(1, 6, 70000)
    d, z, rho, offs = W.batched(len(sizes), 9, sizes=sizes)
    print(f"[batched] {len(sizes)} problems, total n {offs[-1]}", flush=True)
    b = D.eig_batched(d, z, rho, offs)
    for p in list(range(5)) + list(range(65530, 65540)) + [69999]:
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, sizes[p], el, ev)


def test_zeta_spanning_150_decades(D, orc):
    """A batch whose z spans 1e-150..1 (as divide-and-conquer merges produce): every problem
    against the oracle, both signs of rho."""
    d, _, rho, offs = W.batched(24, 60, nmin=2, nmax=400)
    rng = np.random.default_rng(60)
    z = 10.0 ** rng.uniform(-150, 0, d.size) * rng.choice([-1.0, 1.0], d.size)
    rho[::3] *= -1.0
    print(f"[batched] tiny-zeta mix total {offs[-1]}", flush=True)
    b = D.eig_batched(d, z, rho, offs)
    for p in range(24):
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, el, ev)


def test_wide_edge_batch_is_exact_or_reported(D, orc):
    """1500 edge problems in one batch (workloads.extreme_wide: poles over 60 decades or 1e-15
    apart or near 1e-300, |z_j| down to 1e-300, |rho| 1e-12..1e12): every problem is within the
    parity bar of the oracle or reported with DPR1_INFO_RANGE (never a silent failure), and the
    uniform kind is always within the bar."""
    cases = [W.extreme_wide(s) for s in range(1500)]
    sizes = np.array([c[0].size for c in cases])
    offs = np.zeros(1501, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    d = np.concatenate([c[0] for c in cases])
    z = np.concatenate([c[1] for c in cases])
    rho = np.array([c[2] for c in cases])
    print(f"[batched] wide edge batch total {offs[-1]}", flush=True)
    b = D.eig_batched(d, z, rho, offs, check=False)
    info = b.info.cpu().numpy()
    ok = reported = 0
    for p in range(1500):
        dp, zp, rp = cases[p]
        _, _, dg = orc.eig(dp, zp, rp, vectors=False, diags=True)
        cause = range_cause(dp, zp, dg)
        if info[p] == 5:
            assert p % 5 != 0, p
            assert cause is not None, (p, "reported without a cause")
            reported += 1
            continue
        assert info[p] == 0, (p, info[p])
        assert cause is None or cause.endswith("tip b beyond binary64"), (p, cause)
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, el, ev)
        ok += 1
    print(f"[batched] wide edge batch: {ok} within the bar, {reported} reported", flush=True)


def test_range_reports(D):
    """A z_j whose square is not a normal number, and two poles closer than 2^-1000, are reported."""
    r = D.eig([1.0, 0.5, 0.0], [1.0, 1e-160, 1.0], 1.0, check=False)
    assert int(r.info.item()) == 5
    r = D.eig([1.0, 2e-302, 1e-302, -1.0], [1.0, 1.0, 1.0, 1.0], 1.0, check=False)
    assert int(r.info.item()) == 5
    r = D.eig([1.0, 0.5, 0.0], [1.0, 1e-150, 1.0], 1.0, check=False)
    assert int(r.info.item()) == 0


def test_large_edge_batch(D, orc):
    """20 edge problems of 100-2000 poles in one batch (workloads.extreme_large): each within the
    parity bar element by element (eigenvalues, eigenvectors, shifted representation), or reported
    with DPR1_INFO_RANGE for a cause the oracle confirms -- never a silent failure, never a report
    without a cause, never a missed report."""
    cases = [W.extreme_large(s) for s in range(20)]
    offs = np.zeros(21, dtype=np.int64)
    offs[1:] = np.cumsum([c[0].size for c in cases])
    d = np.concatenate([c[0] for c in cases])
    z = np.concatenate([c[1] for c in cases])
    rho = np.array([c[2] for c in cases])
    print(f"[batched] large edge batch total {offs[-1]}", flush=True)
    b = D.eig_batched(d, z, rho, offs, check=False)
    info = b.info.cpu().numpy()
    ok = reported = 0
    for p in range(20):
        dp, zp, rp = cases[p]
        _, _, dg = orc.eig(dp, zp, rp, vectors=False, diags=True)
        cause = range_cause(dp, zp, dg)
        if info[p] == 5:
            assert cause is not None, (p, "reported without a cause")
            reported += 1
            continue
        assert info[p] == 0, (p, info[p])
        assert cause is None or cause.endswith("tip b beyond binary64"), (p, cause)
        el, ev = check_problem(b, orc, d, z, rho, offs, p)
        assert el <= LAM_TOL and ev <= VEC_TOL, (p, el, ev)
        ok += 1
    print(f"[batched] large edge batch: {ok} within the bar, {reported} reported", flush=True)
