"""Autotuned launch shapes (dpr1_autotune, dpr1_batched_autotune): the chosen settings are among the
candidates, the tuned solves keep parity with the oracle, and the cache reproduces the tuned plan."""
import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W

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


def test_autotune_single_problem(D, orc):
    d, z, rho = W.uniform(3000, 21)
    print("[tuning] single n=3000", flush=True)
    o, ms = D.autotune(d, z, rho, reps=2)
    print(f"[tuning] split {o.split} waves/SIMD {o.waves_per_simd} main_passes {o.main_passes} {ms:.3f} ms",
          flush=True)
    assert o.split in (1, 2, 4, 8, 12, 16) and o.waves_per_simd in (4, 6, 8) and o.main_passes in (2, 3)
    assert ms > 0
    r = D.eig(d, z, rho, opts=o)
    lo, Vo = orc.eig(d, z, rho)
    assert np.max(np.abs(r.lam.cpu().numpy() - lo) / np.abs(lo)) <= LAM_TOL
    assert np.max(np.abs(r.V.cpu().numpy() - Vo) / np.abs(Vo)) <= VEC_TOL


def test_autotune_chooses_the_write(D, tmp_path):
    """At n >= 8192 with eigenvectors the tuner also chooses the write (vwrite 0: after the
    eigenvalue kernel, 2: overlapped in two chunks); the cache keeps the choice, and the tuned
    solve gives the outputs of the other write mode bit for bit."""
    import torch
    from paper_1405_7537_amd import tuning as T
    n = 8192
    d, z, rho = W.uniform(n, 23)
    path = str(tmp_path / "tuning.json")
    o, entry, hit = T.tuned_opts(d, z, rho, reps=1, path=path)
    print(f"[tuning] n={n}: {entry}", flush=True)
    assert not hit and o.vwrite in (0, 2) and entry["vwrite"] == o.vwrite
    o2, entry2, hit2 = T.tuned_opts(d, z, rho, reps=1, path=path)
    assert hit2 and (o2.split, o2.waves_per_simd, o2.main_passes, o2.vwrite) == (o.split, o.waves_per_simd,
                                                                                 o.main_passes, o.vwrite)
    r = D.eig(d, z, rho, opts=o)
    other = D.opts(split=o.split, waves_per_simd=o.waves_per_simd, main_passes=o.main_passes,
                   vwrite=2 if o.vwrite == 0 else 0)
    r2 = D.eig(d, z, rho, opts=other)
    torch.cuda.synchronize()
    assert torch.equal(r.lam, r2.lam) and torch.equal(r.V, r2.V)


def test_autotune_batched_and_cache(D, orc, tmp_path):
    import torch
    from paper_1405_7537_amd import tuning as T
    d_h, z_h, rho_h, offs = W.batched(300, 22, nmin=16, nmax=700)
    dev = torch.device("cuda")
    d = torch.as_tensor(d_h, device=dev)
    z = torch.as_tensor(z_h, device=dev)
    rho = torch.as_tensor(rho_h, device=dev)
    path = str(tmp_path / "tuning.json")
    print(f"[tuning] batched 300 problems total {offs[-1]}", flush=True)
    b, entry, hit = T.tuned_batch(offs, d, z, rho, reps=2, path=path)
    print(f"[tuning] batched entry {entry} from cache {hit}", flush=True)
    assert not hit
    assert b.plan.split in (1, 2, 4, 8, 12, 16) and b.plan.opts.main_passes in (2, 3, 4)
    assert b.plan.opts.waves_per_simd in (4, 6, 8)
    b.solve(d, z, rho)
    b.check()
    for p in (0, 1, 150, 299):
        a, e = offs[p], offs[p + 1]
        lo, Vo = orc.eig(d_h[a:e], z_h[a:e], rho_h[p])
        assert np.max(np.abs(b.lam[a:e].cpu().numpy() - lo) / np.abs(lo)) <= LAM_TOL
        assert np.max(np.abs(b.vblock(p).cpu().numpy() - Vo) / np.abs(Vo)) <= VEC_TOL
    lam1 = b.lam.clone()
    V1 = b.V.clone()
    # the cache gives the same plan, hence bit-identical results
    b2, entry2, hit2 = T.tuned_batch(offs, d, z, rho, path=path)
    assert hit2 and entry2 == entry
    assert b2.plan.split == b.plan.split and b2.plan.grid == b.plan.grid
    b2.solve(d, z, rho)
    b2.check()
    assert torch.equal(b2.lam, lam1) and torch.equal(b2.V, V1)
