"""GPU reverse mode (FP64 MFMA GEMMs + epilogues) against the oracle's dense backward,
finite differences, and the autograd wrappers."""
import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_7537_amd.dpr1 as D
    D.lib()
    return D


def scales(V, lam, lb, Vb, z, rho):
    """Magnitudes |V||X||V|^T (diag), rho |V|(|X|+|X|^T)|y|, |y|^T|X||y| for the tolerances, with
    |X| = |F| o (|V|^T |V_bar|) off the diagonal: the rounding error of the product V^T V_bar is
    bounded by n eps times the product of the magnitudes, which can exceed |V^T V_bar| where the
    sum cancels (standard error analysis of inner products)."""
    n = lam.size
    gap = lam[None, :] - lam[:, None]
    np.fill_diagonal(gap, 1.0)
    Pa = np.abs(V).T @ np.abs(Vb) if Vb is not None else np.zeros((n, n))
    Xa = Pa / np.abs(gap)
    np.fill_diagonal(Xa, np.abs(lb) if lb is not None else 0.0)
    Va = np.abs(V)
    y = np.abs(V.T @ z)
    Md = np.sum((Va @ Xa) * Va, axis=1)
    Mz = abs(rho) * Va @ ((Xa + Xa.T) @ y)
    Mr = y @ Xa @ y
    return Md, Mz, Mr


def gpu_backward(D, d, z, rho, lb, Vb):
    import torch
    n = len(d)
    r = D.eig(d, z, rho)
    Vs = r.V.t().contiguous()
    dt = torch.as_tensor(d, device="cuda").view(1, n)
    zt = torch.as_tensor(z, device="cuda").view(1, n)
    rt = torch.tensor([rho], dtype=torch.float64, device="cuda")
    lbt = torch.as_tensor(lb, device="cuda").view(1, n) if lb is not None else None
    Vbt = torch.as_tensor(np.asfortranarray(Vb).T.copy(), device="cuda") if Vb is not None else None
    db, zb, rb = D.backward_batched(dt, zt, rt, r.shift_idx.view(1, n), r.mu.view(1, n), r.xnorm.view(1, n),
                                    Vs, lbt, Vbt)
    return db.cpu().numpy()[0], zb.cpu().numpy()[0], float(rb.cpu().numpy()[0])


@pytest.mark.parametrize("n,seed", [(16, 5), (64, 1), (100, 2), (130, 3), (257, 4)])
def test_backward_vs_oracle(D, orc, n, seed):
    d, z, rho = W.uniform(n, seed)
    rng = np.random.default_rng(seed + 10)
    lb = rng.standard_normal(n)
    Vb = rng.standard_normal((n, n))
    lo, Vo, dg = orc.eig(d, z, rho, diags=True)
    db_o, zb_o, rb_o = orc.backward(d, z, rho, [x["sigma"] for x in dg], [x["mu"] for x in dg], Vo,
                                    lam_bar=lb, V_bar=Vb)
    db, zb, rb = gpu_backward(D, d, z, rho, lb, Vb)
    Md, Mz, Mr = scales(Vo, lo, lb, Vb, z, rho)
    ed = np.max(np.abs(db - db_o) / Md)
    ez = np.max(np.abs(zb - zb_o) / Mz)
    er = abs(rb - rb_o) / Mr
    print(f"[backward] n={n}: d {ed:.2e} z {ez:.2e} rho {er:.2e} (relative to magnitude sums)", flush=True)
    tol = 64 * n * EPS
    assert ed <= tol and ez <= tol and er <= tol


def test_backward_eigenvalue_part_only(D, orc):
    """V_bar = None: the closed-form eigenvalue terms."""
    d, z, rho = W.uniform(90, 6)
    lb = np.random.default_rng(0).standard_normal(90)
    lo, Vo, dg = orc.eig(d, z, rho, diags=True)
    xn = np.array([x["xnorm"] for x in dg])
    db, zb, rb = gpu_backward(D, d, z, rho, lb, None)
    np.testing.assert_allclose(db, (Vo ** 2) @ lb, rtol=1e-12, atol=1e-14 * np.max(np.abs(lb)))
    assert rb == pytest.approx(np.sum(lb / (rho * xn) ** 2), rel=1e-12)
    np.testing.assert_allclose(zb, -2 * Vo @ (lb / xn), rtol=1e-11, atol=1e-13 * np.max(np.abs(zb)))


def test_finite_differences_gpu(D):
    """Central differences (h = 1e-6) of the GPU forward vs the GPU adjoint, n = 16 (seed 5)."""
    d, z, rho = W.uniform(16, 5)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(16)
    Wm = rng.standard_normal((16, 16))

    def loss(d_, z_, r_):
        r = D.eig(d_, z_, r_)
        return float(np.dot(w, r.lam.cpu().numpy()) + np.sum(Wm * r.V.cpu().numpy()))

    db, zb, rb = gpu_backward(D, d, z, rho, w, Wm)
    h = 1e-6
    fd_d = np.array([(loss(d + h * e, z, rho) - loss(d - h * e, z, rho)) / (2 * h) for e in np.eye(16)])
    fd_z = np.array([(loss(d, z + h * e, rho) - loss(d, z - h * e, rho)) / (2 * h) for e in np.eye(16)])
    fd_r = (loss(d, z, rho + h) - loss(d, z, rho - h)) / (2 * h)
    scale = max(np.max(np.abs(db)), np.max(np.abs(zb)), abs(rb))
    print(f"[backward] FD: d {np.max(np.abs(fd_d - db)) / scale:.2e} z {np.max(np.abs(fd_z - zb)) / scale:.2e} "
          f"rho {abs(fd_r - rb) / scale:.2e}", flush=True)
    assert np.max(np.abs(fd_d - db)) < 1e-6 * scale
    assert np.max(np.abs(fd_z - zb)) < 1e-6 * scale
    assert abs(fd_r - rb) < 1e-6 * scale


def test_autograd_single_and_batched(D):
    import torch
    d, z, rho = W.uniform(40, 9)
    rng = np.random.default_rng(9)
    w = torch.as_tensor(rng.standard_normal(40), device="cuda")
    Wm = torch.as_tensor(rng.standard_normal((40, 40)), device="cuda")
    dt = torch.as_tensor(d, device="cuda").requires_grad_()
    zt = torch.as_tensor(z, device="cuda").requires_grad_()
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda").requires_grad_()
    lam, V = D.DPR1Eig.apply(dt, zt, rt)
    L = (w * lam).sum() + (Wm * V).sum()
    gd, gz, gr = torch.autograd.grad(L, (dt, zt, rt))
    db, zb, rb = gpu_backward(D, d, z, rho, w.cpu().numpy(), Wm.cpu().numpy())
    np.testing.assert_allclose(gd.cpu().numpy(), db, rtol=0, atol=0)
    np.testing.assert_allclose(gz.cpu().numpy(), zb, rtol=0, atol=0)
    assert float(gr) == rb
    # batched: 3 problems of n = 40 must give the single-problem gradients
    dB, zB, rB = W.uniform_batch(3, 40, 11)
    dBt = torch.as_tensor(dB, device="cuda").requires_grad_()
    zBt = torch.as_tensor(zB, device="cuda").requires_grad_()
    rBt = torch.as_tensor(rB, device="cuda").requires_grad_()
    lamB, VB = D.DPR1EigBatched.apply(dBt, zBt, rBt)
    LB = (lamB * torch.arange(40, device="cuda")).sum() + VB[:, :, 0].sum()
    g = torch.autograd.grad(LB, (dBt, zBt, rBt))
    for p in range(3):
        dp = torch.as_tensor(dB[p], device="cuda").requires_grad_()
        zp = torch.as_tensor(zB[p], device="cuda").requires_grad_()
        rp = torch.tensor(rB[p], dtype=torch.float64, device="cuda").requires_grad_()
        lp, Vp = D.DPR1Eig.apply(dp, zp, rp)
        Lp = (lp * torch.arange(40, device="cuda")).sum() + Vp[:, 0].sum()
        gp = torch.autograd.grad(Lp, (dp, zp, rp))
        for a, b in zip(g, gp):
            np.testing.assert_allclose(a[p].cpu().numpy(), b.cpu().numpy(), rtol=1e-13, atol=1e-13)


def test_config_fwd_bwd_sampled(D, orc):
    """256 problems of n = 512 (seed 4): batched forward + backward; 33 problems (every 8th and the
    last) checked in full against the oracle's dense backward."""
    import torch
    nb, n = 256, 512
    dB, zB, rB = W.uniform_batch(nb, n, 4)
    rng = np.random.default_rng(104)
    w = rng.standard_normal((nb, n))
    Wcm = rng.standard_normal((nb, n, n))          # column-major blocks: Wcm[b, k, j] = V_bar_b[j, k]
    offs = np.arange(nb + 1, dtype=np.int64) * n
    b = D.Batch(offs)
    dt, zt, rt = (torch.as_tensor(x, device="cuda") for x in (dB, zB, rB))
    b.solve(dt, zt, rt)
    db, zb, rb = D.backward_batched(dt, zt, rt, b.shift_idx.view(nb, n), b.mu.view(nb, n), b.xnorm.view(nb, n),
                                    b.V, torch.as_tensor(w, device="cuda"), torch.as_tensor(Wcm, device="cuda"))
    db, zb, rb = db.cpu().numpy(), zb.cpu().numpy(), rb.cpu().numpy()
    for p in list(range(0, nb, 8)) + [nb - 1]:
        lo, Vo, dg = orc.eig(dB[p], zB[p], rB[p], diags=True)
        Vb = Wcm[p].T
        db_o, zb_o, rb_o = orc.backward(dB[p], zB[p], rB[p], [x["sigma"] for x in dg], [x["mu"] for x in dg], Vo,
                                        lam_bar=w[p], V_bar=Vb)
        Md, Mz, Mr = scales(Vo, lo, w[p], Vb, zB[p], rB[p])
        ed = np.max(np.abs(db[p] - db_o) / Md)
        ez = np.max(np.abs(zb[p] - zb_o) / Mz)
        er = abs(rb[p] - rb_o) / Mr
        print(f"[backward] batch problem {p}: d {ed:.2e} z {ez:.2e} rho {er:.2e}", flush=True)
        tol = 64 * n * EPS
        assert ed <= tol and ez <= tol and er <= tol


def gpu_backward_recomputed(D, d, z, rho, lb, Vb):
    """The adjoint with V never stored: an eigenvalues-only forward, V = NULL in the backward."""
    import torch
    n = len(d)
    r = D.eig(d, z, rho, vectors=False)
    dt = torch.as_tensor(d, device="cuda").view(1, n)
    zt = torch.as_tensor(z, device="cuda").view(1, n)
    rt = torch.tensor([rho], dtype=torch.float64, device="cuda")
    lbt = torch.as_tensor(lb, device="cuda").view(1, n) if lb is not None else None
    Vbt = torch.as_tensor(np.asfortranarray(Vb).T.copy(), device="cuda") if Vb is not None else None
    db, zb, rb = D.backward_batched(dt, zt, rt, r.shift_idx.view(1, n), r.mu.view(1, n), r.xnorm.view(1, n),
                                    None, lbt, Vbt)
    return db.cpu().numpy()[0], zb.cpu().numpy()[0], float(rb.cpu().numpy()[0])


@pytest.mark.parametrize("n,seed,rho", [(64, 21, 1.0), (257, 22, 1.0), (600, 23, -0.6), (130, 24, 5.0)])
def test_backward_with_recomputed_v(D, orc, n, seed, rho):
    """V = NULL: the GEMM tile loads rebuild v_k[j] from (z, shift, mu, ||x||); same bar as with V."""
    d, z, _ = W.uniform(n, seed)
    rng = np.random.default_rng(seed + 10)
    lb = rng.standard_normal(n)
    Vb = rng.standard_normal((n, n))
    lo, Vo, dg = orc.eig(d, z, rho, diags=True)
    # the oracle's diagnostics describe the solved problem: for rho < 0 that is the reduced one
    # (-d reversed, -rho), whose shifted pairs are the negated (sigma, mu) of the original
    sg = 1.0 if rho > 0 else -1.0
    db_o, zb_o, rb_o = orc.backward(d, z, rho, [sg * x["sigma"] for x in dg], [sg * x["mu"] for x in dg], Vo,
                                    lam_bar=lb, V_bar=Vb)
    print(f"[backward] recomputed V n={n} rho={rho}", flush=True)
    db, zb, rb = gpu_backward_recomputed(D, d, z, rho, lb, Vb)
    db_s, zb_s, rb_s = gpu_backward(D, d, z, rho, lb, Vb)
    Md, Mz, Mr = scales(Vo, lo, lb, Vb, z, rho)
    tol = 64 * n * EPS
    for got, ref in ((db, db_o), (db_s, db_o), (db, db_s)):
        assert np.max(np.abs(got - ref) / Md) <= tol
    for got, ref in ((zb, zb_o), (zb, zb_s)):
        assert np.max(np.abs(got - ref) / Mz) <= tol
    assert abs(rb - rb_o) / Mr <= tol and abs(rb - rb_s) / Mr <= tol


def test_eigenvalues_only_autograd(D):
    """DPR1EigValues (no V stored) gives the gradient of L = w^T lambda that DPR1Eig gives."""
    import torch
    d, z, rho = W.uniform(300, 31)
    w = torch.as_tensor(np.random.default_rng(31).standard_normal(300), device="cuda")
    dt = torch.as_tensor(d, device="cuda").requires_grad_()
    zt = torch.as_tensor(z, device="cuda").requires_grad_()
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda").requires_grad_()
    lam = D.DPR1EigValues.apply(dt, zt, rt)
    g1 = torch.autograd.grad((w * lam).sum(), (dt, zt, rt))
    lam2, V2 = D.DPR1Eig.apply(dt, zt, rt)
    assert torch.equal(lam, lam2)
    g2 = torch.autograd.grad((w * lam2).sum(), (dt, zt, rt))
    for a, b in zip(g1, g2):
        scale = float(b.abs().max())
        assert float((a - b).abs().max()) <= 1e-12 * scale


@pytest.mark.parametrize("n,seed,rho", [(100, 31, 1.0), (333, 32, -0.7)])
def test_single_problem_entry(D, n, seed, rho):
    """dpr1_eig_backward (one problem, rho a host number, V and V_bar with leading dimensions)
    gives the batched call's results for nb = 1 bit for bit: with V stored (also padded to
    ld = n + 5, V_bar to ld = n + 3), and with V recomputed."""
    import torch
    d, z, _ = W.uniform(n, seed)
    rng = np.random.default_rng(seed)
    r = D.eig(d, z, rho, ldv=n + 5)
    torch.cuda.synchronize()
    dd = torch.as_tensor(d, device="cuda")
    zz = torch.as_tensor(z, device="cuda")
    lb = torch.as_tensor(rng.standard_normal(n), device="cuda")
    Vb = torch.as_tensor(rng.standard_normal((n, n)), device="cuda")
    Vb_pad = torch.empty((n, n + 3), dtype=torch.float64, device="cuda")[:, :n]   # column-major, ld n + 3
    Vb_pad.copy_(Vb.t())
    Vb_cm = Vb_pad.t()                                                             # V_bar[j, k], stride (1, n + 3)
    V = r.V                                                                        # stride (1, n + 5)
    assert V.stride() == (1, n + 5) and Vb_cm.stride() == (1, n + 3)
    rho_t = torch.tensor([rho], dtype=torch.float64, device="cuda")
    for Vin in (V, None):
        ref = D.backward_batched(dd.view(1, n), zz.view(1, n), rho_t, r.shift_idx.view(1, n), r.mu.view(1, n),
                                 r.xnorm.view(1, n), V.contiguous().t().contiguous() if Vin is not None else None,
                                 lb.view(1, n), Vb.t().contiguous())
        got = D.backward(dd, zz, rho, r.shift_idx, r.mu, r.xnorm, Vin, lb, Vb_cm)
        torch.cuda.synchronize()
        print(f"[backward] single entry n={n} rho={rho} V {'stored' if Vin is not None else 'recomputed'}",
              flush=True)
        for a, b in zip(ref, got):
            assert torch.equal(a.reshape(-1), b.reshape(-1))
