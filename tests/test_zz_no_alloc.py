"""dpr1_eig_noalloc (static device scratch, no allocation) against dpr1_eig (caller's workspace).

Both calls go through the C ABI and run the same kernels on the same data, so every output is
compared to the parity bar of the project (eigenvalues 1e-13 relative, eigenvector components
1e-12 relative, shift indices exactly).  Two no-alloc calls in a row, the second on a smaller
problem, check that the shared scratch carries nothing from one call into the next."""
import numpy as np
import pytest
import torch

import paper_1405_7537_amd.dpr1 as D
from paper_1405_7537_amd import workloads as W

pytestmark = pytest.mark.gpu


def _compare(ref, got, n, vectors):
    lr, lg = ref.lam.cpu().numpy(), got.lam.cpu().numpy()
    assert np.all(np.abs(lg - lr) <= 1e-13 * np.abs(lr)), "eigenvalues"
    assert np.array_equal(ref.shift_idx.cpu().numpy(), got.shift_idx.cpu().numpy()), "shift indices"
    mr, mg = ref.mu.cpu().numpy(), got.mu.cpu().numpy()
    assert np.all(np.abs(mg - mr) <= 1e-13 * np.abs(mr)), "mu"
    xr, xg = ref.xnorm.cpu().numpy(), got.xnorm.cpu().numpy()
    assert np.all(np.abs(xg - xr) <= 1e-13 * np.abs(xr)), "||x||"
    if vectors:
        Vr, Vg = ref.V.cpu().numpy(), got.V.cpu().numpy()
        assert Vg.shape == (n, n)
        assert np.all(np.abs(Vg - Vr) <= 1e-12 * np.abs(Vr)), "eigenvectors"


@pytest.mark.parametrize("vectors", [True, False])
def test_noalloc_matches_dpr1_eig_twice(vectors):
    dev = "cuda:0"
    cases = [W.graded(4096, 1), W.uniform(1000, 7, rho=3.0)]   # second call smaller
    for (d, z, rho) in cases:
        n = d.size
        print(f"noalloc vs dpr1_eig: n={n} vectors={vectors}", flush=True)
        ref = D.eig(d, z, rho, vectors=vectors, device=dev)
        got = D.eig_noalloc(d, z, rho, vectors=vectors, device=dev)
        torch.cuda.synchronize()
        assert int(got.info.item()) == 0
        _compare(ref, got, n, vectors)


def test_noalloc_negative_rho_and_max_size():
    dev = "cuda:0"
    d, z, rho = W.uniform(D.NOALLOC_MAX_N, 2, zscale=1.0 / np.sqrt(D.NOALLOC_MAX_N))
    print(f"noalloc at the maximum size n={d.size}", flush=True)
    ref = D.eig(d, z, rho, vectors=False, device=dev)
    got = D.eig_noalloc(d, z, rho, vectors=False, device=dev)
    torch.cuda.synchronize()
    _compare(ref, got, d.size, False)
    d, z, _ = W.uniform(300, 11)
    print("noalloc with rho < 0, n=300", flush=True)
    ref = D.eig(d, z, -2.0, device=dev)
    got = D.eig_noalloc(d, z, -2.0, device=dev)
    torch.cuda.synchronize()
    _compare(ref, got, 300, True)


def test_noalloc_rejects_oversize():
    dev = "cuda:0"
    n = D.NOALLOC_MAX_N + 1
    d = torch.zeros(n, dtype=torch.float64, device=dev)
    with pytest.raises(RuntimeError, match="-1001"):
        D.eig_noalloc(d, d, 1.0, vectors=False, device=dev)
