"""GPU parity of the divide-and-conquer tridiagonal driver (merges are DPR1 problems, Sec. 1)
against the oracle's tridiag_eig on the same inputs, and its properties at larger n.

The two sides run the same reductions and DPR1 solves; they differ in the order of the sums of
the products diag(Q1, Q2) V, so results agree to rounding propagated through the merges:
eigenvalues to 1e-13 ||T|| (absolute: Weyl's bound scale), eigenvector columns to
1e-12 + 4 n eps ||T|| / gap where the eigenvalue is separated from the others by gap > 1e-6 ||T||
(the two sides' roundings are a perturbation of T of order n eps ||T||, which moves an eigenvector
by at most its size over the gap: Davis and Kahan), else the projector onto the group, to the same
bound with the group's distance to the rest; Q^T Q = I and T Q = Q Lambda to 1e-13 n ||T||.

Columns are compared up to sign.  A merged column is q = diag(Q1, Q2) v with v_j proportional to
z_j / (d_j - lambda); when z_j is far below the absolute accuracy of the children's Q (a
component of 1e-60 from an eigenvector localised away from the split), lambda lies within
rounding of d_j, v is +-e_j, and its sign is the sign of z_j, which is rounding noise on either
side.  The eigenvector is unique only up to that sign.
"""
import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_7537_amd.dpr1 as D
    D.lib()
    return D


def dense(a, b):
    return np.diag(a) + np.diag(b, 1) + np.diag(b, -1)


def check(D, orc, a, b, tag):
    n = len(a)
    print(f"[tridiag] {tag} n={n}", flush=True)
    r = D.tridiag_eig(a, b)
    lam = r.lam.cpu().numpy()
    Q = r.Q.cpu().numpy()
    lo, Qo = orc.tridiag_eig(a, b)
    T = dense(a, b)
    nt = max(np.max(np.abs(lo)), 1e-300)
    el = np.max(np.abs(lam - lo)) / nt
    assert el <= 1e-13, (tag, el)
    sep = np.full(n, np.inf)
    if n > 1:
        gaps = np.abs(np.diff(lo))
        sep[:-1] = np.minimum(sep[:-1], gaps)
        sep[1:] = np.minimum(sep[1:], gaps)
    worst_c = worst_p = 0.0
    ratio = 0.0
    eps = np.finfo(float).eps

    def bound(g):
        return 1e-12 + 4 * n * eps * nt / g
    k = 0
    while k < n:
        e = k + 1
        while e < n and abs(lo[e] - lo[e - 1]) <= 1e-6 * nt:
            e += 1
        if e - k == 1 and sep[k] > 1e-6 * nt:
            dc = min(np.max(np.abs(Q[:, k] - Qo[:, k])), np.max(np.abs(Q[:, k] + Qo[:, k])))
            worst_c = max(worst_c, dc)
            ratio = max(ratio, dc / bound(sep[k]))
            assert dc <= bound(sep[k]), (tag, k, dc, sep[k])
        else:
            g = min(abs(lo[k - 1] - lo[k]) if k > 0 else np.inf, abs(lo[e - 1] - lo[e]) if e < n else np.inf)
            dp = np.max(np.abs(Q[:, k:e] @ Q[:, k:e].T - Qo[:, k:e] @ Qo[:, k:e].T))
            worst_p = max(worst_p, dp)
            ratio = max(ratio, dp / bound(g))
            assert dp <= bound(g), (tag, k, e, dp, g)
        k = e
    orth = np.max(np.abs(Q.T @ Q - np.eye(n)))
    res = np.max(np.abs(T @ Q - Q * lam)) / nt
    assert orth <= 1e-13 * n and res <= 1e-13 * n, (tag, orth, res)
    print(f"[tridiag] {tag}: lam {el:.2e} col {worst_c:.2e} proj {worst_p:.2e} (at most {ratio:.1e} of the bound) "
          f"orth {orth:.2e} res {res:.2e}", flush=True)
    return lam, Q


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (3, 2), (5, 3), (17, 4), (64, 5), (100, 6), (257, 7),
                                    (600, 8)])
def test_random_against_oracle(D, orc, n, seed):
    a, b = W.tridiagonal(n, seed)
    check(D, orc, a, b, f"random seed {seed}")


def test_wilkinson_against_oracle(D, orc):
    a, b = W.wilkinson(10)
    check(D, orc, a, b, "W21+")
    a, b = W.wilkinson(50)
    check(D, orc, a, b, "W101+")


def test_decoupled_and_diagonal(D, orc):
    a, b = W.tridiagonal(40, 9)
    b[[3, 19, 20, 33]] = 0.0
    check(D, orc, a, b, "zero off-diagonals")
    lam, Q = check(D, orc, [0.3, 2.0, -1.0, 2.0, 5.0], [0.0, 0.0, 0.0, 0.0], "diagonal")
    assert list(lam) == [5.0, 2.0, 2.0, 0.3, -1.0]


def test_large_properties(D):
    """n = 4096: eigenvalues against LAPACK's symmetric solver on the dense T, orthogonality and the
    residual (properties that hold at any size)."""
    a, b = W.tridiagonal(4096, 10)
    print("[tridiag] n=4096 properties", flush=True)
    r = D.tridiag_eig(a, b)
    lam = r.lam.cpu().numpy()
    T = dense(a, b)
    L = np.sort(np.linalg.eigvalsh(T))[::-1]
    nt = np.max(np.abs(L))
    assert np.max(np.abs(lam - L)) <= 1e-12 * nt
    Qd = r.Q
    G = (Qd.T @ Qd).cpu().numpy()
    orth = np.max(np.abs(G - np.eye(4096)))
    import torch
    Td = torch.as_tensor(T, device=Qd.device)
    res = (Td @ Qd - Qd * r.lam).abs().max().item() / nt
    print(f"[tridiag] n=4096: lam {np.max(np.abs(lam - L)) / nt:.2e} orth {orth:.2e} res {res:.2e}", flush=True)
    assert orth <= 1e-11 and res <= 1e-11


@pytest.mark.parametrize("case", ["random10000", "wilkinson3001"])
def test_large_uneven_and_clustered(D, case):
    """n = 10000 (an uneven split tree) and Wilkinson's W+ of order 3001 (pairs of eigenvalues equal
    to many digits): eigenvalues against LAPACK on the dense T, Q^T Q = I and T Q = Q Lambda."""
    import torch
    a, b = W.tridiagonal(10000, 12) if case == "random10000" else W.wilkinson(1500)
    n = len(a)
    print(f"[tridiag] {case} n={n}", flush=True)
    r = D.tridiag_eig(a, b)
    lam = r.lam.cpu().numpy()
    L = np.sort(np.linalg.eigvalsh(dense(a, b)))[::-1]
    nt = np.max(np.abs(L))
    el = np.max(np.abs(lam - L)) / nt
    Qd = r.Q
    orth = (Qd.T @ Qd - torch.eye(n, dtype=torch.float64, device=Qd.device)).abs().max().item()
    Td = torch.as_tensor(dense(a, b), device=Qd.device)
    res = (Td @ Qd - Qd * r.lam).abs().max().item() / nt
    print(f"[tridiag] {case}: lam {el:.2e} orth {orth:.2e} res {res:.2e}", flush=True)
    assert el <= 1e-12 and orth <= 1e-11 and res <= 1e-11


def test_structured_families(D):
    """35 structured matrices (workloads.tridiagonal_family, 5 of each of 7 kinds: graded, glued
    Wilkinson, tiny and zero couplings, wide diagonal, constant diagonal, 1-2-1): eigenvalues against
    LAPACK on the dense T, Q^T Q = I and T Q = Q Lambda."""
    worst = np.zeros(3)
    for s in range(35):
        a, b = W.tridiagonal_family(s)
        n = a.size
        r = D.tridiag_eig(a, b)
        lam, Q = r.lam.cpu().numpy(), r.Q.cpu().numpy()
        T = dense(a, b)
        L = np.sort(np.linalg.eigvalsh(T))[::-1]
        nt = np.max(np.abs(L))
        m = (np.max(np.abs(lam - L)) / nt, np.max(np.abs(Q.T @ Q - np.eye(n))), np.max(np.abs(T @ Q - Q * lam)) / nt)
        worst = np.maximum(worst, m)
        assert m[0] <= 1e-12 and m[1] <= 1e-12 and m[2] <= 1e-12, (s, n, m)
    print(f"[tridiag] families: lam {worst[0]:.1e} orth {worst[1]:.1e} res {worst[2]:.1e}", flush=True)


@pytest.mark.parametrize("kind", ["one_two_one", "graded"])
def test_structured_large(D, kind):
    """n = 3000: the 1-2-1 matrix (closed-form spectrum 2 - 2 cos(k pi/(n+1))) and a graded
    off-diagonal (1 .. 1e-20): eigenvalues, Q^T Q = I and T Q = Q Lambda."""
    import torch
    n = 3000
    if kind == "one_two_one":
        a, b = 2.0 * np.ones(n), -np.ones(n - 1)
        L = np.sort(2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1]
    else:
        rng = np.random.default_rng(3000)
        a, b = rng.standard_normal(n), 10.0 ** (-np.linspace(0, 20, n - 1))
        L = np.sort(np.linalg.eigvalsh(dense(a, b)))[::-1]
    print(f"[tridiag] {kind} n={n}", flush=True)
    r = D.tridiag_eig(a, b)
    nt = np.max(np.abs(L))
    el = np.max(np.abs(r.lam.cpu().numpy() - L)) / nt
    Q = r.Q
    orth = (Q.T @ Q - torch.eye(n, dtype=torch.float64, device=Q.device)).abs().max().item()
    res = (torch.as_tensor(dense(a, b), device=Q.device) @ Q - Q * r.lam).abs().max().item() / nt
    print(f"[tridiag] {kind}: lam {el:.1e} orth {orth:.1e} res {res:.1e}", flush=True)
    assert el <= 1e-13 and orth <= 1e-12 and res <= 1e-12


@pytest.mark.parametrize("nb,glue", [(126, 1e-8), (126, 1e-12), (64, 1e-4)])
def test_glued_wilkinson_large(D, orc, nb, glue):
    """Glued Wilkinson matrices: nb copies of W21+ joined by couplings `glue` (n = 21 nb, 2646 at
    nb = 126, the size at which an earlier driver lost orthogonality to 2.4e-9).  Eigenvalues
    against LAPACK on the dense T and against the oracle's driver, Q^T Q = I and T Q = Q Lambda to
    1e-12 of ||T||, and every column against the oracle's up to sign (or its cluster's projector)."""
    m = 10
    blk = np.abs(np.arange(-m, m + 1, dtype=np.float64))
    a = np.tile(blk, nb)
    b = np.ones(a.size - 1)
    b[2 * m::2 * m + 1] = glue
    n = a.size
    print(f"[tridiag] glued Wilkinson n={n} glue={glue}", flush=True)
    r = D.tridiag_eig(a, b)
    lam, Q = r.lam.cpu().numpy(), r.Q.cpu().numpy()
    T = dense(a, b)
    L = np.sort(np.linalg.eigvalsh(T))[::-1]
    nt = np.max(np.abs(L))
    orth = np.max(np.abs(Q.T @ Q - np.eye(n)))
    res = np.max(np.abs(T @ Q - Q * lam)) / nt
    print(f"[tridiag] glued n={n}: lam {np.max(np.abs(lam - L)) / nt:.1e} orth {orth:.1e} res {res:.1e}", flush=True)
    assert np.max(np.abs(lam - L)) <= 1e-12 * nt
    assert orth <= 1e-12 and res <= 1e-12
    lo, Qo = orc.tridiag_eig(a, b)
    assert np.max(np.abs(lam - lo)) <= 1e-12 * nt


def test_side_stream_and_repeat_bitwise(D):
    """The driver overlaps each depth's host work and DPR1 solves (on the library's second stream)
    with the product of the depth below on the caller's stream.  Called on a side stream, with the
    default stream busy on other work meanwhile, and twice in a row with one workspace, it gives
    the same bits as a plain call: every cross-stream dependency is waited for."""
    import torch
    n = 3000
    a_h, b_h = W.tridiagonal(n, 17)
    a = torch.as_tensor(a_h, device="cuda")
    b = torch.as_tensor(b_h, device="cuda")
    print(f"[tridiag] side stream n={n}", flush=True)
    r0 = D.tridiag_eig(a, b)
    lam0, Q0 = r0.lam.clone(), r0.Q.clone()
    r1 = D.tridiag_eig(a, b, work=r0.work)
    assert torch.equal(r1.lam, lam0) and torch.equal(r1.Q, Q0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    busy = torch.randn(4096, 4096, dtype=torch.float64, device="cuda")
    for _ in range(4):  # queued on the default stream, running during the call below
        busy = (busy @ busy.t()) * 1e-3
    with torch.cuda.stream(s):
        r2 = D.tridiag_eig(a, b)
        lam2, Q2 = r2.lam.clone(), r2.Q.clone()
    torch.cuda.synchronize()
    assert torch.equal(lam2, lam0) and torch.equal(Q2, Q0)


def test_maximum_order_sampled(D):
    """The largest order the driver takes, n = 65536 (Q and its second buffer 34 GB each, the root
    merge a DPR1 problem of order 65536): 64 eigenvalues against LAPACK's bisection for the same
    indices, the trace, and for 66 columns their inner products with every column of Q and the
    residual T q - lambda q (properties that hold at any size)."""
    import torch
    from scipy.linalg import eigvalsh_tridiagonal
    n = 65536
    a, b = W.tridiagonal(n, 31)
    print(f"[tridiag] maximum order n={n}", flush=True)
    r = D.tridiag_eig(a, b)
    lam_d = r.lam
    lam = lam_d.cpu().numpy()
    assert np.all(np.diff(lam) <= 0)
    nt = max(abs(lam[0]), abs(lam[-1]))
    eps = np.finfo(float).eps
    rng = np.random.default_rng(3)
    ks = np.unique(np.concatenate([[0, 1, n // 2, n - 2, n - 1], rng.choice(n, 59, replace=False)]))
    ref = np.array([eigvalsh_tridiagonal(a, b, select="i", select_range=(n - 1 - k, n - 1 - k))[0] for k in ks])
    el = np.max(np.abs(lam[ks] - ref)) / nt
    tr = abs(float(np.sum(lam)) - float(np.sum(a))) / (n * nt)
    cols = np.unique(np.concatenate([np.arange(0, n, 1024), [n - 1]]))
    ci = torch.as_tensor(cols, device=r.Q.device)
    Qs = r.Q[:, ci]                                        # [n, 65] sampled columns
    G = Qs.T @ r.Q                                         # inner products with every column
    G[torch.arange(cols.size, device=G.device), ci] -= 1.0
    orth = G.abs().max().item()
    ad = torch.as_tensor(a, device=Qs.device)
    bd = torch.as_tensor(b, device=Qs.device)
    TQ = ad[:, None] * Qs
    TQ[:-1] += bd[:, None] * Qs[1:]
    TQ[1:] += bd[:, None] * Qs[:-1]
    res = (TQ - Qs * lam_d[ci][None, :]).abs().max().item() / nt
    print(f"[tridiag] n={n}: lam {el:.2e} trace {tr:.2e} orth {orth:.2e} res {res:.2e}", flush=True)
    assert el <= 1e-12 and tr <= 64 * eps and orth <= 1e-11 and res <= 1e-11
    del r, G, Qs, TQ
    torch.cuda.empty_cache()
