"""GPU parity of the front end for reducible inputs (Sec. 1): unsorted poles, repeated poles and
zero z_j, through dpr1_eig_general, against the oracle's eig_general on the same inputs.

Eigenvalues are compared element by element (relative 1e-13; a deflated pole is returned exactly).
Eigenvectors of a simple eigenvalue of the reduced problem are compared componentwise (relative
1e-12, exact zeros where the oracle has them).  Where several eigenvalues are equal the eigenspace
basis is not unique, and a reflection column has entries 1 - beta u_t^2 that cancel: for those the
projector onto the group's columns is compared instead (1e-13 absolute).  Orthonormality is
checked on the whole matrix.
"""
import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM_TOL = 1e-13
VEC_TOL = 1e-12
PROJ_TOL = 1e-13


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_7537_amd.dpr1 as D
    D.lib()
    return D


def tie_groups(lam):
    """Runs of equal eigenvalues (relative 1e-13) in a decreasing array."""
    out, s = [], 0
    for k in range(1, lam.size + 1):
        if k == lam.size or abs(lam[k] - lam[k - 1]) > LAM_TOL * max(abs(lam[k - 1]), 1e-300):
            out.append((s, k))
            s = k
    return out


def check(D, orc, d, z, rho, tag, hermitian=False):
    print(f"[general] {tag} n={len(d)} rho={rho} hermitian={hermitian}", flush=True)
    r = (D.eig_hermitian if hermitian else D.eig_general)(d, z, rho)
    lam = r.lam.cpu().numpy()
    V = r.V.cpu().numpy()
    lo, Vo = (orc.eig_hermitian if hermitian else orc.eig_general)(d, z, rho)
    den = np.where(lo == 0, 1.0, np.abs(lo))
    el = np.abs(lam - lo) / den
    assert el.max() <= LAM_TOL, (tag, int(np.argmax(el)), el.max())
    n = len(d)
    worst_v = worst_p = 0.0
    poles = set(np.asarray(d, dtype=np.float64).tolist())
    for s, e in tie_groups(lo):
        # a simple eigenvalue equal to a pole is a deflated or reflected column (not from
        # Algorithm 1): entries 1 - beta u_t^2 of a reflection cancel, so compare its projector
        if e - s == 1 and lo[s] not in poles:
            a, b = V[:, s], Vo[:, s]
            zero = b == 0
            assert np.all(a[zero] == 0), (tag, s)
            ev = np.max(np.abs(a[~zero] - b[~zero]) / np.abs(b[~zero])) if np.any(~zero) else 0.0
            worst_v = max(worst_v, ev)
            assert ev <= VEC_TOL, (tag, s, ev)
        else:
            P = V[:, s:e] @ V[:, s:e].conj().T
            Po = Vo[:, s:e] @ Vo[:, s:e].conj().T
            ep = np.max(np.abs(P - Po))
            worst_p = max(worst_p, ep)
            assert ep <= PROJ_TOL, (tag, s, e, ep)
    orth = np.max(np.abs(V.conj().T @ V - np.eye(n)))
    assert orth <= 1e-13, (tag, orth)
    print(f"[general] {tag}: lam {el.max():.2e} V {worst_v:.2e} proj {worst_p:.2e} orth {orth:.2e}", flush=True)
    return lam, V


@pytest.mark.parametrize("n,seed,rho", [(40, 0, 1.0), (300, 1, -0.8), (513, 2, 5.0), (1000, 3, 0.3)])
def test_reducible_against_oracle(D, orc, n, seed, rho):
    d, z, _ = W.reducible(n, seed, rho=rho)
    check(D, orc, d, z, rho, f"reducible seed {seed}")


def test_large_groups_and_many_zeros(D, orc):
    """A few poles repeated many times (groups of tens) and a third of z zero."""
    rng = np.random.default_rng(7)
    vals = rng.uniform(-2, 2, 12)
    d = vals[rng.integers(0, 12, 400)]
    d[:100] = rng.uniform(-2, 2, 100)
    z = rng.standard_normal(400)
    z[rng.choice(400, 130, replace=False)] = 0.0
    check(D, orc, d, z, 1.5, "large groups")


def test_degenerate_inputs(D, orc):
    # n = 1
    check(D, orc, [0.7], [2.0], -1.0, "n1")
    check(D, orc, [0.7], [0.0], 1.0, "n1 zero z")
    # all z zero: V is a permutation, lambda the sorted d
    d = np.array([0.3, -1.0, 2.0, 0.3, 0.0])
    lam, V = check(D, orc, d, np.zeros(5), 1.0, "all z zero")
    assert np.array_equal(lam, np.sort(d)[::-1])
    # all poles equal: one eigenvalue d + rho ||z||^2, the rest d
    z = np.array([1.0, -2.0, 2.0, 0.5])
    lam, V = check(D, orc, np.full(4, 0.25), z, 2.0, "one pole")
    assert abs(lam[0] - (0.25 + 2.0 * np.dot(z, z))) <= 1e-15 * lam[0]
    assert np.all(lam[1:] == 0.25)
    # a group whose z part is partly zero and a zero pole value
    check(D, orc, [0.0, 0.5, 0.0, 0.5, -0.5], [0.0, 1.0, 2.0, 0.0, 1.0], 1.0, "mixed")


def test_irreducible_input_matches_direct_solve(D, orc):
    """A strictly decreasing d with no zero z reduces to itself: the same result as dpr1_eig."""
    d, z, rho = W.uniform(700, 5)
    g = D.eig_general(d, z, rho)
    r = D.eig(d, z, rho)
    assert np.array_equal(g.lam.cpu().numpy(), r.lam.cpu().numpy())
    # V from the shifted representation: the eigenvector writer's quotient, scaled by
    # 1/(mu ||x||) instead of its internal scaled norm (a few ulps)
    ev = np.max(np.abs(g.V.cpu().numpy() - r.V.cpu().numpy()) / np.abs(r.V.cpu().numpy()))
    assert ev <= 1e-14, ev


def test_permuted_input(D, orc):
    """Permuting the input rows permutes the rows of V and leaves lambda unchanged."""
    d, z, rho = W.uniform(500, 6)
    p = np.random.default_rng(6).permutation(500)
    g = D.eig_general(d[p], z[p], rho)
    r = D.eig(d, z, rho)
    assert np.array_equal(g.lam.cpu().numpy(), r.lam.cpu().numpy())
    Vr = r.V.cpu().numpy()[p, :]
    assert np.max(np.abs(g.V.cpu().numpy() - Vr) / np.abs(Vr)) <= 1e-14
    check(D, orc, d[p], z[p], rho, "permuted")


def test_large_reducible_properties(D):
    """n = 8192 with repeated poles and zero z: orthonormality and the residual on sampled
    columns, A v = lambda v (properties that hold at any size), and the eigenvalue sum = trace."""
    import torch
    d, z, rho = W.reducible(8192, 11, rho=-0.7)
    print("[general] n=8192 properties", flush=True)
    r = D.eig_general(d, z, rho)
    lam = r.lam.cpu().numpy()
    Vd = r.V
    G = (Vd.T @ Vd).cpu().numpy()
    orth = np.max(np.abs(G - np.eye(8192)))
    assert orth <= 1e-12, orth
    idx = np.random.default_rng(11).choice(8192, 64, replace=False)
    Vs = Vd[:, torch.as_tensor(idx, device=Vd.device)].cpu().numpy()
    res = d[:, None] * Vs + rho * np.outer(z, z @ Vs) - Vs * lam[idx]
    scale = max(np.max(np.abs(d)), abs(rho) * np.dot(z, z))
    assert np.max(np.abs(res)) <= 1e-13 * scale, np.max(np.abs(res))
    tr = np.sum(d) + rho * np.dot(z, z)
    assert abs(np.sum(lam) - tr) <= 1e-11 * scale
    assert np.all(np.diff(lam) <= 0)
    print(f"[general] n=8192: orth {orth:.2e} residual {np.max(np.abs(res)) / scale:.2e}", flush=True)


def test_nonfinite_input_is_reported(D):
    r = D.eig_general([1.0, np.nan, 0.0], [1.0, 1.0, 1.0], 1.0, check=False)
    assert int(r.info.item()) == 3


def _complex_z(z, seed):
    return np.asarray(z) * np.exp(1j * np.random.default_rng(seed).uniform(0, 2 * np.pi, len(z)))


@pytest.mark.parametrize("n,seed,rho", [(40, 30, 1.0), (300, 31, -0.8), (777, 32, 2.5)])
def test_hermitian_against_oracle(D, orc, n, seed, rho):
    """Complex z with repeated poles and zero entries: the Hermitian entry point against the oracle."""
    d, z, _ = W.reducible(n, seed, rho=rho)
    check(D, orc, d, _complex_z(z, seed), rho, f"hermitian seed {seed}", hermitian=True)


def test_hermitian_degenerate(D, orc):
    check(D, orc, [0.5], [0.0 + 0.0j], 1.0, "hermitian n1 zero", hermitian=True)
    check(D, orc, [0.5], [0.3 - 0.4j], 2.0, "hermitian n1", hermitian=True)
    check(D, orc, np.full(5, -0.25), [1j, 0, -1, 0.5 + 0.5j, 2], 1.0, "hermitian one pole", hermitian=True)


def test_hermitian_real_z_is_the_real_problem(D):
    """Real z: the same eigenvalues as the real front end with |z|, and V the real V with each row
    multiplied by sign(z_j), bit for bit (the same kernels on the same |z|)."""
    d, z, rho = W.reducible(600, 33, rho=0.7)
    h = D.eig_hermitian(d, z.astype(complex), rho)
    g = D.eig_general(d, np.abs(z), rho)
    assert np.array_equal(h.lam.cpu().numpy(), g.lam.cpu().numpy())
    Vh = h.V.cpu().numpy()
    sgn = np.where(z < 0, -1.0, 1.0)
    assert np.array_equal(Vh.real, sgn[:, None] * g.V.cpu().numpy())
    assert np.all(Vh.imag == 0)


def test_hermitian_large_properties(D):
    """n = 4096 complex: V^H V = I, and A v = lambda v on sampled columns."""
    import torch
    d, z, rho = W.reducible(4096, 34, rho=1.3)
    zc = _complex_z(z, 34)
    print("[general] hermitian n=4096 properties", flush=True)
    r = D.eig_hermitian(d, zc, rho)
    lam = r.lam.cpu().numpy()
    G = (r.V.conj().T @ r.V).cpu().numpy()
    orth = np.max(np.abs(G - np.eye(4096)))
    assert orth <= 1e-12, orth
    idx = np.random.default_rng(34).choice(4096, 64, replace=False)
    Vs = r.V[:, torch.as_tensor(idx, device=r.V.device)].cpu().numpy()
    res = d[:, None] * Vs + rho * np.outer(zc, zc.conj() @ Vs) - Vs * lam[idx]
    scale = max(np.max(np.abs(d)), abs(rho) * np.sum(np.abs(zc) ** 2))
    assert np.max(np.abs(res)) <= 1e-13 * scale, np.max(np.abs(res))
    print(f"[general] hermitian n=4096: orth {orth:.2e} residual {np.max(np.abs(res)) / scale:.2e}", flush=True)


@pytest.mark.parametrize("hermitian", [False, True])
def test_zeta_spanning_150_decades(D, orc, hermitian):
    """Front end (and Hermitian case) with repeated poles, zero z_j and |z_j| spanning 1e-150..1."""
    d, z, _ = W.reducible(500, 61, rho=-1.3)
    rng = np.random.default_rng(61)
    z = np.where(z == 0, 0.0, 10.0 ** rng.uniform(-150, 0, 500) * np.sign(z))
    if hermitian:
        z = _complex_z(z, 61)
    check(D, orc, d, z, -1.3, f"tiny zeta hermitian={hermitian}", hermitian=hermitian)


def test_subnormal_square_is_deflated(D, orc):
    """The front end deflates |z_j| < 2^-511 (its square is not a normal number), as the oracle does."""
    d = np.array([0.9, 0.3, -0.2, -0.8, 0.1])
    z = np.array([1.0, 1e-160, 0.7, -3e-200, 0.4])
    lam, V = check(D, orc, d, z, 1.1, "subnormal squares")
    assert 0.3 in lam and -0.8 in lam
