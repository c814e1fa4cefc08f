"""GPU parity of K_nu (eq. K0) and of the remedies (R1)/(R2) of Sec. 2 (Algorithm 1, last branch)
against the CPU oracle, which is pinned to the 256-bit truth tool (test_oracle_pins.py)."""
import math

import numpy as np
import pytest

from paper_1405_7537_amd import workloads as W
from test_gpu_parity import compare, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1405_7537_amd.dpr1 as D
    D.lib()
    return D


CASES = {
    "C1 n256": lambda: W.uniform(256, 0),
    "graded1024": lambda: W.graded(1024, 1),
    "rho10 n512": lambda: W.uniform(512, 11, rho=10.0),
    "rho<0 n300": lambda: (W.uniform(300, 8)[0], W.uniform(300, 8)[1], -3.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_knu_matches_oracle(D, orc, case):
    """K_nu of every eigenpair (the optional knu output, caller's order) against the oracle's, and
    the count of K_nu > 32 in the stats."""
    d, z, rho = CASES[case]()
    print(f"[remedy] K_nu {case}", flush=True)
    r = D.eig(d, z, rho, want_knu=True, want_stats=True)
    kg = r.knu.cpu().numpy()
    _, _, dg = orc.eig(d, z, rho, vectors=False, diags=True)
    ko = np.array([g["Knu"] for g in dg])
    # both are ratios of distances from the shifted representations; where the other eigenvalue is
    # represented from another pole the distance carries its cancellation, so the bar is loose
    assert np.all(rel(kg, ko) <= 1e-8), (np.argmax(rel(kg, ko)), rel(kg, ko).max())
    far = np.abs(np.log(ko / 32.0)) > 1e-6
    assert r.stats_dict()["knu_gt"] == int(np.sum(kg > 32.0))
    assert np.array_equal((kg > 32)[far], (ko > 32)[far])
    print(f"[remedy] {case}: K_nu max {ko.max():.3g}, {int(np.sum(ko > 32))} above 32", flush=True)


PROBLEMS = {
    "C1 n256": lambda: W.uniform(256, 0),
    "C2 graded4096": lambda: W.graded(4096, 1),
    "rho10 n512": lambda: W.uniform(512, 11, rho=10.0),
    "uniform z/sqrt(n) 2048": lambda: W.uniform(2048, 2, zscale=1 / math.sqrt(2048)),
    "rho<0 n300": lambda: (W.uniform(300, 8)[0], W.uniform(300, 8)[1], -3.0),
    "extreme 92": lambda: W.extreme(92),
    "extreme 128": lambda: W.extreme(128),
    "extreme 182": lambda: W.extreme(182),
}


@pytest.mark.parametrize("case", list(PROBLEMS))
def test_remedies_with_polish_off(D, orc, case):
    """The double-double polish off, the remedies on: every eigenpair (eigenvalue, eigenvector,
    shift index, mu, ||x||) within the parity bar of the oracle run with the same options; the
    remedied pairs are the oracle's."""
    d, z, rho = PROBLEMS[case]()
    r, lo, Vo, dg = compare(D, orc, d, z, rho, opts=D.opts(polish=0, remedy=1),
                            oopts=orc.make_opts(polish=0, remedy=1), tag=f"remedy {case}")
    st = r.stats_dict()
    nrem = st["remedy_r1"] + st["remedy_r2"]
    nrem_o = sum(1 for g in dg if g["remedied"])
    print(f"[remedy] {case}: GPU R1 {st['remedy_r1']} R2 {st['remedy_r2']}, oracle {nrem_o}", flush=True)
    assert st["polished"] == 0
    assert abs(nrem - nrem_o) <= max(2, nrem_o // 20)
