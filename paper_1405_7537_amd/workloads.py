"""Seeded synthetic DPR1 inputs.

Pure input generation (NumPy PCG64 streams): no arithmetic of the eigensolver
lives here.  Both the GPU path and the CPU oracle are fed from these arrays.

Workload families (all float64):

* ``uniform``  -- d sorted-descending distinct draws from U[-1, 1],
  z ~ N(0, 1) (optionally scaled by 1/sqrt(n)), rho given;
* ``graded``   -- d_i = 10^(-12 (i-1)/(n-1)), every 64th pole pushed to a
  relative gap of 1e-10 from its predecessor, |z_i| = 10^U(-8, 0) with fair
  random signs, rho = 1e-3;
* ``batched``  -- many independent uniform problems with sizes log-uniform in
  [16, 2048] and rho ~ U[0.1, 10], packed back to back with int64 offsets;
* paper examples 1-4 (Sec. 3), built from their printed definitions.
"""
from __future__ import annotations

import math

import numpy as np


def _sorted_distinct_uniform(rng, n, lo=-1.0, hi=1.0):
    while True:
        d = np.sort(rng.uniform(lo, hi, n))[::-1].copy()
        if n < 2 or np.all(d[:-1] > d[1:]):
            return d


def uniform(n, seed, rho=1.0, zscale=1.0):
    rng = np.random.default_rng(seed)
    d = _sorted_distinct_uniform(rng, n)
    z = rng.standard_normal(n) * zscale
    z[z == 0.0] = 1e-300
    return d, z, float(rho)


def graded(n, seed, rho=1e-3, pair_every=64, pair_gap=1e-10):
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    d = 10.0 ** (-12.0 * i / (n - 1))
    for p in range(pair_every, n, pair_every):          # 1-based p = 64, 128, ...
        d[p] = d[p - 1] * (1.0 - pair_gap)               # d_{p+1} = d_p (1 - gap)
    mag = 10.0 ** rng.uniform(-8.0, 0.0, n)
    sgn = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    z = mag * sgn
    assert np.all(d[:-1] > d[1:])
    return d, z, float(rho)


def batched_sizes(nprob, seed, nmin=16, nmax=2048):
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), nprob))).astype(np.int64), rng


def batched(nprob, seed, nmin=16, nmax=2048, rho_lo=0.1, rho_hi=10.0, sizes=None):
    """Packed ragged batch: returns (d, z, rho[nprob], offs[nprob+1])."""
    if sizes is None:
        sizes, rng = batched_sizes(nprob, seed, nmin, nmax)
    else:
        sizes = np.asarray(sizes, dtype=np.int64)
        rng = np.random.default_rng(seed)
    offs = np.zeros(nprob + 1, dtype=np.int64)
    offs[1:] = np.cumsum(sizes)
    d = np.empty(offs[-1])
    z = np.empty(offs[-1])
    rho = np.empty(nprob)
    for p in range(nprob):
        a, b = offs[p], offs[p + 1]
        d[a:b] = _sorted_distinct_uniform(rng, b - a)
        zz = rng.standard_normal(b - a)
        zz[zz == 0.0] = 1e-300
        z[a:b] = zz
        rho[p] = rng.uniform(rho_lo, rho_hi)
    return d, z, rho, offs


def uniform_batch(nprob, n, seed, rho=1.0):
    """nprob problems of equal size n, d U[-1,1] sorted, z ~ N(0,1): arrays [nprob, n]."""
    rng = np.random.default_rng(seed)
    d = np.empty((nprob, n))
    z = np.empty((nprob, n))
    for p in range(nprob):
        d[p] = _sorted_distinct_uniform(rng, n)
        z[p] = rng.standard_normal(n)
    z[z == 0.0] = 1e-300
    return d, z, np.full(nprob, float(rho))


# ----------------------------------------------------------- paper examples
def example1():
    """Sec. 3, Example 1: D = diag(1e10, 5, 4e-3, 0, -4e-3, -5), z = (1e10,1,1,1e-7,1,1), rho = 1."""
    d = np.array([1e10, 5.0, 4e-3, 0.0, -4e-3, -5.0])
    z = np.array([1e10, 1.0, 1.0, 1e-7, 1.0, 1.0])
    return d, z, 1.0


def example2():
    """Sec. 3, Example 2: D = 1 + (40, 30, 20, 10) * 2^-52, z = (1, 2, 2, 1), rho = 1."""
    e = 2.0 ** -52
    d = np.array([1 + 40 * e, 1 + 30 * e, 1 + 20 * e, 1 + 10 * e])
    z = np.array([1.0, 2.0, 2.0, 1.0])
    return d, z, 1.0


def example3(beta=1e-7):
    """Sec. 3, Example 3: D = diag(10/3, 2+beta, 2-beta, 1), z = (2, beta, beta, 2), rho = 1."""
    d = np.array([10.0 / 3.0, 2.0 + beta, 2.0 - beta, 1.0])
    z = np.array([2.0, beta, beta, 2.0])
    return d, z, 1.0


def example4(beta, m=100):
    """Sec. 3, Example 4: D = {1, 2 +- j beta (j = 1..m), 10/3}, z = (2, beta, ..., beta, 2),
    put in decreasing order of D (symmetric permutation, Sec. 1)."""
    dd = [1.0]
    zz = [2.0]
    for j in range(1, m + 1):
        dd += [2.0 + j * beta, 2.0 - j * beta]
        zz += [beta, beta]
    dd.append(10.0 / 3.0)
    zz.append(2.0)
    dd, zz = np.array(dd), np.array(zz)
    order = np.argsort(-dd, kind="stable")
    return dd[order].copy(), zz[order].copy(), 1.0


def reducible(n, seed, groups=None, zeros=None, rho=1.0):
    """Unsorted poles with repeated values and some zero z_j (the input of the front end of Sec. 1):
    `groups` poles get the value of another pole (groups of 2 and more), `zeros` entries of z are 0.
    Defaults: n // 10 of each."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, n)
    groups = n // 10 if groups is None else groups
    zeros = n // 10 if zeros is None else zeros
    if n >= 2:
        for _ in range(groups):
            a, b = rng.choice(n, 2, replace=False)
            d[b] = d[a]
    z = rng.standard_normal(n)
    if zeros:
        z[rng.choice(n, min(zeros, n), replace=False)] = 0.0
    return d, z, rho


def tridiagonal(n, seed):
    """Symmetric tridiagonal T: diagonal and off-diagonal ~ N(0, 1) (seed), the input of the
    divide-and-conquer driver whose merges are DPR1 problems."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n), rng.standard_normal(max(n - 1, 0))


def wilkinson(m):
    """Wilkinson's W_{2m+1}^+: diagonal |m|, ..., 1, 0, 1, ..., m, off-diagonal ones (close pairs)."""
    return np.abs(np.arange(-m, m + 1, dtype=np.float64)), np.ones(2 * m)


def extreme(seed):
    """A small problem at the edges of the binary64 range (seeded): 2-40 distinct poles, sorted
    decreasingly, either uniform in [-1, 1], spread over 20 decades with both signs, or clustered
    (gaps 1e-14..1e-1 above 1); |z_j| = 10^U(-150, 0) with random signs; |rho| = 10^U(-8, 8), either
    sign."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 40))
    kind = seed % 3
    if kind == 0:
        d = rng.uniform(-1, 1, n)
    elif kind == 1:
        d = 10.0 ** rng.uniform(-10, 10, n) * rng.choice([-1.0, 1.0], n)
    else:
        d = 1.0 + np.cumsum(10.0 ** rng.uniform(-14, -1, n))
    d = np.unique(d)[::-1].copy()
    z = 10.0 ** rng.uniform(-150, 0, d.size) * rng.choice([-1.0, 1.0], d.size)
    rho = 10.0 ** rng.uniform(-8, 8) * rng.choice([-1.0, 1.0])
    return d, z, float(rho)


def extreme_wide(seed):
    """A wider edge problem (seeded): 1-59 distinct poles, uniform in [-1, 1] with |z_j| down to 1e-20,
    or (other kinds) spread over 60 decades, clustered to gaps of 1e-15, half near 1e-300, or normal
    times 10^(-5..5), each with |z_j| down to 1e-300; |rho| = 10^U(-12, 12), either sign."""
    rng = np.random.default_rng(10_000 + seed)
    n = int(rng.integers(1, 60))
    kind = seed % 5
    if kind == 0:
        d = rng.uniform(-1, 1, n)
    elif kind == 1:
        d = 10.0 ** rng.uniform(-30, 30, n) * rng.choice([-1.0, 1.0], n)
    elif kind == 2:
        d = 1.0 + np.cumsum(10.0 ** rng.uniform(-15, -1, n))
    elif kind == 3:
        d = np.concatenate([rng.uniform(-1, 1, n // 2), 1e-300 * rng.uniform(-1, 1, n - n // 2)])
    else:
        d = rng.standard_normal(n) * 10.0 ** rng.integers(-5, 6)
    d = np.unique(d)[::-1].copy()
    zl = rng.uniform(-300, 0, d.size) if kind != 0 else rng.uniform(-20, 0, d.size)
    z = 10.0 ** zl * rng.choice([-1.0, 1.0], d.size)
    rho = 10.0 ** rng.uniform(-12, 12) * rng.choice([-1.0, 1.0])
    return d, z, float(rho)


def tridiagonal_family(seed):
    """Structured symmetric tridiagonal matrices that stress divide-and-conquer merges (seeded):
    kind = seed % 7: 0 random, 1 graded off-diagonal (1 .. 1e-20), 2 glued Wilkinson W21+ blocks
    (couplings 1e-8), 3 couplings 10^U(-300, 0) with 10 % zeros, 4 diagonal over 20 decades,
    5 constant diagonal with 1e-6 couplings, 6 the 1-2-1 matrix.  Returns (a, b)."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(2, 700))
    k = seed % 7
    if k == 0:
        a, b = rng.standard_normal(n), rng.standard_normal(n - 1)
    elif k == 1:
        a, b = rng.standard_normal(n), 10.0 ** (-np.linspace(0, 20, n - 1))
    elif k == 2:
        m = 10
        blk = np.abs(np.arange(-m, m + 1, dtype=np.float64))
        a = np.tile(blk, max(1, n // 21))
        b = np.ones(a.size - 1)
        b[20::21] = 1e-8
    elif k == 3:
        a, b = rng.standard_normal(n), rng.standard_normal(n - 1) * 10.0 ** rng.uniform(-300, 0, n - 1)
        b[rng.random(n - 1) < 0.1] = 0.0
    elif k == 4:
        a, b = 10.0 ** rng.uniform(-10, 10, n) * rng.choice([-1.0, 1.0], n), rng.standard_normal(n - 1)
    elif k == 5:
        a, b = np.ones(n), 1e-6 * rng.standard_normal(n - 1)
    else:
        a, b = 2.0 * np.ones(n), -np.ones(n - 1)
    return a, b


def extreme_large(seed):
    """Larger edge problems (seeded): 100-2000 distinct poles, uniform, clustered (gaps 1e-13..1e-2
    above 1), over 16 decades with both signs, or half in a 1e-9 cluster at 0.3; |z_j| = 10^U(-150, 0)
    with random signs; |rho| = 10^U(-6, 6), either sign."""
    rng = np.random.default_rng(77_000 + seed)
    n = int(rng.integers(100, 2000))
    kind = seed % 4
    if kind == 0:
        d = rng.uniform(-1, 1, n)
    elif kind == 1:
        d = 1.0 + np.cumsum(10.0 ** rng.uniform(-13, -2, n))
    elif kind == 2:
        d = np.sort(10.0 ** rng.uniform(-8, 8, n) * rng.choice([-1.0, 1.0], n))
    else:
        d = np.concatenate([rng.uniform(-1, 1, n // 2), rng.uniform(0.3, 0.3 + 1e-9, n - n // 2)])
    d = np.unique(d)[::-1].copy()
    z = 10.0 ** rng.uniform(-150, 0, d.size) * rng.choice([-1.0, 1.0], d.size)
    rho = 10.0 ** rng.uniform(-6, 6) * rng.choice([-1.0, 1.0])
    return d, z, float(rho)
