// Forward-stable DPR1 eigensolver: gfx950 kernels and the C ABI.
//
// Paper: Jakovcevic Stor, Slapnicar, Barlow, "Forward stable eigenvalue
// decomposition of rank-one modifications of diagonal matrices" (Alg. 1).
//
// Kernels (all FP64; double-double where the paper asks for double the
// working precision):
//   k_prep  -- per problem: checks of Sec. 1, the rho < 0 reduction, staging
//              of (d_j, zeta_j^2) pairs and the low parts of zeta_j^2.
//   k_eig   -- one lane per eigenvalue, 64 eigenvalues per block; W waves of
//              a block split the inner index j.  All lanes of a wave read the
//              same (d_j, zeta_j^2) at the same time, so the data arrive
//              through scalar loads and feed the FP64 VALU as SGPR operands.
//              Per eigenvalue: shift test, tip b in double-double, extreme
//              root of the arrowhead secular function (model passes, the
//              last one with compensated summation), near-zero test, ||x||.
//              Instances for 4, 6 and 8 waves per SIMD (register budgets);
//              the split W, the budget and the pass count are options that
//              dpr1_autotune / dpr1_batched_autotune choose by timing.
//   k_out   -- user outputs in the caller's index order.
//   k_fix   -- one 256-thread block at a time per flagged eigenpair: root
//              search continued past k_eig's pass budget, double-double
//              Newton polish, and the near-zero recomputation of eq. (gamma).
//   k_fixvec -- k_fix's work and the eigenvector writer in one launch: a few
//              blocks finish the flagged eigenpairs while the others write V,
//              one block per column group and row range, non-temporal stores
//              in windows aligned to whole cache lines; flagged columns are
//              left to k_fixout.
//   k_fixout -- outputs and V columns of the flagged eigenpairs.
#include <float.h>
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/dpr1.h"
#include "dd.h"

namespace dpr1 {

constexpr int WAVE = 64;
constexpr int MAXW = 16;
constexpr double GROW = 1.0 + 0x1p-40;

typedef const __attribute__((address_space(4))) double cdouble;

// Wave-uniform load through the scalar data cache (idx must be uniform).
__device__ __forceinline__ double ldu(const double* base, int64_t idx) {
  return ((cdouble*)base)[idx];
}

struct Meta {
  int64_t off;   // first element of the problem in the packed arrays
  int32_t n;
  int32_t neg;   // rho < 0: solved as (-d reversed, z reversed, -rho)
  int32_t info;
  int32_t pad;
  double rho;    // |rho|
  double zz;     // sum zeta_j^2
  double zabs;   // sum |zeta_j| (K_z of eq. knu2)
};

enum : int32_t { FIX_POLISH = 1, FIX_NEARZERO = 2, FIX_CONTINUE = 4 };

// A flagged eigenpair: polish, near-zero rule, or a rational iteration still
// running when the eigenvalue kernel reached its pass budget (then cnu, cL,
// cU, cprev, iters hold the iteration's state).
struct FixItem {
  int32_t p, k, i, flags;
  int32_t iters, pad;
  double nu0, nu1, bhi, blo, lo, hi;
  double cnu, cL, cU, cprev;
};

struct KArgs {
  const Meta* meta;
  const double* pairs;  // [2N]: (d'_j, zeta'_j^2)
  const double* z2lo;   // [N]  low part of zeta'_j^2
  const double* sd;     // [N]  d'
  const double* sz;     // [N]  zeta'
  int32_t* ii;          // [N]  shift index (within the problem)
  double* mu;           // [N]
  double* xs;           // [N]  |mu| * ||x||_2
  double* lam;          // [N]
  FixItem* fix;         // [N]
  uint8_t* vflag;       // [N]  1: eigenpair finished in k_fix (its V column written after)
  int32_t* ctr;         // [0] fix count, [1] queue head, [2] k_fix queue head
  int32_t* stats;       // nullable
  const int2* items;    // batched queue (p, k0) or nullptr
  int32_t nitems;
  int32_t nfixcap;  // capacity of `fix` (one slot per eigenvalue)
  int32_t W;
  int32_t mode_b, root, polish;
  int32_t main_passes;
  double kappa_polish, nearzero;
  int32_t g0;           // single problem: first group of 64 eigenvalues of this launch
  int32_t remedy;       // apply (R1)/(R2) where K_nu > knu_thr
  double knu_thr;
  double* knu;          // optional output: K_nu per eigenpair (caller's order)
};

// ------------------------------------------------------------ bit helpers
__device__ __forceinline__ uint64_t bits(double x) { return (uint64_t)__double_as_longlong(x); }
__device__ __forceinline__ double unbits(uint64_t u) { return __longlong_as_double((long long)u); }

// midpoint in the order of binary64 numbers, 0 < lo < hi
__device__ __forceinline__ double fmid(double lo, double hi) {
  uint64_t a = bits(lo), b = bits(hi);
  return unbits(a + (b - a) / 2);
}
__device__ __forceinline__ bool adjacent(double lo, double hi) { return bits(hi) - bits(lo) <= 1; }
// the same for lo < hi of one sign (both negative: the bit patterns run backwards)
__device__ __forceinline__ bool adjacent_signed(double lo, double hi) {
  return lo > 0.0 ? bits(hi) - bits(lo) <= 1 : bits(lo) - bits(hi) <= 1;
}
__device__ __forceinline__ double fmid_signed(double lo, double hi) {
  return lo > 0.0 ? fmid(lo, hi) : -fmid(-hi, -lo);
}

// Reciprocal from the hardware estimate refined by one Newton step: for the
// signs that steer bisection, and as the seed of a quotient that is then
// corrected by its residual (within about half an ulp more than correct
// rounding).  v_rcp_f64 is specified to 2^29 ulp (2^-23 relative) and
// measured at 2^-24.4 on gfx950 over random normal inputs; one Newton step
// gives 2^-48.7.  The IEEE divide costs about twice as many instructions on
// this ISA.
__device__ __forceinline__ double rcp_1nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE); }
__device__ __forceinline__ int lane_id() { return threadIdx.x % WAVE; }
__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// ------------------------------------------------- cross-wave reductions
// Every wave of the block ends with the same sums, added in the same order,
// so all waves keep identical per-lane state.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], int W, int wv, int lane, double* red) {
  static_assert(NV <= 4, "the reduction buffer holds four values per lane and wave");
  if (W == 1) return;
#pragma unroll
  for (int q = 0; q < NV; ++q) red[(q * W + wv) * WAVE + lane] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = red[(q * W) * WAVE + lane];
    for (int w = 1; w < W; ++w) s += red[(q * W + w) * WAVE + lane];
    v[q] = s;
  }
  __syncthreads();
}

// (s, c) Neumaier partials -> combined with TwoSum in wave order.
__device__ __forceinline__ void wg_sum_comp(double& s, double& c, int W, int wv, int lane, double* red) {
  if (W == 1) return;
  red[(0 * W + wv) * WAVE + lane] = s;
  red[(1 * W + wv) * WAVE + lane] = c;
  __syncthreads();
  double S = red[lane], C = red[W * WAVE + lane];
  for (int w = 1; w < W; ++w) {
    dd t = two_sum(S, red[w * WAVE + lane]);
    S = t.hi;
    C += red[(W + w) * WAVE + lane] + t.lo;
  }
  s = S;
  c = C;
  __syncthreads();
}

// same-signed double-double partials
__device__ __forceinline__ void wg_sum_dd(dd& a, int W, int wv, int lane, double* red) {
  if (W == 1) return;
  red[(0 * W + wv) * WAVE + lane] = a.hi;
  red[(1 * W + wv) * WAVE + lane] = a.lo;
  __syncthreads();
  dd s = {red[lane], red[W * WAVE + lane]};
  for (int w = 1; w < W; ++w) s = dd_add_same(s, dd{red[w * WAVE + lane], red[(W + w) * WAVE + lane]});
  a = s;
  __syncthreads();
}

// Walk the wave's slice [j0, j1) of the inner index in three segments:
// below the window of shift indices this wave can own (seg 0: every lane has
// j < i), inside it (seg 1: per-lane test), above it (seg 2: every lane has
// j > i).  j is wave-uniform in all three loops.  f(j, seg, d_j, zeta_j^2,
// low part of zeta_j^2 (0 unless asked for), u) with u the position of the
// pair in its block (a compile-time constant once unrolled), or -1 for the
// pairs after the last whole block.
template <bool LO, class F>
__device__ __forceinline__ void sweep_seg(const double* P, const double* Zl, int a, int b, int seg, F& f) {
  // Blocks of B pairs (with LO also the B low parts of zeta_j^2), software-
  // pipelined: the scalar loads of the next block are issued before the
  // current block is computed, so their latency hides behind that work.  A
  // wait for scalar loads covers all of them, so no load may be waited for
  // inside the computation; with LO the blocks are halved to keep both
  // blocks in scalar registers.
  constexpr int B = LO ? 4 : 8;
  constexpr int NV = LO ? 3 * B : 2 * B;
  auto load = [](double (&c)[NV], const double* q, const double* ql) {
#pragma unroll
    for (int t = 0; t < 2 * B; ++t) c[t] = ldu(q, t);
    if constexpr (LO) {
#pragma unroll
      for (int t = 0; t < B; ++t) c[2 * B + t] = ldu(ql, t);
    }
  };
  const double* q = P + 2 * (int64_t)a;
  const double* ql = LO ? Zl + a : nullptr;
  int j = a;
  if (j + B <= b) {
    double c[NV];
    load(c, q, ql);
    // wait for the first block here (s_waitcnt lgkmcnt(0)): otherwise the wait
    // for it lands inside the loop, where it also waits for the prefetch
    __builtin_amdgcn_s_waitcnt(0xC07F);
    for (; j + 2 * B <= b; j += B, q += 2 * B, ql += LO ? B : 0) {
      double nx[NV];
      load(nx, q + 2 * B, LO ? ql + B : nullptr);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < B; ++u) f(j + u, seg, c[2 * u], c[2 * u + 1], LO ? c[2 * B + u] : 0.0, u);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < NV; ++t) c[t] = nx[t];
    }
#pragma unroll
    for (int u = 0; u < B; ++u) f(j + u, seg, c[2 * u], c[2 * u + 1], LO ? c[2 * B + u] : 0.0, u);
    j += B;
    q += 2 * B;
    ql += LO ? B : 0;
  }
  for (; j < b; ++j, q += 2, ql += LO ? 1 : 0)
    f(j, seg, ldu(q, 0), ldu(q, 1), LO ? ldu(ql, 0) : 0.0, -1);
}

template <class F>
__device__ __forceinline__ void sweep(const double* P, int j0, int j1, int wlo, int whi, F&& f) {
  sweep_seg<false>(P, nullptr, j0, min(j1, wlo), 0, f);
  sweep_seg<false>(P, nullptr, max(j0, wlo), min(j1, whi), 1, f);
  sweep_seg<false>(P, nullptr, max(j0, whi), j1, 2, f);
}

// the same walk, also handing f the low part of zeta_j^2 from Zl
template <class F>
__device__ __forceinline__ void sweep_lo(const double* P, const double* Zl, int j0, int j1, int wlo, int whi,
                                         F&& f) {
  sweep_seg<true>(P, Zl, j0, min(j1, wlo), 0, f);
  sweep_seg<true>(P, Zl, max(j0, wlo), min(j1, whi), 1, f);
  sweep_seg<true>(P, Zl, max(j0, whi), j1, 2, f);
}

// ------------------------------------------------------------------ prep
// nsplit == 1: block p stages problem p and writes its meta.  nsplit > 1 (a
// single problem): block b stages one slice and leaves its partial sum and
// flags in `part`; the last block to finish adds the partials in slice order
// (so the result does not depend on the order the blocks ran in) and writes
// the meta.
constexpr int PREP_MAX_SPLIT = 64;
__global__ void __launch_bounds__(256) k_prep(int nprob, int nsplit, const int64_t* __restrict__ offs,
                                              int64_t n_single, const double* __restrict__ d,
                                              const double* __restrict__ z, const double* __restrict__ rho_dev,
                                              double rho_host, Meta* __restrict__ meta, double* __restrict__ sd,
                                              double* __restrict__ sz, double* __restrict__ pairs,
                                              double* __restrict__ z2lo, int32_t* __restrict__ info,
                                              double* __restrict__ part, int32_t* __restrict__ done_ctr) {
  const int p = nsplit == 1 ? (int)blockIdx.x : 0;
  const int bs = nsplit == 1 ? 0 : (int)blockIdx.x;
  if (p >= nprob) return;
  const int64_t off = offs ? offs[p] : 0;
  const int64_t n = offs ? offs[p + 1] - offs[p] : n_single;
  const double rho = rho_dev ? rho_dev[p] : rho_host;
  const int neg = rho < 0;
  const int64_t chunk = (n + nsplit - 1) / nsplit;
  const int64_t ja = min(n, (int64_t)bs * chunk), jb = min(n, ja + chunk);
  __shared__ double red[256], red2[256];
  __shared__ int flags, last;
  if (threadIdx.x == 0) flags = 0;
  __syncthreads();
  int f = 0;
  double acc = 0.0, acc2 = 0.0;
  for (int64_t j = ja + threadIdx.x; j < jb; j += blockDim.x) {
    int64_t src = neg ? n - 1 - j : j;
    double dj = d[off + src], zj = z[off + src];
    if (!isfinite(dj) || !isfinite(zj)) f |= 4;
    if (zj == 0.0) f |= 2;
    // zeta_j^2 must be a normal number (the sums are taken in squares), and
    // two poles closer than 2^-1000 would put 1/(d_j - d_i) and nu beyond the
    // binary64 range
    if (zj != 0.0 && fabs(zj) < 0x1p-511) f |= 8;
    if (j + 1 < n) {
      double dn = d[off + src + (neg ? -1 : 1)];
      // staged order must be strictly decreasing: d_j > d_{j+1} (or -d reversed)
      if (!(neg ? (-dj > -dn) : (dj > dn))) f |= 1;
      else if (fabs(dj - dn) < 0x1p-1000) f |= 8;
    }
    double ds = neg ? -dj : dj;
    double z2 = zj * zj;
    sd[off + j] = ds;
    sz[off + j] = zj;
    pairs[2 * (off + j)] = ds;
    pairs[2 * (off + j) + 1] = z2;
    z2lo[off + j] = __builtin_fma(zj, zj, -z2);
    acc += z2;
    acc2 += fabs(zj);
  }
  if (f) atomicOr(&flags, f);
  red[threadIdx.x] = acc;
  red2[threadIdx.x] = acc2;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      red2[threadIdx.x] += red2[threadIdx.x + s];
    }
    __syncthreads();
  }
  double zz = red[0], za = red2[0];
  int fl = flags;
  if (nsplit > 1) {
    // part: (sum zeta^2, sum |zeta|, flags) per slice
    if (threadIdx.x == 0) {
      part[3 * bs] = zz;
      part[3 * bs + 1] = za;
      part[3 * bs + 2] = (double)fl;
      __threadfence();
      last = atomicAdd(done_ctr, 1) == nsplit - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    if (threadIdx.x == 0) {
      const volatile double* vp = part;
      zz = 0.0;
      za = 0.0;
      fl = 0;
      for (int q = 0; q < nsplit; ++q) {
        zz += vp[3 * q];
        za += vp[3 * q + 1];
        fl |= (int)vp[3 * q + 2];
      }
    }
  }
  if (threadIdx.x == 0) {
    int code = 0;
    if (!isfinite(rho) || rho == 0.0) code = DPR1_INFO_BAD_RHO;
    else if (fl & 4) code = DPR1_INFO_NONFINITE;
    else if (fl & 1) code = DPR1_INFO_UNSORTED;
    else if (fl & 2) code = DPR1_INFO_ZERO_Z;
    else if (fl & 8) code = DPR1_INFO_RANGE;
    Meta m;
    m.off = off;
    m.n = (int32_t)n;
    m.neg = neg;
    m.info = code;
    m.pad = 0;
    m.rho = fabs(rho);
    m.zz = zz;
    m.zabs = za;
    meta[p] = m;
    if (info) info[p] = code;
  }
}

__global__ void k_zero(int32_t* __restrict__ a, int n) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = 0;
}

// ------------------------------------------------------------------- eig
// Root of the model of g at the current iterate m.  Written in poles,
// g(t) = b' - t + sum_j w_j/(t - xi_j) with xi_j = 1/delta'_j and
// w_j = zeta_j^2/(delta'_j^2 zeta_i^2); the wanted root lies right of every
// pole.  The model keeps the nearest pole xm with its exact weight sw^2 and
// replaces the rest of the sum, R(t), by sa^2/(t - p) + B fitted to R's
// value, slope and curvature at m (Sz, Spz, Sppz are the moments of the whole
// sum: S/zeta_i^2, sum w/(m - xi)^2, sum w/(m - xi)^3).  Every other pole
// lies left of xm, so the fitted pole does too; the model is then convex and
// decreasing right of its poles and its root is found by Newton's method
// inside the bracket (L, U).  The model matches g to second order at m, so
// the outer iteration converges cubically.  Both weights are carried as
// square roots: with zeta_i near 1e-148 beside a pole 1e-13 away a weight
// reaches 1e322 while every term weight/(t - pole) of the model is finite.
__device__ __forceinline__ double model_root(double m, double Sz, double Spz, double Sppz, double bp, double xm,
                                             double sw, double L, double U) {
  double Rs = Sz, Rp = Spz, Rpp = Sppz;
  if (sw > 0.0) {
    const double ie = 1.0 / (m - xm);
    const double a = sw * ie;
    Rs -= sw * a;
    Rp -= a * a;
    Rpp -= (a * a) * ie;
  }
  double p = xm, sa = 0.0, B = Rs;
  if (Rp > 0.0 && Rpp > 0.0) {
    p = fmin(m - Rp / Rpp, xm);
    const double x = m - p;
    sa = sqrt(Rp) * x;
    B = Rs - Rp * x;
  }
  // a model whose parameters are not finite says nothing: NaN makes the
  // caller take a bisection step instead of reading a zero step as
  // convergence
  if (!(sa < INFINITY) || !(fabs(B) < INFINITY) || !(sw < INFINITY)) return NAN;
  double lo = fmax(L, fmax(xm, p)), hi = U;
  double t = m;
  for (int q = 0; q < 40; ++q) {
    const double e1 = 1.0 / (t - xm), e2 = 1.0 / (t - p);
    const double s1 = sw * e1, s2 = sa * e2;
    const double h = ((bp - t) + B) + (sw * s1 + sa * s2);
    if (!(h == h)) return NAN;
    if (h == 0.0) break;  // t is a root of the model
    const double hp = -1.0 - (s1 * s1 + s2 * s2);
    if (h > 0.0) lo = t; else hi = t;
    double tn = t - h / hp;
    // a step below the resolution of t ends the iteration (t may sit on the
    // bracket end it has just set, where tn == t would fail the test below)
    if (fabs(tn - t) <= 0x1p-52 * t) {
      t = tn;
      break;
    }
    if (!(tn > lo && tn < hi)) tn = (hi < INFINITY) ? 0.5 * (lo + hi) : 2.0 * t;
    t = tn;
  }
  return t;
}

// One step of the safeguarded iteration for the rightmost root of g from its
// value g and moments at m (the bracket [L, U] already updated with the sign
// of g).  A model root outside (L, U) is replaced by the bit midpoint, and so
// is the next iterate of a two-cycle: g changed sign at the last two steps
// while |g| fell by less than a factor 10 on the same side (g1, g2 keep the
// two previous values of g).
__device__ __forceinline__ void model_step(double m, double g, double Sz, double Spz, double Sppz, double bp,
                                           double xm, double sw, int iters, double L, double U, double& nu,
                                           double& nu0, double& prevstep, double& g1, double& g2, bool& done,
                                           double tol = 0x1p-20) {
  if (g == 0.0) {
    done = true;
    nu0 = m;
    return;
  }
  const bool cycle = (g * g1 < 0.0) && (g1 * g2 < 0.0) && (fabs(g) > 0.1 * fabs(g2));
  g2 = g1;
  g1 = g;
  const double nn0 = model_root(m, Sz, Spz, Sppz, bp, xm, sw, L, U);
  double nn = nn0;
  const double step = fabs(nn - m);
  // Cubic convergence: a step e leaves a model error of about 8 e^3 (the
  // shift keeps every pole at least nu/2 from the root), so after a step
  // below 2^-20 the new iterate is exact to rounding.  The same tolerance
  // accepts the step of the accurate last pass.
  if (step <= tol * m) {
    done = true;
    nu0 = (nn >= L && nn <= U) ? nn : m;
    return;
  }
  if (!(nn > L && nn < U) || cycle) {
    if (adjacent(L, U)) {
      done = true;
      nu0 = U;
      return;
    }
    nn = fmid(L, U);
  } else if (iters >= 8 && step > 0.5 * prevstep) {
    done = true;  // rounding noise dominates g: leave it to the checks after
    nu0 = nn;
    return;
  }
  if (iters >= 40) {
    done = true;
    nu0 = nn;
    return;
  }
  prevstep = fabs(nn - m);
  nu = nn;
}

// One block of 64 eigenvalues (k0 .. k0+63) of problem p, W waves.
__device__ void eig_block(const KArgs& A, int p, int k0, double* red) {
  const int W = A.W;
  const int wv = wave_id();
  const int lane = lane_id();
  const Meta M = A.meta[p];
  if (M.info != 0) return;
  const int n = M.n;
  const int64_t off = M.off;
  const double* P = A.pairs + 2 * off;
  const double* Zl = A.z2lo + off;
  const double* Dv = A.sd + off;
  const double* Zv = A.sz + off;
  const double rho = M.rho;
  const int k = k0 + lane;
  const bool valid = k < n;
  const int kk = valid ? k : n - 1;

  // wave slice of the inner index and the window of possible shift indices
  const int chunk = (n + W - 1) / W;
  const int j0 = min(n, wv * chunk);
  const int j1 = min(n, j0 + chunk);
  const int wlo = max(0, k0 - 1);
  const int whi = min(n, k0 + WAVE);

  if (n == 1) {
    // 1x1: lambda = d_1 + rho zeta_1^2, x = zeta_1/(d_1 - lambda)
    if (wv == 0 && lane == 0) {
      double z0 = Zv[0];
      double m = rho * (z0 * z0);
      A.ii[off] = 0;
      A.vflag[off] = 0;
      A.mu[off] = m;
      A.xs[off] = fabs(z0);
      A.lam[off] = Dv[0] + m;
    }
    return;
  }

  const double dk = Dv[kk];
  const double dkm1 = kk > 0 ? Dv[kk - 1] : 0.0;

  // bracket of the exterior root (k = 1): d_1 + rho zeta_1^2 <= lambda_1 <=
  // d_1 + rho ||z||^2, in nu = 1/(lambda_1 - d_1)
  double Lx = 0.0, Ux = 0.0, nux = 0.0;
  if (kk == 0) {
    const double z0 = Zv[0];
    Lx = (1.0 / (rho * M.zz)) / GROW;
    Ux = (1.0 / (rho * (z0 * z0))) * GROW;
    nux = A.root ? Ux : fmid(Lx, Ux);
  }

  // ---- shift (Alg. 1): F = 1 + rho sum zeta_j^2/((d_j - d_k) - tau)
  // The same pass also sums |terms| and terms/den (f' at the midpoint): the
  // midpoint is the first probe of the root finder, so its evaluation is reused.
  // For k = 1 there is no shift to choose; the pass evaluates f at the first
  // point of the root search instead, lambda = d_1 + 1/nux.
  const double tau = kk > 0 ? (dkm1 - dk) / 2 : 1.0 / nux;
  // Only the sign of F and a first model step are taken from these sums, so
  // the reciprocal is the hardware estimate alone (relative error below
  // 2^-23): the bounds taken from the probe allow for it.
  // The terms are positive for j < k (pole above the midpoint) and negative
  // for j >= k, so their sum and the sum of their magnitudes come from the
  // two one-signed partial sums Fs[0] (j < k) and Fs[1] (j >= k); below the
  // window every lane has j < k, above it j > k.
  double Fs[4] = {0.0, 0.0, 0.0, 0.0};
  sweep(P, j0, j1, wlo, whi, [&](int j, int seg, double dj, double z2, double, int) {
    double r = __builtin_amdgcn_rcp((dj - dk) - tau);
    double t = z2 * r;
    double tr = t * r;
    if (seg == 0) {
      Fs[0] += t;
    } else if (seg == 2) {
      Fs[1] += t;
    } else {
      const bool up = j < kk;
      Fs[0] += up ? t : 0.0;
      Fs[1] += up ? 0.0 : t;
    }
    Fs[2] += tr;
    Fs[3] = __builtin_fma(tr, r, Fs[3]);
  });
  wg_sum<4>(Fs, W, wv, lane, red);
  {
    const double sp = Fs[0], sn = Fs[1];
    Fs[0] = sp + sn;  // sum of the terms
    Fs[1] = sp - sn;  // sum of their magnitudes
  }
  double F = 1.0 + rho * Fs[0];
  // The estimated reciprocals leave the sign of F open when |F| is within
  // their error (2^-23 of the sum of |terms|, taken with a margin of 8): such
  // lanes repeat the test with corrected quotients, so that the shift pole
  // differs from a serial IEEE evaluation only where F is zero to rounding
  // (the eigenvalue at the midpoint of its gap: either pole is then nearest).
  // Every wave of the block holds the same per-lane state, so all take the
  // branch together.
  const bool open = valid && kk > 0 && fabs(F) <= 0x1p-20 * (1.0 + rho * Fs[1]);
  if (wave_any(open)) {
    double Fr[1] = {0.0};
    sweep(P, j0, j1, wlo, whi, [&](int, int, double dj, double z2, double, int) {
      const double den = (dj - dk) - tau;
      const double r = rcp_1nr(den);
      double t = z2 * r;
      t = __builtin_fma(__builtin_fma(-t, den, z2), r, t);
      Fr[0] += t;
    });
    wg_sum<1>(Fr, W, wv, lane, red);
    if (open) F = 1.0 + rho * Fr[0];
  }
  const bool right = (kk == 0) || (F > 0);
  const int i = right ? kk : kk - 1;
  const double s = right ? 1.0 : -1.0;
  const double sigma = right ? dk : dkm1;
  const double zi = Zv[i];
  const double zi2 = zi * zi;

  // ---- tip b of A_i^{-1} (eq. b_ob) in double-double, plus the binary64 sums
  // of eq. (knu2).  P collects j < i (delta > 0), N collects j > i.
  // Each term zeta_j^2/(d_j - sigma) is formed as q1 + q2 from the exact
  // difference (TwoSum), the exact square (hi + lo) and one residual
  // correction, relative error about 2^-100.  P and N each add terms of one
  // sign (N adds the negated terms), so max/min by value orders the operands
  // by magnitude: each sum is a Neumaier compensated sum of the q1 whose
  // compensation also collects the q2.  Its error is O(n eps^2) of the sum,
  // as for a double-double accumulation, at 7 operations a term instead of 11.
  double ps = 0.0, pc = 0.0, ns = 0.0, nc = 0.0;
  auto acc = [](double& a, double& c, double q1, double q2) {
    const double hi = fmax(a, q1), lo = fmin(a, q1);
    const double y = hi + lo;
    c += ((hi - y) + lo) + q2;
    a = y;
  };
  sweep_lo(P, Zl, j0, j1, wlo, whi, [&](int j, int seg, double dj, double z2, double z2l, int) {
    dd dl = two_sum(dj, -sigma);  // exact d_j - sigma
    double r = rcp_1nr(dl.hi);
    double q1 = z2 * r;
    double e = __builtin_fma(-q1, dl.hi, z2);
    e = __builtin_fma(-q1, dl.lo, e + z2l);
    double q2 = e * r;
    if (seg == 0) {
      acc(ps, pc, q1, q2);
    } else if (seg == 2) {
      acc(ns, nc, -q1, -q2);
    } else if (j != i) {
      const bool up = j < i;
      double a = up ? ps : ns, c = up ? pc : nc;
      acc(a, c, up ? q1 : -q1, up ? q2 : -q2);
      if (up) { ps = a; pc = c; } else { ns = a; nc = c; }
    }
  });
  dd Pd = fast_two_sum(ps, pc);
  dd Nd = fast_two_sum(-ns, -nc);
  wg_sum_dd(Pd, W, wv, lane, red);
  wg_sum_dd(Nd, W, wv, lane, red);
  const dd rr = dd_div(dd{1.0, 0.0}, dd{rho, 0.0});
  const dd num = dd_add(dd_add_same(rr, Pd), Nd);
  const dd bdd = dd_div_sq(num, zi);
  const double Pr = rho * Pd.hi, Nr = rho * Nd.hi;
  const double Kb64 = (1.0 + Pr - Nr) / fabs(1.0 + Pr + Nr);
  bool use_ext = A.mode_b == 0 || (A.mode_b == 1 && Kb64 > 100.0);
  if (A.mode_b == 3) {
    // Algorithm 1's gate: the bound of eq. (knu2) from the standard-precision
    // K_b above 100 (n+4) sqrt(n) (K_b > 100 unless K_z shows that b cannot
    // influence ||A_i^{-1}||)
    const double sn = sqrt((double)n), azi = fabs(zi);
    const double Kz = (M.zabs - azi) / azi;
    const double k1 = (n + 4) * sn * Kb64, k2 = 3.0 * sn + (n + 4) * (1.0 + 2.0 * Kz);
    use_ext = fmin(k1, k2) > 100.0 * (n + 4) * sn;
  }
  const double rzi = 1.0 / zi;
  const double b64 = ((1.0 / rho + Pd.hi) + Nd.hi) * (rzi * rzi);
  const double bh = use_ext ? bdd.hi : b64;
  const double bl = use_ext ? bdd.lo : 0.0;
  const double bp = s * bh;  // b' of the mirrored (rightmost) problem

  // ---- extreme root nu' > 0 of g(nu') = b' - nu' + S(nu')/zeta_i^2,
  // S(nu') = sum_{j!=i} zeta_j^2/(delta'_j (nu' delta'_j - 1)), delta' = s (d_j - sigma).
  const double nss = -s * sigma;
  const bool interior = kk > 0;
  const double xm = interior ? 1.0 / (dkm1 - dk) : 0.0;  // pole nearest to the root
  // the square root of its weight zeta_jm^2/(delta'_jm^2 zeta_i^2), jm the
  // other end of the gap
  const double zjm = interior ? Zv[right ? kk - 1 : kk] : 0.0;
  const double sw = interior ? fabs(zjm * xm) / fabs(zi) : 0.0;
  double L, U, nu;
  if (interior) {
    L = xm;
    U = INFINITY;
    nu = 2.0 * xm;  // mu at the midpoint of the gap: the nearest-pole bound
  } else {
    L = Lx;
    U = Ux;
    nu = nux;
  }
  // the rigorous bracket [L0, U0] (set below) is kept for the double-double
  // polish: the signs of g seen by the binary64 iteration can be wrong when g
  // is badly conditioned
  bool done = !valid;
  int iters = 0;
  double nu0 = nu, prevstep = INFINITY, g1 = 0.0, g2 = 0.0;
  const double rz2 = 1.0 / zi2;

  // First probe from the shift pass: g(nu') = f(lambda)/(rho zeta_i^2) up to
  // the sign s (eqs. secAi, Pick).  For an interior root lambda is the gap
  // midpoint, so g >= 0 there by the choice of the shift; b' + S/zeta_i^2 =
  // g + nu' is then an upper bound of the root (S decreases).  If rounding
  // leaves the sign of g open the pole is kept as the lower end.  For k = 1
  // the probe may lie on either side of the root.
  bool pre = valid;
  double pre_Sz = 0.0, pre_Spz = 0.0, pre_Sppz = 0.0, pre_g = 0.0;
  if (pre) {
    // error of f(lambda) from the estimated reciprocals: 2^-23 of |terms|,
    // taken with a margin of 8
    const double gerr = 0x1p-20 * (1.0 + rho * Fs[1]) / (rho * zi2);
    pre_g = s * (1.0 + rho * Fs[0]) / (rho * zi2);
    pre_Sz = (pre_g - bp) + nu;
    // g' = -F2/(zeta_i^2 nu^2) and g'' = 2 (s F3/nu^4 + F2/nu^3)/zeta_i^2 with
    // F2, F3 the sums of zeta_j^2/(d_j - lambda)^2 and ^3 (lambda = sigma + s/nu)
    const double inu = 1.0 / nu;
    pre_Spz = fmax(Fs[2] / (zi2 * nu * nu) - 1.0, 0.0);
    pre_Sppz = (((s * Fs[3]) * inu + Fs[2]) * (inu * inu * inu)) / zi2;
    if (interior) {
      U = (nu + fmax(pre_g, 0.0) + gerr) * GROW;
      if (pre_g > gerr) L = nu;
    } else if (pre_g > gerr) {
      L = nu;
      U = fmin(U, (nu + pre_g + gerr) * GROW);
    } else if (pre_g < -gerr) {
      U = nu;
    }
  }
  const double L0 = L, U0 = U;

  if (A.root == 0) {
    // -------- bisection in the order of the binary64 numbers
    while (wave_any(!done)) {
      double m = nu;
      double S[1] = {0.0};
      if (wave_any(!done && !pre)) {
        sweep(P, j0, j1, wlo, whi, [&](int j, int seg, double dj, double z2, double, int) {
          double dl = __builtin_fma(s, dj, nss);
          double pp = __builtin_fma(m, dl, -1.0);
          double t = z2 * rcp_1nr(dl * pp);
          if (seg == 1 && j == i) t = 0.0;
          S[0] += t;
        });
        wg_sum<1>(S, W, wv, lane, red);
        ++iters;
      }
      if (!done) {
        double Sz = S[0] * rz2;
        double g = (bp - m) + Sz;
        if (pre) {
          g = pre_g;
          pre = false;  // bracket already set from the probe
        } else {
          if (g > 0) L = m; else U = m;
        }
        if (adjacent(L, U) || iters >= 200) {
          done = true;
          nu0 = U;
        } else {
          nu = fmid(L, U);
        }
      }
    }
  } else {
    // -------- safeguarded model iteration: every pass gives the value, slope
    // and curvature of the sum term at nu; the root of the model built from
    // them (the nearest pole exact, the rest one fitted pole) is the next
    // iterate.  The last pass of the budget is the accurate one below.
    // The step from the probe costs no pass and is always taken.
    const int budget = max(A.main_passes, 1);
    int passes = 0;
    while (wave_any(!done) && (passes < budget - 1 || wave_any(pre))) {
      double m = nu;
      double S[3] = {0.0, 0.0, 0.0};
      if (wave_any(!done && !pre)) {
        sweep(P, j0, j1, wlo, whi, [&](int j, int seg, double dj, double z2, double, int) {
          double dl = __builtin_fma(s, dj, nss);
          double pp = __builtin_fma(m, dl, -1.0);
          double rq = __builtin_amdgcn_rcp(dl * pp);
          double t = z2 * rq;           // w_j/(m - xi_j)
          double u = (dl * rq) * dl;    // delta'_j/pp = 1/(m - xi_j)
          double tp = t * u;            // w_j/(m - xi_j)^2
          if (seg == 1 && j == i) {     // (dl = 0 there: u is NaN)
            t = 0.0;
            tp = 0.0;
            u = 0.0;
          }
          S[0] += t;
          S[1] += tp;
          S[2] = __builtin_fma(tp, u, S[2]);  // w_j/(m - xi_j)^3
        });
        wg_sum<3>(S, W, wv, lane, red);
        ++iters;
        ++passes;
      }
      if (!done) {
        double Sz = S[0] * rz2;
        double Spz = S[1] * rz2;  // -dS/dnu / zeta_i^2
        double Sppz = S[2] * rz2;
        double g = (bp - m) + Sz;
        if (pre) {
          Sz = pre_Sz;
          Spz = pre_Spz;
          Sppz = pre_Sppz;
          g = pre_g;
          pre = false;  // bracket already set from the probe
        } else {
          // the terms of a plain pass carry the error of the estimated
          // reciprocal (below 2^-23, all terms positive): a sign of g within
          // that error leaves the bracket as it is
          const double gtol = 0x1p-20 * Sz + 0x1p-50 * fabs(bp);
          if (g > gtol) L = m; else if (g < -gtol) U = m;
        }
        model_step(m, g, Sz, Spz, Sppz, bp, xm, sw, iters, L, U, nu, nu0, prevstep, g1, g2, done);
      }
    }
  }

  // ---- accurate pass at m: compensated sum of the secular terms (each a
  // corrected quotient), the moments for the last step, the amplification
  // estimate kappa_g = (|b| + |nu| + S)/(|nu| |g'|) and ||x||.  After
  // bisection m is the converged bracket end and the last step is Newton's;
  // in the model iteration m is the converged iterate (or the next one for a
  // lane that has not converged) and the last step is the model's, which is
  // accepted when it is below 2^-20 relative.  Right of every pole all terms
  // are positive: the eight terms of a block are added as a tree of depth 3
  // (error at most 3 eps of the block sum), and the block sums go into a
  // Neumaier sum, which takes the larger operand first by value.
  const double m = (A.root == 0 || done) ? nu0 : nu;
  double cs = 0.0, cc = 0.0;
  double Sp[3] = {0.0, 0.0, 0.0};
  double ga = 0.0, gb = 0.0, gc = 0.0;
  auto neu = [&](double t) {
    const double hi = fmax(cs, t), lo = fmin(cs, t);
    const double y = hi + lo;
    cc += (hi - y) + lo;
    cs = y;
  };
  sweep(P, j0, j1, wlo, whi, [&](int j, int seg, double dj, double z2, double, int ub) {
    double dl = __builtin_fma(s, dj, nss);
    double pp = __builtin_fma(m, dl, -1.0);
    // q > 0; beyond binary64 (a far pole with nu near 1e300) it is held at the
    // largest finite number, where the quotient is 0 to working precision and
    // the correction below stays finite (0 * inf would be NaN)
    double q = fmin(dl * pp, DBL_MAX);
    double r = rcp_1nr(q);
    double t = z2 * r;
    t = __builtin_fma(__builtin_fma(-t, q, z2), r, t);  // corrected quotient
    double u = (dl * r) * dl;                           // 1/(m - xi_j)
    double tp = t * u;                                  // zeta_j^2/pp^2
    double tp3 = tp * u;                                // zeta_j^2 delta'_j/pp^3
    if (seg == 1 && j == i) {                           // (dl = 0 there: u is NaN)
      t = 0.0;
      tp = 0.0;
      tp3 = 0.0;
      u = 0.0;
    }
    switch (ub) {
      case 0: ga = t; break;
      case 1: ga += t; break;
      case 2: gb = t; break;
      case 3: gb += t; ga += gb; break;
      case 4: gb = t; break;
      case 5: gb += t; break;
      case 6: gc = t; break;
      case 7: gc += t; gb += gc; ga += gb; neu(ga); break;
      default: neu(t);
    }
    Sp[0] += tp;
    Sp[1] += tp3;
    Sp[2] = __builtin_fma(tp3, u, Sp[2]);               // zeta_j^2 delta'_j^2/pp^4
  });
  wg_sum_comp(cs, cc, W, wv, lane, red);
  wg_sum<3>(Sp, W, wv, lane, red);
  const double Sz = (cs + cc) / zi2;
  const double g = (bp - m) + Sz;
  const double gp = -1.0 - Sp[0] / zi2;
  // divided in two steps: m |g'| overflows when nu nears 1e304
  const double kap = ((fabs(bp) + m + Sz) / m) / fabs(gp);
  double nu1 = m;
  bool fin = true;
  if (A.root == 0) {
    nu1 = m - g / gp;
  } else if (valid) {
    fin = false;
    if (g > 0) L = m; else if (g < 0) U = m;
    double nn = m;
    model_step(m, g, Sz, Sp[0] / zi2, Sp[1] / zi2, bp, xm, sw, iters, L, U, nu, nn, prevstep, g1, g2, fin);
    if (fin) nu1 = nn;
  }
  const bool cont = valid && !fin;  // unfinished: continued in k_fix
  double muv = s / nu1;
  double lam = sigma + muv;
  double amp = fabs(muv / lam);
  if (!(amp > 1.0)) amp = 1.0;
  const bool pol = valid && !cont && A.polish && (kap * amp > A.kappa_polish);
  bool nz = false;
  if (valid && !cont && !pol && A.nearzero > 0) {
    double gap = fabs(lam - dk);
    if (kk > 0) gap = fmin(gap, fabs(lam - dkm1));
    nz = A.nearzero * fabs(lam) < gap;
  }

  // ---- ||x|| scaled by |mu|: with delta_j - mu = s (delta'_j - 1/nu) one has
  // mu/(delta_j - mu) = 1/(nu delta'_j - 1), so |mu|^2 ||x||^2 =
  // zeta_i^2 + sum_{j != i} zeta_j^2/pp_j^2, the S' sum of the accurate pass.
  // That sum is taken at m and carried to nu1 = m + h by its Taylor series to
  // second order (derivatives -2 sum zeta^2 delta'/pp^3 and 6 sum zeta^2
  // delta'^2/pp^4; |h|/(m - xi_j) <= 2^-19, so the error is below 2^-55).
  // The products are formed as h (h S) so that an h near 1e300 (nu = 1/mu
  // for a mu near 1e-300, beside a zeta_i near 1e-150) meets the underflowed
  // sums before it is squared: h h would overflow and inf * 0 be NaN.
  const double h = nu1 - m;
  double Nx[1] = {zi2 + ((Sp[0] - 2.0 * (h * Sp[1])) + 3.0 * (h * (h * Sp[2])))};
  if (wv == 0 && valid) {
    A.ii[off + k] = i;
    A.vflag[off + k] = (pol || nz || cont) ? 1 : 0;
    A.mu[off + k] = muv;
    // a tip b' beyond binary64 (zeta_i near 1e-150 beside a pole 1e-13 away
    // with an O(1) zeta) leaves g undefined: the NaN norm makes the output
    // check report DPR1_INFO_RANGE instead of a wrong vector
    A.xs[off + k] = fabs(bp) < INFINITY ? sqrt(Nx[0]) : NAN;
    A.lam[off + k] = lam;
    if (pol || nz || cont) {
      // the long items (polish, near-zero recomputation) fill the list from
      // the front, roots only continued fill it from the back, so that the
      // queue of k_fix hands out the long ones first
      const bool longer = pol || nz;
      int e = longer ? atomicAdd(&A.ctr[0], 1) : A.nfixcap - 1 - atomicAdd(&A.ctr[3], 1);
      FixItem it;
      it.p = p;
      it.k = k;
      it.i = i;
      it.flags = (pol ? FIX_POLISH : 0) | (nz ? FIX_NEARZERO : 0) | (cont ? FIX_CONTINUE : 0);
      it.iters = iters;
      it.pad = 0;
      it.nu0 = m;
      it.nu1 = nu1;
      it.bhi = bp;
      it.blo = s * bl;
      it.lo = L0;
      it.hi = U0;
      it.cnu = nu;
      it.cL = L;
      it.cU = U;
      it.cprev = prevstep;
      A.fix[e] = it;
    }
  }
  if (A.stats && wv == 0) {
    bool kb = valid && Kb64 > 100.0;
    unsigned long long bal = __ballot(kb);
    const unsigned long long bext = __ballot(valid && use_ext);
    int itv = valid ? iters : 0;
    int imax = itv, isum = itv;
    for (int o = 32; o > 0; o >>= 1) {
      imax = max(imax, __shfl_xor(imax, o));
      isum += __shfl_xor(isum, o);
    }
    if (lane == 0) {
      if (bal) atomicAdd(&A.stats[DPR1_STAT_KB_GT_100], __popcll(bal));
      if (bext) atomicAdd(&A.stats[DPR1_STAT_EXT_B], __popcll(bext));
      atomicMax(&A.stats[DPR1_STAT_ITERS_MAX], imax);
      atomicAdd(&A.stats[DPR1_STAT_ITERS_SUM], isum);
    }
  }
}

// OCC: waves per SIMD the register allocation is made for (4: up to 128
// VGPRs; 6: 80; 8: 64, the outer state then partly in scratch, the inner
// sweeps unchanged), so that more waves can hide the FP64 latencies.
template <int OCC>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) k_eig(KArgs A) {
  extern __shared__ double red[];
  if (A.items == nullptr) {
    eig_block(A, 0, (A.g0 + (int)blockIdx.x) * WAVE, red);
    return;
  }
  // persistent: take (problem, first eigenvalue) items from the queue
  __shared__ int item;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(&A.ctr[1], 1);
    __syncthreads();
    int it = item;
    __syncthreads();
    if (it >= A.nitems) break;
    int2 pk = A.items[it];
    eig_block(A, pk.x, pk.y, red);
  }
}

// ------------------------------------------------------------------- fix
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ dd wave_sum_same(dd a) {
  for (int o = 32; o > 0; o >>= 1) {
    dd b = {__shfl_xor(a.hi, o), __shfl_xor(a.lo, o)};
    a = dd_add_same(a, b);
  }
  return a;
}
__device__ __forceinline__ dd wave_sum_dd(dd a) {
  for (int o = 32; o > 0; o >>= 1) {
    dd b = {__shfl_xor(a.hi, o), __shfl_xor(a.lo, o)};
    a = dd_add(a, b);
  }
  return a;
}
// Neumaier partials of the lanes, combined in a fixed butterfly order

// Block-wide sums over FIXT threads (4 waves) in a fixed order; every thread
// receives the total.
constexpr int FIXT = 256;
__device__ __forceinline__ double block_sum(double v, double* sm) {
  v = wave_sum(v);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) sm[wv] = v;
  __syncthreads();
  return (sm[0] + sm[1]) + (sm[2] + sm[3]);
}
__device__ __forceinline__ double block_min(double v, double* sm) {
  v = wave_min(v);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) sm[wv] = v;
  __syncthreads();
  return fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3]));
}
__device__ __forceinline__ dd block_sum_same(dd a, double* sm) {
  a = wave_sum_same(a);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) {
    sm[wv] = a.hi;
    sm[4 + wv] = a.lo;
  }
  __syncthreads();
  dd r = dd_add_same(dd{sm[0], sm[4]}, dd{sm[1], sm[5]});
  r = dd_add_same(r, dd{sm[2], sm[6]});
  return dd_add_same(r, dd{sm[3], sm[7]});
}
__device__ __forceinline__ dd block_sum_dd(dd a, double* sm) {
  a = wave_sum_dd(a);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) {
    sm[wv] = a.hi;
    sm[4 + wv] = a.lo;
  }
  __syncthreads();
  dd r = dd_add(dd{sm[0], sm[4]}, dd{sm[1], sm[5]});
  r = dd_add(r, dd{sm[2], sm[6]});
  return dd_add(r, dd{sm[3], sm[7]});
}
__device__ __forceinline__ double block_sum_comp(double s, double c, double* sm) {
  // Neumaier partials: wave butterflies, then the four wave results in order
  for (int o = 32; o > 0; o >>= 1) {
    double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
    dd t = two_sum(s, s2);
    s = t.hi;
    c = c + c2 + t.lo;
  }
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) {
    sm[wv] = s;
    sm[4 + wv] = c;
  }
  __syncthreads();
  double S = sm[0], C = sm[4];
  for (int w = 1; w < 4; ++w) {
    dd t = two_sum(S, sm[w]);
    S = t.hi;
    C += sm[4 + w] + t.lo;
  }
  return S + C;
}

// One block of FIXT threads per flagged eigenpair at a time; the inner index
// is strided over the block and every pass ends in a block-wide sum.
// The four sums of a continued pass in one exchange: the Neumaier partials
// (s, c) combined as in block_sum_comp and three plain sums a, b, e as in
// block_sum (same orders, so the same results), with one pair of barriers
// instead of four.  sm holds 20 values.
__device__ __forceinline__ double block_sum_comp3(double s, double c, double& a, double& b, double& e,
                                                  double* sm) {
  for (int o = 32; o > 0; o >>= 1) {
    const double s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
    const dd t = two_sum(s, s2);
    s = t.hi;
    c = c + c2 + t.lo;
  }
  a = wave_sum(a);
  b = wave_sum(b);
  e = wave_sum(e);
  const int wv = threadIdx.x / WAVE;
  __syncthreads();
  if (threadIdx.x % WAVE == 0) {
    sm[wv] = s;
    sm[4 + wv] = c;
    sm[8 + wv] = a;
    sm[12 + wv] = b;
    sm[16 + wv] = e;
  }
  __syncthreads();
  double S = sm[0], C = sm[4];
  for (int w = 1; w < 4; ++w) {
    dd t = two_sum(S, sm[w]);
    S = t.hi;
    C += sm[4 + w] + t.lo;
  }
  a = (sm[8] + sm[9]) + (sm[10] + sm[11]);
  b = (sm[12] + sm[13]) + (sm[14] + sm[15]);
  e = (sm[16] + sm[17]) + (sm[18] + sm[19]);
  return S + C;
}

// Safeguarded iteration for the extreme root of g (eq. secAi) at the shift
// pole d_i (side s), g evaluated in double-double: far from the root the
// rational model step of the main solver, close to it Newton (g exact to
// ~2^-100, so the last step lands on the rounded root).  b' = s b in
// double-double, xm the nearest pole of g (in nu), (lo0, hi0) a rigorous
// bracket, cur the start.  Returns the last iterate; *last receives the
// Newton correction at it (nu = cur + *last to about 2^-100), *steps the
// number of double-double evaluations.  All threads of the block call it and
// return the same values.
__device__ double dd_polish(const double2* Z2v, const double* Zl, int n, int i, double s, double sigma, double zi,
                           dd bdd, double xm, double lo0, double hi0, double cur, double* last, int* steps,
                           double* sm) {
  const int tid = threadIdx.x;
  const double zi2 = zi * zi;
  double lo = lo0, hi = hi0;
  if (!(cur > lo && cur < hi)) cur = fmid(lo, hi);
  // progress guard: when |g| has not halved over two steps away from the
  // final Newton phase, the model is not describing g (a pole one ulp from
  // the shift pole dominates it), and the step is a bisection
  double gprev = INFINITY, newton = 0.0;
  int slow = 0, pit;
  for (pit = 0; pit < 100; ++pit) {
    dd acc = {0.0, 0.0};
    double sp = 0.0;
#pragma unroll 4
    for (int j = tid; j < n; j += FIXT) {
      if (j == i) continue;
      const double2 pj = Z2v[j];
      double dj = pj.x, z2 = pj.y;
      dd dl = two_sum(s * dj, -s * sigma);               // delta'_j exactly
      dd pp = dd_add(dd_mul_d(dl, cur), dd{-1.0, 0.0});   // nu delta' - 1
      dd q = dd_mul(dl, pp);
      if (!(q.hi < DBL_MAX)) q = {DBL_MAX, 0.0};  // beyond binary64: the term is 0
      // (zeta_j^2 hi + lo)/q: leading quotient from the refined reciprocal
      // (2^-48.7) and one residual correction, about 2^-97
      const double r = rcp_1nr(q.hi);
      const double q1 = z2 * r;
      double e = __builtin_fma(-q1, q.hi, z2);
      e = __builtin_fma(-q1, q.lo, e + Zl[j]);
      dd t = fast_two_sum(q1, e * r);
      acc = dd_add_same(acc, t);
      sp += z2 * rcp_1nr(pp.hi * pp.hi);  // g' only steers the step
    }
    acc = block_sum_same(acc, sm);
    sp = block_sum(sp, sm);
    dd Sdd = dd_div_sq(acc, zi);
    dd gd = dd_add(dd_add(bdd, dd{-cur, 0.0}), Sdd);
    double Spz = sp / zi2;
    double gpv = -1.0 - Spz;
    newton = 0.0;
    if (gd.hi == 0.0) break;
    if (gd.hi > 0) lo = cur; else hi = cur;
    const double ag = fabs(gd.hi);
    slow = ag > 0.5 * gprev ? slow + 1 : 0;
    gprev = ag;
    newton = -(gd.hi + gd.lo) / gpv;
    double t;
    if (fabs(newton) <= 0x1p-30 * cur) {
      t = cur + newton;
    } else {
      double x = cur - xm;
      double Am = Spz * x * x;
      double C = (bdd.hi + (Sdd.hi - Spz * x)) - xm;
      double disc = sqrt(C * C + 4.0 * Am);
      double u = C >= 0 ? (C + disc) * 0.5 : (2.0 * Am) / (disc - C);
      t = xm + u;
    }
    // stay inside the sign bracket and off the pole / rigorous lower end
    if (!(t >= lo && t <= hi) || !(t > lo0) || !(t < INFINITY) || (slow >= 2 && fabs(newton) > 0x1p-30 * cur)) {
      t = fmid(lo, hi);
      slow = 0;
    }
    if (t == cur) break;
    cur = t;
  }
  *last = fabs(newton) <= 0x1p-30 * cur ? newton : 0.0;
  *steps = pit;
  return cur;
}

// Item e of the list: the n0 long items sit at the front, the others at the
// back in reverse order.
__device__ __forceinline__ int fix_slot(const KArgs& A, int n0, int e) {
  return e < n0 ? e : A.nfixcap - 1 - (e - n0);
}

__device__ void fix_items(const KArgs& A) {
  __shared__ double sm[20];
  __shared__ int next;
  const int tid = threadIdx.x;
  const int n0 = A.ctr[0];
  const int cnt = n0 + A.ctr[3];
  for (;;) {
    // items are taken from a queue, long ones first, so a block that drew
    // cheap items takes more of them (polish steps cost several times a
    // continued root's)
    if (tid == 0) next = atomicAdd(&A.ctr[2], 1);
    __syncthreads();
    const int e = next;
    __syncthreads();
    if (e >= cnt) break;
    const FixItem it = A.fix[fix_slot(A, n0, e)];
    const Meta M = A.meta[it.p];
    const int n = M.n;
    const int64_t off = M.off;
    const double* Dv = A.sd + off;
    const double* Zv = A.sz + off;
    const double* Z2 = A.pairs + 2 * off;
    const double2* Z2v = reinterpret_cast<const double2*>(Z2);  // (d_j, zeta_j^2), 16-byte aligned
    const double* Zl = A.z2lo + off;
    const double rho = M.rho;
    const int k = it.k, i = it.i;
    const double s = (i == k) ? 1.0 : -1.0;
    const double sigma = Dv[i];
    const double zi = Zv[i];
    const double zi2 = zi * zi;
    double muv = A.mu[off + k];
    double lam = A.lam[off + k];
    bool nz = (it.flags & FIX_NEARZERO) != 0;
    bool pol = (it.flags & FIX_POLISH) != 0;
    bool polished = false;
    int singular = 0;
    int pit = 0;  // double-double steps of the polish
    double nu0 = it.nu0, nu1 = it.nu1;
    double xsv = 0.0;
    bool have_xs = false;

    if (it.flags & FIX_CONTINUE) {
      // the root search continued with block-wide sums; every pass is the
      // accurate one of the eigenvalue kernel (compensated sum, corrected
      // quotients, derivative sums up to the third), so the pass whose model
      // step is accepted also gives kappa_g and ||x||
      const double xm = (k > 0) ? 1.0 / (Dv[k - 1] - Dv[k]) : 0.0;
      const double zjm = (k > 0) ? Zv[i == k ? k - 1 : k] : 0.0;
      const double sw = (k > 0) ? fabs(zjm * xm) / fabs(zi) : 0.0;
      const double bp = it.bhi;
      double nu = it.cnu, L = it.cL, U = it.cU, prevstep = it.cprev, g1 = 0.0, g2 = 0.0;
      int iters = it.iters;
      bool done = false;
      double m = nu, Sz = 0.0, sp = 0.0, sp3 = 0.0, sp4 = 0.0;
      while (!done) {
        m = nu;
        double cs = 0.0, cc = 0.0;
        sp = 0.0;
        sp3 = 0.0;
        sp4 = 0.0;
#pragma unroll 4
        for (int j = tid; j < n; j += FIXT) {
          if (j == i) continue;
          const double2 pj = Z2v[j];
          const double dl = __builtin_fma(s, pj.x, -s * sigma);
          const double pp = __builtin_fma(m, dl, -1.0);
          const double q = fmin(dl * pp, DBL_MAX);  // as in k_eig's accurate pass
          const double r = rcp_1nr(q);
          double t = pj.y * r;
          t = __builtin_fma(__builtin_fma(-t, q, pj.y), r, t);  // corrected quotient
          const double u = (dl * r) * dl;                       // 1/(m - xi_j)
          const double tp = t * u;
          const double tp3 = tp * u;
          const double hi = fmax(cs, t), lo = fmin(cs, t);     // positive terms
          const double y = hi + lo;
          cc += (hi - y) + lo;
          cs = y;
          sp += tp;
          sp3 += tp3;
          sp4 = __builtin_fma(tp3, u, sp4);
        }
        Sz = block_sum_comp3(cs, cc, sp, sp3, sp4, sm) / zi2;
        ++iters;
        const double g = (bp - m) + Sz;
        if (g > 0) L = m; else if (g < 0) U = m;
        model_step(m, g, Sz, sp / zi2, sp3 / zi2, bp, xm, sw, iters, L, U, nu, nu0, prevstep, g1, g2, done);
      }
      nu1 = nu0;
      const double gp = -1.0 - sp / zi2;
      const double kap = ((fabs(bp) + m + Sz) / m) / fabs(gp);  // as in k_eig
      muv = s / nu1;
      lam = sigma + muv;
      double amp = fabs(muv / lam);
      if (!(amp > 1.0)) amp = 1.0;
      pol = A.polish && (kap * amp > A.kappa_polish);
      if (!pol && A.nearzero > 0) {
        double gap = fabs(lam - Dv[k]);
        if (k > 0) gap = fmin(gap, fabs(lam - Dv[k - 1]));
        nz = A.nearzero * fabs(lam) < gap;
      }
      // ||x|| carried from m to the root to second order, as in k_eig
      const double h = nu1 - m;
      xsv = sqrt(zi2 + ((sp - 2.0 * (h * sp3)) + 3.0 * (h * (h * sp4))));
      nu0 = m;
      have_xs = true;
    }

    if (pol) {
      const dd bdd = {it.bhi, it.blo};
      const double xm = (k > 0) ? 1.0 / (Dv[k - 1] - Dv[k]) : 0.0;
      double cur = nu1;
      if (!(cur > it.lo && cur < it.hi)) cur = nu0;
      double last;
      cur = dd_polish(Z2v, Zl, n, i, s, sigma, zi, bdd, xm, it.lo, it.hi, cur, &last, &pit, sm);
      muv = s / cur;
      lam = sigma + muv;
      polished = true;
      if (A.nearzero > 0) {
        double gap = fabs(lam - Dv[k]);
        if (k > 0) gap = fmin(gap, fabs(lam - Dv[k - 1]));
        nz = A.nearzero * fabs(lam) < gap;
      }
    }

    if (nz) {
      // eq. (gamma): f(0) = 1 + rho z^T D^{-1} z in double-double
      dd f0 = {0.0, 0.0};
      double uu = 0.0, dmin = INFINITY;
      #pragma unroll 4
        for (int j = tid; j < n; j += FIXT) {
        const double2 pj = Z2v[j];
          double dj = pj.x, z2 = pj.y;
        dd t = dd_div(dd{z2, Zl[j]}, dd{dj, 0.0});
        f0 = dd_add(f0, t);
        double u = Zv[j] / dj;
        uu += u * u;
        dmin = fmin(dmin, fabs(dj));
      }
      f0 = block_sum_dd(f0, sm);
      uu = block_sum(uu, sm);
      dmin = block_min(dmin, sm);
      f0 = dd_add(dd{1.0, 0.0}, dd_mul_d(f0, rho));
      double f0d = f0.hi + f0.lo;
      if (f0d == 0.0) {
        lam = 0.0;
        singular = 1;
      } else {
        const double gam = -rho / f0d;
        const double sh = (f0d < 0) ? 1.0 : -1.0;  // sign of lambda
        const double gt = sh * gam;
        // eta~ = sh/lambda > 0 on the right branch of
        // h(eta~) = 1 + gt sum zeta_j^2/(d~_j (1 - eta~ d~_j)),  d~ = sh d
        double lo;
        if (sh > 0) lo = (k > 0) ? 1.0 / Dv[k - 1] : 4.9406564584124654e-324;
        else lo = -1.0 / Dv[k];
        double hi = (1.0 / dmin + fabs(gam) * uu) * GROW;
        if (!(lo > 0)) lo = 4.9406564584124654e-324;
        if (!(hi > lo)) hi = lo * 2.0;
        for (int hit = 0; hit < 200 && !adjacent(lo, hi); ++hit) {
          double m = fmid(lo, hi);
          double acc = 0.0;
          #pragma unroll 4
        for (int j = tid; j < n; j += FIXT) {
            const double2 pj = Z2v[j];
            double dt = sh * pj.x, z2 = pj.y;
            acc += z2 / (dt * __builtin_fma(-m, dt, 1.0));
          }
          acc = block_sum(acc, sm);
          double hv = 1.0 + gt * acc;
          if (hv < 0) lo = m; else hi = m;
        }
        const double e0 = hi;
        double cs = 0.0, cc = 0.0, sp = 0.0;
        #pragma unroll 4
        for (int j = tid; j < n; j += FIXT) {
          const double2 pj = Z2v[j];
            double dt = sh * pj.x, z2 = pj.y;
          double om = __builtin_fma(-e0, dt, 1.0);
          double t = z2 / (dt * om);
          double y = cs + t;
          cc += (fabs(cs) >= fabs(t)) ? ((cs - y) + t) : ((t - y) + cs);
          cs = y;
          sp += z2 / (om * om);
        }
        double S = block_sum_comp(cs, cc, sm);
        sp = block_sum(sp, sm);
        double hv = 1.0 + gt * S;
        double hp = gt * sp;
        double e1 = e0 - hv / hp;
        lam = sh / e1;
      }
    }

    if (polished) {
      double acc = 0.0;
      #pragma unroll 4
        for (int j = tid; j < n; j += FIXT) {
        double r = muv / ((Dv[j] - sigma) - muv);
        double z2 = Z2[2 * j + 1];
        acc = __builtin_fma(z2 * r, r, acc);
      }
      xsv = sqrt(block_sum(acc, sm));
    }
    if (tid == 0) {
      A.lam[off + k] = lam;
      if (nz) A.vflag[off + k] = 2;  // lambda from eq. (gamma): no remedy of K_nu
      if (polished || have_xs) {
        A.mu[off + k] = muv;
        A.xs[off + k] = fabs(it.bhi) < INFINITY ? xsv : NAN;
      }
      if (A.stats) {
        if (polished) {
          atomicAdd(&A.stats[DPR1_STAT_POLISHED], 1);
          atomicMax(&A.stats[DPR1_STAT_POLISH_STEPS_MAX], min(pit + 1, 100));
        }
        if (it.flags & FIX_CONTINUE) atomicAdd(&A.stats[DPR1_STAT_CONTINUED], 1);
        if (nz) atomicAdd(&A.stats[DPR1_STAT_NEARZERO], 1);
        if (singular) atomicAdd(&A.stats[DPR1_STAT_SINGULAR], 1);
      }
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(FIXT) k_fix(KArgs A) { fix_items(A); }

// ------------------------------------------------------------------- out
// The shifted representation of an eigenpair is usable when lambda is finite,
// mu is a normal number and |mu| ||x|| is finite and positive.  It leaves the
// binary64 range when |delta_j / mu| exceeds it (mu beside a pole with zeta
// near 1e-150 while the poles spread over many decades): the problem's info
// then reports DPR1_INFO_RANGE instead of returning NaN silently.
__device__ __forceinline__ bool range_ok(double lam, double mu, double xs) {
  return fabs(lam) < INFINITY && fabs(mu) >= 2.2250738585072014e-308 && fabs(mu) < INFINITY && xs > 0.0 &&
         xs < INFINITY;
}

// user outputs in the caller's order (rho < 0 maps k -> n-1-k, lambda -> -lambda)
__global__ void __launch_bounds__(256) k_out(const Meta* __restrict__ meta, int nprob,
                                             const int32_t* __restrict__ ii, const double* __restrict__ mu,
                                             const double* __restrict__ xs, const double* __restrict__ lam,
                                             const double* __restrict__ sd, double* __restrict__ csig,
                                             double* __restrict__ cinv, double* __restrict__ lam_out,
                                             int32_t* __restrict__ idx_out, double* __restrict__ mu_out,
                                             double* __restrict__ xn_out, const uint8_t* __restrict__ vflag,
                                             int32_t* __restrict__ info_out, int kb, int ke) {
  // a batch: block p handles problem p; one problem: the grid strides over
  // its eigenvalues kb .. ke-1
  const int p = nprob > 1 ? (int)blockIdx.x : 0;
  const int k0 = nprob > 1 ? (int)threadIdx.x : (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int kstep = nprob > 1 ? (int)blockDim.x : (int)(gridDim.x * blockDim.x);
  if (p >= nprob) return;
  const Meta M = meta[p];
  const int n = M.n;
  if (M.info != 0) {
    // rejected problem: the solver wrote nothing; leave defined outputs
    // (NaN values, in-range shift indices) and no eigenvector constants
    for (int k = k0; k < n; k += kstep) {
      int64_t b = M.off + k;
      lam_out[b] = NAN;
      if (idx_out) idx_out[b] = k;
      if (mu_out) mu_out[b] = NAN;
      if (xn_out) xn_out[b] = NAN;
    }
    return;
  }
  for (int k = kb + k0; k < min(n, ke); k += kstep) {
    int ko = M.neg ? n - 1 - k : k;
    int64_t a = M.off + k, b = M.off + ko;
    double sg = M.neg ? -1.0 : 1.0;
    lam_out[b] = sg * lam[a];
    // per-column constants of the eigenvector kernel: sigma_k and
    // w_k = 1/||x_k|| = |mu|/(|mu| ||x||), so that v_j = zeta_j (w_k/(delta_j -
    // mu)).  The quotient w/(delta_j - mu) = v_j/zeta_j is at most 1/|zeta_j|
    // and underflows only where v_j/zeta_j does; mu/(delta_j - mu) alone would
    // be subnormal beside a distant pole when mu is tiny (1e-304 against
    // delta_j = 1e10) and lose bits although v_j is a normal number
    csig[a] = sd[M.off + ii[a]];
    cinv[a] = fabs(mu[a]) / xs[a];
    if (idx_out) idx_out[b] = M.neg ? n - 1 - ii[a] : ii[a];
    if (mu_out) mu_out[b] = sg * mu[a];
    if (xn_out) xn_out[b] = xs[a] / fabs(mu[a]);
    // flagged pairs are finished (and checked) by k_fix / k_fixout
    if (!vflag[a] && !range_ok(lam[a], mu[a], xs[a])) info_out[p] = DPR1_INFO_RANGE;
  }
}

// ------------------------------------------------------------------- vec
// v_j = zeta_j w/(delta_j - mu), w = 1/||x|| (eq. eigenvecAi).  A block owns up
// to CB columns of one problem over up to ROWS consecutive positions of each
// column.  The (d_j, zeta_j) of those positions are staged in LDS once; each
// wave then writes 64-element windows aligned to 512 bytes of V, so every
// store instruction covers whole cache lines whatever the column's offset
// (a packed ragged batch puts most columns at odd offsets; misaligned
// non-temporal stores write partial lines and halve the write bandwidth).
// Only the first and last window of a column segment are partial.  The
// single-problem launch derives (column group, row tile) from the block
// index; the batched launch reads (problem, first column, columns, first
// row) from a table built by the plan.
constexpr int VEC_T = 256;
constexpr int VEC_ROWS = 2048;
// columns per block: 32 for a batch as for one problem (64 measured 4-7 %
// slower on the 2048-problem mix and on 4 problems of n = 16384, 16 no faster)
constexpr int VEC_C_SINGLE = 32, VEC_C_BATCH = 32;
// most chunks of the overlapped single-problem solve (opts.vwrite)
constexpr int VEC_CHUNKS_MAX = 8;

// Arguments of the eigenvector writer.  Columns flagged in vflag belong to
// eigenpairs that k_fix finishes; they are skipped here and written by
// k_fixout once their values are final.
struct VArgs {
  const Meta* meta;
  const int4* groups;  // batched: (problem, first column, columns, first row) per block
  int64_t ncolgroups;  // single problem: column groups per row tile
  const double* sd;
  const double* sz;
  const double* mu;
  const double* csig;
  const double* cinv;
  const uint8_t* vflag;
  double* V;
  const int64_t* voffs;
  int64_t ldv;
  int32_t cbase, cend;  // single problem: columns cbase .. cend-1
  int32_t prio;         // k_vec: raise the waves' issue priority
  int32_t sweep;        // single problem: waves of vec_sweep (0: vec_block)
};

template <int CB>
__device__ void vec_block(unsigned bid, const VArgs& v) {
  __shared__ double ld_d[VEC_ROWS], ld_z[VEC_ROWS];
  __shared__ double lsig[CB], lmu[CB], linv[CB];
  __shared__ uint8_t lskip[CB];
  const Meta* __restrict__ meta = v.meta;
  const int4* __restrict__ groups = v.groups;
  const int64_t ncolgroups = v.ncolgroups;
  const double* __restrict__ sd = v.sd;
  const double* __restrict__ sz = v.sz;
  double* __restrict__ V = v.V;
  const int64_t* __restrict__ voffs = v.voffs;
  const int64_t ldv = v.ldv;
  int p, c0, nc;
  int64_t r0;
  if (groups) {
    const int4 g = groups[bid];
    p = g.x;
    c0 = g.y;
    nc = g.z;
    r0 = g.w;
  } else {
    p = 0;
    c0 = v.cbase + (int)(bid % ncolgroups) * CB;
    r0 = (int64_t)(bid / ncolgroups) * VEC_ROWS;
    nc = 0;
  }
  const Meta M = meta[p];
  if (M.info != 0) return;
  const int n = M.n;
  if (!groups) nc = min(CB, min(n, v.cend) - c0);
  const int nr = (int)min((int64_t)VEC_ROWS, (int64_t)n - r0);
  if (nc <= 0 || nr <= 0) return;
  const double sg = M.neg ? -1.0 : 1.0;
  // stage positions r0 .. r0+nr-1 (position = row in memory order; a
  // reversed problem stores row j at position n-1-j)
  for (int t = threadIdx.x; t < nr; t += VEC_T) {
    const int64_t pos = r0 + t;
    const int64_t j = M.neg ? n - 1 - pos : pos;
    ld_d[t] = sd[M.off + j];
    ld_z[t] = sg * sz[M.off + j];
  }
  if (threadIdx.x < nc) {
    const int64_t a = M.off + c0 + threadIdx.x;
    lsig[threadIdx.x] = v.csig[a];
    lmu[threadIdx.x] = v.mu[a];
    linv[threadIdx.x] = v.cinv[a];
    lskip[threadIdx.x] = v.vflag ? v.vflag[a] : 0;
  }
  __syncthreads();
  const int64_t ld = voffs ? (int64_t)n : ldv;
  const int64_t base = voffs ? voffs[p] : 0;
  const int wv = wave_id(), lane = threadIdx.x % WAVE;
  constexpr int NW = VEC_T / WAVE;
  if (r0 == 0 && nr == n && ld == n) {
    // Whole columns of a packed block: the group's columns are one
    // contiguous range of nc n elements, written in aligned windows with
    // (column, position) recovered per element.  nc n <= CB VEC_ROWS < 2^24,
    // so the float quotient is off by at most one and corrected exactly.
    const int64_t kolo = M.neg ? (int64_t)n - c0 - nc : c0;
    const int64_t S = base + kolo * n;
    const int len = nc * n;
    const int64_t Sal = S & ~(int64_t)(WAVE - 1);
    const int nwin = (int)((S + len - Sal + WAVE - 1) / WAVE);
    const float inv_n = 1.0f / (float)n;
    for (int w = wv; w < nwin; w += NW) {
      const int64_t e = Sal + (int64_t)w * WAVE + lane;
      const int64_t l64 = e - S;
      if (l64 >= 0 && l64 < len) {
        const int local = (int)l64;
        int q = (int)((float)local * inv_n);
        int pos = local - q * n;
        if (pos < 0) {
          pos += n;
          --q;
        } else if (pos >= n) {
          pos -= n;
          ++q;
        }
        const int ko = (int)kolo + q;
        const int c = (M.neg ? n - 1 - ko : ko) - c0;
        if (lskip[c]) continue;
        const double w = linv[c];
        const double den = (ld_d[pos] - lsig[c]) - lmu[c];
        const double rc = rcp_1nr(den);
        double qq = w * rc;
        qq = __builtin_fma(__builtin_fma(-qq, den, w), rc, qq);  // corrected quotient
        __builtin_nontemporal_store(ld_z[pos] * qq, &V[e]);
      }
    }
    return;
  }
  // Column segments: wave w writes columns w, w + NW, ... of the group, each
  // in windows of 128 elements aligned to 1 KB, two consecutive elements per
  // lane in one 16-byte store (the column's address set up once, then a plain
  // loop; a window's lane with only one element in the segment stores it
  // alone).
  typedef double vdbl2 __attribute__((ext_vector_type(2)));
  constexpr int WE = 2 * WAVE;
  for (int c = wv; c < nc; c += NW) {
    if (lskip[c]) continue;
    const int k = c0 + c;
    const int64_t ko = M.neg ? n - 1 - k : k;
    const int64_t s0 = base + ko * ld + r0;  // element index of the segment's first position
    // windows aligned on the address (V itself need only be 8-byte aligned)
    const int64_t sal = s0 - (int64_t)(((uintptr_t)(V + s0) >> 3) & (WE - 1));
    const int nwin = (int)((s0 + nr - sal + WE - 1) / WE);
    const double m = lmu[c], sc = lsig[c], iv = linv[c];
    double* vp = V + sal + 2 * lane;
    int rel = (int)(sal - s0) + 2 * lane;
    for (int w = 0; w < nwin; ++w, vp += WE, rel += WE) {
      const bool a0 = rel >= 0 && rel < nr, a1 = rel + 1 >= 0 && rel + 1 < nr;
      if (!a0 && !a1) continue;
      const int r0c = a0 ? rel : rel + 1, r1c = a1 ? rel + 1 : rel;
      const double den0 = (ld_d[r0c] - sc) - m, den1 = (ld_d[r1c] - sc) - m;
      const double rc0 = rcp_1nr(den0), rc1 = rcp_1nr(den1);
      double q0 = iv * rc0, q1 = iv * rc1;
      q0 = __builtin_fma(__builtin_fma(-q0, den0, iv), rc0, q0);  // corrected quotients
      q1 = __builtin_fma(__builtin_fma(-q1, den1, iv), rc1, q1);
      const double v0 = ld_z[r0c] * q0, v1 = ld_z[r1c] * q1;
      if (a0 && a1) {
        const vdbl2 vv = {v0, v1};
        __builtin_nontemporal_store(vv, reinterpret_cast<vdbl2*>(vp));
      } else if (a0) {
        __builtin_nontemporal_store(v0, vp);
      } else {
        __builtin_nontemporal_store(v1, vp + 1);
      }
    }
  }
}


// The eigenvector writer of one problem in address order, for a V whose
// columns all start 16-byte aligned (the other case, and batches, take
// vec_block).  HBM takes writes fastest when the whole GPU's write front
// moves through memory in order, as a fill does (a standalone test: 6.3
// TB/s against 5.4 for column groups written independently): wave g keeps
// positions 128 (g % wpc) .. + 127 of every column it writes, their d and
// zeta in registers, two per lane in one 16-byte non-temporal store, and writes the
// groups of SWEEP_U consecutive columns g / wpc, g / wpc + m, ... (m waves
// per position range, nw = m wpc waves in all), the next group's column
// constants loaded while the current one is written.  The arithmetic is
// vec_block's.
constexpr int SWEEP_U = 8, SWEEP_WAVES = 2048;
// lane l's value to every lane (an SGPR), l a compile-time constant
__device__ __forceinline__ double lane_value(double x, int l) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ void vec_sweep(const VArgs& v, int g, int nw) {
  const Meta M = v.meta[0];
  if (M.info != 0) return;
  const int n = M.n;
  const int wpc = (n + 2 * WAVE - 1) / (2 * WAVE);
  const int m = nw / wpc;
  const int r = g % wpc, cg = g / wpc;
  if (cg >= m) return;
  const int lane = lane_id();
  const int pos = 2 * WAVE * r + 2 * lane;
  const bool a0 = pos < n, a1 = pos + 1 < n;
  const double sg = M.neg ? -1.0 : 1.0;
  const int64_t j0 = M.neg ? n - 1 - pos : pos, j1 = M.neg ? n - 2 - pos : pos + 1;
  const double d0 = a0 ? v.sd[M.off + j0] : 0.0, z0 = a0 ? sg * v.sz[M.off + j0] : 0.0;
  const double d1 = a1 ? v.sd[M.off + j1] : 0.0, z1 = a1 ? sg * v.sz[M.off + j1] : 0.0;
  const int cb = v.cbase, ce = min(n, v.cend);
  const int ngrp = (ce - cb + SWEEP_U - 1) / SWEEP_U;
  // the constants of group q in one load across the wave: lane u + 8 t
  // holds, for column cb + q SWEEP_U + u, sigma (t = 0), mu (1), 1/||x||
  // (2) or 1 for a column to skip (3: past the range, or one k_fixout
  // writes)
  auto load = [&](int q) {
    const int u = lane & (SWEEP_U - 1), t = lane / SWEEP_U;
    const int k = cb + q * SWEEP_U + u;
    const int64_t a = M.off + min(k, ce - 1);
    double x = 0.0;
    if (t == 0) x = v.csig[a];
    else if (t == 1) x = v.mu[a];
    else if (t == 2) x = v.cinv[a];
    else if (t == 3) x = (k >= ce || (v.vflag && v.vflag[a])) ? 1.0 : 0.0;
    return x;
  };
  double cur = cg < ngrp ? load(cg) : 0.0;
  for (int q = cg; q < ngrp; q += m) {
    const bool more = q + m < ngrp;
    const double nxt = more ? load(q + m) : 0.0;
#pragma unroll
    for (int u = 0; u < SWEEP_U; ++u) {
      if (lane_value(cur, 3 * SWEEP_U + u) != 0.0) continue;
      const double sc = lane_value(cur, u), mm = lane_value(cur, SWEEP_U + u), iv = lane_value(cur, 2 * SWEEP_U + u);
      const int k = cb + q * SWEEP_U + u;
      const int64_t ko = M.neg ? n - 1 - k : k;
      const double den0 = (d0 - sc) - mm, den1 = (d1 - sc) - mm;
      const double rc0 = rcp_1nr(den0), rc1 = rcp_1nr(den1);
      double q0 = iv * rc0, q1 = iv * rc1;
      q0 = __builtin_fma(__builtin_fma(-q0, den0, iv), rc0, q0);  // corrected quotients
      q1 = __builtin_fma(__builtin_fma(-q1, den1, iv), rc1, q1);
      double* vp = v.V + ko * v.ldv + pos;
      if (a1) {
        typedef double vdbl2 __attribute__((ext_vector_type(2)));
        const vdbl2 vv = {z0 * q0, z1 * q1};
        __builtin_nontemporal_store(vv, reinterpret_cast<vdbl2*>(vp));
      } else if (a0) {
        __builtin_nontemporal_store(z0 * q0, vp);
      }
    }
    cur = nxt;
  }
}

// Waves of the address-ordered writer for a problem of order n: about
// SWEEP_WAVES, a whole number m >= 1 of waves per position range.
static int64_t sweep_waves(int64_t n) {
  const int64_t wpc = (n + 2 * WAVE - 1) / (2 * WAVE);
  const int64_t m = std::min<int64_t>(std::max<int64_t>(1, SWEEP_WAVES / wpc), (n + SWEEP_U - 1) / SWEEP_U);
  return wpc * m;
}

// The eigenvector writer alone (single problem, a range of columns).
template <int CB>
__global__ void __launch_bounds__(VEC_T) k_vec(VArgs v) {
  // beside the eigenvalue kernel of the next chunk its waves issue first, so
  // that the stores keep flowing while the sweeps take the remaining issue
  // slots; beside k_fix (the last chunk) they do not, since k_fix is latency-
  // bound and would starve
  if (v.prio) __builtin_amdgcn_s_setprio(3);
  if (v.sweep)
    vec_sweep(v, __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (VEC_T / WAVE) + threadIdx.x / WAVE)), v.sweep);
  else
    vec_block<CB>(blockIdx.x, v);
}

// k_fix and the eigenvector writer in one launch: the first nfix blocks take
// flagged eigenpairs from the queue (latency-bound work), the others write V
// (HBM-bound), so the two overlap.
template <int CB>
__global__ void __launch_bounds__(VEC_T) k_fixvec(KArgs A, VArgs v, int nfix) {
  if (blockIdx.x < (unsigned)nfix)
    fix_items(A);
  else if (v.sweep)
    vec_sweep(v, __builtin_amdgcn_readfirstlane((int)((blockIdx.x - nfix) * (VEC_T / WAVE) + threadIdx.x / WAVE)),
              v.sweep);
  else
    vec_block<CB>(blockIdx.x - nfix, v);
}

// Outputs and V columns of the eigenpairs finished in k_fix, in the same
// arithmetic as k_out and the eigenvector writer.
__global__ void __launch_bounds__(256) k_fixout(KArgs A, double* __restrict__ lam_out,
                                                int32_t* __restrict__ idx_out, double* __restrict__ mu_out,
                                                double* __restrict__ xn_out, double* __restrict__ V,
                                                const int64_t* __restrict__ voffs, int64_t ldv,
                                                int32_t* __restrict__ info_out) {
  const int n0 = A.ctr[0];
  const int cnt = n0 + A.ctr[3];
  for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
    const FixItem it = A.fix[fix_slot(A, n0, e)];
    const Meta M = A.meta[it.p];
    const int n = M.n, k = it.k;
    const int64_t a = M.off + k;
    const int ii = A.ii[a];
    const double m = A.mu[a], xs = A.xs[a];
    const int ko = M.neg ? n - 1 - k : k;
    const double sg = M.neg ? -1.0 : 1.0;
    if (threadIdx.x == 0) {
      const int64_t b = M.off + ko;
      lam_out[b] = sg * A.lam[a];
      if (idx_out) idx_out[b] = M.neg ? n - 1 - ii : ii;
      if (mu_out) mu_out[b] = sg * m;
      if (!range_ok(A.lam[a], m, xs)) info_out[it.p] = DPR1_INFO_RANGE;
      if (xn_out) xn_out[b] = xs / fabs(m);
    }
    if (V) {
      const double sc = A.sd[M.off + ii];
      const double iv = fabs(m) / xs;  // 1/||x||, as in k_out
      const int64_t ld = voffs ? (int64_t)n : ldv;
      double* col = V + (voffs ? voffs[it.p] : 0) + (int64_t)ko * ld;
#pragma unroll 8
      for (int pos = threadIdx.x; pos < n; pos += 256) {
        const int j = M.neg ? n - 1 - pos : pos;
        const double den = (A.sd[M.off + j] - sc) - m;
        const double rc = rcp_1nr(den);
        double q = iv * rc;
        q = __builtin_fma(__builtin_fma(-q, den, iv), rc, q);  // corrected quotient
        __builtin_nontemporal_store((sg * A.sz[M.off + j]) * q, &col[pos]);
      }
    }
  }
}

// ------------------------------------------------------- K_nu, remedies
// K_nu of eq. (K0) for eigenpair k shifted to d_i: ||A_i^{-1}||_2 =
// 1/min_j |lambda_j - d_i|, and by the interlacing (eq. interlace) the
// minimum is taken at lambda_k or at the other eigenvalue beside the pole,
// lambda_o (o = k+1 if i = k, o = k-1 if i = k-1), so
// K_nu = |lambda_k - d_i| / min(|lambda_k - d_i|, |lambda_o - d_i|), with the
// distances from the shifted representations in double-double.  knu_pole
// gives it for any neighbouring pole p of lambda_k (remedy (R1) compares the
// two).
__device__ double knu_pole(const double* Dv, const int32_t* ii, const double* mu, int n, int k, int p) {
  const dd lk = dd_add(two_sum(Dv[ii[k]], -Dv[p]), dd{mu[k], 0.0});
  const double ak = fabs(lk.hi + lk.lo);
  const int o = (p == k) ? k + 1 : k - 1;
  if (o < 0 || o >= n || ak == 0.0) return 1.0;
  const dd lo = dd_add(two_sum(Dv[ii[o]], -Dv[p]), dd{mu[o], 0.0});
  const double ao = fabs(lo.hi + lo.lo);
  if (ao >= ak) return 1.0;
  return ao > 0.0 ? ak / ao : INFINITY;
}

// A remedy: eigenpair k of problem p, nearest pole i; po the other
// neighbouring pole for (R1), -1 for (R2).
struct RemItem {
  int32_t p, k, i, po;
};

// One thread per eigenpair (a batch: block p takes problem p): K_nu to the
// optional output, the count of K_nu > knu_thr, and with opts.remedy the
// remedy list (in the eigenpair list's memory, free once k_fix has run).
// Pairs whose eigenvalue came from eq. (gamma) (vflag 2) keep it.
__global__ void __launch_bounds__(256) k_knu(KArgs A, int nprob) {
  const int p = nprob > 1 ? (int)blockIdx.x : 0;
  const int k0 = nprob > 1 ? (int)threadIdx.x : (int)(blockIdx.x * blockDim.x + threadIdx.x);
  const int kstep = nprob > 1 ? (int)blockDim.x : (int)(gridDim.x * blockDim.x);
  if (p >= nprob) return;
  const Meta M = A.meta[p];
  if (M.info != 0) return;
  const int n = M.n;
  const int64_t off = M.off;
  const double* Dv = A.sd + off;
  const int32_t* ii = A.ii + off;
  const double* mu = A.mu + off;
  RemItem* list = reinterpret_cast<RemItem*>(A.fix);
  for (int k = k0; k < n; k += kstep) {
    const int i = ii[k];
    const double K = n > 1 ? knu_pole(Dv, ii, mu, n, k, i) : 1.0;
    if (A.knu) A.knu[off + (M.neg ? n - 1 - k : k)] = K;
    if (!(K > A.knu_thr)) continue;
    if (A.stats) atomicAdd(&A.stats[DPR1_STAT_KNU_GT], 1);
    if (!A.remedy || A.vflag[off + k] == 2) continue;
    const int po = (i == k) ? k - 1 : k;  // the other neighbouring pole
    int use = -1;
    if (k >= 1 && po >= 0) {
      const double K2 = knu_pole(Dv, ii, mu, n, k, po);
      if (K2 < K && K2 <= A.knu_thr) use = po;
    }
    const int e = atomicAdd(&A.ctr[4], 1);
    list[e] = RemItem{p, k, i, use};
  }
}

// Outputs written by the remedy kernel.
struct OArgs {
  double* lam_out;
  int32_t* idx_out;
  double* mu_out;
  double* xn_out;
  double* V;
  const int64_t* voffs;
  int64_t ldv;
  int32_t* info_out;
};

// Remedies of Sec. 2 (Algorithm 1, last branch), one block of FIXT threads
// per listed eigenpair:
//  (R1) the other neighbouring pole d_po: its tip b (eq. b_ob) in
//       double-double, the extreme root of its g refined in double-double
//       (dd_polish from the current eigenvalue), and mu_i = (d_po - d_i) +
//       mu_po in double-double: mu_i inherits mu_po's absolute error, so the
//       root is carried to about 2^-100;
//  (R2) A - sigma I with sigma = d_i + mu (1 - 2^-e) between d_i and lambda
//       (e = 20, or smaller when the sign of f(sigma) shows sigma past
//       lambda): its inverse E + gamma u u^T with e_j = 1/(d_j - sigma), u_j =
//       zeta_j e_j, gamma = -rho/f(sigma), f(sigma) = 1 + rho sum
//       zeta_j^2/(d_j - sigma) in double-double from the exact differences;
//       eta = 1/(lambda - sigma) is its exterior eigenvalue (right of every
//       e_j when mu > 0, left when mu < 0), found by safeguarded Newton steps
//       from the current estimate; mu_i = (sigma - d_i) + 1/eta.
// The eigenpair keeps its nearest pole; ||x||, the outputs and its column of
// V are recomputed from the new mu.
__global__ void __launch_bounds__(FIXT) k_remedy(KArgs A, OArgs O) {
  __shared__ double sm[20];
  const int tid = threadIdx.x;
  const int cnt = A.ctr[4];
  const RemItem* list = reinterpret_cast<const RemItem*>(A.fix);
  for (int e = blockIdx.x; e < cnt; e += gridDim.x) {
    const RemItem it = list[e];
    const Meta M = A.meta[it.p];
    const int n = M.n;
    const int64_t off = M.off;
    const double* Dv = A.sd + off;
    const double* Zv = A.sz + off;
    const double2* Z2v = reinterpret_cast<const double2*>(A.pairs + 2 * off);
    const double* Zl = A.z2lo + off;
    const double rho = M.rho;
    const int k = it.k, i = it.i;
    const double muk = A.mu[off + k];
    double newmu = NAN;
    int how = 0;
    if (it.po >= 0) {
      // ---- (R1)
      const int po = it.po;
      const double s = (po == k) ? 1.0 : -1.0;
      const double sigma = Dv[po], zp = Zv[po];
      dd acc = {0.0, 0.0};
      for (int j = tid; j < n; j += FIXT) {
        if (j == po) continue;
        const double2 pj = Z2v[j];
        const dd dl = two_sum(pj.x, -sigma);
        const double r = rcp_1nr(dl.hi);
        const double q1 = pj.y * r;
        double er = __builtin_fma(-q1, dl.hi, pj.y);
        er = __builtin_fma(-q1, dl.lo, er + Zl[j]);
        acc = dd_add(acc, fast_two_sum(q1, er * r));
      }
      acc = block_sum_dd(acc, sm);
      const dd num = dd_add(dd_div(dd{1.0, 0.0}, dd{rho, 0.0}), acc);
      const dd b = dd_div_sq(num, zp);
      const dd bdd = {s * b.hi, s * b.lo};
      const double xm = 1.0 / (Dv[k - 1] - Dv[k]);
      // nu at d_po from the current eigenvalue: 1/(s (lambda - d_po))
      const dd lp = dd_add(two_sum(Dv[i], -sigma), dd{muk, 0.0});
      double cur = 1.0 / (s * (lp.hi + lp.lo));
      double last;
      int steps;
      cur = dd_polish(Z2v, Zl, n, po, s, sigma, zp, bdd, xm, xm, INFINITY, cur, &last, &steps, sm);
      const dd nu = fast_two_sum(cur, last);
      const dd mup = dd_div(dd{s, 0.0}, nu);
      const dd mi = dd_add(two_sum(sigma, -Dv[i]), mup);
      newmu = mi.hi + mi.lo;
      how = 1;
    } else {
      // ---- (R2)
      const bool pos = muk > 0;
      for (int ex = 20; ex >= 2; ex -= 6) {
        const double ms = muk * (1.0 - ldexp(1.0, -ex));  // sigma - d_i
        dd fs = {0.0, 0.0};
        double uu = 0.0, emax = -INFINITY, emin = INFINITY, emag = 0.0;
        for (int j = tid; j < n; j += FIXT) {
          const double2 pj = Z2v[j];
          const dd dl = dd_add(two_sum(pj.x, -Dv[i]), dd{-ms, 0.0});  // d_j - sigma
          const double r = rcp_1nr(dl.hi);
          const double q1 = pj.y * r;
          double er = __builtin_fma(-q1, dl.hi, pj.y);
          er = __builtin_fma(-q1, dl.lo, er + Zl[j]);
          fs = dd_add(fs, fast_two_sum(q1, er * r));
          const double dr = dl.hi + dl.lo, ej = 1.0 / dr, uj = Zv[j] / dr;
          uu += uj * uj;
          emax = fmax(emax, ej);
          emin = fmin(emin, ej);
          emag = fmax(emag, fabs(ej));
        }
        fs = block_sum_dd(fs, sm);
        uu = block_sum(uu, sm);
        emax = -block_min(-emax, sm);
        emin = block_min(emin, sm);
        emag = -block_min(-emag, sm);
        const dd F = dd_add(dd{1.0, 0.0}, dd_mul_d(fs, rho));
        if (pos ? !(F.hi < 0.0) : !(F.hi > 0.0)) continue;  // sigma is past lambda
        const double gam = -rho / (F.hi + F.lo);
        const double ub = (emag + fabs(gam) * uu) * GROW;
        double lo, hi;
        if (pos) {
          lo = emax > 0.0 ? emax : 4.9406564584124654e-324;
          hi = ub;
        } else {
          lo = -ub;
          hi = emin < 0.0 ? emin : -4.9406564584124654e-324;
        }
        // eta from the current estimate 1/(mu - ms), kept in the bracket
        double cur = 1.0 / (muk - ms);
        for (int st = 0; st < 80; ++st) {
          if (!(cur > lo && cur < hi)) cur = fmid_signed(lo, hi);
          double hs = 0.0, hc = 0.0, hp = 0.0;
          for (int j = tid; j < n; j += FIXT) {
            const double2 pj = Z2v[j];
            const dd dl = dd_add(two_sum(pj.x, -Dv[i]), dd{-ms, 0.0});
            const double dr = dl.hi + dl.lo, ej = 1.0 / dr, uj = Zv[j] / dr;
            const double den = ej - cur;
            const double t = (uj * uj) / den;
            const double y = hs + t;
            hc += (fabs(hs) >= fabs(t)) ? ((hs - y) + t) : ((t - y) + hs);
            hs = y;
            hp += (uj * uj) / (den * den);
          }
          const double S = block_sum_comp(hs, hc, sm);
          hp = block_sum(hp, sm);
          const double h = 1.0 + gam * S;
          if (h == 0.0) break;
          // right branch: h rises, the root is above where h < 0; left branch:
          // h falls, the root is above where h > 0
          if (pos ? (h < 0.0) : (h > 0.0)) lo = cur; else hi = cur;
          const double step = -h / (gam * hp);
          double t = cur + step;
          if (!(t > lo && t < hi)) t = fmid_signed(lo, hi);
          if (t == cur || fabs(step) <= 0x1p-53 * fabs(cur) || adjacent_signed(lo, hi)) {
            cur = t > lo && t < hi ? t : cur;
            break;
          }
          cur = t;
        }
        newmu = ms + 1.0 / cur;
        how = 2;
        break;
      }
    }
    if (!(newmu == newmu) || newmu == 0.0 || !(fabs(newmu) < INFINITY)) continue;
    // ||x|| scaled by |mu| from the new mu, as after the polish
    double acc = 0.0;
    for (int j = tid; j < n; j += FIXT) {
      const double r = (j == i) ? -1.0 : newmu / ((Dv[j] - Dv[i]) - newmu);
      acc = __builtin_fma(Z2v[j].y * r, r, acc);
    }
    const double xsv = sqrt(block_sum(acc, sm));
    const double lam = Dv[i] + newmu;
    const int ko = M.neg ? n - 1 - k : k;
    const double sg = M.neg ? -1.0 : 1.0;
    if (tid == 0) {
      A.mu[off + k] = newmu;
      A.xs[off + k] = xsv;
      A.lam[off + k] = lam;
      const int64_t b = off + ko;
      O.lam_out[b] = sg * lam;
      if (O.idx_out) O.idx_out[b] = M.neg ? n - 1 - i : i;
      if (O.mu_out) O.mu_out[b] = sg * newmu;
      if (O.xn_out) O.xn_out[b] = xsv / fabs(newmu);
      if (!range_ok(lam, newmu, xsv)) O.info_out[it.p] = DPR1_INFO_RANGE;
      if (A.stats) atomicAdd(&A.stats[how == 1 ? DPR1_STAT_REMEDY_R1 : DPR1_STAT_REMEDY_R2], 1);
    }
    if (O.V) {
      const double sc = Dv[i];
      const double iv = fabs(newmu) / xsv;
      const int64_t ld = O.voffs ? (int64_t)n : O.ldv;
      double* col = O.V + (O.voffs ? O.voffs[it.p] : 0) + (int64_t)ko * ld;
      for (int pos = tid; pos < n; pos += FIXT) {
        const int j = M.neg ? n - 1 - pos : pos;
        const double den = (Dv[j] - sc) - newmu;
        const double rc = rcp_1nr(den);
        double q = iv * rc;
        q = __builtin_fma(__builtin_fma(-q, den, iv), rc, q);
        __builtin_nontemporal_store((sg * Zv[j]) * q, &col[pos]);
      }
    }
  }
}

// ===================================================================== host
struct Layout {
  size_t meta, sd, sz, pairs, z2lo, ii, mu, xs, lam, csig, cinv, fix, vflag, items, groups, part, ctr, total;
};

static constexpr size_t al(size_t x) { return (x + 255) & ~size_t(255); }

static constexpr Layout layout(int64_t nprob, int64_t N, int64_t nitems, int64_t ngroups = 0) {
  Layout L{};
  size_t o = 0;
  L.meta = o; o = al(o + sizeof(Meta) * nprob);
  L.sd = o; o = al(o + 8 * N);
  L.sz = o; o = al(o + 8 * N);
  L.pairs = o; o = al(o + 16 * N);
  L.z2lo = o; o = al(o + 8 * N);
  L.ii = o; o = al(o + 4 * N);
  L.mu = o; o = al(o + 8 * N);
  L.xs = o; o = al(o + 8 * N);
  L.lam = o; o = al(o + 8 * N);
  L.csig = o; o = al(o + 8 * N);
  L.cinv = o; o = al(o + 8 * N);
  L.fix = o; o = al(o + sizeof(FixItem) * N);
  L.vflag = o; o = al(o + N);
  L.items = o; o = al(o + sizeof(int2) * nitems);
  L.groups = o; o = al(o + sizeof(int4) * ngroups);
  L.part = o; o = al(o + 3 * sizeof(double) * PREP_MAX_SPLIT);
  L.ctr = o; o = al(o + 64);
  L.total = o;
  return L;
}

static void fill_opts(const dpr1_opts* in, dpr1_opts* o) {
  dpr1_default_opts(o);
  if (in) {
    *o = *in;
    if (!(o->kappa_polish > 0)) o->kappa_polish = 16.0;
    if (o->nearzero < 0) o->nearzero = 10.0;
    if (!(o->knu_thr > 0)) o->knu_thr = 32.0;
  }
}

// The split when the options leave it open: the W that ends the launch
// soonest, with a block of W waves taking time in proportion to its slice
// n/W and each of the 256 CUs holding floor(4 occ / W) blocks at a time (a
// block's waves stay on one CU, 4 occ wave slots per CU): minimise
// ceil(nblocks / (256 floor(4 occ / W))) / W, the smaller W on a tie (fewer
// partial sums), keeping slices of at least 256 terms.  (Filling the wave
// slots alone is not enough: 423 blocks at W = 10 fit one block per CU and
// take two rounds, 1.6 times longer than W = 8 in one.)
static int pick_split(int64_t nblocks, int64_t nmax, int occ) {
  int best = 1;
  double bc = 1e300;
  for (int w = 1; w <= MAXW; ++w) {
    if (w > 1 && nmax / w < 256) break;
    const int64_t per_cu = (4 * (int64_t)occ) / w;
    if (per_cu < 1) break;
    const double c = std::ceil((double)std::max<int64_t>(nblocks, 1) / (256.0 * (double)per_cu)) / w;
    if (c < bc * (1.0 - 1e-9)) {
      bc = c;
      best = w;
    }
  }
  return best;
}

// k_eig occupancy variant of the options: 4 (default), 6 or 8 waves per SIMD.
static int occ_of(const dpr1_opts& o) { return o.waves_per_simd == 0 ? 4 : o.waves_per_simd; }
static bool occ_valid(int32_t w) { return w == 0 || w == 4 || w == 6 || w == 8; }

// Blocks of the persistent batched k_eig: as many W-wave blocks as the 256
// CUs hold at the variant's occupancy (4 SIMDs x occ waves per CU), never
// more blocks than work items.
static int32_t persistent_grid_for(int64_t nitems, int W, int occ) {
  const int64_t per_cu = std::max<int64_t>(1, (4 * occ) / W);
  return (int32_t)std::min<int64_t>(nitems, 256 * per_cu);
}

// ------------------------------------------------------------ autotuning
// Mean duration in ms of `reps` calls of `solve` after one untimed call,
// between two events on stream st.
template <class F>
static int time_calls(F&& solve, int reps, hipStream_t st, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return DPR1_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return DPR1_EHIP;
  }
  int rc = solve();
  if (rc == 0 && hipEventRecord(e0, st) != hipSuccess) rc = DPR1_EHIP;
  for (int r = 0; r < reps && rc == 0; ++r) rc = solve();
  if (rc == 0 && hipEventRecord(e1, st) != hipSuccess) rc = DPR1_EHIP;
  if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = DPR1_EHIP;
  float t = 0.0f;
  if (rc == 0 && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = DPR1_EHIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return rc;
}

// Candidate splits for inner length nmax (the largest problem): W waves
// share one block of 64 eigenvalues (W threads per eigenvalue), and every
// wave's slice of the inner sum keeps at least 64 terms.  Candidate
// occupancy variants of k_eig: 4, 6 and 8 waves per SIMD.
static int split_candidates(int64_t nmax, int* out) {
  static const int cand[6] = {1, 2, 4, 8, 12, 16};
  int c = 0;
  for (int w : cand)
    if (w <= MAXW && (w == 1 || nmax / w >= 64)) out[c++] = w;
  return c;
}
static const int OCC_CAND[3] = {4, 6, 8};
// The 6- and 8-wave register budgets spill part of k_eig's state to scratch
// (about 7 to 18 times the HBM bytes of the 4-wave variant at n = 32768):
// they are chosen only when at least 4 % faster, beyond the 2-3 % by which
// one shape's time moves between runs, not on timing noise.
static double occ_margin(int oc) { return oc > 4 ? 0.96 : 1.0; }

// Number of (problem, column group, row tile) blocks of the batched
// eigenvector launch.
static int64_t count_groups(int64_t nprob, const int64_t* offs) {
  int64_t c = 0;
  for (int64_t p = 0; p < nprob; ++p) {
    const int64_t np = offs[p + 1] - offs[p];
    c += ((np + VEC_C_BATCH - 1) / VEC_C_BATCH) * ((np + VEC_ROWS - 1) / VEC_ROWS);
  }
  return c;
}

// LDS of k_eig's cross-wave reductions: the widest, wg_sum<RED_NV>, stores
// RED_NV values per lane and wave.
constexpr int RED_NV = 4;
static size_t red_bytes(int W) { return W > 1 ? sizeof(double) * RED_NV * W * WAVE : 0; }

// Workspace of dpr1_eig_noalloc: a device array of the library, sized for the
// largest problem it accepts.  Every GPU holds its own copy for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device (the name itself is a host-side
// stand-in, not a device address).
constexpr size_t NOALLOC_BYTES = layout(1, DPR1_NOALLOC_MAX_N, 0).total;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex scratch_mutex;
static void* scratch_ptr[NOALLOC_MAX_DEVICES];

// Device address of `scratch` on the current device, resolved once per device
// (nullptr on a HIP error or an out-of-range device index).
static void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

}  // namespace dpr1

using namespace dpr1;

extern "C" {

void dpr1_default_opts(dpr1_opts* o) {
  o->mode_b = 0;
  o->root = 1;
  o->polish = 1;
  o->split = 0;
  o->kappa_polish = 16.0;
  o->nearzero = 10.0;
  o->main_passes = 0;
  o->waves_per_simd = 0;
  o->events = nullptr;
  o->vwrite = 0;
  o->remedy = 0;
  o->knu_thr = 32.0;
  o->knu = nullptr;
}

size_t dpr1_workspace_size(int64_t n) {
  if (n < 1) return 0;
  return layout(1, n, 0).total;
}

#define HIPCHECK(x)                           \
  do {                                        \
    if ((x) != hipSuccess) return DPR1_EHIP;  \
  } while (0)

// Second stream of the current device for the overlapped eigenvector write:
// created once per device (default priority, non-blocking) and kept until the
// process ends; nullptr if it cannot be created.
constexpr int AUX_MAX_DEVICES = 64;
static std::mutex aux_mutex;
static hipStream_t aux_streams[AUX_MAX_DEVICES];
static hipStream_t aux_stream() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= AUX_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(aux_mutex);
  if (!aux_streams[dev]) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    aux_streams[dev] = s;
  }
  return aux_streams[dev];
}

static int launch_solve(const Layout& L, char* w, int64_t nprob, int64_t N, const int64_t* offs,
                        int64_t n_single, const double* d, const double* z, const double* rho_dev,
                        double rho_host, double* lambda, double* V, const int64_t* voffs, int64_t ldv,
                        int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, int32_t* stats,
                        const dpr1_opts& o, int W, int64_t nitems, int persistent_grid, int64_t ngroups,
                        hipStream_t st, bool aux_ok = true) {
  Meta* meta = (Meta*)(w + L.meta);
  KArgs A;
  A.meta = meta;
  A.pairs = (const double*)(w + L.pairs);
  A.z2lo = (const double*)(w + L.z2lo);
  A.sd = (const double*)(w + L.sd);
  A.sz = (const double*)(w + L.sz);
  A.ii = (int32_t*)(w + L.ii);
  A.mu = (double*)(w + L.mu);
  A.xs = (double*)(w + L.xs);
  A.lam = (double*)(w + L.lam);
  A.fix = (FixItem*)(w + L.fix);
  A.vflag = (uint8_t*)(w + L.vflag);
  A.ctr = (int32_t*)(w + L.ctr);
  A.stats = stats;
  A.items = persistent_grid ? (const int2*)(w + L.items) : nullptr;
  A.nitems = (int32_t)nitems;
  A.nfixcap = (int32_t)N;
  A.W = W;
  A.mode_b = o.mode_b;
  A.root = o.root;
  A.polish = o.polish;
  A.kappa_polish = o.kappa_polish;
  A.nearzero = o.nearzero;
  // Default budget: 2 passes (one plain, one accurate) for a single problem,
  // whose stragglers (under a tenth of the roots) are finished beside the V
  // write; a batch runs one more, since its many small problems would queue
  // their stragglers in k_fix.
  A.main_passes = o.main_passes > 0 ? o.main_passes : (persistent_grid ? 3 : 2);
  A.remedy = o.remedy;
  A.knu_thr = o.knu_thr;
  A.knu = o.knu;

  hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, A.ctr, 16);
  if (stats) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, stats, DPR1_NSTATS);
  const int nsplit = nprob == 1 ? (int)std::min<int64_t>(PREP_MAX_SPLIT, std::max<int64_t>(1, N / 512)) : 1;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)(nsplit > 1 ? nsplit : nprob)), dim3(256), 0, st, (int)nprob, nsplit,
                     offs, n_single, d, z, rho_dev, rho_host, meta, (double*)A.sd, (double*)A.sz,
                     (double*)A.pairs, (double*)A.z2lo, info, (double*)(w + L.part), A.ctr + 8);
  HIPCHECK(hipGetLastError());
  hipEvent_t* ev = (hipEvent_t*)o.events;
  double* csig = (double*)(w + L.csig);
  double* cinv = (double*)(w + L.cinv);
  VArgs va;
  va.meta = meta;
  va.sd = A.sd;
  va.sz = A.sz;
  va.mu = A.mu;
  va.csig = csig;
  va.cinv = cinv;
  va.vflag = A.vflag;
  va.V = V;
  va.voffs = voffs;
  va.ldv = ldv;
  va.cbase = 0;
  va.cend = (int32_t)N;
  va.prio = 0;
  // one problem whose columns all start 16-byte aligned: the address-ordered writer
  va.sweep = (V && !persistent_grid && ((uintptr_t)V & 15) == 0 && (ldv & 1) == 0) ? (int32_t)sweep_waves(N) : 0;
  const unsigned sweep_blocks = (unsigned)((va.sweep + VEC_T / WAVE - 1) / (VEC_T / WAVE));
  auto launch_eig = [&](unsigned grid, int g0, int occ) {
    A.g0 = g0;
    switch (occ) {
      case 6: hipLaunchKernelGGL(k_eig<6>, dim3(grid), dim3(64 * W), red_bytes(W), st, A); break;
      case 8: hipLaunchKernelGGL(k_eig<8>, dim3(grid), dim3(64 * W), red_bytes(W), st, A); break;
      default: hipLaunchKernelGGL(k_eig<4>, dim3(grid), dim3(64 * W), red_bytes(W), st, A); break;
    }
  };
  // user outputs of eigenvalues kb .. ke-1 (those of flagged ones are
  // rewritten by k_fixout once k_fix has finished them) and the per-column
  // constants of the eigenvector writer
  auto launch_out = [&](int64_t kb, int64_t ke) {
    const int64_t cnt = nprob > 1 ? N : ke - kb;
    hipLaunchKernelGGL(k_out,
                       dim3(nprob > 1 ? (unsigned)nprob : (unsigned)std::min<int64_t>((cnt + 255) / 256, 1024)),
                       dim3(256), 0, st, meta, (int)nprob, A.ii, A.mu, A.xs, A.lam, A.sd, csig, cinv, lambda,
                       shift_idx, mu, xnorm, A.vflag, info, (int)kb, (int)ke);
  };
  // K_nu of every eigenpair and, with opts.remedy, the remedies (after every
  // eigenpair and column is final, on `stream`)
  auto launch_knu = [&]() {
    hipLaunchKernelGGL(k_knu, dim3(nprob > 1 ? (unsigned)nprob : (unsigned)std::min<int64_t>((N + 255) / 256, 1024)),
                       dim3(256), 0, st, A, (int)nprob);
    if (o.remedy) {
      OArgs oa;
      oa.lam_out = lambda;
      oa.idx_out = shift_idx;
      oa.mu_out = mu;
      oa.xn_out = xnorm;
      oa.V = V;
      oa.voffs = voffs;
      oa.ldv = ldv;
      oa.info_out = info;
      hipLaunchKernelGGL(k_remedy, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(N / 16, 1), 2048)),
                         dim3(FIXT), 0, st, A, oa);
    }
  };
  auto launch_vec = [&](int64_t cb, int64_t ce, hipStream_t s2, bool prio) {
    const int64_t cg = (ce - cb + VEC_C_SINGLE - 1) / VEC_C_SINGLE;
    const int64_t rt = (N + VEC_ROWS - 1) / VEC_ROWS;
    VArgs vb = va;
    vb.groups = nullptr;
    vb.ncolgroups = cg;
    vb.cbase = (int32_t)cb;
    vb.cend = (int32_t)ce;
    vb.prio = prio ? 1 : 0;
    hipLaunchKernelGGL((k_vec<VEC_C_SINGLE>), dim3(vb.sweep ? sweep_blocks : (unsigned)(cg * rt)), dim3(VEC_T), 0, s2,
                       vb);
  };

  // A single problem with eigenvectors and opts.vwrite = K >= 2: the
  // eigenvalue kernel runs in K launches over consecutive chunks of its
  // groups of 64 eigenvalues, and the columns of chunk c are written on a
  // second stream while chunk c + 1 is solved, so that the HBM-bound stores
  // overlap the ALU-bound sweeps; the last chunk's columns are written beside
  // k_fix.  Flagged columns are left to k_fixout, as in the sequential path.
  // The default (0 or 1) writes V after the eigenvalue kernel, which measured
  // faster at every order tried (n = 8192 .. 65536) since the address-ordered
  // writer; below 8192 eigenpairs the write is short and the fork costs more
  // than it hides in any case.
  const int nchunks = o.vwrite <= 1 ? 1 : o.vwrite;
  bool overlap = V && !persistent_grid && nchunks >= 2 && aux_ok && N >= 8192 && nitems >= nchunks;
  hipStream_t st2 = overlap ? aux_stream() : nullptr;
  if (overlap && !st2) overlap = false;
  if (overlap) {
    hipEvent_t evs[VEC_CHUNKS_MAX + 1];
    int nev = 0, rc = DPR1_OK;
    for (; nev <= nchunks; ++nev)
      if (hipEventCreateWithFlags(&evs[nev], hipEventDisableTiming) != hipSuccess) {
        rc = DPR1_EHIP;
        break;
      }
    if (rc == DPR1_OK && ev && hipEventRecord(ev[0], st) != hipSuccess) rc = DPR1_EHIP;
    for (int c = 0; c < nchunks && rc == DPR1_OK; ++c) {
      const int64_t ga = nitems * c / nchunks, gb = nitems * (c + 1) / nchunks;
      const int64_t ka = ga * WAVE, kb = std::min<int64_t>(gb * WAVE, N);
      // the chunks solved beside the writer take at least the 6-wave register
      // budget, so that writer waves fit next to a 16-wave block
      launch_eig((unsigned)(gb - ga), (int)ga, c == 0 ? occ_of(o) : std::max(occ_of(o), 6));
      if (c == nchunks - 1 && ev && hipEventRecord(ev[1], st) != hipSuccess) rc = DPR1_EHIP;
      launch_out(ka, kb);
      if (hipGetLastError() != hipSuccess || hipEventRecord(evs[c], st) != hipSuccess ||
          hipStreamWaitEvent(st2, evs[c], 0) != hipSuccess)
        rc = DPR1_EHIP;
      if (rc == DPR1_OK) launch_vec(ka, kb, st2, c < nchunks - 1);
    }
    if (rc == DPR1_OK && ev && hipEventRecord(ev[2], st) != hipSuccess) rc = DPR1_EHIP;
    if (rc == DPR1_OK) {
      unsigned fgrid = (unsigned)std::min<int64_t>(std::max<int64_t>(N, 1), 2048);
      hipLaunchKernelGGL(k_fix, dim3(fgrid), dim3(FIXT), 0, st, A);
      hipLaunchKernelGGL(k_fixout, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(N, 1), 2048)), dim3(256), 0,
                         st, A, lambda, shift_idx, mu, xnorm, V, voffs, ldv, info);
      if (hipGetLastError() != hipSuccess || hipEventRecord(evs[nchunks], st2) != hipSuccess ||
          hipStreamWaitEvent(st, evs[nchunks], 0) != hipSuccess || (ev && hipEventRecord(ev[3], st) != hipSuccess))
        rc = DPR1_EHIP;
    }
    if (rc == DPR1_OK) {
      launch_knu();
      if (hipGetLastError() != hipSuccess) rc = DPR1_EHIP;
    }
    for (int e = 0; e < nev; ++e) (void)hipEventDestroy(evs[e]);
    return rc;
  }

  unsigned grid = persistent_grid ? (unsigned)persistent_grid : (unsigned)nitems;
  if (ev) HIPCHECK(hipEventRecord(ev[0], st));
  launch_eig(grid, 0, occ_of(o));
  HIPCHECK(hipGetLastError());
  if (ev) HIPCHECK(hipEventRecord(ev[1], st));
  launch_out(0, N);
  HIPCHECK(hipGetLastError());
  if (ev) HIPCHECK(hipEventRecord(ev[2], st));
  if (V) {
    // k_fix overlapped with the eigenvector writer: a few blocks take the
    // flagged eigenpairs, the rest write every other column
    const int nfix = persistent_grid ? 512 : 256;
    if (persistent_grid) {
      va.groups = (const int4*)(w + L.groups);
      va.ncolgroups = ngroups;
      hipLaunchKernelGGL((k_fixvec<VEC_C_BATCH>), dim3((unsigned)(nfix + ngroups)), dim3(VEC_T), 0, st, A, va, nfix);
    } else {
      const int64_t cg = (N + VEC_C_SINGLE - 1) / VEC_C_SINGLE;
      const int64_t rt = (N + VEC_ROWS - 1) / VEC_ROWS;
      va.groups = nullptr;
      va.ncolgroups = cg;
      hipLaunchKernelGGL((k_fixvec<VEC_C_SINGLE>), dim3(nfix + (va.sweep ? sweep_blocks : (unsigned)(cg * rt))),
                         dim3(VEC_T), 0, st, A, va,
                         nfix);
    }
  } else {
    unsigned fgrid = (unsigned)std::min<int64_t>(std::max<int64_t>(N, 1), 2048);
    hipLaunchKernelGGL(k_fix, dim3(fgrid), dim3(FIXT), 0, st, A);
  }
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(k_fixout, dim3((unsigned)std::min<int64_t>(std::max<int64_t>(N, 1), 2048)), dim3(256), 0, st,
                     A, lambda, shift_idx, mu, xnorm, V, voffs, ldv, info);
  HIPCHECK(hipGetLastError());
  if (ev) HIPCHECK(hipEventRecord(ev[3], st));
  launch_knu();
  HIPCHECK(hipGetLastError());
  return DPR1_OK;
}

int dpr1_eig(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V, int64_t ldv,
             int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, int32_t* stats,
             const dpr1_opts* opts, void* work, size_t work_bytes, void* stream) {
  if (!d) return -1;
  if (!z) return -2;
  if (!(rho == rho) || rho == 0.0 || rho == INFINITY || rho == -INFINITY) return -3;
  if (n < 1 || n > (int64_t)INT32_MAX / 2) return -4;
  if (!lambda) return -5;
  if (V && ldv < n) return -7;
  if (!info) return -11;
  Layout L = layout(1, n, 0);
  if (!work) return -14;
  if (work_bytes < L.total) return -15;
  dpr1_opts o;
  fill_opts(opts, &o);
  if (!occ_valid(o.waves_per_simd) || o.vwrite < 0 || o.vwrite > VEC_CHUNKS_MAX || o.mode_b < 0 || o.mode_b > 3)
    return -13;
  int64_t nblocks = (n + WAVE - 1) / WAVE;
  int W = o.split > 0 ? std::min(o.split, MAXW) : pick_split(nblocks, n, occ_of(o));
  return launch_solve(L, (char*)work, 1, n, nullptr, n, d, z, nullptr, rho, lambda, V, nullptr, ldv, shift_idx,
                      mu, xnorm, info, stats, o, W, nblocks, 0, 0, (hipStream_t)stream);
}

size_t dpr1_noalloc_scratch_bytes(void) { return NOALLOC_BYTES; }

// dpr1_eig on the library's static device scratch instead of a workspace
// argument: the same checks, kernels and results; no allocation of any kind.
int dpr1_eig_noalloc(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                     int64_t ldv, int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, int32_t* stats,
                     const dpr1_opts* opts, void* stream) {
  if (!d) return -1;
  if (!z) return -2;
  if (!(rho == rho) || rho == 0.0 || rho == INFINITY || rho == -INFINITY) return -3;
  if (n < 1) return -4;
  if (n > DPR1_NOALLOC_MAX_N) return DPR1_ETOOBIG;
  if (!lambda) return -5;
  if (V && ldv < n) return -7;
  if (!info) return -11;
  dpr1_opts o;
  fill_opts(opts, &o);
  if (!occ_valid(o.waves_per_simd) || o.vwrite < 0 || o.vwrite > VEC_CHUNKS_MAX || o.mode_b < 0 || o.mode_b > 3)
    return -13;
  void* work = scratch_on_current_device();
  if (!work) return DPR1_EHIP;
  const Layout L = layout(1, n, 0);
  int64_t nblocks = (n + WAVE - 1) / WAVE;
  int W = o.split > 0 ? std::min(o.split, MAXW) : pick_split(nblocks, n, occ_of(o));
  return launch_solve(L, (char*)work, 1, n, nullptr, n, d, z, nullptr, rho, lambda, V, nullptr, ldv, shift_idx,
                      mu, xnorm, info, stats, o, W, nblocks, 0, 0, (hipStream_t)stream,
                      /*aux_ok=*/false);
}

// ------------------------------------------------------------ batched
size_t dpr1_batched_workspace_size(int64_t nprob, const int64_t* offs_host) {
  if (nprob < 1 || !offs_host || offs_host[0] != 0) return 0;
  for (int64_t p = 0; p < nprob; ++p)
    if (offs_host[p + 1] - offs_host[p] < 1) return 0;
  int64_t ntotal = offs_host[nprob];
  int64_t nitems = ntotal / WAVE + nprob;  // upper bound of sum ceil(n_p/64)
  return layout(nprob, ntotal, nitems, count_groups(nprob, offs_host)).total;
}

int dpr1_batched_plan(int64_t nprob, const int64_t* offs_host, const dpr1_opts* opts, dpr1_plan* plan,
                      void* work, size_t work_bytes, void* stream) {
  if (nprob < 1 || nprob > (1 << 24)) return -1;
  if (!offs_host) return -2;
  if (!plan) return -4;
  if (!work) return -5;
  if (offs_host[0] != 0) return -2;
  int64_t nmax = 0;
  for (int64_t p = 0; p < nprob; ++p) {
    int64_t np = offs_host[p + 1] - offs_host[p];
    if (np < 1 || np > (int64_t)INT32_MAX / 2) return -2;
    nmax = std::max(nmax, np);
  }
  int64_t N = offs_host[nprob];
  if (N > (int64_t)INT32_MAX) return -2;
  Layout L0 = layout(nprob, N, N / WAVE + nprob, count_groups(nprob, offs_host));
  if (work_bytes < L0.total) return -6;
  dpr1_opts o;
  fill_opts(opts, &o);
  if (!occ_valid(o.waves_per_simd) || o.mode_b < 0 || o.mode_b > 3) return -3;
  // longest-processing-time order: larger problems first
  std::vector<int32_t> order(nprob);
  for (int64_t p = 0; p < nprob; ++p) order[p] = (int32_t)p;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return offs_host[a + 1] - offs_host[a] > offs_host[b + 1] - offs_host[b];
  });
  std::vector<int2> items;
  for (int32_t p : order) {
    int64_t np = offs_host[p + 1] - offs_host[p];
    for (int64_t k0 = 0; k0 < np; k0 += WAVE) items.push_back(make_int2(p, (int)k0));
  }
  int64_t nitems = (int64_t)items.size();
  int W = o.split > 0 ? std::min(o.split, MAXW) : pick_split(nitems, nmax, occ_of(o));
  // blocks of the eigenvector kernel: (problem, first column, columns,
  // first row), largest problems first
  std::vector<int4> groups;
  for (int32_t p : order) {
    const int64_t np = offs_host[p + 1] - offs_host[p];
    for (int64_t c0 = 0; c0 < np; c0 += VEC_C_BATCH)
      for (int64_t r0 = 0; r0 < np; r0 += VEC_ROWS)
        groups.push_back(make_int4(p, (int)c0, (int)std::min<int64_t>(VEC_C_BATCH, np - c0), (int)r0));
  }
  hipStream_t st = (hipStream_t)stream;
  HIPCHECK(hipMemcpyAsync((char*)work + L0.items, items.data(), sizeof(int2) * nitems, hipMemcpyHostToDevice, st));
  HIPCHECK(hipMemcpyAsync((char*)work + L0.groups, groups.data(), sizeof(int4) * groups.size(),
                          hipMemcpyHostToDevice, st));
  HIPCHECK(hipStreamSynchronize(st));
  plan->ngroups = (int64_t)groups.size();
  plan->nprob = nprob;
  plan->ntotal = N;
  plan->nitems = nitems;
  plan->nmax = nmax;
  plan->split = W;
  plan->grid = persistent_grid_for(nitems, W, occ_of(o));
  plan->opts = o;
  return DPR1_OK;
}

int dpr1_eig_batched(const dpr1_plan* plan, const int64_t* offs, const double* d, const double* z,
                     const double* rho, double* lambda, double* V, const int64_t* voffs, int32_t* shift_idx,
                     double* mu, double* xnorm, int32_t* info, int32_t* stats, void* work, size_t work_bytes,
                     void* stream) {
  if (!plan || plan->nprob < 1) return -1;
  if (!offs) return -2;
  if (!d) return -3;
  if (!z) return -4;
  if (!rho) return -5;
  if (!lambda) return -6;
  if (V && !voffs) return -8;
  if (!info) return -12;
  if (!work) return -14;
  Layout L = layout(plan->nprob, plan->ntotal, plan->ntotal / WAVE + plan->nprob, plan->ngroups);
  if (work_bytes < L.total) return -15;
  return launch_solve(L, (char*)work, plan->nprob, plan->ntotal, offs, 0, d, z, rho, 0.0, lambda, V, voffs, 0,
                      shift_idx, mu, xnorm, info, stats, plan->opts, plan->split, plan->nitems, plan->grid,
                      plan->ngroups, (hipStream_t)stream);
}

// Autotuning: every candidate (split, occupancy variant, pass budget) is
// timed on the caller's data and the fastest kept; ties keep the earlier
// candidate.
int dpr1_autotune(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                  int64_t ldv, int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, dpr1_opts* opts,
                  int32_t reps, double* best_ms, void* work, size_t work_bytes, void* stream) {
  if (!opts) return -12;
  if (reps < 0) return -13;
  if (reps == 0) reps = 3;
  dpr1_opts o;
  fill_opts(opts, &o);
  o.events = nullptr;
  int ws[8];
  const int nw = split_candidates(n, ws);
  const int passes[2] = {2, 3};
  const int np = o.root == 1 ? 2 : 1;
  // with eigenvectors at n >= 8192 also the write: after the eigenvalue
  // kernel (0) or overlapped in two chunks (2)
  const int vws[2] = {0, 2};
  const int nv = (V && n >= 8192) ? 2 : 1;
  double best = INFINITY;
  int bw = ws[0], bp = o.main_passes, bo = 4, bv = o.vwrite;
  for (int a = 0; a < nw; ++a)
    for (int oc : OCC_CAND)
      for (int b = 0; b < np; ++b)
        for (int e = 0; e < nv; ++e) {
        dpr1_opts c = o;
        c.split = ws[a];
        c.waves_per_simd = oc;
        if (o.root == 1) c.main_passes = passes[b];
        if (nv > 1) c.vwrite = vws[e];
        double ms = 0.0;
        int rc = time_calls([&]() { return dpr1_eig(d, z, rho, n, lambda, V, ldv, shift_idx, mu, xnorm, info,
                                                    nullptr, &c, work, work_bytes, stream); },
                            reps, (hipStream_t)stream, &ms);
        if (rc != 0) return rc;
        if (ms < best * occ_margin(oc)) {
          best = ms;
          bw = c.split;
          bp = c.main_passes;
          bo = oc;
          bv = c.vwrite;
        }
      }
  opts->split = bw;
  opts->main_passes = bp;
  opts->waves_per_simd = bo;
  opts->vwrite = bv;
  if (best_ms) *best_ms = best;
  return DPR1_OK;
}

int dpr1_batched_autotune(dpr1_plan* plan, const int64_t* offs, const double* d, const double* z,
                          const double* rho, double* lambda, double* V, const int64_t* voffs,
                          int32_t* shift_idx, double* mu, double* xnorm, int32_t* info, int32_t reps,
                          double* best_ms, void* work, size_t work_bytes, void* stream) {
  if (!plan || plan->nprob < 1) return -1;
  if (reps < 0) return -13;
  if (reps == 0) reps = 3;
  const dpr1_plan base = *plan;
  int ws[8];
  const int nw = split_candidates(base.nmax, ws);
  const int passes[3] = {2, 3, 4};
  const int np = base.opts.root == 1 ? 3 : 1;
  double best = INFINITY;
  dpr1_plan bestp = base;
  for (int a = 0; a < nw; ++a)
    for (int oc : OCC_CAND)
      for (int b = 0; b < np; ++b) {
        dpr1_plan c = base;
        c.split = ws[a];
        c.opts.waves_per_simd = oc;
        c.grid = persistent_grid_for(c.nitems, ws[a], oc);
        c.opts.events = nullptr;
        if (base.opts.root == 1) c.opts.main_passes = passes[b];
        double ms = 0.0;
        int rc = time_calls([&]() { return dpr1_eig_batched(&c, offs, d, z, rho, lambda, V, voffs, shift_idx, mu,
                                                            xnorm, info, nullptr, work, work_bytes, stream); },
                            reps, (hipStream_t)stream, &ms);
        if (rc != 0) return rc;
        if (ms < best * occ_margin(oc)) {
          best = ms;
          bestp = c;
        }
      }
  bestp.opts.events = base.opts.events;
  *plan = bestp;
  if (best_ms) *best_ms = best;
  return DPR1_OK;
}

const char* dpr1_strerror(int code) {
  switch (code) {
    case DPR1_OK: return "ok";
    case DPR1_EHIP: return "a HIP runtime call or kernel launch failed";
    case DPR1_ETOOBIG: return "n exceeds DPR1_NOALLOC_MAX_N, the size of the static scratch of dpr1_eig_noalloc";
    case DPR1_INFO_UNSORTED: return "info: d is not strictly decreasing";
    case DPR1_INFO_ZERO_Z: return "info: some z_j is zero (reducible problem)";
    case DPR1_INFO_NONFINITE: return "info: non-finite input";
    case DPR1_INFO_BAD_RHO: return "info: rho is zero or not finite";
    case DPR1_INFO_RANGE: return "info: a shifted representation left the binary64 range";
    default: return code < 0 ? "invalid argument (see the argument position -code)" : "unknown code";
  }
}

}  // extern "C"
