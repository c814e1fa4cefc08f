// Front end for reducible inputs (Sec. 1 of the paper): any finite d (any
// order, repeated values) and any finite z (zeros allowed); and the Hermitian
// case A = D + rho z z^H with complex z, which a diagonal unitary similarity
// turns into the real problem with |z| (the extension the paper's closing
// remarks mention).
//
// The reduction is host work on n numbers: sort the poles decreasingly,
// deflate a pole whose z_j is zero (eigenpair (d_j, e_j)), and merge a group of
// equal poles by a Householder reflection of its block that maps its part w
// of z onto a multiple of e_first: the pole enters the reduced problem once,
// with z = ||w||, and the other columns of the reflection are eigenvectors for
// the same eigenvalue.  The reduced problem (strictly decreasing, no zero z)
// is solved on the GPU by dpr1_eig without eigenvectors; k_assemble then
// writes every column of V in the caller's row order.
//
// A column k of the reduced problem needs no gather: in the caller's rows its
// components are those of eq. (eigenvecAi) evaluated on the original d and z,
//   v_k[i] = z_i / (((d_i - sigma_k) - mu_k) ||x_k||),
// because a member i of a merged group has d_i = the group's pole and carries
// z_i = (w_i / ||w||) ||w||, and a deflated row has z_i = 0.  So each thread
// keeps (d_i, z_i) of its row in registers and writes whole column segments
// (coalesced, streaming stores), HBM-bound like the eigenvector writer.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/dpr1.h"
#include "reduce.h"

namespace dpr1 {
namespace gen {

using fe::COL_REDUCED;
using fe::COL_REFLECT;
using fe::COL_UNIT;

// Per original row i: rgrp its group id, rpos its position in the group, ru
// the reflection vector's component there (0 for groups without reflection).
// Per final column c:
//   COL_REDUCED  csig = sigma_k (the shift pole), cmu = mu_k,
//                cic = 1 / ||x_k||
//   COL_UNIT     cidx = original row of the unit vector
//   COL_REFLECT  cidx = group id, ct = column t of the reflection,
//                cub = beta u_t
struct AsmArgs {
  int64_t n, ldv;
  const double* d;
  const double* z;
  const int32_t* rgrp;
  const int32_t* rpos;
  const double* ru;
  const int32_t* ckind;
  const int32_t* cidx;
  const int32_t* ct;
  const double* csig;
  const double* cmu;
  const double* cic;
  const double* cub;
  const double* ph;  // [2n] unit phases z_i / |z_i| (Hermitian case), else null
  double* V;
};

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// Tile: ASM_CB columns x ASM_T * ASM_R rows.  The block stages the column
// parameters in LDS once; each thread keeps ASM_R rows in registers and, per
// column, issues ASM_R streaming stores, each a contiguous, aligned 512-byte
// window per wave when ldv is a multiple of 64.
constexpr int ASM_T = 256, ASM_R = 4, ASM_CB = 16;

typedef double dbl2 __attribute__((ext_vector_type(2)));

// CPLX: V is complex (interleaved re, im; element (i, c) at 2 (i + c ldv)) and
// row i is multiplied by the phase of z_i.
template <bool CPLX>
__global__ void __launch_bounds__(ASM_T) k_assemble(AsmArgs a) {
  __shared__ int s_kind[ASM_CB], s_idx[ASM_CB], s_t[ASM_CB];
  __shared__ double s_sig[ASM_CB], s_mu[ASM_CB], s_ic[ASM_CB], s_ub[ASM_CB];
  const int64_t n = a.n;
  const int64_t r0 = (int64_t)blockIdx.x * (ASM_T * ASM_R);
  double di[ASM_R], zi[ASM_R], ui[ASM_R], pr[ASM_R], pm[ASM_R];
  int gi[ASM_R], pi[ASM_R];
#pragma unroll
  for (int j = 0; j < ASM_R; ++j) {
    const int64_t i = r0 + threadIdx.x + j * ASM_T;
    const bool ok = i < n;
    if (CPLX) {
      pr[j] = ok ? a.ph[2 * i] : 0.0;
      pm[j] = ok ? a.ph[2 * i + 1] : 0.0;
    }
    di[j] = ok ? a.d[i] : 0.0;
    zi[j] = ok ? a.z[i] : 0.0;
    ui[j] = ok ? a.ru[i] : 0.0;
    gi[j] = ok ? a.rgrp[i] : -1;
    pi[j] = ok ? a.rpos[i] : -1;
  }
  const int64_t ncg = (n + ASM_CB - 1) / ASM_CB;
  for (int64_t cg = blockIdx.y; cg < ncg; cg += gridDim.y) {
    const int64_t c0 = cg * ASM_CB;
    const int nc = (int)min((int64_t)ASM_CB, n - c0);
    __syncthreads();  // the previous group's parameters are no longer read
    if (threadIdx.x < nc) {
      const int64_t c = c0 + threadIdx.x;
      s_kind[threadIdx.x] = a.ckind[c];
      s_idx[threadIdx.x] = a.cidx[c];
      s_t[threadIdx.x] = a.ct[c];
      s_sig[threadIdx.x] = a.csig[c];
      s_mu[threadIdx.x] = a.cmu[c];
      s_ic[threadIdx.x] = a.cic[c];
      s_ub[threadIdx.x] = a.cub[c];
    }
    __syncthreads();
    for (int cc = 0; cc < nc; ++cc) {
      const int kind = s_kind[cc];
      const int64_t e0 = (c0 + cc) * a.ldv + r0 + threadIdx.x;
      double v[ASM_R];
      if (kind == COL_REDUCED) {
        const double m = s_mu[cc], sg = s_sig[cc], ic = s_ic[cc];
#pragma unroll
        for (int j = 0; j < ASM_R; ++j) {
          // mu / den with one residual correction, then the scaled norm; a
          // row with z_i == 0 (deflated, or a zero member of a merged group)
          // is exactly 0 whatever den is
          const double den = (di[j] - sg) - m;
          const double rc = rcp_nr(den);
          double q = ic * rc;
          q = __builtin_fma(__builtin_fma(-q, den, ic), rc, q);
          v[j] = zi[j] != 0.0 ? zi[j] * q : 0.0;
        }
      } else if (kind == COL_UNIT) {
        const int64_t at = s_idx[cc];
#pragma unroll
        for (int j = 0; j < ASM_R; ++j) v[j] = (r0 + threadIdx.x + j * ASM_T == at) ? 1.0 : 0.0;
      } else {
        // column t of H = I - beta u u^T restricted to the group
        const int g = s_idx[cc], t = s_t[cc];
        const double ub = s_ub[cc];
#pragma unroll
        for (int j = 0; j < ASM_R; ++j) v[j] = gi[j] == g ? (pi[j] == t ? 1.0 : 0.0) - ub * ui[j] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < ASM_R; ++j) {
        if (r0 + threadIdx.x + j * ASM_T >= n) continue;
        if (CPLX) {
          const dbl2 cv = {v[j] * pr[j], v[j] * pm[j]};
          __builtin_nontemporal_store(cv, (dbl2*)(a.V + 2 * (e0 + j * ASM_T)));
        } else {
          __builtin_nontemporal_store(v[j], a.V + e0 + j * ASM_T);
        }
      }
    }
  }
}

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct GLayout {
  size_t dr, zr, lamr, sidx, mu, xn, inf, rgrp, rpos, ru, ckind, cidx, ct, csig, cmu, cic, cub, zabs, ph, solver,
      total;
};
static GLayout glayout(int64_t n) {
  GLayout L;
  size_t o = 0;
  L.dr = o; o = al(o + 8 * n);
  L.zr = o; o = al(o + 8 * n);
  L.lamr = o; o = al(o + 8 * n);
  L.sidx = o; o = al(o + 4 * n);
  L.mu = o; o = al(o + 8 * n);
  L.xn = o; o = al(o + 8 * n);
  L.inf = o; o = al(o + 8);
  L.rgrp = o; o = al(o + 4 * n);
  L.rpos = o; o = al(o + 4 * n);
  L.ru = o; o = al(o + 8 * n);
  L.ckind = o; o = al(o + 4 * n);
  L.cidx = o; o = al(o + 4 * n);
  L.ct = o; o = al(o + 4 * n);
  L.csig = o; o = al(o + 8 * n);
  L.cmu = o; o = al(o + 8 * n);
  L.cic = o; o = al(o + 8 * n);
  L.cub = o; o = al(o + 8 * n);
  L.zabs = o; o = al(o + 8 * n);
  L.ph = o; o = al(o + 16 * n);
  L.solver = o; o = al(o + dpr1_workspace_size(n));
  L.total = o;
  return L;
}

}  // namespace gen
}  // namespace dpr1

using namespace dpr1::gen;
namespace fe = dpr1::fe;

#define GCHECK(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return DPR1_EHIP; \
  } while (0)

extern "C" {

size_t dpr1_general_workspace_size(int64_t n) {
  if (n < 1) return 0;
  return glayout(n).total;
}

}  // extern "C"

// Argument checks shared by the two entry points (same positions).
static int check_args(const double* d, const void* z, double rho, int64_t n, const double* lambda,
                      const double* V, int64_t ldv, const int32_t* info, const dpr1_opts* opts, const void* work,
                      size_t work_bytes) {
  if (!d) return -1;
  if (!z) return -2;
  if (!(rho == rho) || rho == 0.0 || rho == INFINITY || rho == -INFINITY) return -3;
  if (n < 1 || n > (int64_t)INT32_MAX / 2) return -4;
  if (!lambda) return -5;
  if (V && ldv < n) return -7;
  if (!info) return -8;
  if (opts && opts->waves_per_simd != 0 && opts->waves_per_simd != 4 && opts->waves_per_simd != 6 &&
      opts->waves_per_simd != 8)
    return -9;
  if (!work) return -10;
  if (work_bytes < glayout(n).total) return -11;
  return 0;
}

static int set_info(int32_t* info, int32_t code, hipStream_t st) {
  GCHECK(hipMemcpyAsync(info, &code, 4, hipMemcpyHostToDevice, st));
  GCHECK(hipStreamSynchronize(st));
  return DPR1_OK;
}

// The reduction, the reduced solve and the assembly.  hd, hz: host copies of
// the poles and of the (real, here nonnegative in the Hermitian case) z; zdev
// the same z on the device; ph the device phases for a complex V, else null.
static int front_end(const double* d, const double* zdev, const std::vector<double>& hd,
                     const std::vector<double>& hz, const double* ph, double rho, int64_t n, double* lambda,
                     double* V, int64_t ldv, int32_t* info, const dpr1_opts* opts, char* w, const GLayout& L,
                     hipStream_t st, void* stream) {
  // |z_j| < 2^-511 counts as zero: its square is not a normal number, and
  // the eigenvalue beside d_j would lie within rho z_j^2 of it; the assembly
  // then reads this deflated z from the workspace
  std::vector<double> hz0(hz);
  for (double& x : hz0)
    if (std::fabs(x) < 0x1p-511) x = 0.0;
  double* zdef = (double*)(w + L.zabs);
  GCHECK(hipMemcpyAsync(zdef, hz0.data(), 8 * n, hipMemcpyHostToDevice, st));
  zdev = zdef;
  std::vector<double> rd, rz;
  std::vector<int32_t> rgrp(n), rpos(n);
  std::vector<double> ru(n);
  std::vector<fe::Col> cols;
  cols.reserve(n);
  fe::reduce(hd.data(), hz0.data(), n, false, rd, rz, rgrp.data(), rpos.data(), ru.data(), cols);
  const int64_t m = (int64_t)rd.size();

  // the reduced problem on the GPU: eigenvalues and the shifted representation
  // (sigma_k, mu_k, ||x_k||) from which k_assemble evaluates the vectors
  std::vector<double> lamr(m), mur(m), xnr(m);
  std::vector<int32_t> sir(m);
  std::vector<char> mir;
  if (m > 0) {
    double* ddr = (double*)(w + L.dr);
    double* dzr = (double*)(w + L.zr);
    double* dlr = (double*)(w + L.lamr);
    int32_t* dsi = (int32_t*)(w + L.sidx);
    double* dmu = (double*)(w + L.mu);
    double* dxn = (double*)(w + L.xn);
    int32_t* dinf = (int32_t*)(w + L.inf);
    // the inputs [dr, zr] and the outputs [lamr, inf] are contiguous in the
    // workspace: one copy each way through a host mirror
    mir.resize(std::max(L.zr + 8 * m - L.dr, L.inf + 4 - L.lamr));
    memcpy(mir.data(), rd.data(), 8 * m);
    memcpy(mir.data() + (L.zr - L.dr), rz.data(), 8 * m);
    GCHECK(hipMemcpyAsync(ddr, mir.data(), L.zr + 8 * m - L.dr, hipMemcpyHostToDevice, st));
    const int rc = dpr1_eig(ddr, dzr, rho, m, dlr, nullptr, m, V ? dsi : nullptr, V ? dmu : nullptr,
                            V ? dxn : nullptr, dinf, nullptr, opts, w + L.solver, dpr1_workspace_size(m), stream);
    if (rc != DPR1_OK) return rc;
    int32_t hinf = 0;
    GCHECK(hipMemcpyAsync(mir.data(), dlr, L.inf + 4 - L.lamr, hipMemcpyDeviceToHost, st));
    GCHECK(hipStreamSynchronize(st));
    memcpy(lamr.data(), mir.data(), 8 * m);
    if (V) {
      memcpy(sir.data(), mir.data() + (L.sidx - L.lamr), 4 * m);
      memcpy(mur.data(), mir.data() + (L.mu - L.lamr), 8 * m);
      memcpy(xnr.data(), mir.data() + (L.xn - L.lamr), 8 * m);
    }
    memcpy(&hinf, mir.data() + (L.inf - L.lamr), 4);
    if (hinf != DPR1_INFO_OK) return set_info(info, hinf, st);
  }
  {
    std::vector<fe::Col> all;
    fe::merge_cols(cols, lamr.data(), m, all);
    cols.swap(all);
  }
  std::vector<double> lam(n), csig(n, 0.0), cmu(n, 0.0), cic(n, 0.0), cub(n, 0.0);
  std::vector<int32_t> ckind(n), cidx(n), ct(n);
  for (int64_t c = 0; c < n; ++c) {
    const fe::Col& q = cols[c];
    lam[c] = q.val;
    ckind[c] = q.kind;
    cidx[c] = q.idx;
    ct[c] = q.t;
    cub[c] = q.ub;
    if (V && q.kind == COL_REDUCED) {
      csig[c] = rd[sir[q.idx]];
      cmu[c] = mur[q.idx];
      cic[c] = 1.0 / xnr[q.idx];
    }
  }
  GCHECK(hipMemcpyAsync(lambda, lam.data(), 8 * n, hipMemcpyHostToDevice, st));
  if (V) {
    AsmArgs a;
    a.n = n;
    a.ldv = ldv;
    a.d = d;
    a.z = zdev;
    a.ph = ph;
    a.rgrp = (int32_t*)(w + L.rgrp);
    a.rpos = (int32_t*)(w + L.rpos);
    a.ru = (double*)(w + L.ru);
    a.ckind = (int32_t*)(w + L.ckind);
    a.cidx = (int32_t*)(w + L.cidx);
    a.ct = (int32_t*)(w + L.ct);
    a.csig = (double*)(w + L.csig);
    a.cmu = (double*)(w + L.cmu);
    a.cic = (double*)(w + L.cic);
    a.cub = (double*)(w + L.cub);
    a.V = V;
    // the ten column tables [rgrp, cub] are contiguous: one copy
    mir.resize(L.cub + 8 * n - L.rgrp);
    auto put = [&](size_t off, const void* src, size_t bytes) { memcpy(mir.data() + (off - L.rgrp), src, bytes); };
    put(L.rgrp, rgrp.data(), 4 * n);
    put(L.rpos, rpos.data(), 4 * n);
    put(L.ru, ru.data(), 8 * n);
    put(L.ckind, ckind.data(), 4 * n);
    put(L.cidx, cidx.data(), 4 * n);
    put(L.ct, ct.data(), 4 * n);
    put(L.csig, csig.data(), 8 * n);
    put(L.cmu, cmu.data(), 8 * n);
    put(L.cic, cic.data(), 8 * n);
    put(L.cub, cub.data(), 8 * n);
    GCHECK(hipMemcpyAsync(w + L.rgrp, mir.data(), mir.size(), hipMemcpyHostToDevice, st));
    const int64_t rows = ASM_T * ASM_R;
    const int64_t rtiles = (n + rows - 1) / rows;
    // about 512 blocks, each looping over every gy-th column group: the grid's
    // write front then moves through V in order, which HBM takes faster than
    // one block per column group (n = 32768: 5.42 against 5.6 ms per call)
    const int64_t gy = std::min<int64_t>(std::max<int64_t>(16, (512 + rtiles - 1) / rtiles),
                                         std::min<int64_t>((n + ASM_CB - 1) / ASM_CB, 65535));
    const dim3 grid((unsigned)rtiles, (unsigned)gy);
    if (ph)
      hipLaunchKernelGGL(k_assemble<true>, grid, dim3(ASM_T), 0, st, a);
    else
      hipLaunchKernelGGL(k_assemble<false>, grid, dim3(ASM_T), 0, st, a);
    GCHECK(hipGetLastError());
  }
  // set_info waits for the stream: the host vectors above are sources of the
  // copies and must outlive them
  return set_info(info, DPR1_INFO_OK, st);
}

extern "C" {

int dpr1_eig_general(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                     int64_t ldv, int32_t* info, const dpr1_opts* opts, void* work, size_t work_bytes,
                     void* stream) {
  const int bad = check_args(d, z, rho, n, lambda, V, ldv, info, opts, work, work_bytes);
  if (bad) return bad;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> hd(n), hz(n);
  GCHECK(hipMemcpyAsync(hd.data(), d, 8 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipMemcpyAsync(hz.data(), z, 8 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipStreamSynchronize(st));
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(hd[j]) || !std::isfinite(hz[j])) return set_info(info, DPR1_INFO_NONFINITE, st);
  return front_end(d, z, hd, hz, nullptr, rho, n, lambda, V, ldv, info, opts, (char*)work, glayout(n), st, stream);
}

int dpr1_eig_hermitian(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                       int64_t ldv, int32_t* info, const dpr1_opts* opts, void* work, size_t work_bytes,
                       void* stream) {
  const int bad = check_args(d, z, rho, n, lambda, V, ldv, info, opts, work, work_bytes);
  if (bad) return bad;
  hipStream_t st = (hipStream_t)stream;
  const GLayout L = glayout(n);
  char* w = (char*)work;
  std::vector<double> hd(n), hzc(2 * n);
  GCHECK(hipMemcpyAsync(hd.data(), d, 8 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipMemcpyAsync(hzc.data(), z, 16 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipStreamSynchronize(st));
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(hd[j]) || !std::isfinite(hzc[2 * j]) || !std::isfinite(hzc[2 * j + 1]))
      return set_info(info, DPR1_INFO_NONFINITE, st);
  // z = Phi |z| with Phi = diag(z_j / |z_j|) unitary (1 where z_j = 0), and
  // Phi D Phi^H = D: A = Phi (D + rho |z| |z|^T) Phi^H, so the eigenvalues are
  // those of the real problem with |z| and v = Phi v_real
  std::vector<double> ha(n), hph(2 * n);
  for (int64_t j = 0; j < n; ++j) {
    const double re = hzc[2 * j], im = hzc[2 * j + 1];
    const double r = std::hypot(re, im);
    ha[j] = r;
    hph[2 * j] = r > 0.0 ? re / r : 1.0;
    hph[2 * j + 1] = r > 0.0 ? im / r : 0.0;
  }
  double* za = (double*)(w + L.zabs);
  double* ph = (double*)(w + L.ph);
  GCHECK(hipMemcpyAsync(za, ha.data(), 8 * n, hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(ph, hph.data(), 16 * n, hipMemcpyHostToDevice, st));
  // front_end synchronises before it returns, so ha and hph outlive the copies
  return front_end(d, za, hd, ha, ph, rho, n, lambda, V, ldv, info, opts, w, L, st, stream);
}

}  // extern "C"
