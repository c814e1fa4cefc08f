// Front end for reducible inputs (Sec. 1 of the paper): any finite d (any
// order, repeated values) and any finite z (zeros allowed).
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
#include <numeric>
#include <vector>

#include "../../include/dpr1.h"

namespace dpr1 {
namespace gen {

enum : int32_t { COL_REDUCED = 0, COL_UNIT = 1, COL_REFLECT = 2 };

// Per original row i: rgrp its group id, rpos its position in the group, ru
// the reflection vector's component there (0 for groups without reflection).
// Per final column c:
//   COL_REDUCED  csig = sigma_k (the shift pole), cmu = mu_k,
//                cic = 1 / (mu_k ||x_k||)
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
  double* V;
};

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

__global__ void __launch_bounds__(256) k_assemble(AsmArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double di = a.d[i], zi = a.z[i];
  const int g = a.rgrp[i], p = a.rpos[i];
  const double u = a.ru[i];
  for (int64_t c = blockIdx.y; c < a.n; c += gridDim.y) {
    const int kind = a.ckind[c];
    double v = 0.0;
    if (kind == COL_REDUCED) {
      if (zi != 0.0) {
        // mu / den with one residual correction, then the scaled norm
        const double m = a.cmu[c];
        const double den = (di - a.csig[c]) - m;
        const double rc = rcp_nr(den);
        double q = m * rc;
        q = __builtin_fma(__builtin_fma(-q, den, m), rc, q);
        v = (zi * q) * a.cic[c];
      }
    } else if (kind == COL_UNIT) {
      v = (i == a.cidx[c]) ? 1.0 : 0.0;
    } else if (g == a.cidx[c]) {
      // column t of H = I - beta u u^T restricted to the group
      v = (p == a.ct[c] ? 1.0 : 0.0) - a.cub[c] * u;
    }
    __builtin_nontemporal_store(v, &a.V[i + c * a.ldv]);
  }
}

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct GLayout {
  size_t dr, zr, lamr, sidx, mu, xn, inf, rgrp, rpos, ru, ckind, cidx, ct, csig, cmu, cic, cub, solver, total;
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
  L.solver = o; o = al(o + dpr1_workspace_size(n));
  L.total = o;
  return L;
}

}  // namespace gen
}  // namespace dpr1

using namespace dpr1::gen;

#define GCHECK(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return DPR1_EHIP; \
  } while (0)

extern "C" {

size_t dpr1_general_workspace_size(int64_t n) {
  if (n < 1) return 0;
  return glayout(n).total;
}

int dpr1_eig_general(const double* d, const double* z, double rho, int64_t n, double* lambda, double* V,
                     int64_t ldv, int32_t* info, const dpr1_opts* opts, void* work, size_t work_bytes,
                     void* stream) {
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
  const GLayout L = glayout(n);
  if (work_bytes < L.total) return -11;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)work;

  std::vector<double> hd(n), hz(n);
  GCHECK(hipMemcpyAsync(hd.data(), d, 8 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipMemcpyAsync(hz.data(), z, 8 * n, hipMemcpyDeviceToHost, st));
  GCHECK(hipStreamSynchronize(st));
  int32_t code = DPR1_INFO_OK;
  for (int64_t j = 0; j < n; ++j)
    if (!std::isfinite(hd[j]) || !std::isfinite(hz[j])) code = DPR1_INFO_NONFINITE;
  if (code != DPR1_INFO_OK) {
    GCHECK(hipMemcpyAsync(info, &code, 4, hipMemcpyHostToDevice, st));
    GCHECK(hipStreamSynchronize(st));
    return DPR1_OK;
  }

  // sorted position s -> original row order[s]
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return hd[a] > hd[b]; });
  std::vector<double> rd, rz;
  std::vector<int32_t> rgrp(n, -1), rpos(n, 0);
  std::vector<double> ru(n, 0.0);
  struct Col {
    double val;
    int32_t kind, idx, t;
    double ub;
  };
  std::vector<Col> cols;
  cols.reserve(n);
  int32_t ngrp = 0;
  for (int64_t s = 0; s < n;) {
    int64_t e = s + 1;
    while (e < n && hd[order[e]] == hd[order[s]]) ++e;
    const double dv = hd[order[s]];
    // ||w|| scaled by the largest |w_t|, so that no square overflows
    double big = 0.0, nw = 0.0;
    for (int64_t t = s; t < e; ++t) big = std::max(big, std::fabs(hz[order[t]]));
    if (big > 0.0) {
      double acc = 0.0;
      for (int64_t t = s; t < e; ++t) {
        const double q = hz[order[t]] / big;
        acc += q * q;
      }
      nw = big * std::sqrt(acc);
    }
    const int32_t g = ngrp++;
    for (int64_t t = s; t < e; ++t) {
      rgrp[order[t]] = g;
      rpos[order[t]] = (int32_t)(t - s);
    }
    if (nw == 0.0) {
      for (int64_t t = s; t < e; ++t) cols.push_back({dv, COL_UNIT, (int32_t)order[t], 0, 0.0});
    } else if (e - s == 1) {
      rd.push_back(dv);
      rz.push_back(hz[order[s]]);
    } else {
      rd.push_back(dv);
      rz.push_back(nw);
      // u = w/||w|| + sign(u_first) e_first, H = I - beta u u^T, beta = 2/(u^T u)
      std::vector<double> u(e - s);
      for (int64_t t = s; t < e; ++t) u[t - s] = hz[order[t]] / nw;
      u[0] += u[0] >= 0.0 ? 1.0 : -1.0;
      double uu = 0.0;
      for (double x : u) uu += x * x;
      const double beta = 2.0 / uu;
      for (int64_t t = s; t < e; ++t) ru[order[t]] = u[t - s];
      for (int64_t t = 1; t < e - s; ++t) cols.push_back({dv, COL_REFLECT, g, (int32_t)t, beta * u[t]});
    }
    s = e;
  }
  const int64_t m = (int64_t)rd.size();

  // the reduced problem on the GPU: eigenvalues and the shifted representation
  // (sigma_k, mu_k, ||x_k||) from which k_assemble evaluates the vectors
  std::vector<double> lamr(m), mur(m), xnr(m);
  std::vector<int32_t> sir(m);
  if (m > 0) {
    double* ddr = (double*)(w + L.dr);
    double* dzr = (double*)(w + L.zr);
    double* dlr = (double*)(w + L.lamr);
    int32_t* dsi = (int32_t*)(w + L.sidx);
    double* dmu = (double*)(w + L.mu);
    double* dxn = (double*)(w + L.xn);
    int32_t* dinf = (int32_t*)(w + L.inf);
    GCHECK(hipMemcpyAsync(ddr, rd.data(), 8 * m, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync(dzr, rz.data(), 8 * m, hipMemcpyHostToDevice, st));
    const int rc = dpr1_eig(ddr, dzr, rho, m, dlr, nullptr, m, V ? dsi : nullptr, V ? dmu : nullptr,
                            V ? dxn : nullptr, dinf, nullptr, opts, w + L.solver, dpr1_workspace_size(m), stream);
    if (rc != DPR1_OK) return rc;
    int32_t hinf = 0;
    GCHECK(hipMemcpyAsync(lamr.data(), dlr, 8 * m, hipMemcpyDeviceToHost, st));
    if (V) {
      GCHECK(hipMemcpyAsync(sir.data(), dsi, 4 * m, hipMemcpyDeviceToHost, st));
      GCHECK(hipMemcpyAsync(mur.data(), dmu, 8 * m, hipMemcpyDeviceToHost, st));
      GCHECK(hipMemcpyAsync(xnr.data(), dxn, 8 * m, hipMemcpyDeviceToHost, st));
    }
    GCHECK(hipMemcpyAsync(&hinf, dinf, 4, hipMemcpyDeviceToHost, st));
    GCHECK(hipStreamSynchronize(st));
    if (hinf != DPR1_INFO_OK) {
      GCHECK(hipMemcpyAsync(info, &hinf, 4, hipMemcpyHostToDevice, st));
      GCHECK(hipStreamSynchronize(st));
      return DPR1_OK;
    }
    for (int64_t k = 0; k < m; ++k) cols.push_back({lamr[k], COL_REDUCED, (int32_t)k, 0, 0.0});
  }
  std::stable_sort(cols.begin(), cols.end(), [](const Col& a, const Col& b) { return a.val > b.val; });

  std::vector<double> lam(n), csig(n, 0.0), cmu(n, 0.0), cic(n, 0.0), cub(n, 0.0);
  std::vector<int32_t> ckind(n), cidx(n), ct(n);
  for (int64_t c = 0; c < n; ++c) {
    const Col& q = cols[c];
    lam[c] = q.val;
    ckind[c] = q.kind;
    cidx[c] = q.idx;
    ct[c] = q.t;
    cub[c] = q.ub;
    if (V && q.kind == COL_REDUCED) {
      csig[c] = rd[sir[q.idx]];
      cmu[c] = mur[q.idx];
      cic[c] = 1.0 / (mur[q.idx] * xnr[q.idx]);
    }
  }
  GCHECK(hipMemcpyAsync(lambda, lam.data(), 8 * n, hipMemcpyHostToDevice, st));
  if (V) {
    AsmArgs a;
    a.n = n;
    a.ldv = ldv;
    a.d = d;
    a.z = z;
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
    GCHECK(hipMemcpyAsync((void*)a.rgrp, rgrp.data(), 4 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.rpos, rpos.data(), 4 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.ru, ru.data(), 8 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.ckind, ckind.data(), 4 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.cidx, cidx.data(), 4 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.ct, ct.data(), 4 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.csig, csig.data(), 8 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.cmu, cmu.data(), 8 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.cic, cic.data(), 8 * n, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync((void*)a.cub, cub.data(), 8 * n, hipMemcpyHostToDevice, st));
    const unsigned gy = (unsigned)std::min<int64_t>(n, 4096);
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((n + 255) / 256), gy), dim3(256), 0, st, a);
    GCHECK(hipGetLastError());
  }
  code = DPR1_INFO_OK;
  GCHECK(hipMemcpyAsync(info, &code, 4, hipMemcpyHostToDevice, st));
  // the host vectors above are sources of the copies: wait before they go
  GCHECK(hipStreamSynchronize(st));
  return DPR1_OK;
}

}  // extern "C"
