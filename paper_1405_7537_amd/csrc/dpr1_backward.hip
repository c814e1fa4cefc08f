// Reverse mode of the DPR1 eigendecomposition on gfx950.
//
// For L(Lambda, V):  Abar = V X V^T,  X = diag(lambda_bar) + F o (V^T V_bar),
// F_lk = 1/(lambda_k - lambda_l) for l != k (first-order perturbation of a
// symmetric eigendecomposition with simple eigenvalues; the interlacing of
// Sec. 1 makes every eigenvalue of an irreducible DPR1 matrix simple).  With
// dA = diag(dd) + drho z z^T + rho (dz z^T + z dz^T):
//   d_bar_j = Abar_jj = sum_k (V X)_jk V_jk
//   rho_bar = z^T Abar z = y^T X y,            y = V^T z
//   z_bar   = rho (Abar + Abar^T) z = rho V (X + X^T) y
// and y_k = v_k^T z = -1/(rho ||x_k||) because f(lambda_k) = 0 (eq. Pick,
// Aeigenvec), which avoids the cancellation of the sum v_k^T z.  The gaps
// lambda_k - lambda_l come from the shifted representation
// (d_{i_k} + mu_k) - (d_{i_l} + mu_l), added in double-double, so clustered
// eigenvalues keep their relative gap accuracy.
//
// Kernels:
//   k_gemm<EPI_X>  P = V^T V_bar on FP64 matrix cores, epilogue X = F o P +
//                  diag(lambda_bar), partial sums of X y (rows) and X^T y (cols)
//   k_bwd_u        u = (X + X^T) y and rho_bar = y^T X y from those partials
//   k_gemm<EPI_D>  Q = V X on FP64 matrix cores, epilogue partial row sums of
//                  Q o V (for d_bar) and of V diag(u) (for z_bar)
//   k_bwd_final    d_bar, z_bar = rho V u from the partials
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/dpr1.h"
#include "dd.h"

namespace dpr1 {
namespace bwd {

// Block tile 128 x 128 (2 x WNW waves of 64 x TN, each 4 x TN/16 blocks of
// the 16x16x4 FP64 MFMA), K staged through LDS in slices of 16,
// double-buffered.
constexpr int BM = 128, BN = 128, BK = 16;
constexpr int WNW = 4;               // waves along n
constexpr int TN = BN / WNW;         // columns per wave
constexpr int NBT = TN / 16;         // MFMA blocks per wave along n
constexpr int NT = 128 * WNW;
constexpr int PAD = 2;   // LDS row padding (doubles)
constexpr int NXCD = 8;  // workgroups are dealt round-robin to the 8 XCDs

typedef double double4_t __attribute__((ext_vector_type(4)));

enum { EPI_X = 0, EPI_D = 1 };

struct GArgs {
  int64_t n;
  int nb;
  const double* A;   // V (both GEMMs), or null: V recomputed from (z, shift, mu, ||x||)
  const double* z;      // [nb*n]  (used when A is null)
  const double* sig;    // [nb*n]  d_{i_k}, the shift of eigenvalue k (used when A is null)
  const double* ixn;    // [nb*n]  1/||x_k|| (used when A is null)
  const double* B;   // V_bar (EPI_X, column-major) or X (EPI_D, row-major)
  double* C;         // X (EPI_X), stored row-major
  // EPI_X
  const double* lam_bar;  // [nb*n] or null
  const double* d;        // [nb*n]
  const int32_t* sidx;    // [nb*n]
  const double* mu;       // [nb*n]
  const double* y;        // [nb*n]
  double* part_r;         // [nb][ntile][n]  sum_k X_lk y_k over the tile's k range
  double* part_c;         // [nb][ntile][n]  sum_l X_lk y_l over the tile's l range
  // EPI_D
  const double* u;        // [nb*n]  (X + X^T) y
  double* part_d;         // [nb][ntile][n]  sum_k Q_jk V_jk
  double* part_z;         // [nb][ntile][n]  sum_k V_jk u_k
  int has_B;              // 0: V_bar is null, P = 0
  int64_t lda;            // leading dimension of V (A), column-major
  int64_t ldb;            // leading dimension of V_bar (EPI_X's B), column-major
};

// Element (j, k) of V for problem offset vo, recomputed from the forward's
// shifted representation: v_k[j] = z_j / (((d_j - d_{i_k}) - mu_k) ||x_k||)
// (eq. eigenvecAi), so that a caller short of memory need not keep V between
// the forward and the backward.  d_{i_k} and 1/||x_k|| come precomputed
// (k_bwd_y); the quotient is the refined reciprocal with one residual
// correction, as in the forward's eigenvector writer.
__device__ __forceinline__ double v_from(double dj, double zj, double sk, double mk, double ik) {
  const double den = (dj - sk) - mk;
  double r = __builtin_amdgcn_rcp(den);
  r = __builtin_fma(r, __builtin_fma(-den, r, 1.0), r);
  double q = zj * r;
  q = __builtin_fma(__builtin_fma(-q, den, zj), r, q);
  return q * ik;
}
__device__ __forceinline__ double v_elem(const GArgs& g, int64_t vo, int64_t j, int64_t k) {
  return v_from(g.d[vo + j], g.z[vo + j], g.sig[vo + k], g.mu[vo + k], g.ixn[vo + k]);
}

// Column-major n x n matrices (V with ld = lda, V_bar with ld = ldb; a
// batch's problems lda * n and ldb * n apart; X row-major with ld = n).
// EPI_X computes op(A) = A^T (A = V),
// EPI_D op(A) = A.  The linear block index is mapped so that all tiles of a
// problem run on one XCD and share its L2.
// RV: V is not passed in; its elements are rebuilt by v_elem (a separate
// instance, so that the path with V keeps its plain loads).
// Two blocks per CU (66.5 KB of LDS each, 68 KB where V^T is rebuilt) are 4
// waves per SIMD, which leaves 128 VGPRs a lane: the bound asks for that
// budget.
template <int EPI, bool RV>
__global__ void __launch_bounds__(NT, 4) k_gemm(GArgs g) {
  const int64_t n = g.n;
  const int tiles = (int)((n + BM - 1) / BM);
  const int T = tiles * tiles;
  const int B_ = blockIdx.x;
  const int xcd = B_ % NXCD, slot = B_ / NXCD;
  const int t = slot % T;
  const int pb = NXCD * (slot / T) + xcd;
  if (pb >= g.nb) return;
  const int tm = t % tiles, tn = t / tiles;
  const int64_t mo = (int64_t)pb * n * n;
  const int64_t vo = (int64_t)pb * n;
  const double* A = RV ? nullptr : g.A + (int64_t)pb * g.lda * n;
  const double* Bm = g.B + (EPI == EPI_X ? (int64_t)pb * g.ldb * n : mo);
  const int64_t lda = g.lda, ldb = g.ldb;
  const int m0 = tm * BM, n0 = tn * BN;
  const int tid = threadIdx.x;
  const int wv = tid / 64, lane = tid % 64;
  const int wm = (wv & 1) * 64, wn = (wv >> 1) * TN;

  // one LDS buffer: the double-buffered operand tiles during the K loop,
  // the epilogue's per-row / per-column arrays after it
  constexpr int TILE_D = 2 * BK * (BM + PAD);
  constexpr int EPI_D_N = 3 * BM + 4 * BN + 2 * WNW * BM + 2 * BN;
  constexpr int SMEM_D = 2 * TILE_D > EPI_D_N ? 2 * TILE_D : EPI_D_N;
  __shared__ double smem[SMEM_D];
  double(*As)[BK][BM + PAD] = reinterpret_cast<double(*)[BK][BM + PAD]>(smem);
  double(*Bs)[BK][BN + PAD] = reinterpret_cast<double(*)[BK][BN + PAD]>(smem + TILE_D);

  double4_t acc[4][NBT];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NBT; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};

  constexpr int PER = (BM * BK) / NT;  // elements of each operand per thread
  static_assert(BM == BN && NT % BM == 0 && NT % BK == 0, "tile shape");
  // Element e2 of a thread: EPI_X: k = ek, m (or c) = em + STEP e2; EPI_D: m (or
  // c) = em, k = ek + STEP e2.  The per-thread part of each address is formed
  // once; what changes with k0 and e2 is uniform across the block.
  constexpr int STEP = EPI == EPI_X ? NT / BK : NT / BM;
  const int ek = EPI == EPI_X ? tid % BK : tid / BM;
  const int em = EPI == EPI_X ? tid / BK : tid % BM;
  const double* pA = RV ? nullptr : (EPI == EPI_X ? A + ek + (m0 + em) * lda : A + (m0 + em) + ek * lda);
  const double* pB = EPI == EPI_X ? Bm + ek + (n0 + em) * ldb : Bm + (int64_t)ek * n + (n0 + em);
  double ra[PER], rb[PER];
  // V^T rebuilt (EPI_X): the tile's columns k = m0 .. m0 + BM - 1 keep their
  // (d_{i_k}, mu_k, 1/||x_k||) in LDS for the whole K loop, and a thread's
  // elements of one K step share their row j, so d_j and z_j load once
  __shared__ double colc[RV && EPI == EPI_X ? 3 : 1][RV && EPI == EPI_X ? BM : 1];
  // V rebuilt (EPI_D): a thread's elements all lie in its row j = m0 + em
  double djr = 0.0, zjr = 0.0;
  if constexpr (RV && EPI == EPI_D) {
    if (m0 + em < n) {
      djr = g.d[vo + m0 + em];
      zjr = g.z[vo + m0 + em];
    }
  }
  if constexpr (RV && EPI == EPI_X) {
    for (int t = tid; t < BM; t += NT) {
      const int64_t gm = m0 + t;
      const bool ok = gm < n;
      colc[0][t] = ok ? g.sig[vo + gm] : 0.0;
      colc[1][t] = ok ? g.mu[vo + gm] : 0.0;
      colc[2][t] = ok ? g.ixn[vo + gm] : 0.0;
    }
    __syncthreads();
  }
  auto gload = [&](int64_t k0) {
    double dj = 0.0, zj = 0.0;
    if constexpr (RV && EPI == EPI_X) {
      const int64_t gk = k0 + ek;
      if (gk < n) {
        dj = g.d[vo + gk];
        zj = g.z[vo + gk];
      }
    }
#pragma unroll
    for (int e2 = 0; e2 < PER; ++e2) {
      if (EPI == EPI_X) {
        // A^T(m, k) = V[k + m lda] and V_bar(k, c) = V_bar[k + c ldb], contiguous along k
        const int64_t gk = k0 + ek, gm = m0 + em + STEP * e2, gc = n0 + em + STEP * e2;
        const int ml = em + STEP * e2;
        ra[e2] = (gm < n && gk < n)
                     ? (RV ? v_from(dj, zj, colc[0][RV ? ml : 0], colc[1][RV ? ml : 0], colc[2][RV ? ml : 0])
                           : pA[k0 + STEP * e2 * lda])
                     : 0.0;
        rb[e2] = (gk < n && gc < n) ? pB[k0 + STEP * e2 * ldb] : 0.0;
      } else {
        // A(m, k) = V[m + k lda], contiguous along m; X(k, c) = X[k n + c] (row-major), contiguous along c
        const int64_t gk = k0 + ek + STEP * e2, gm = m0 + em, gc = n0 + em;
        ra[e2] = (gm < n && gk < n)
                     ? (RV ? v_from(djr, zjr, g.sig[vo + gk], g.mu[vo + gk], g.ixn[vo + gk]) : pA[(k0 + STEP * e2) * lda])
                     : 0.0;
        rb[e2] = (gk < n && gc < n) ? pB[(k0 + STEP * e2) * n] : 0.0;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e2 = 0; e2 < PER; ++e2) {
      int e = tid + e2 * NT;
      if (EPI == EPI_X) {
        As[buf][e % BK][e / BK] = ra[e2];
        Bs[buf][e % BK][e / BK] = rb[e2];
      } else {
        As[buf][e / BM][e % BM] = ra[e2];
        Bs[buf][e / BN][e % BN] = rb[e2];
      }
    }
  };

  const bool doB = (EPI == EPI_D) || g.has_B;
  if (doB) {
    gload(0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < n; k0 += BK) {
      const bool more = k0 + BK < n;
      if (more) gload(k0 + BK);  // next slice in flight during this one
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        // 16x16x4 FP64 MFMA: lane holds A(row = lane%16, k = lane/16) and
        // B(k = lane/16, col = lane%16)
        const int r = lane % 16, q = lane / 16;
        double af[4], bf[NBT];
#pragma unroll
        for (int x = 0; x < 4; ++x) af[x] = As[buf][ks + q][wm + 16 * x + r];
#pragma unroll
        for (int x = 0; x < NBT; ++x) bf[x] = Bs[buf][ks + q][wn + 16 * x + r];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < NBT; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      if (more) {
        sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }
  }

  // Epilogue.  Accumulator element q of a lane holds row lane/16 + 4q,
  // column lane%16 of its 16x16 block (checked on gfx950 with a probe that
  // multiplies A(:,0) = 2^i by B(0,:) = 3^j).  The per-row and per-column
  // quantities of this tile are staged in LDS first; per-row / per-column
  // partial sums go back through LDS.
  __syncthreads();  // every wave is done with the operand tiles
  double* rsig = smem;
  double* rmu = rsig + BM;
  double* ry = rmu + BM;
  double* csig = ry + BM;
  double* cmu = csig + BN;
  double* cy = cmu + BN;
  double* clb = cy + BN;
  double(*rowp)[WNW][BM] = reinterpret_cast<double(*)[WNW][BM]>(clb + BN);  // [quantity][wave along n][row]
  double(*colp)[BN] = reinterpret_cast<double(*)[BN]>(clb + BN + 2 * WNW * BM);  // [wave along m][col]
  // shift indices come from the caller: clamped so that a bad one cannot
  // address outside the problem
  auto sidx = [&](int64_t k) { return (int64_t)min(max(g.sidx[vo + k], 0), (int)(n - 1)); };
  if (tid < BM) {
    int64_t row = m0 + tid;
    if (row < n) {
      if (EPI == EPI_X) {
        rsig[tid] = g.d[vo + sidx(row)];
        rmu[tid] = g.mu[vo + row];
        ry[tid] = g.y[vo + row];
      }
    }
  } else if (tid < BM + BN) {
    int c = tid - BM;
    int64_t col = n0 + c;
    if (col < n) {
      if (EPI == EPI_X) {
        csig[c] = g.d[vo + sidx(col)];
        cmu[c] = g.mu[vo + col];
        cy[c] = g.y[vo + col];
        clb[c] = g.lam_bar ? g.lam_bar[vo + col] : 0.0;
      } else {
        cy[c] = g.u[vo + col];
      }
    }
  }
  __syncthreads();
  const int half_n = wv >> 1, half_m = wv & 1;  // wave index along n, along m
  double cs[NBT];
#pragma unroll
  for (int b = 0; b < NBT; ++b) cs[b] = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double rs1[4] = {0.0, 0.0, 0.0, 0.0}, rs2[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
      const int cl = wn + b * 16 + lane % 16;
      const int64_t col = n0 + cl;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rl = wm + a * 16 + (lane / 16) + 4 * q;
        const int64_t row = m0 + rl;
        if (row >= n || col >= n) continue;
        double v = acc[a][b][q];
        if (EPI == EPI_X) {
          // X(row = l, col = k), stored row-major (consecutive lanes on
          // consecutive columns)
          double x;
          if (row == col) {
            x = clb[cl];
          } else {
            dd gap = dd_add(two_sum(csig[cl], -rsig[rl]), two_sum(cmu[cl], -rmu[rl]));
            x = v / (gap.hi + gap.lo);
          }
          g.C[mo + row * n + col] = x;
          rs1[q] += x * cy[cl];
          cs[b] += x * ry[rl];
        } else {
          // Q(row = j, col = k) V(j, k) for d_bar, V(j, k) u_k for z_bar
          double vjk = RV ? v_elem(g, vo, row, col) : A[row + col * lda];
          rs1[q] += v * vjk;
          rs2[q] += vjk * cy[cl];
        }
      }
    }
    // reduce over the 16 lanes sharing a row (same lane/16)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double s1 = rs1[q], s2 = rs2[q];
      for (int o = 1; o < 16; o <<= 1) {
        s1 += __shfl_xor(s1, o);
        if (EPI == EPI_D) s2 += __shfl_xor(s2, o);
      }
      if (lane % 16 == 0) {
        int r = wm + a * 16 + (lane / 16) + 4 * q;
        rowp[0][half_n][r] = s1;
        rowp[1][half_n][r] = s2;
      }
    }
  }
  if (EPI == EPI_X) {
    // columns: reduce over the 4 lane groups sharing a column (same lane%16)
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
      double c = cs[b];
      c += __shfl_xor(c, 16);
      c += __shfl_xor(c, 32);
      if (lane < 16) colp[half_m][wn + b * 16 + lane] = c;
    }
  }
  __syncthreads();
  const int ntile = tiles;
  if (tid < BM) {
    int64_t row = m0 + tid;
    if (row < n) {
      int64_t a = ((int64_t)pb * ntile + tn) * n + row;
      double s1 = rowp[0][0][tid], s2 = rowp[1][0][tid];
      for (int w = 1; w < WNW; ++w) {
        s1 += rowp[0][w][tid];
        s2 += rowp[1][w][tid];
      }
      if (EPI == EPI_X) {
        g.part_r[a] = s1;
      } else {
        g.part_d[a] = s1;
        g.part_z[a] = s2;
      }
    }
  } else if (EPI == EPI_X && tid < BM + BN) {
    int c = tid - BM;
    int64_t col = n0 + c;
    if (col < n) g.part_c[((int64_t)pb * ntile + tm) * n + col] = colp[0][c] + colp[1][c];
  }
}

// y_k = v_k^T z = -1/(rho ||x_k||); for the products without a stored V also
// the shift d_{i_k} (index clamped to the problem) and 1/||x_k||
__global__ void __launch_bounds__(256) k_bwd_y(int64_t n, int64_t nb, const double* __restrict__ rho,
                                               const double* __restrict__ xnorm, const double* __restrict__ d,
                                               const int32_t* __restrict__ sidx, double* __restrict__ y,
                                               double* __restrict__ sig, double* __restrict__ ixn) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  int64_t p = t / n;
  y[t] = -1.0 / (rho[p] * xnorm[t]);
  if (sig) {
    const int64_t ik = (int64_t)min(max(sidx[t], 0), (int)(n - 1));
    sig[t] = d[p * n + ik];
    ixn[t] = 1.0 / xnorm[t];
  }
}

// u = X y + X^T y and rho_bar = y^T X y from the partials of the first GEMM
__global__ void __launch_bounds__(256) k_bwd_u(int64_t n, int ntile, const double* __restrict__ part_r,
                                               const double* __restrict__ part_c, const double* __restrict__ y,
                                               double* __restrict__ u, double* __restrict__ rho_bar) {
  const int pb = blockIdx.x;
  const int64_t vo = (int64_t)pb * n;
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    double r = 0.0, c = 0.0;
    for (int t = 0; t < ntile; ++t) {
      int64_t a = ((int64_t)pb * ntile + t) * n + j;
      r += part_r[a];
      c += part_c[a];
    }
    u[vo + j] = r + c;
    acc += y[vo + j] * r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) rho_bar[pb] = red[0];
}

// d_bar_j = sum_k (V X)_jk V_jk and z_bar = rho V u from the second GEMM's partials
__global__ void __launch_bounds__(256) k_bwd_final(int64_t n, int64_t nb, int ntile, const double* __restrict__ rho,
                                                   const double* __restrict__ part_d,
                                                   const double* __restrict__ part_z, double* __restrict__ d_bar,
                                                   double* __restrict__ z_bar) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  int64_t pb = t / n, j = t % n;
  double sd = 0.0, sz = 0.0;
  for (int q = 0; q < ntile; ++q) {
    int64_t a = (pb * ntile + q) * n + j;
    sd += part_d[a];
    sz += part_z[a];
  }
  d_bar[t] = sd;
  z_bar[t] = rho[pb] * sz;
}

// Without V_bar only the eigenvalue part remains, in closed form (O(n^2) per
// problem instead of two n^3 products): d_bar_j = sum_k lam_bar_k v_jk^2,
// z_bar_j = -2 sum_k lam_bar_k v_jk / ||x_k|| (from v_k^T z = -1/(rho ||x_k||)),
// rho_bar = sum_k lam_bar_k / (rho ||x_k||)^2.  Grid (row blocks, problems);
// the first row block of a problem also forms rho_bar.
__global__ void __launch_bounds__(256) k_bwd_eigonly(GArgs g, const double* __restrict__ lam_bar,
                                                     const double* __restrict__ xnorm,
                                                     const double* __restrict__ rho, double* __restrict__ d_bar,
                                                     double* __restrict__ z_bar, double* __restrict__ rho_bar) {
  const int64_t n = g.n;
  const int64_t p = blockIdx.y;
  const int64_t vo = p * n;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) {
      const double lb = lam_bar ? lam_bar[vo + k] : 0.0;
      const double yk = 1.0 / (rho[p] * xnorm[vo + k]);
      acc += lb * (yk * yk);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) rho_bar[p] = red[0];
  }
  if (j >= n) return;
  double sd = 0.0, sz = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double lb = lam_bar ? lam_bar[vo + k] : 0.0;
    const double v = g.A ? g.A[p * g.lda * n + j + k * g.lda] : v_elem(g, vo, j, k);
    const double t = lb * v;
    sd = __builtin_fma(t, v, sd);
    sz += t / xnorm[vo + k];
  }
  d_bar[vo + j] = sd;
  z_bar[vo + j] = -2.0 * sz;
}

// rho of the single-problem call, moved to the device as a kernel argument
// (no copy from host memory, so the call can be captured in a graph)
__global__ void k_set_rho(double* __restrict__ dst, double v) { *dst = v; }

struct BLayout {
  size_t X, y, u, pr, pc, pd, pz, sig, ixn, rho, total;
};
static size_t al(size_t x) { return (x + 255) & ~size_t(255); }
static BLayout blayout(int64_t n, int64_t nb) {
  BLayout L;
  int64_t nt = (n + BM - 1) / BM;
  size_t o = 0;
  L.X = o; o = al(o + sizeof(double) * n * n * nb);
  L.y = o; o = al(o + sizeof(double) * n * nb);
  L.u = o; o = al(o + sizeof(double) * n * nb);
  L.pr = o; o = al(o + sizeof(double) * n * nt * nb);
  L.pc = o; o = al(o + sizeof(double) * n * nt * nb);
  L.pd = o; o = al(o + sizeof(double) * n * nt * nb);
  L.pz = o; o = al(o + sizeof(double) * n * nt * nb);
  L.sig = o; o = al(o + sizeof(double) * n * nb);
  L.ixn = o; o = al(o + sizeof(double) * n * nb);
  L.rho = o; o = al(o + sizeof(double));
  L.total = o;
  return L;
}

// The launches of both entry points (arguments checked there).
static int run_backward(int64_t nbatch, int64_t n, const double* d, const double* z, const double* rho,
                        const int32_t* shift_idx, const double* mu, const double* xnorm, const double* V, int64_t lda,
                        const double* lambda_bar, const double* V_bar, int64_t ldb, double* d_bar, double* z_bar,
                        double* rho_bar, void* work, const BLayout& L, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)work;
  double* X = (double*)(w + L.X);
  double* y = (double*)(w + L.y);
  double* u = (double*)(w + L.u);
  double* pr = (double*)(w + L.pr);
  double* pc = (double*)(w + L.pc);
  double* pd = (double*)(w + L.pd);
  double* pz = (double*)(w + L.pz);
  const int tiles = (int)((n + BM - 1) / BM);
  const int64_t nbpad = (nbatch + NXCD - 1) / NXCD * NXCD;
  const unsigned ggrid = (unsigned)(nbpad * tiles * tiles);

  double* sig = V ? nullptr : (double*)(w + L.sig);
  double* ixn = V ? nullptr : (double*)(w + L.ixn);
  hipLaunchKernelGGL(k_bwd_y, dim3((unsigned)((n * nbatch + 255) / 256)), dim3(256), 0, st, n, nbatch, rho, xnorm, d,
                     shift_idx, y, sig, ixn);
  GArgs g;
  g.n = n;
  g.nb = (int)nbatch;
  g.A = V;
  g.z = z;
  g.sig = sig;
  g.ixn = ixn;
  g.B = V_bar;
  g.C = X;
  g.lam_bar = lambda_bar;
  g.d = d;
  g.sidx = shift_idx;
  g.mu = mu;
  g.y = y;
  g.part_r = pr;
  g.part_c = pc;
  g.u = u;
  g.part_d = pd;
  g.part_z = pz;
  g.has_B = V_bar != nullptr;
  g.lda = lda;
  g.ldb = ldb;
  if (!V_bar) {
    hipLaunchKernelGGL(k_bwd_eigonly, dim3((unsigned)((n + 255) / 256), (unsigned)nbatch), dim3(256), 0, st, g,
                       lambda_bar, xnorm, rho, d_bar, z_bar, rho_bar);
    if (hipGetLastError() != hipSuccess) return DPR1_EHIP;
    return DPR1_OK;
  }
  if (V)
    hipLaunchKernelGGL((k_gemm<EPI_X, false>), dim3(ggrid), dim3(NT), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm<EPI_X, true>), dim3(ggrid), dim3(NT), 0, st, g);
  if (hipGetLastError() != hipSuccess) return DPR1_EHIP;
  hipLaunchKernelGGL(k_bwd_u, dim3((unsigned)nbatch), dim3(256), 0, st, n, tiles, pr, pc, y, u, rho_bar);
  g.B = X;
  if (V)
    hipLaunchKernelGGL((k_gemm<EPI_D, false>), dim3(ggrid), dim3(NT), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm<EPI_D, true>), dim3(ggrid), dim3(NT), 0, st, g);
  if (hipGetLastError() != hipSuccess) return DPR1_EHIP;
  hipLaunchKernelGGL(k_bwd_final, dim3((unsigned)((n * nbatch + 255) / 256)), dim3(256), 0, st, n, nbatch, tiles,
                     rho, pd, pz, d_bar, z_bar);
  if (hipGetLastError() != hipSuccess) return DPR1_EHIP;
  return DPR1_OK;
}

}  // namespace bwd
}  // namespace dpr1

using namespace dpr1::bwd;

extern "C" {

size_t dpr1_backward_workspace_size(int64_t n, int64_t nbatch) {
  if (n < 1 || nbatch < 1) return 0;
  return blayout(n, nbatch).total;
}

int dpr1_eig_backward_batched(int64_t nbatch, int64_t n, const double* d, const double* z, const double* rho,
                              const int32_t* shift_idx, const double* mu, const double* xnorm, const double* V,
                              const double* lambda_bar, const double* V_bar, double* d_bar, double* z_bar,
                              double* rho_bar, void* work, size_t work_bytes, void* stream) {
  if (nbatch < 1 || nbatch > 65535) return -1;
  if (n < 1 || n > (1 << 20)) return -2;
  if (!d) return -3;
  if (!z && !V) return -4;
  if (!rho) return -5;
  if (!shift_idx) return -6;
  if (!mu) return -7;
  if (!xnorm) return -8;
  if (!d_bar) return -12;
  if (!z_bar) return -13;
  if (!rho_bar) return -14;
  if (!work) return -15;
  BLayout L = blayout(n, nbatch);
  if (work_bytes < L.total) return -16;
  return run_backward(nbatch, n, d, z, rho, shift_idx, mu, xnorm, V, n, lambda_bar, V_bar, n, d_bar, z_bar, rho_bar,
                      work, L, stream);
}

int dpr1_eig_backward(const double* d, const double* z, double rho, int64_t n, const int32_t* shift_idx,
                      const double* mu, const double* xnorm, const double* V, int64_t ldv, const double* lambda_bar,
                      const double* V_bar, int64_t ldvb, double* d_bar, double* z_bar, double* rho_bar, void* work,
                      size_t work_bytes, void* stream) {
  if (!d) return -1;
  if (!z && !V) return -2;
  if (!(rho == rho) || rho == 0.0 || rho == INFINITY || rho == -INFINITY) return -3;
  if (n < 1 || n > (1 << 20)) return -4;
  if (!shift_idx) return -5;
  if (!mu) return -6;
  if (!xnorm) return -7;
  if (V && ldv < n) return -9;
  if (V_bar && ldvb < n) return -12;
  if (!d_bar) return -13;
  if (!z_bar) return -14;
  if (!rho_bar) return -15;
  if (!work) return -16;
  BLayout L = blayout(n, 1);
  if (work_bytes < L.total) return -17;
  double* drho = (double*)((char*)work + L.rho);
  hipLaunchKernelGGL(k_set_rho, dim3(1), dim3(1), 0, (hipStream_t)stream, drho, rho);
  if (hipGetLastError() != hipSuccess) return DPR1_EHIP;
  return run_backward(1, n, d, z, drho, shift_idx, mu, xnorm, V, V ? ldv : n, lambda_bar, V_bar, V_bar ? ldvb : n,
                      d_bar, z_bar, rho_bar, work, L, stream);
}

}  // extern "C"
