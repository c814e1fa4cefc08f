// Divide-and-conquer eigensolver for a real symmetric tridiagonal matrix T,
// the application of DPR1 eigenproblems named in Sec. 1 of the paper: every
// merge of two halves is a DPR1 problem.
//
// Split a block at m = size/2 with beta = its off-diagonal there:
//   T = diag(T1 - beta e_m e_m^T, T2 - beta e_1 e_1^T) + beta u u^T,
//   u = e_m + e_{m+1}.
// With T_h = Q_h Lambda_h Q_h^T the merged block is
//   Q (diag(Lambda1, Lambda2) + beta z z^T) Q^T, Q = diag(Q1, Q2),
//   z = Q^T u = [last row of Q1, first row of Q2],
// and its eigenvectors are Q V for the DPR1 eigenvectors V.  The split tree
// goes down to 1 x 1 leaves; all merges of one depth are done together:
//   1. z of every merge: a 1 x 1 child gives 1; the row of a larger child's Q
//      was formed by k_zrows when that child was merged, straight from its
//      children's Q and its V, so it is on the host before that child's
//      product (step 5) has finished;
//   2. the host reduces each merge as in Sec. 1 (unsorted poles, equal poles,
//      zero z_j: reduce.h), a z_j below 2^-300 max|z| counting as zero and
//      poles within 8 eps max|d| merged like equal ones;
//   3. one batched launch of the DPR1 solver (dpr1_eig_batched, eigenvalues
//      and the shifted representation only) solves all reduced problems;
//   4. k_tri_assemble writes every merge's V (eq. (eigenvecAi) on the merge's
//      own poles and z, unit and reflection columns);
//   5. k_dgemm forms diag(Q1, Q2) V for every merge into the other Q buffer
//      (two products per merge, one batched launch over 128 x 128 tiles on
//      FP64 matrix cores).
// The two Q buffers alternate between depths so that the root's product
// lands in the caller's Q.  A block is written only by its own merge and read
// only by its parent's, and a leaf's 1 x 1 block (= 1) is set in both buffers
// at the start, so no buffer is ever cleared.
// Steps 2 and 3 of a depth overlap the product of the depth below: the
// host work runs while that product occupies the caller's stream, and the
// DPR1 solves go to a second stream of the library (nothing they read or
// write is touched by the assembly or the products).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/dpr1.h"
#include "reduce.h"

namespace dpr1 {
namespace tri {

using fe::COL_REDUCED;
using fe::COL_REFLECT;
using fe::COL_UNIT;

struct Node {
  int64_t start, size, m;
  int depth;
  int side;  // 0 the root, 1 the left child of its parent, 2 the right child
};

static void build_tree(int64_t start, int64_t size, int depth, std::vector<Node>& out, int& maxd, int side = 0) {
  if (size < 2) return;
  const int64_t m = size / 2;
  out.push_back({start, size, m, depth, side});
  maxd = std::max(maxd, depth);
  build_tree(start, m, depth + 1, out, maxd, 1);
  build_tree(start + m, size - m, depth + 1, out, maxd, 2);
}

// The diagonal of every leaf after the splits above it: each split subtracts
// beta from the two diagonal entries beside it, the split nearer the root
// first (the order of the recursion).
static void modify_diag(std::vector<double>& a, const std::vector<double>& b, int64_t start, int64_t size) {
  if (size < 2) return;
  const int64_t m = size / 2;
  const double beta = b[start + m - 1];
  a[start + m - 1] -= beta;
  a[start + m] -= beta;
  modify_diag(a, b, start, m);
  modify_diag(a, b, start + m, size - m);
}

// --------------------------------------------------------------- kernels
__global__ void k_diag_one(double* Q, int64_t ld, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Q[i + i * ld] = 1.0;
}

// The row of a merged block's Q that its parent's z takes (the last row for a
// left child, the first for a right one), formed from the same operands as
// the block's product: row r of diag(Q1, Q2) V is row r of the child block
// that holds r times that block's rows of V.  One item is up to ZC columns of
// one merge; the row segment is staged in LDS in chunks of ZCH, and wave w
// takes columns w, w + 4, ... with its lanes along the segment.
struct ZItem {
  int64_t q;    // Q-buffer offset of the segment's first element: r + kbeg ldq
  int64_t v;    // offset in the merges' V of element (kbeg - start, c0) of this merge's V
  int32_t len;  // segment length (rows of the child block holding r)
  int32_t ldv;  // leading dimension of this merge's V (its size)
  int32_t z0;   // output index of column c0 (start + c0)
  int32_t nc;   // columns of the item, <= ZC
};
constexpr int ZC = 16, ZT = 256, ZCH = 2048;

__global__ void __launch_bounds__(ZT) k_zrows(const ZItem* __restrict__ items, const double* __restrict__ Q,
                                              int64_t ldq, const double* __restrict__ V, double* __restrict__ z) {
  __shared__ double row[ZCH];
  const ZItem it = items[blockIdx.x];
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  constexpr int PW = ZC / (ZT / 64);  // columns per wave
  double acc[PW];
#pragma unroll
  for (int c = 0; c < PW; ++c) acc[c] = 0.0;
  for (int k0 = 0; k0 < it.len; k0 += ZCH) {
    const int kn = min(ZCH, it.len - k0);
    __syncthreads();  // the previous chunk is consumed
    for (int k = threadIdx.x; k < kn; k += ZT) row[k] = Q[it.q + (int64_t)(k0 + k) * ldq];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < PW; ++c) {
      const int col = wv + (ZT / 64) * c;
      if (col < it.nc) {
        const double* vc = V + it.v + (int64_t)col * it.ldv + k0;
        double a = acc[c];
        for (int k = lane; k < kn; k += 64) a = __builtin_fma(row[k], vc[k], a);
        acc[c] = a;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < PW; ++c) {
    double a = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
    const int col = wv + (ZT / 64) * c;
    if (lane == 0 && col < it.nc) z[it.z0 + col] = a;
  }
}

struct ANode {
  int64_t start, size, voff;
};

// Arrays indexed by the merged block's global row/column start + local index.
struct TArgs {
  const double* d;  // the merge's poles (its children's eigenvalues), unsorted
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
  double* V;  // merge p's size x size V at voff (ld = size)
};

__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

constexpr int TA_T = 256, TA_R = 4, TA_CB = 16;

// One block = (merge, 16 columns, 1024 rows), as the front end's assembly.
__global__ void __launch_bounds__(TA_T) k_tri_assemble(const ANode* __restrict__ nodes, const int4* __restrict__ tab,
                                                       TArgs a) {
  __shared__ int s_kind[TA_CB], s_idx[TA_CB], s_t[TA_CB];
  __shared__ double s_sig[TA_CB], s_mu[TA_CB], s_ic[TA_CB], s_ub[TA_CB];
  const int4 e = tab[blockIdx.x];
  const ANode nd = nodes[e.x];
  const int64_t n = nd.size, o = nd.start;
  const int64_t c0 = (int64_t)e.y * TA_CB;
  const int64_t r0 = (int64_t)e.z * (TA_T * TA_R);
  const int nc = (int)min((int64_t)TA_CB, n - c0);
  if (threadIdx.x < nc) {
    const int64_t c = o + c0 + threadIdx.x;
    s_kind[threadIdx.x] = a.ckind[c];
    s_idx[threadIdx.x] = a.cidx[c];
    s_t[threadIdx.x] = a.ct[c];
    s_sig[threadIdx.x] = a.csig[c];
    s_mu[threadIdx.x] = a.cmu[c];
    s_ic[threadIdx.x] = a.cic[c];
    s_ub[threadIdx.x] = a.cub[c];
  }
  double di[TA_R], zi[TA_R], ui[TA_R];
  int gi[TA_R], pi[TA_R];
#pragma unroll
  for (int j = 0; j < TA_R; ++j) {
    const int64_t i = r0 + threadIdx.x + j * TA_T;
    const bool ok = i < n;
    di[j] = ok ? a.d[o + i] : 0.0;
    zi[j] = ok ? a.z[o + i] : 0.0;
    ui[j] = ok ? a.ru[o + i] : 0.0;
    gi[j] = ok ? a.rgrp[o + i] : -1;
    pi[j] = ok ? a.rpos[o + i] : -1;
  }
  __syncthreads();
  double* V = a.V + nd.voff;
  for (int cc = 0; cc < nc; ++cc) {
    const int kind = s_kind[cc];
    double v[TA_R];
    if (kind == COL_REDUCED) {
      const double m = s_mu[cc], sg = s_sig[cc], ic = s_ic[cc];
#pragma unroll
      for (int j = 0; j < TA_R; ++j) {
        const double den = (di[j] - sg) - m;
        const double rc = rcp_nr(den);
        double q = ic * rc;
        q = __builtin_fma(__builtin_fma(-q, den, ic), rc, q);
        v[j] = zi[j] != 0.0 ? zi[j] * q : 0.0;
      }
    } else if (kind == COL_UNIT) {
      const int64_t at = s_idx[cc];
#pragma unroll
      for (int j = 0; j < TA_R; ++j) v[j] = (r0 + threadIdx.x + j * TA_T == at) ? 1.0 : 0.0;
    } else {
      const int g = s_idx[cc], t = s_t[cc];
      const double ub = s_ub[cc];
#pragma unroll
      for (int j = 0; j < TA_R; ++j) v[j] = gi[j] == g ? (pi[j] == t ? 1.0 : 0.0) - ub * ui[j] : 0.0;
    }
    double* col = V + (c0 + cc) * n + r0 + threadIdx.x;
#pragma unroll
    for (int j = 0; j < TA_R; ++j)
      if (r0 + threadIdx.x + j * TA_T < n) col[j * TA_T] = v[j];
  }
}

// C (M x N, ldc) = A (M x K, lda) B (K x N, ldb), column-major, FP64.
struct GDesc {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int32_t M, N, K, pad;
};

constexpr int GT = 128, GKS = 16, GNT = 512, GPAD = 2;
typedef double dbl4 __attribute__((ext_vector_type(4)));

// One 512-thread block (8 waves) per 128 x 128 tile of C (tile table entry:
// descriptor, tile row, tile column), on FP64 matrix cores
// (v_mfma_f64_16x16x4f64).  Wave w owns rows 64 (w & 1) .. +63 and columns
// 32 (w >> 1) .. +31 of the tile: 4 x 2 blocks of 16 x 16.  K advances in
// steps of 16 through two LDS buffers; the next step's operands are loaded
// into registers while the current one is multiplied.  Lane layout of the
// 16x16x4 instruction: A(row = lane % 16, k = lane / 16), B(k = lane / 16,
// col = lane % 16); accumulator element q of a lane is row lane / 16 + 4 q,
// column lane % 16 of its block.
// Two blocks per CU (66.5 KB of LDS each) are 4 waves per SIMD: the bound keeps
// the kernel within the 128 VGPRs a lane that this leaves.
__global__ void __launch_bounds__(GNT, 4) k_dgemm(const GDesc* __restrict__ desc, const int4* __restrict__ tiles) {
  __shared__ double As[2][GKS][GT + GPAD];
  __shared__ double Bs[2][GKS][GT + GPAD];
  const int4 t = tiles[blockIdx.x];
  const GDesc g = desc[t.x];
  const int r0 = t.y * GT, c0 = t.z * GT;
  const int tid = threadIdx.x;
  const int wv = tid / 64, lane = tid % 64;
  const int wm = (wv & 1) * 64, wn = (wv >> 1) * 32;
  dbl4 acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = (dbl4){0.0, 0.0, 0.0, 0.0};
  constexpr int PER = GT * GKS / GNT;  // 4 elements of each operand per thread
  static_assert(GNT % GT == 0 && GNT % GKS == 0, "tile shape");
  // Element e2 of a thread: A(m, k) with m = tid % GT, k = tid / GT + (GNT / GT) e2
  // (consecutive threads along m); B(k, c) with k = tid % GKS, c = tid / GKS +
  // (GNT / GKS) e2 (consecutive threads along k).  The per-thread part of each
  // address is formed once; what changes with k0 and e2 is uniform.
  const int ma = tid % GT, ka = tid / GT, kb = tid % GKS, cb = tid / GKS;
  const double* pA = g.A + (r0 + ma) + (int64_t)ka * g.lda;
  const double* pB = g.B + kb + (int64_t)(c0 + cb) * g.ldb;
  const bool rowA = r0 + ma < g.M;
  double ra[PER], rb[PER];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e2 = 0; e2 < PER; ++e2) {
      const int gka = k0 + ka + (GNT / GT) * e2;
      ra[e2] = (rowA && gka < g.K) ? pA[(int64_t)(k0 + (GNT / GT) * e2) * g.lda] : 0.0;
      const int gkb = k0 + kb, gc = c0 + cb + (GNT / GKS) * e2;
      rb[e2] = (gkb < g.K && gc < g.N) ? pB[k0 + (int64_t)((GNT / GKS) * e2) * g.ldb] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int e2 = 0; e2 < PER; ++e2) {
      const int e = tid + e2 * GNT;
      As[buf][e / GT][e % GT] = ra[e2];
      Bs[buf][e % GKS][e / GKS] = rb[e2];
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < g.K; k0 += GKS) {
    const bool more = k0 + GKS < g.K;
    if (more) gload(k0 + GKS);
#pragma unroll
    for (int ks = 0; ks < GKS; ks += 4) {
      const int r = lane % 16, q = lane / 16;
      double af[4], bf[2];
#pragma unroll
      for (int x = 0; x < 4; ++x) af[x] = As[buf][ks + q][wm + 16 * x + r];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = Bs[buf][ks + q][wn + 16 * y + r];
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    if (more) {
      sstore(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int gc = c0 + wn + 16 * y + lane % 16;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gr = r0 + wm + 16 * x + lane / 16 + 4 * q;
        if (gr < g.M && gc < g.N) g.C[gr + (int64_t)gc * g.ldc] = acc[x][y][q];
      }
    }
}

// ------------------------------------------------------------ workspace
static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct TLayout {
  size_t Qw, Vw, rd, rz, lamr, mur, xnr, sidx, infop, rhop, offsp, zl, dl, rgrp, rpos, ru, ckind, cidx, ct,
      csig, cmu, cic, cub, anodes, atab, gdesc, gtab, zit, solver, total;
  int64_t maxV, maxAsm, maxTiles, maxNodes, maxZ;
  size_t solver_bytes;
};

static TLayout tlayout(int64_t n, const std::vector<Node>& nodes, int maxd) {
  TLayout L;
  L.maxV = 0;
  L.maxAsm = 0;
  L.maxTiles = 0;
  L.maxNodes = 0;
  L.maxZ = 0;
  L.solver_bytes = 0;
  std::vector<int64_t> offs;
  for (int D = maxd; D >= 0; --D) {
    int64_t v = 0, as = 0, ti = 0, cnt = 0, zi = 0;
    offs.assign(1, 0);
    for (const Node& nd : nodes) {
      if (nd.depth != D) continue;
      ++cnt;
      v += nd.size * nd.size;
      as += cdiv(nd.size, TA_CB) * cdiv(nd.size, TA_T * TA_R);
      ti += (cdiv(nd.m, GT) + cdiv(nd.size - nd.m, GT)) * cdiv(nd.size, GT);
      if (nd.side) zi += cdiv(nd.size, ZC);
      offs.push_back(offs.back() + nd.size);
    }
    if (!cnt) continue;
    L.maxV = std::max(L.maxV, v);
    L.maxAsm = std::max(L.maxAsm, as);
    L.maxTiles = std::max(L.maxTiles, ti);
    L.maxNodes = std::max(L.maxNodes, cnt);
    L.maxZ = std::max(L.maxZ, zi);
    // the reduced problems of a depth are no more and no larger than its merges
    L.solver_bytes = std::max(L.solver_bytes, dpr1_batched_workspace_size(cnt, offs.data()));
  }
  const int64_t P = std::max<int64_t>(L.maxNodes, 1);
  size_t o = 0;
  L.Qw = o; o = al(o + 8 * (size_t)n * n);
  L.Vw = o; o = al(o + 8 * (size_t)L.maxV);
  L.rd = o; o = al(o + 8 * n);
  L.rz = o; o = al(o + 8 * n);
  L.lamr = o; o = al(o + 8 * n);
  L.mur = o; o = al(o + 8 * n);
  L.xnr = o; o = al(o + 8 * n);
  L.sidx = o; o = al(o + 4 * n);
  L.infop = o; o = al(o + 4 * P);
  L.rhop = o; o = al(o + 8 * P);
  L.offsp = o; o = al(o + 8 * (P + 1));
  L.zl = o; o = al(o + 8 * n);
  L.dl = o; o = al(o + 8 * n);
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
  L.anodes = o; o = al(o + sizeof(ANode) * P);
  L.atab = o; o = al(o + sizeof(int4) * std::max<int64_t>(L.maxAsm, 1));
  L.gdesc = o; o = al(o + sizeof(GDesc) * 2 * P);
  L.gtab = o; o = al(o + sizeof(int4) * std::max<int64_t>(L.maxTiles, 1));
  L.zit = o; o = al(o + sizeof(ZItem) * std::max<int64_t>(L.maxZ, 1));
  L.solver = o; o = al(o + L.solver_bytes);
  L.total = o;
  return L;
}

}  // namespace tri
}  // namespace dpr1

using namespace dpr1::tri;
namespace fe = dpr1::fe;

#define TCHECK(x)                            \
  do {                                       \
    if ((x) != hipSuccess) return DPR1_EHIP; \
  } while (0)

static int tri_set_info(int32_t* info, int32_t code, hipStream_t st) {
  TCHECK(hipMemcpyAsync(info, &code, 4, hipMemcpyHostToDevice, st));
  TCHECK(hipStreamSynchronize(st));
  return DPR1_OK;
}

// Second stream of the current device for the merges' DPR1 solves: created
// once per device (default priority, non-blocking) and kept until the
// process ends; nullptr if it cannot be created.
constexpr int TRI_MAX_DEVICES = 64;
static std::mutex tri_mutex;
static hipStream_t tri_streams[TRI_MAX_DEVICES];
static hipStream_t tri_aux_stream() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= TRI_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(tri_mutex);
  if (!tri_streams[dev]) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    tri_streams[dev] = s;
  }
  return tri_streams[dev];
}

// On every return: wait for both streams (the host buffers that their copies
// use are freed after this) and release the event.
struct TriDone {
  hipStream_t st, st2;
  hipEvent_t ev = nullptr;
  ~TriDone() {
    (void)hipStreamSynchronize(st2);
    (void)hipStreamSynchronize(st);
    if (ev) (void)hipEventDestroy(ev);
  }
};

extern "C" {

size_t dpr1_tridiag_workspace_size(int64_t n) {
  if (n < 1 || n > 65536) return 0;
  std::vector<Node> nodes;
  int maxd = 0;
  build_tree(0, n, 0, nodes, maxd);
  return tlayout(n, nodes, maxd).total;
}

int dpr1_tridiag_eig(const double* a, const double* b, int64_t n, double* lambda, double* Q, int64_t ldq,
                     int32_t* info, const dpr1_opts* opts, void* work, size_t work_bytes, void* stream) {
  if (!a) return -1;
  if (!b && n > 1) return -2;
  if (n < 1 || n > 65536) return -3;
  if (!lambda) return -4;
  if (!Q) return -5;
  if (ldq < n) return -6;
  if (!info) return -7;
  if (opts && opts->waves_per_simd != 0 && opts->waves_per_simd != 4 && opts->waves_per_simd != 6 &&
      opts->waves_per_simd != 8)
    return -8;
  if (!work) return -9;
  std::vector<Node> nodes;
  int maxd = 0;
  build_tree(0, n, 0, nodes, maxd);
  const TLayout L = tlayout(n, nodes, maxd);
  if (work_bytes < L.total) return -10;
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)work;

  std::vector<double> ha(n), hb(std::max<int64_t>(n - 1, 0));
  TCHECK(hipMemcpyAsync(ha.data(), a, 8 * n, hipMemcpyDeviceToHost, st));
  if (n > 1) TCHECK(hipMemcpyAsync(hb.data(), b, 8 * (n - 1), hipMemcpyDeviceToHost, st));
  TCHECK(hipStreamSynchronize(st));
  for (double x : ha)
    if (!std::isfinite(x)) return tri_set_info(info, DPR1_INFO_NONFINITE, st);
  for (double x : hb)
    if (!std::isfinite(x)) return tri_set_info(info, DPR1_INFO_NONFINITE, st);

  // leaves: the diagonal after every split's modification, Q = 1 in both buffers
  std::vector<double> hlam = ha;
  modify_diag(hlam, hb, 0, n);
  TCHECK(hipMemcpyAsync(lambda, hlam.data(), 8 * n, hipMemcpyHostToDevice, st));
  double* Qw = (double*)(w + L.Qw);
  const unsigned g1 = (unsigned)cdiv(n, 256);
  hipLaunchKernelGGL(k_diag_one, dim3(g1), dim3(256), 0, st, Q, ldq, n);
  hipLaunchKernelGGL(k_diag_one, dim3(g1), dim3(256), 0, st, Qw, n, n);
  TCHECK(hipGetLastError());

  double* zl = (double*)(w + L.zl);
  double* dl = (double*)(w + L.dl);
  TArgs ta;
  ta.d = dl;
  ta.z = zl;
  ta.rgrp = (int32_t*)(w + L.rgrp);
  ta.rpos = (int32_t*)(w + L.rpos);
  ta.ru = (double*)(w + L.ru);
  ta.ckind = (int32_t*)(w + L.ckind);
  ta.cidx = (int32_t*)(w + L.cidx);
  ta.ct = (int32_t*)(w + L.ct);
  ta.csig = (double*)(w + L.csig);
  ta.cmu = (double*)(w + L.cmu);
  ta.cic = (double*)(w + L.cic);
  ta.cub = (double*)(w + L.cub);
  ta.V = (double*)(w + L.Vw);

  // host staging, reused by every depth: each buffer is rewritten only after
  // the copies that use it have finished (the event waited for at the start of
  // a depth follows the previous depth's copies on the caller's stream; the
  // second stream is synchronised after each depth's solves)
  std::vector<int32_t> hgrp(n, 0), hpos(n, 0), hkind(n, 0), hidx(n, 0), hct(n, 0);
  std::vector<double> hz(n), hzr(n, 0.0), hru(n, 0.0), hsig(n, 0.0), hmu(n, 0.0), hic(n, 0.0), hub(n, 0.0);
  std::vector<ZItem> zit;
  std::vector<double> rd, rz, lamr, mur, xnr, rhop;
  std::vector<int32_t> sidx, infop;
  std::vector<int64_t> offs;
  std::vector<ANode> anodes;
  std::vector<int4> atab, gtab;
  std::vector<GDesc> gdesc;
  std::vector<fe::Col> all;
  std::vector<int64_t> roff, rcnt;  // per merge: offset and size of its reduced problem
  std::vector<std::vector<fe::Col>> mcols;
  std::vector<double> hnew(n), hpole(n), gval(n);
  std::vector<char> seen(n);
  fe::Scratch scr;
  dpr1_plan plan;
  // host mirrors of contiguous workspace regions, so that each region moves
  // in one copy per depth: the solver's inputs [rd, offsp], its outputs
  // [lamr, infop], and the merges' z and poles with the assembly, GEMM and
  // z-row arrays [zl, zit]
  const int64_t P = std::max<int64_t>(L.maxNodes, 1);
  std::vector<char> mirA(L.offsp + 8 * (P + 1) - L.rd), mirB(L.infop + 4 * P - L.lamr), mirC(L.solver - L.zl);
  auto put = [](std::vector<char>& mir, size_t base, size_t off, const void* src, size_t bytes) {
    if (bytes) memcpy(mir.data() + (off - base), src, bytes);
  };
  hipStream_t st2 = tri_aux_stream();
  if (!st2) return DPR1_EHIP;
  TriDone fin{st, st2};
  TCHECK(hipEventCreateWithFlags(&fin.ev, hipEventDisableTiming));
  bool zpending = false;  // rows of this depth's z in flight to hzr (event fin.ev)

  for (int D = maxd; D >= 0; --D) {
    std::vector<const Node*> lv;
    for (const Node& nd : nodes)
      if (nd.depth == D) lv.push_back(&nd);
    if (lv.empty()) continue;
    // buffers: the root (D = 0) writes the caller's Q
    double* Qn = (D % 2 == 0) ? Q : Qw;
    const int64_t ldn = (D % 2 == 0) ? ldq : n;
    double* Qc = (D % 2 == 0) ? Qw : Q;
    const int64_t ldc = (D % 2 == 0) ? n : ldq;

    // 1. z of every merge: the rows k_zrows formed for its merged children
    // (copied to hzr), 1 for a 1 x 1 child; 0 outside this depth's merges
    if (zpending) {
      TCHECK(hipEventSynchronize(fin.ev));
      zpending = false;
    }
    std::fill(hz.begin(), hz.end(), 0.0);
    for (const Node* nd : lv) {
      const int64_t o = nd->start, m = nd->m, s2 = nd->size - nd->m;
      if (m == 1) hz[o] = 1.0; else std::copy(hzr.begin() + o, hzr.begin() + o + m, hz.begin() + o);
      if (s2 == 1) hz[o + m] = 1.0; else std::copy(hzr.begin() + o + m, hzr.begin() + o + m + s2, hz.begin() + o + m);
    }

    // 2. reduce each merge (hlam holds the current eigenvalues of every block)
    rd.clear();
    rz.clear();
    rhop.clear();
    offs.assign(1, 0);
    roff.assign(lv.size(), 0);
    rcnt.assign(lv.size(), 0);
    mcols.resize(lv.size());
    for (size_t p = 0; p < lv.size(); ++p) {
      const Node& nd = *lv[p];
      const double beta = hb[nd.start + nd.m - 1];
      const size_t before = rd.size();
      // a component below 2^-300 of the largest is taken as 0: it lies far
      // below the absolute accuracy of the children's eigenvectors it comes
      // from, and kept it would put an eigenvalue within ~beta z_j^2 (below
      // 1e-180) of its pole, where binary64 loses the shifted representation
      // Also a component whose share of the rank-one term is negligible,
      // |beta z_j| <= 2 eps max|d| (zeroing it changes T by at most
      // 2 sqrt(2) |beta z_j|, within the children's accuracy), as divide and
      // conquer codes deflate.
      double zmax = 0.0, dm = 0.0;
      for (int64_t i = nd.start; i < nd.start + nd.size; ++i) {
        zmax = std::max(zmax, std::fabs(hz[i]));
        dm = std::max(dm, std::fabs(hlam[i]));
      }
      const double ztiny = std::max(std::ldexp(zmax, -300), 2.0 * 0x1p-52 * dm / std::fabs(beta));
      for (int64_t i = nd.start; i < nd.start + nd.size; ++i)
        if (std::fabs(hz[i]) < ztiny) hz[i] = 0.0;
      mcols[p].clear();
      // poles within 8 eps max|d| of each other are merged like equal ones (the
      // perturbation is within the accuracy of the children's eigenvalues);
      // each member then takes its group's pole, in hpole for the assembly
      double dmax = 0.0;
      for (int64_t i = nd.start; i < nd.start + nd.size; ++i) dmax = std::max(dmax, std::fabs(hlam[i]));
      const double ptol = 8.0 * 0x1p-52 * dmax;
      // a coupling |beta| <= 8 eps max|d| decouples the halves (the matrix
      // changes by less than the children's accuracy)
      const bool decoupled = std::fabs(beta) <= ptol;
      // the children's eigenvalues are each decreasing: their order is one merge
      fe::reduce(hlam.data() + nd.start, hz.data() + nd.start, nd.size, decoupled, rd, rz,
                 hgrp.data() + nd.start, hpos.data() + nd.start, hru.data() + nd.start, mcols[p], ptol, nd.m,
                 &scr);
      {
        std::fill(seen.begin(), seen.begin() + nd.size, 0);
        for (int64_t i = 0; i < nd.size; ++i) {
          const int g = hgrp[nd.start + i];
          if (!seen[g] || hlam[nd.start + i] > gval[g]) gval[g] = hlam[nd.start + i];
          seen[g] = 1;
        }
        for (int64_t i = 0; i < nd.size; ++i) hpole[nd.start + i] = gval[hgrp[nd.start + i]];
      }
      roff[p] = (int64_t)before;
      rcnt[p] = (int64_t)(rd.size() - before);
      if (rcnt[p] > 0) {
        offs.push_back(offs.back() + rcnt[p]);
        rhop.push_back(beta);
      }
    }
    const int64_t nprob = (int64_t)rhop.size();
    const int64_t mtot = (int64_t)rd.size();

    // 3. one batched solve of the reduced problems
    lamr.resize(mtot);
    mur.resize(mtot);
    xnr.resize(mtot);
    sidx.resize(mtot);
    if (nprob > 0) {
      infop.assign(nprob, 0);
      const int prc = dpr1_batched_plan(nprob, offs.data(), opts, &plan, w + L.solver, L.solver_bytes, (void*)st2);
      if (prc != DPR1_OK) return prc == DPR1_EHIP ? DPR1_EHIP : -10;
      double* drd = (double*)(w + L.rd);
      double* drz = (double*)(w + L.rz);
      double* dlr = (double*)(w + L.lamr);
      double* dmu = (double*)(w + L.mur);
      double* dxn = (double*)(w + L.xnr);
      int32_t* dsi = (int32_t*)(w + L.sidx);
      int32_t* dinf = (int32_t*)(w + L.infop);
      double* drho = (double*)(w + L.rhop);
      int64_t* doffs = (int64_t*)(w + L.offsp);
      put(mirA, L.rd, L.rd, rd.data(), 8 * mtot);
      put(mirA, L.rd, L.rz, rz.data(), 8 * mtot);
      put(mirA, L.rd, L.rhop, rhop.data(), 8 * nprob);
      put(mirA, L.rd, L.offsp, offs.data(), 8 * (nprob + 1));
      TCHECK(hipMemcpyAsync(w + L.rd, mirA.data(), L.offsp + 8 * (nprob + 1) - L.rd, hipMemcpyHostToDevice, st2));
      const int rc = dpr1_eig_batched(&plan, doffs, drd, drz, drho, dlr, nullptr, nullptr, dsi, dmu, dxn, dinf,
                                      nullptr, w + L.solver, L.solver_bytes, (void*)st2);
      if (rc != DPR1_OK) return rc;
      TCHECK(hipMemcpyAsync(mirB.data(), w + L.lamr, mirB.size(), hipMemcpyDeviceToHost, st2));
      TCHECK(hipStreamSynchronize(st2));
      memcpy(lamr.data(), mirB.data() + (L.lamr - L.lamr), 8 * mtot);
      memcpy(mur.data(), mirB.data() + (L.mur - L.lamr), 8 * mtot);
      memcpy(xnr.data(), mirB.data() + (L.xnr - L.lamr), 8 * mtot);
      memcpy(sidx.data(), mirB.data() + (L.sidx - L.lamr), 4 * mtot);
      memcpy(infop.data(), mirB.data() + (L.infop - L.lamr), 4 * nprob);
      for (int32_t x : infop)
        if (x != DPR1_INFO_OK) return tri_set_info(info, x, st);
    }

    // 4. columns of every merge, the new eigenvalues, the assembly and GEMM tables
    put(mirC, L.zl, L.zl, hz.data(), 8 * n);     // z as reduced
    put(mirC, L.zl, L.dl, hpole.data(), 8 * n);  // the merges' poles (grouped)
    anodes.clear();
    atab.clear();
    gdesc.clear();
    gtab.clear();
    zit.clear();
    int64_t voff = 0;
    hnew = hlam;
    for (size_t p = 0; p < lv.size(); ++p) {
      const Node& nd = *lv[p];
      const int64_t o = nd.start, s = nd.size;
      fe::merge_cols(mcols[p], lamr.data() + roff[p], rcnt[p], all, &scr);
      for (int64_t c = 0; c < s; ++c) {
        const fe::Col& q = all[c];
        hnew[o + c] = q.val;
        hkind[o + c] = q.kind;
        hidx[o + c] = q.idx;
        hct[o + c] = q.t;
        hub[o + c] = q.ub;
        hsig[o + c] = hmu[o + c] = hic[o + c] = 0.0;
        if (q.kind == COL_REDUCED) {
          const int64_t k = roff[p] + q.idx;
          hsig[o + c] = rd[roff[p] + sidx[k]];
          hmu[o + c] = mur[k];
          hic[o + c] = 1.0 / xnr[k];
        }
      }
      const int32_t q = (int32_t)anodes.size();
      anodes.push_back({o, s, voff});
      for (int32_t cg = 0; cg < (int32_t)cdiv(s, TA_CB); ++cg)
        for (int32_t rc = 0; rc < (int32_t)cdiv(s, TA_T * TA_R); ++rc) atab.push_back({q, cg, rc, 0});
      const double* Vp = ta.V + voff;
      // rows of the left child: Q1 (m x m) times V's first m rows
      GDesc g1d = {Qc + o + o * ldc, Vp, Qn + o + o * ldn, ldc, s, ldn, (int32_t)nd.m, (int32_t)s,
                   (int32_t)nd.m, 0};
      // rows of the right child: Q2 ((s-m) x (s-m)) times V's last s - m rows
      const int64_t o2 = o + nd.m;
      GDesc g2d = {Qc + o2 + o2 * ldc, Vp + nd.m, Qn + o2 + o * ldn, ldc, s, ldn, (int32_t)(s - nd.m), (int32_t)s,
                   (int32_t)(s - nd.m), 0};
      const int32_t d1 = (int32_t)gdesc.size();
      gdesc.push_back(g1d);
      gdesc.push_back(g2d);
      for (int32_t tr = 0; tr < (int32_t)cdiv(nd.m, GT); ++tr)
        for (int32_t tc = 0; tc < (int32_t)cdiv(s, GT); ++tc) gtab.push_back({d1, tr, tc, 0});
      for (int32_t tr = 0; tr < (int32_t)cdiv(s - nd.m, GT); ++tr)
        for (int32_t tc = 0; tc < (int32_t)cdiv(s, GT); ++tc) gtab.push_back({d1 + 1, tr, tc, 0});
      // the row of this block's Q that the parent's z takes: the last (left
      // child, in the Q2 block) or the first (right child, in the Q1 block)
      if (nd.side) {
        const int64_t r = nd.side == 1 ? o + s - 1 : o;
        const int64_t kbeg = nd.side == 1 ? o2 : o, len = nd.side == 1 ? s - nd.m : nd.m;
        for (int64_t c0 = 0; c0 < s; c0 += ZC)
          zit.push_back({r + kbeg * ldc, voff + (kbeg - o) + c0 * s, (int32_t)len, (int32_t)s, (int32_t)(o + c0),
                         (int32_t)std::min<int64_t>(ZC, s - c0)});
      }
      voff += s * s;
    }
    if (voff > L.maxV || (int64_t)atab.size() > L.maxAsm || (int64_t)gtab.size() > L.maxTiles ||
        (int64_t)zit.size() > L.maxZ)
      return -10;
    hlam.swap(hnew);
    put(mirC, L.zl, L.rgrp, hgrp.data(), 4 * n);
    put(mirC, L.zl, L.rpos, hpos.data(), 4 * n);
    put(mirC, L.zl, L.ru, hru.data(), 8 * n);
    put(mirC, L.zl, L.ckind, hkind.data(), 4 * n);
    put(mirC, L.zl, L.cidx, hidx.data(), 4 * n);
    put(mirC, L.zl, L.ct, hct.data(), 4 * n);
    put(mirC, L.zl, L.csig, hsig.data(), 8 * n);
    put(mirC, L.zl, L.cmu, hmu.data(), 8 * n);
    put(mirC, L.zl, L.cic, hic.data(), 8 * n);
    put(mirC, L.zl, L.cub, hub.data(), 8 * n);
    put(mirC, L.zl, L.anodes, anodes.data(), sizeof(ANode) * anodes.size());
    put(mirC, L.zl, L.atab, atab.data(), sizeof(int4) * atab.size());
    put(mirC, L.zl, L.gdesc, gdesc.data(), sizeof(GDesc) * gdesc.size());
    put(mirC, L.zl, L.gtab, gtab.data(), sizeof(int4) * gtab.size());
    put(mirC, L.zl, L.zit, zit.data(), sizeof(ZItem) * zit.size());
    TCHECK(hipMemcpyAsync(w + L.zl, mirC.data(),
                          (zit.empty() ? L.gtab + sizeof(int4) * gtab.size() : L.zit + sizeof(ZItem) * zit.size()) -
                              L.zl,
                          hipMemcpyHostToDevice, st));
    ANode* danodes = (ANode*)(w + L.anodes);
    int4* datab = (int4*)(w + L.atab);
    GDesc* dgdesc = (GDesc*)(w + L.gdesc);
    int4* dgtab = (int4*)(w + L.gtab);
    hipLaunchKernelGGL(k_tri_assemble, dim3((unsigned)atab.size()), dim3(TA_T), 0, st, danodes, datab, ta);
    TCHECK(hipGetLastError());
    // the parents' z rows (after the assembly, which reads this depth's z
    // from the same buffer), on the host before the product below ends
    if (!zit.empty()) {
      hipLaunchKernelGGL(k_zrows, dim3((unsigned)zit.size()), dim3(ZT), 0, st, (const ZItem*)(w + L.zit), Qc, ldc,
                         (const double*)ta.V, zl);
      TCHECK(hipGetLastError());
      TCHECK(hipMemcpyAsync(hzr.data(), zl, 8 * n, hipMemcpyDeviceToHost, st));
      TCHECK(hipEventRecord(fin.ev, st));
      zpending = true;
    }
    // 5. Q = diag(Q1, Q2) V for every merge
    hipLaunchKernelGGL(k_dgemm, dim3((unsigned)gtab.size()), dim3(GNT), 0, st, dgdesc, dgtab);
    TCHECK(hipGetLastError());
  }
  // the eigenvalues once, after the root merge (no kernel reads them)
  if (!nodes.empty()) TCHECK(hipMemcpyAsync(lambda, hlam.data(), 8 * n, hipMemcpyHostToDevice, st));
  // tri_set_info waits for the stream: the host staging above must outlive
  // its copies
  return tri_set_info(info, DPR1_INFO_OK, st);
}

}  // extern "C"
