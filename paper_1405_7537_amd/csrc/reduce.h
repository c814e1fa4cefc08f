// Host side of the reduction of Sec. 1 for one DPR1 problem: sort the poles
// decreasingly, deflate a pole whose z_j is zero, merge each group of equal
// poles by one Householder reflection (the reduced problem keeps the pole
// once, with z = ||w||).  Used by the front end (dpr1_general.hip) and by the
// divide-and-conquer driver (dpr1_tridiag.hip), one problem at a time.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace dpr1 {
namespace fe {

enum : int32_t { COL_REDUCED = 0, COL_UNIT = 1, COL_REFLECT = 2 };

// One eigenvector column of the reduced-and-deflated problem:
//   COL_REDUCED  idx = eigenpair k of the reduced problem
//   COL_UNIT     idx = row of the unit vector (a deflated pole)
//   COL_REFLECT  idx = group id, t = column t of the group's reflection,
//                ub = beta u_t
struct Col {
  double val;
  int32_t kind, idx, t;
  double ub;
};

// Stable sort of the poles in decreasing order: order[s] = the row with the
// s-th largest d (equal values keep their row order, -0 and +0 are equal).
// LSD radix sort on order-preserving 64-bit keys, 11 bits a pass (a pass
// whose digit is the same for every key is skipped); insertion sort up to 256.
inline void sort_decreasing(const double* d, int64_t n, std::vector<int64_t>& order) {
  if (n <= 256) {
    // small problems (the many merges near the leaves of a divide and
    // conquer): an insertion sort, stable, with -0 = +0 by value comparison
    order.resize(n);
    for (int64_t j = 0; j < n; ++j) {
      int64_t t = j;
      while (t > 0 && d[order[t - 1]] < d[j]) {
        order[t] = order[t - 1];
        --t;
      }
      order[t] = j;
    }
    return;
  }
  std::vector<uint64_t> k(n), k2(n);
  std::vector<int64_t> o2(n);
  order.resize(n);
  for (int64_t j = 0; j < n; ++j) {
    const double x = d[j] == 0.0 ? 0.0 : d[j];
    uint64_t b;
    memcpy(&b, &x, 8);
    b = (b >> 63) ? ~b : (b | (uint64_t(1) << 63));  // increasing with x
    k[j] = ~b;                                        // decreasing with x
    order[j] = j;
  }
  if (n < 2) return;
  std::vector<int64_t> cnt(2048);
  for (int sh = 0; sh < 64; sh += 11) {
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int64_t j = 0; j < n; ++j) ++cnt[(k[j] >> sh) & 2047];
    if (cnt[(k[0] >> sh) & 2047] == n) continue;
    int64_t acc = 0;
    for (int b = 0; b < 2048; ++b) {
      const int64_t c = cnt[b];
      cnt[b] = acc;
      acc += c;
    }
    for (int64_t j = 0; j < n; ++j) {
      const int64_t at = cnt[(k[j] >> sh) & 2047]++;
      k2[at] = k[j];
      o2[at] = order[j];
    }
    k.swap(k2);
    order.swap(o2);
  }
}

// The same order when d[0 .. m) and d[m .. n) are each non-increasing (the
// children's eigenvalues in a divide-and-conquer merge): one stable merge,
// the first run first among equal values, as the stable sort orders them.
inline void merge_decreasing(const double* d, int64_t n, int64_t m, std::vector<int64_t>& order) {
  order.resize(n);
  int64_t a = 0, b = m, s = 0;
  while (a < m && b < n) order[s++] = (d[b] > d[a]) ? b++ : a++;
  while (a < m) order[s++] = a++;
  while (b < n) order[s++] = b++;
}

// Work buffers of reduce and merge_cols, kept by a caller that reduces many
// problems so that they are allocated once.
struct Scratch {
  std::vector<int64_t> order;
  std::vector<double> u;
  std::vector<Col> red;
};

// Reduce one problem (host d, z of length n; zero_all treats every z_j as 0;
// poles within tol of a group's largest are merged into that group; runs >= 0:
// d[0 .. runs) and d[runs .. n) are each non-increasing).
// Appends the reduced poles and z to rd, rz (decreasing poles, no zero z);
// writes per row i: rgrp[i] group id (local), rpos[i] position in the group,
// ru[i] reflection component (0 for groups without one); appends the
// deflated and reflected columns to cols in decreasing pole order.
inline void reduce(const double* hd, const double* hz, int64_t n, bool zero_all, std::vector<double>& rd,
                   std::vector<double>& rz, int32_t* rgrp, int32_t* rpos, double* ru, std::vector<Col>& cols,
                   double tol = 0.0, int64_t runs = -1, Scratch* scratch = nullptr) {
  Scratch local;
  Scratch& sc = scratch ? *scratch : local;
  std::vector<int64_t>& order = sc.order;
  if (runs >= 0)
    merge_decreasing(hd, n, runs, order);
  else
    sort_decreasing(hd, n, order);
  std::vector<double>& u = sc.u;
  int32_t ngrp = 0;
  for (int64_t s = 0; s < n;) {
    int64_t e = s + 1;
    // tol = 0: equal poles only (Sec. 1); tol > 0 (divide and conquer): poles
    // within tol of the group's first join it and take its value
    while (e < n && hd[order[s]] - hd[order[e]] <= tol) ++e;
    const double dv = hd[order[s]];
    // ||w|| scaled by the largest |w_t|, so that no square overflows
    double big = 0.0, nw = 0.0;
    if (!zero_all)
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
      ru[order[t]] = 0.0;
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
      u.resize(e - s);
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
}

// Both lists are decreasing: merge the deflated/reflected columns with the
// reduced eigenvalues lamr[0..m) (deflated and reflected first among equal
// values).
inline void merge_cols(const std::vector<Col>& cols, const double* lamr, int64_t m, std::vector<Col>& out,
                       Scratch* scratch = nullptr) {
  Scratch local;
  std::vector<Col>& red = (scratch ? *scratch : local).red;
  red.resize(m);
  for (int64_t k = 0; k < m; ++k) red[k] = {lamr[k], COL_REDUCED, (int32_t)k, 0, 0.0};
  out.resize(cols.size() + m);
  std::merge(cols.begin(), cols.end(), red.begin(), red.end(), out.begin(),
             [](const Col& a, const Col& b) { return a.val > b.val; });
}

}  // namespace fe
}  // namespace dpr1
