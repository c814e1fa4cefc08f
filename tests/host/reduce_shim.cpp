// C entry points over the front end's host reduction (reduce.h), for CPU tests.
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../paper_1405_7537_amd/csrc/reduce.h"

extern "C" {

void shim_sort(const double* d, int64_t n, int64_t* order) {
  std::vector<int64_t> o;
  dpr1::fe::sort_decreasing(d, n, o);
  memcpy(order, o.data(), 8 * n);
}

// Returns the reduced size m; fills rd, rz [m], rgrp, rpos, ru [n], and the
// deflated/reflected columns (kind, idx, t, val, ub) [n - m], which are merged
// with the given reduced eigenvalues lamr [m] into the final column list
// (out_kind, out_idx, out_val) [n].
int64_t shim_reduce(const double* d, const double* z, int64_t n, int zero_all, double* rd, double* rz,
                    int32_t* rgrp, int32_t* rpos, double* ru, int32_t* ckind, int32_t* cidx, int32_t* ct,
                    double* cval, double* cub) {
  std::vector<double> vrd, vrz;
  std::vector<dpr1::fe::Col> cols;
  dpr1::fe::reduce(d, z, n, zero_all != 0, vrd, vrz, rgrp, rpos, ru, cols);
  const int64_t m = (int64_t)vrd.size();
  memcpy(rd, vrd.data(), 8 * m);
  memcpy(rz, vrz.data(), 8 * m);
  for (size_t c = 0; c < cols.size(); ++c) {
    ckind[c] = cols[c].kind;
    cidx[c] = cols[c].idx;
    ct[c] = cols[c].t;
    cval[c] = cols[c].val;
    cub[c] = cols[c].ub;
  }
  return m;
}

void shim_merge(const int32_t* ckind, const int32_t* cidx, const int32_t* ct, const double* cval, const double* cub,
                int64_t ncols, const double* lamr, int64_t m, int32_t* okind, int32_t* oidx, double* oval) {
  std::vector<dpr1::fe::Col> cols(ncols), out;
  for (int64_t c = 0; c < ncols; ++c) cols[c] = {cval[c], ckind[c], cidx[c], ct[c], cub[c]};
  dpr1::fe::merge_cols(cols, lamr, m, out);
  for (size_t c = 0; c < out.size(); ++c) {
    okind[c] = out[c].kind;
    oidx[c] = out[c].idx;
    oval[c] = out[c].val;
  }
}
}
