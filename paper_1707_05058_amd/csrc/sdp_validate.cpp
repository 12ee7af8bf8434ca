// Validation of one SDP instance and its host-side index structures (entry
// selectors, overlap counts): plain C++, no device work.
#include "sdp_host.h"

#include <algorithm>
#include <cmath>

namespace sdp_host {

int validate_and_index(const sdp_instance &I, int max_clique, HostInst &H) {
  H.src = &I;
  if (I.n <= 0 || I.m <= 0 || I.nnz_pattern <= 0 || I.p <= 0 || !I.pat_row || !I.pat_col ||
      !I.clique_ptr || !I.clique_vert || !I.a_val || !I.b || !I.c ||
      (I.a_format != SDP_A_DENSE && I.a_format != SDP_A_CSR) ||
      (I.a_format == SDP_A_CSR && (!I.a_rowptr || !I.a_col)))
    fail(SDP_ERR_ARG, "invalid sizes, pointers or A format");
  if (I.nnz_pattern >= (int64_t)1 << 31) fail(SDP_ERR_ARG, "pattern too large");
  const int n = I.n;
  const int64_t nnz = I.nnz_pattern;
  int ndiag = 0;
  for (int64_t j = 0; j < nnz; ++j) {
    const int r = I.pat_row[j], c = I.pat_col[j];
    if (r < 0 || r >= n || c < 0 || c > r) fail(SDP_ERR_ARG, "pattern coordinate out of range or not lower");
    if (j > 0) {
      const int pr = I.pat_row[j - 1], pc = I.pat_col[j - 1];
      if (c < pc || (c == pc && r <= pr)) fail(SDP_ERR_ARG, "pattern not sorted by (col, row)");
    }
    if (r == c) ++ndiag;
  }
  if (ndiag != n) fail(SDP_ERR_ARG, "pattern misses a diagonal entry");
  if (I.clique_ptr[0] != 0) fail(SDP_ERR_ARG, "clique_ptr[0] != 0");
  for (int k = 0; k < I.p; ++k)
    if (I.clique_ptr[k + 1] - I.clique_ptr[k] <= 0) fail(SDP_ERR_ARG, "empty clique");
  for (int k = 0; k < I.p; ++k) {
    const int s = I.clique_ptr[k + 1] - I.clique_ptr[k];
    const int32_t *v = I.clique_vert + I.clique_ptr[k];
    for (int a = 0; a < s; ++a) {
      if (v[a] < 0 || v[a] >= n) fail(SDP_ERR_CLIQUE_ORDER, "clique vertex out of range");
      if (a > 0 && v[a] <= v[a - 1]) fail(SDP_ERR_CLIQUE_ORDER, "clique vertices not increasing");
    }
  }
  const int smax = max_clique;
  for (int k = 0; k < I.p; ++k)
    if (I.clique_ptr[k + 1] - I.clique_ptr[k] > smax)
      fail(SDP_ERR_UNSUPPORTED, "clique larger than " + std::to_string(smax) +
                                    " for this projection precision");
  int64_t annz;
  if (I.a_format == SDP_A_CSR) {
    if (I.a_rowptr[0] != 0) fail(SDP_ERR_ARG, "a_rowptr[0] != 0");
    for (int i = 0; i < I.m; ++i)
      if (I.a_rowptr[i + 1] < I.a_rowptr[i]) fail(SDP_ERR_ARG, "a_rowptr not monotone");
    annz = I.a_rowptr[I.m];
    for (int64_t t = 0; t < annz; ++t)
      if (I.a_col[t] < 0 || I.a_col[t] >= nnz) fail(SDP_ERR_ARG, "a_col out of range");
  } else {
    annz = (int64_t)I.m * nnz;
  }
  for (int64_t t = 0; t < annz; ++t)
    if (!std::isfinite(I.a_val[t])) fail(SDP_ERR_NONFINITE, "non-finite value in A");
  for (int i = 0; i < I.m; ++i)
    if (!std::isfinite(I.b[i])) fail(SDP_ERR_NONFINITE, "non-finite value in b");
  for (int64_t j = 0; j < nnz; ++j)
    if (!std::isfinite(I.c[j])) fail(SDP_ERR_NONFINITE, "non-finite value in C");

  // column starts of the sorted pattern, for coordinate lookup
  std::vector<int64_t> colstart(n + 1, 0);
  for (int64_t j = 0; j < nnz; ++j) colstart[I.pat_col[j] + 1]++;
  for (int c = 0; c < n; ++c) colstart[c + 1] += colstart[c];
  auto lookup = [&](int r, int c) -> int64_t {
    const int32_t *b = I.pat_row + colstart[c], *e = I.pat_row + colstart[c + 1];
    const int32_t *it = std::lower_bound(b, e, r);
    if (it == e || *it != r) return -1;
    return colstart[c] + (it - b);
  };
  H.n = n; H.m = I.m; H.p = I.p; H.fmt = I.a_format; H.nnz = nnz;
  H.ld = (int32_t)round_up(nnz, 64);
  H.ldm = (int32_t)round_up(I.m, 64);
  H.cl_off.resize(I.p + 1);
  H.cl_off[0] = 0;
  for (int k = 0; k < I.p; ++k) {
    const int64_t s = I.clique_ptr[k + 1] - I.clique_ptr[k];
    H.cl_off[k + 1] = H.cl_off[k] + s * (s + 1) / 2;
  }
  H.npk = H.cl_off[I.p];
  H.blk_loc.resize(H.npk);
  H.D.assign(nnz, 0);
  // entry selectors E_Ck: packed block entry (a, b), a >= b, of clique k is
  // the pattern coordinate (v_a, v_b) (v_a > v_b since vertices increase)
  for (int k = 0; k < I.p; ++k) {
    const int s = I.clique_ptr[k + 1] - I.clique_ptr[k];
    const int32_t *v = I.clique_vert + I.clique_ptr[k];
    int64_t e = H.cl_off[k];
    for (int a = 0; a < s; ++a)
      for (int b = 0; b <= a; ++b, ++e) {
        const int64_t j = lookup(v[a], v[b]);
        if (j < 0) fail(SDP_ERR_OFF_PATTERN, "clique pair outside the pattern");
        H.blk_loc[e] = (int32_t)j;
      }
  }
  for (int64_t e = 0; e < H.npk; ++e) H.D[H.blk_loc[e]]++;
  for (int64_t j = 0; j < nnz; ++j)
    if (H.D[j] == 0) fail(SDP_ERR_PATTERN_UNCOVERED, "pattern coordinate covered by no clique");
  return SDP_OK;
}

}  // namespace sdp_host
