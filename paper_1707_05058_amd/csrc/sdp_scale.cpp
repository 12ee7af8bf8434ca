// Data scaling of an SDP instance (host code).
//
// Section 7.1.3 rescales the decomposed problem by positive diagonal D (on
// the variable, preserving the cone), E (on the equality constraints) and by
// positive scalars multiplying b and C, choosing them so that the rows of the
// scaled A and b have norms near one and the columns of A and c have similar
// norms (the equilibration scheme of SCS, which the paper cites).  Here D is a
// congruence X -> S X S by one positive diagonal S over the vertices: it maps
// every clique block to a PSD block and keeps the pattern, so the scaled
// instance is solved by the unchanged solver.
//
//   A'_i = e_i S A_i S,   b'_i = rho_b e_i b_i,   C' = sigma_c S C S
//
// e and s come from Ruiz iterations (both norms taken on the current scaled
// A, then e_i /= sqrt(||A'_i||_F), s_v /= sqrt(norm of row v over all A'_i),
// clamped to [1e-4, 1e4]); rho_b and sigma_c equalise ||b'|| and ||C'||_F
// with the mean row and vertex norms.  A solution of the scaled problem maps
// back by X = S X' S / rho_b, y = E y' / sigma_c, Z = S^-1 Z' S^-1 / sigma_c.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "sdp.h"

void sdp_set_last_error(const std::string &msg);   // sdp_api.cpp

namespace {

constexpr double kScaleMin = 1e-4, kScaleMax = 1e4;

struct ScaleError : std::runtime_error {
  int code;
  ScaleError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// Visits every stored A entry as f(i, j, value) with j the pattern coordinate.
template <typename F>
void for_each_a(const sdp_instance &I, F &&f) {
  if (I.a_format == SDP_A_DENSE) {
    for (int32_t i = 0; i < I.m; ++i)
      for (int64_t j = 0; j < I.nnz_pattern; ++j) f(i, j, I.a_val[(int64_t)i * I.nnz_pattern + j]);
  } else {
    for (int32_t i = 0; i < I.m; ++i)
      for (int64_t t = I.a_rowptr[i]; t < I.a_rowptr[i + 1]; ++t) f(i, (int64_t)I.a_col[t], I.a_val[t]);
  }
}

int64_t a_count(const sdp_instance &I) {
  return I.a_format == SDP_A_DENSE ? (int64_t)I.m * I.nnz_pattern : I.a_rowptr[I.m];
}

void check(const sdp_instance *in) {
  if (!in) throw ScaleError(SDP_ERR_ARG, "NULL instance");
  const sdp_instance &I = *in;
  if (I.n <= 0 || I.m <= 0 || I.nnz_pattern <= 0 || !I.pat_row || !I.pat_col || !I.a_val || !I.b ||
      !I.c || (I.a_format != SDP_A_DENSE && I.a_format != SDP_A_CSR) ||
      (I.a_format == SDP_A_CSR && (!I.a_rowptr || !I.a_col)))
    throw ScaleError(SDP_ERR_ARG, "invalid sizes, pointers or A format");
  for (int64_t j = 0; j < I.nnz_pattern; ++j) {
    const int32_t r = I.pat_row[j], c = I.pat_col[j];
    if (r < 0 || r >= I.n || c < 0 || c > r) throw ScaleError(SDP_ERR_ARG, "pattern coordinate out of range or not lower");
    if (!std::isfinite(I.c[j])) throw ScaleError(SDP_ERR_NONFINITE, "non-finite value in C");
  }
  if (I.a_format == SDP_A_CSR) {
    if (I.a_rowptr[0] != 0) throw ScaleError(SDP_ERR_ARG, "a_rowptr[0] != 0");
    for (int32_t i = 0; i < I.m; ++i)
      if (I.a_rowptr[i + 1] < I.a_rowptr[i]) throw ScaleError(SDP_ERR_ARG, "a_rowptr not monotone");
    for (int64_t t = 0; t < I.a_rowptr[I.m]; ++t)
      if (I.a_col[t] < 0 || I.a_col[t] >= I.nnz_pattern) throw ScaleError(SDP_ERR_ARG, "a_col out of range");
  }
  for (int64_t t = 0; t < a_count(I); ++t)
    if (!std::isfinite(I.a_val[t])) throw ScaleError(SDP_ERR_NONFINITE, "non-finite value in A");
  for (int32_t i = 0; i < I.m; ++i)
    if (!std::isfinite(I.b[i])) throw ScaleError(SDP_ERR_NONFINITE, "non-finite value in b");
}

double clamp_scale(double x) { return std::min(kScaleMax, std::max(kScaleMin, x)); }

// Squared row norms r2[i] = ||A'_i||_F^2 and vertex norms q2[v] of the
// current scaled A.
void norms(const sdp_instance &I, const std::vector<double> &e, const std::vector<double> &s,
           std::vector<double> &r2, std::vector<double> &q2) {
  std::fill(r2.begin(), r2.end(), 0.0);
  std::fill(q2.begin(), q2.end(), 0.0);
  for_each_a(I, [&](int32_t i, int64_t j, double a) {
    const int32_t r = I.pat_row[j], c = I.pat_col[j];
    const double v = e[i] * s[r] * s[c] * a, v2 = v * v;
    if (r == c) {
      r2[i] += v2;
      q2[r] += v2;
    } else {
      r2[i] += 2.0 * v2;
      q2[r] += v2;
      q2[c] += v2;
    }
  });
}

template <typename F>
int run(F &&f) {
  try {
    sdp_set_last_error("");
    f();
    return SDP_OK;
  } catch (ScaleError &e) {
    sdp_set_last_error(e.what());
    return e.code;
  } catch (std::bad_alloc &) {
    sdp_set_last_error("host allocation failed");
    return SDP_ERR_OOM;
  } catch (std::exception &e) {
    sdp_set_last_error(e.what());
    return SDP_ERR_ARG;
  }
}

}  // namespace

extern "C" {

int sdp_scale_compute(const sdp_instance *inst, int32_t iters, double *row_scale, double *vertex_scale,
                      double *rho_b, double *sigma_c) {
  return run([&] {
    check(inst);
    if (iters < 0 || !row_scale || !vertex_scale || !rho_b || !sigma_c)
      throw ScaleError(SDP_ERR_ARG, "invalid iteration count or NULL output");
    const sdp_instance &I = *inst;
    std::vector<double> e(I.m, 1.0), s(I.n, 1.0), r2(I.m), q2(I.n);
    for (int32_t it = 0; it < iters; ++it) {
      norms(I, e, s, r2, q2);
      for (int32_t i = 0; i < I.m; ++i)
        if (r2[i] > 0) e[i] = clamp_scale(e[i] / std::sqrt(std::sqrt(r2[i])));
      for (int32_t v = 0; v < I.n; ++v)
        if (q2[v] > 0) s[v] = clamp_scale(s[v] / std::sqrt(std::sqrt(q2[v])));
    }
    norms(I, e, s, r2, q2);
    double rmean = 0, qmean = 0, nb2 = 0, nc2 = 0;
    for (int32_t i = 0; i < I.m; ++i) rmean += std::sqrt(r2[i]);
    for (int32_t v = 0; v < I.n; ++v) qmean += std::sqrt(q2[v]);
    rmean /= I.m;
    qmean /= I.n;
    for (int32_t i = 0; i < I.m; ++i) nb2 += (e[i] * I.b[i]) * (e[i] * I.b[i]);
    for (int64_t j = 0; j < I.nnz_pattern; ++j) {
      const int32_t r = I.pat_row[j], c = I.pat_col[j];
      const double v = s[r] * s[c] * I.c[j];
      nc2 += (r == c ? 1.0 : 2.0) * v * v;
    }
    *rho_b = clamp_scale(rmean / std::max(std::sqrt(nb2), kScaleMin));
    *sigma_c = clamp_scale(qmean / std::max(std::sqrt(nc2), kScaleMin));
    std::copy(e.begin(), e.end(), row_scale);
    std::copy(s.begin(), s.end(), vertex_scale);
  });
}

int sdp_scale_apply(const sdp_instance *inst, const double *row_scale, const double *vertex_scale,
                    double rho_b, double sigma_c, double *a_val_out, double *b_out, double *c_out) {
  return run([&] {
    check(inst);
    if (!row_scale || !vertex_scale || !(rho_b > 0) || !(sigma_c > 0))
      throw ScaleError(SDP_ERR_ARG, "invalid scaling");
    const sdp_instance &I = *inst;
    if (a_val_out) {
      int64_t t = 0;
      for_each_a(I, [&](int32_t i, int64_t j, double a) {
        a_val_out[t++] = row_scale[i] * vertex_scale[I.pat_row[j]] * vertex_scale[I.pat_col[j]] * a;
      });
    }
    if (b_out)
      for (int32_t i = 0; i < I.m; ++i) b_out[i] = rho_b * row_scale[i] * I.b[i];
    if (c_out)
      for (int64_t j = 0; j < I.nnz_pattern; ++j)
        c_out[j] = sigma_c * vertex_scale[I.pat_row[j]] * vertex_scale[I.pat_col[j]] * I.c[j];
  });
}

int sdp_scale_recover(const sdp_instance *inst, const double *row_scale, const double *vertex_scale,
                      double rho_b, double sigma_c, double *x, double *y, double *z) {
  return run([&] {
    if (!inst || !inst->pat_row || !inst->pat_col || inst->nnz_pattern < 0 || inst->m < 0 ||
        inst->n <= 0 || !row_scale || !vertex_scale || !(rho_b > 0) || !(sigma_c > 0))
      throw ScaleError(SDP_ERR_ARG, "invalid instance or scaling");
    const sdp_instance &I = *inst;
    for (int64_t j = 0; j < I.nnz_pattern; ++j) {
      const int32_t r = I.pat_row[j], c = I.pat_col[j];
      if (r < 0 || r >= I.n || c < 0 || c >= I.n) throw ScaleError(SDP_ERR_ARG, "pattern coordinate out of range");
      const double ss = vertex_scale[r] * vertex_scale[c];
      if (x) x[j] = ss * x[j] / rho_b;
      if (z) z[j] = z[j] / (ss * sigma_c);
    }
    if (y)
      for (int32_t i = 0; i < I.m; ++i) y[i] = row_scale[i] * y[i] / sigma_c;
  });
}

}  // extern "C"
