// Host-code driver for the sanitizer test: runs libsdp's host-only code (the
// instance validation with its entry selectors, the chordal extension and
// maximal cliques, the data scaling) on valid and invalid inputs.  Built with
// -fsanitize=address,undefined by test_sanitize_cpu.py; exits non-zero on a
// wrong status code or result, and the sanitizers abort on any memory error
// or undefined behaviour.  No device code is involved.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "sdp.h"
#include "sdp_host.h"

static std::string g_msg;
void sdp_set_last_error(const std::string &msg) { g_msg = msg; }

static int g_fail = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++g_fail;                                                         \
    }                                                                   \
  } while (0)

struct Inst {
  int n = 0, m = 0;
  std::vector<int32_t> row, col, cptr, cvert;
  std::vector<int64_t> arp;
  std::vector<int32_t> acol;
  std::vector<double> aval, b, c;
  int fmt = SDP_A_DENSE;
  sdp_instance view() const {
    sdp_instance I{};
    I.n = n;
    I.m = m;
    I.p = (int32_t)cptr.size() - 1;
    I.nnz_pattern = (int64_t)row.size();
    I.pat_row = row.data();
    I.pat_col = col.data();
    I.clique_ptr = cptr.data();
    I.clique_vert = cvert.data();
    I.a_format = fmt;
    I.a_rowptr = fmt == SDP_A_CSR ? arp.data() : nullptr;
    I.a_col = fmt == SDP_A_CSR ? acol.data() : nullptr;
    I.a_val = aval.data();
    I.b = b.data();
    I.c = c.data();
    return I;
  }
};

// banded pattern of half-bandwidth w, cliques {i, ..., i + w}
static Inst banded(int n, int w, int m, unsigned seed, bool csr) {
  Inst I;
  I.n = n;
  I.m = m;
  for (int cc = 0; cc < n; ++cc)
    for (int r = cc; r < n && r - cc <= w; ++r) {
      I.row.push_back(r);
      I.col.push_back(cc);
    }
  I.cptr.push_back(0);
  for (int i = 0; i + w < n; ++i) {
    for (int v = i; v <= i + w; ++v) I.cvert.push_back(v);
    I.cptr.push_back((int32_t)I.cvert.size());
  }
  std::mt19937 rng(seed);
  std::normal_distribution<double> N01;
  std::uniform_real_distribution<double> U;
  const int64_t nnz = (int64_t)I.row.size();
  if (csr) {
    I.fmt = SDP_A_CSR;
    I.arp.push_back(0);
    for (int i = 0; i < m; ++i) {
      for (int64_t j = 0; j < nnz; ++j)
        if (U(rng) < 0.1 || j == (i * 7) % nnz) {
          I.acol.push_back((int32_t)j);
          I.aval.push_back(N01(rng));
        }
      I.arp.push_back((int64_t)I.acol.size());
    }
  } else {
    I.aval.resize((size_t)m * nnz);
    for (double &v : I.aval) v = N01(rng);
  }
  I.b.resize(m);
  for (double &v : I.b) v = N01(rng);
  I.c.resize(nnz);
  for (double &v : I.c) v = N01(rng);
  return I;
}

static int validate(const Inst &I, int max_clique, sdp_host::HostInst *out = nullptr) {
  sdp_host::HostInst H;
  try {
    const sdp_instance v = I.view();
    sdp_host::validate_and_index(v, max_clique, H);
  } catch (sdp_host::SdpError &e) {
    return e.code;
  }
  if (out) *out = H;
  return SDP_OK;
}

static void test_validation() {
  for (int csr = 0; csr < 2; ++csr) {
    const int n = 40, w = 5;
    Inst I = banded(n, w, 12, 7 + csr, csr != 0);
    sdp_host::HostInst H;
    CHECK(validate(I, 128, &H) == SDP_OK);
    const int p = n - w;
    CHECK(H.npk == (int64_t)p * (w + 1) * (w + 2) / 2);
    CHECK(H.ld % 64 == 0 && H.ld >= (int64_t)I.row.size());
    // D counts the cliques covering each coordinate: diagonal entry v lies
    // in min(v, w, n-1-v, n-1-w) + 1 cliques
    for (size_t j = 0; j < I.row.size(); ++j) CHECK(H.D[j] >= 1 && H.D[j] <= w + 1);
    CHECK(validate(I, w, nullptr) == SDP_ERR_UNSUPPORTED);   // cliques of w + 1
    {   // unsorted pattern
      Inst J = I;
      std::swap(J.row[1], J.row[2]);
      CHECK(validate(J, 128) == SDP_ERR_ARG);
    }
    {   // a coordinate above the diagonal
      Inst J = I;
      J.row[1] = 0;
      J.col[1] = 1;
      CHECK(validate(J, 128) == SDP_ERR_ARG);
    }
    {   // clique vertices out of order
      Inst J = I;
      std::swap(J.cvert[0], J.cvert[1]);
      CHECK(validate(J, 128) == SDP_ERR_CLIQUE_ORDER);
    }
    {   // vertex out of range
      Inst J = I;
      J.cvert.back() = n;
      CHECK(validate(J, 128) == SDP_ERR_CLIQUE_ORDER);
    }
    {   // non-finite data
      Inst J = I;
      J.c[3] = NAN;
      CHECK(validate(J, 128) == SDP_ERR_NONFINITE);
      Inst K = I;
      K.aval[5] = INFINITY;
      CHECK(validate(K, 128) == SDP_ERR_NONFINITE);
    }
    {   // a clique pair outside the pattern: drop coordinate (1, 0)
      Inst J = I;
      J.row.erase(J.row.begin() + 1);
      J.col.erase(J.col.begin() + 1);
      J.c.erase(J.c.begin() + 1);
      if (!csr) {
        J.aval.clear();
        const int64_t nnz = (int64_t)J.row.size();
        J.aval.assign((size_t)J.m * nnz, 0.5);
      } else {
        for (auto &a : J.acol) a = a > 0 ? a - 1 : 0;
      }
      CHECK(validate(J, 128) == SDP_ERR_OFF_PATTERN);
    }
    {   // a pattern coordinate no clique covers: drop the first clique
      Inst J = I;
      J.cvert.erase(J.cvert.begin(), J.cvert.begin() + (w + 1));
      J.cptr.erase(J.cptr.begin());
      for (auto &q : J.cptr) q -= w + 1;
      CHECK(validate(J, 128) == SDP_ERR_PATTERN_UNCOVERED);
    }
    if (csr) {   // CSR column out of range, rows not monotone
      Inst J = I;
      J.acol[0] = (int32_t)I.row.size();
      CHECK(validate(J, 128) == SDP_ERR_ARG);
      Inst K = I;
      K.arp[1] = K.arp[2] + 1;
      CHECK(validate(K, 128) == SDP_ERR_ARG);
    }
    {   // missing pointers and sizes
      Inst J = I;
      J.b.clear();
      sdp_instance v = J.view();
      v.b = nullptr;
      sdp_host::HostInst HH;
      int code = SDP_OK;
      try {
        sdp_host::validate_and_index(v, 128, HH);
      } catch (sdp_host::SdpError &e) {
        code = e.code;
      }
      CHECK(code == SDP_ERR_ARG);
    }
  }
}

// chordal extension of grids, cycles and random graphs: every clique pair is
// in the extension, every original coordinate maps into it
static void check_pattern(int n, const std::vector<int32_t> &r, const std::vector<int32_t> &c) {
  sdp_pattern *P = nullptr;
  CHECK(sdp_pattern_create(n, (int64_t)r.size(), r.data(), c.data(), &P) == SDP_OK);
  if (!P) return;
  int64_t ne = 0, tot = 0;
  int32_t p = 0;
  CHECK(sdp_pattern_sizes(P, &ne, &p, &tot) == SDP_OK);
  std::vector<int32_t> er(ne), ec(ne), cp(p + 1), cv(tot);
  std::vector<int64_t> idx(r.size());
  CHECK(sdp_pattern_get(P, er.data(), ec.data(), cp.data(), cv.data(), (int64_t)r.size(), r.data(),
                        c.data(), idx.data()) == SDP_OK);
  std::vector<std::vector<char>> in(n, std::vector<char>(n, 0));
  for (int64_t j = 0; j < ne; ++j) {
    CHECK(er[j] >= ec[j] && er[j] < n);
    in[er[j]][ec[j]] = 1;
  }
  for (int k = 0; k < p; ++k)
    for (int a = cp[k]; a < cp[k + 1]; ++a)
      for (int b2 = cp[k]; b2 <= a; ++b2) CHECK(in[cv[a]][cv[b2]] || in[cv[b2]][cv[a]]);
  for (size_t j = 0; j < r.size(); ++j) {
    const int rr = std::max(r[j], c[j]), cc = std::min(r[j], c[j]);
    CHECK(idx[j] >= 0 && idx[j] < ne && er[idx[j]] == rr && ec[idx[j]] == cc);
  }
  sdp_pattern_destroy(P);
}

static void test_pattern() {
  for (int g = 3; g <= 12; g += 3) {   // g x g grid
    std::vector<int32_t> r, c;
    for (int i = 0; i < g; ++i)
      for (int j = 0; j < g; ++j) {
        const int v = i * g + j;
        if (j + 1 < g) { r.push_back(v + 1); c.push_back(v); }
        if (i + 1 < g) { r.push_back(v + g); c.push_back(v); }
      }
    check_pattern(g * g, r, c);
  }
  for (int n = 4; n <= 30; n += 5) {   // chordless cycles (upper coordinates too)
    std::vector<int32_t> r, c;
    for (int v = 0; v < n; ++v) {
      r.push_back(v);
      c.push_back((v + 1) % n);
    }
    check_pattern(n, r, c);
  }
  std::mt19937 rng(3);
  for (int t = 0; t < 5; ++t) {   // random sparse graphs with repeats and diagonals
    const int n = 20 + 15 * t;
    std::uniform_int_distribution<int> V(0, n - 1);
    std::vector<int32_t> r, c;
    for (int e = 0; e < 2 * n; ++e) {
      r.push_back(V(rng));
      c.push_back(V(rng));
    }
    check_pattern(n, r, c);
  }
  sdp_pattern *P = nullptr;
  const int32_t bad_r[1] = {5}, bad_c[1] = {0};
  CHECK(sdp_pattern_create(3, 1, bad_r, bad_c, &P) == SDP_ERR_ARG && P == nullptr);
  CHECK(sdp_pattern_create(0, 0, nullptr, nullptr, &P) == SDP_ERR_ARG);
  sdp_pattern_destroy(nullptr);
}

static void test_scaling() {
  for (int csr = 0; csr < 2; ++csr) {
    Inst I = banded(30, 4, 10, 11 + csr, csr != 0);
    const sdp_instance v = I.view();
    std::vector<double> e(I.m), s(I.n);
    double rb = 0, sc = 0;
    CHECK(sdp_scale_compute(&v, 10, e.data(), s.data(), &rb, &sc) == SDP_OK);
    for (double x : e) CHECK(std::isfinite(x) && x > 0);
    for (double x : s) CHECK(std::isfinite(x) && x > 0);
    CHECK(rb > 0 && sc > 0);
    std::vector<double> a2(I.aval.size()), b2(I.m), c2(I.c.size());
    CHECK(sdp_scale_apply(&v, e.data(), s.data(), rb, sc, a2.data(), b2.data(), c2.data()) ==
          SDP_OK);
    std::vector<double> x(I.c.size(), 1.0), y(I.m, 1.0), z(I.c.size(), 1.0);
    CHECK(sdp_scale_recover(&v, e.data(), s.data(), rb, sc, x.data(), y.data(), z.data()) == SDP_OK);
    for (double q : x) CHECK(std::isfinite(q));
    Inst J = I;
    J.b[0] = NAN;
    const sdp_instance vj = J.view();
    CHECK(sdp_scale_compute(&vj, 10, e.data(), s.data(), &rb, &sc) != SDP_OK);
  }
}

int main() {
  test_validation();
  test_pattern();
  test_scaling();
  std::printf("sanitize driver: %d failed checks\n", g_fail);
  return g_fail ? 1 : 0;
}
