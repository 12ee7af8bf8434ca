// Chordal extension and maximal cliques of a sparsity pattern (host code).
//
// The decomposition needs a chordal aggregate pattern and its maximal
// cliques (Theorem 1 and Section 7.1.1: a nonchordal pattern is first
// extended).  Here the extension is the filled graph of a symbolic Cholesky
// elimination under a greedy minimum-degree order: eliminating a vertex makes
// its remaining neighbours pairwise adjacent.  The elimination order is then a
// perfect elimination order of the filled graph, and its maximal cliques are
// the sets C(v) = {v} u adj+(v) (adj+ = neighbours eliminated after v) that
// are not contained in C(u) for a vertex u whose first later neighbour is v
// with |adj+(u)| = |adj+(v)| + 1.
#include <algorithm>
#include <cstdint>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "sdp.h"

void sdp_set_last_error(const std::string &msg);   // sdp_api.cpp

struct sdp_pattern {
  int32_t n = 0;
  std::vector<int32_t> pat_row, pat_col;            // lower coordinates, sorted (col, row)
  std::vector<int32_t> clique_ptr, clique_vert;
};

namespace {

struct PatternError : std::runtime_error {
  int code;
  PatternError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void build(sdp_pattern &P, int32_t n, int64_t nnz, const int32_t *row, const int32_t *col) {
  if (n <= 0 || nnz < 0 || (nnz > 0 && (!row || !col)))
    throw PatternError(SDP_ERR_ARG, "invalid pattern arguments");
  std::vector<std::set<int32_t>> adj(n);
  for (int64_t k = 0; k < nnz; ++k) {
    const int32_t r = row[k], c = col[k];
    if (r < 0 || r >= n || c < 0 || c >= n) throw PatternError(SDP_ERR_ARG, "coordinate out of range");
    if (r != c) {
      adj[r].insert(c);
      adj[c].insert(r);
    }
  }
  // greedy minimum degree on the elimination graph (ties: smallest label)
  std::vector<char> gone(n, 0);
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<std::vector<int32_t>> higher(n);     // adj+(v) at elimination time
  std::set<std::pair<int32_t, int32_t>> queue;     // (degree, vertex)
  for (int32_t v = 0; v < n; ++v) queue.insert({(int32_t)adj[v].size(), v});
  while (!queue.empty()) {
    const int32_t v = queue.begin()->second;
    queue.erase(queue.begin());
    gone[v] = 1;
    order.push_back(v);
    std::vector<int32_t> nb(adj[v].begin(), adj[v].end());
    higher[v] = nb;
    for (int32_t a : nb) {
      queue.erase({(int32_t)adj[a].size(), a});
      adj[a].erase(v);
    }
    for (size_t i = 0; i < nb.size(); ++i)
      for (size_t j = i + 1; j < nb.size(); ++j) {
        adj[nb[i]].insert(nb[j]);
        adj[nb[j]].insert(nb[i]);
      }
    for (int32_t a : nb) queue.insert({(int32_t)adj[a].size(), a});
  }
  // maximal cliques from the perfect elimination order
  std::vector<int32_t> pos(n);
  for (int32_t i = 0; i < n; ++i) pos[order[i]] = i;
  std::vector<char> maximal(n, 1);
  for (int32_t u = 0; u < n; ++u) {
    if (higher[u].empty()) continue;
    int32_t parent = higher[u][0];
    for (int32_t a : higher[u])
      if (pos[a] < pos[parent]) parent = a;
    if (higher[u].size() == higher[parent].size() + 1) maximal[parent] = 0;
  }
  std::vector<std::vector<int32_t>> cliques;
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = order[i];
    if (!maximal[v]) continue;
    std::vector<int32_t> c = higher[v];
    c.push_back(v);
    std::sort(c.begin(), c.end());
    cliques.push_back(std::move(c));
  }
  std::sort(cliques.begin(), cliques.end());
  P.n = n;
  P.clique_ptr.assign(1, 0);
  P.clique_vert.clear();
  std::vector<int64_t> keys;
  for (const auto &c : cliques) {
    for (size_t a = 0; a < c.size(); ++a)
      for (size_t b = 0; b <= a; ++b) keys.push_back((int64_t)c[b] * n + c[a]);   // (col, row)
    P.clique_vert.insert(P.clique_vert.end(), c.begin(), c.end());
    P.clique_ptr.push_back((int32_t)P.clique_vert.size());
  }
  for (int32_t v = 0; v < n; ++v) keys.push_back((int64_t)v * n + v);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  P.pat_row.resize(keys.size());
  P.pat_col.resize(keys.size());
  for (size_t k = 0; k < keys.size(); ++k) {
    P.pat_col[k] = (int32_t)(keys[k] / n);
    P.pat_row[k] = (int32_t)(keys[k] % n);
  }
}

template <typename F>
int run(F &&f) {
  try {
    sdp_set_last_error("");
    f();
    return SDP_OK;
  } catch (PatternError &e) {
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

int sdp_pattern_create(int32_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                       sdp_pattern **out) {
  if (!out) return SDP_ERR_ARG;
  *out = nullptr;
  sdp_pattern *P = nullptr;
  const int rc = run([&] {
    P = new sdp_pattern();
    build(*P, n, nnz, row, col);
  });
  if (rc != SDP_OK) {
    delete P;
    return rc;
  }
  *out = P;
  return SDP_OK;
}

int sdp_pattern_sizes(const sdp_pattern *pat, int64_t *nnz_ext, int32_t *p, int64_t *clique_total) {
  return run([&] {
    if (!pat) throw PatternError(SDP_ERR_ARG, "NULL pattern");
    if (nnz_ext) *nnz_ext = (int64_t)pat->pat_row.size();
    if (p) *p = (int32_t)pat->clique_ptr.size() - 1;
    if (clique_total) *clique_total = (int64_t)pat->clique_vert.size();
  });
}

int sdp_pattern_get(const sdp_pattern *pat, int32_t *pat_row, int32_t *pat_col, int32_t *clique_ptr,
                    int32_t *clique_vert, int64_t nnz, const int32_t *row, const int32_t *col,
                    int64_t *index_out) {
  return run([&] {
    if (!pat) throw PatternError(SDP_ERR_ARG, "NULL pattern");
    if (pat_row) std::copy(pat->pat_row.begin(), pat->pat_row.end(), pat_row);
    if (pat_col) std::copy(pat->pat_col.begin(), pat->pat_col.end(), pat_col);
    if (clique_ptr) std::copy(pat->clique_ptr.begin(), pat->clique_ptr.end(), clique_ptr);
    if (clique_vert) std::copy(pat->clique_vert.begin(), pat->clique_vert.end(), clique_vert);
    if (index_out && nnz > 0) {
      if (!row || !col) throw PatternError(SDP_ERR_ARG, "coordinates missing for the index map");
      const int64_t n = pat->n;
      std::vector<int64_t> keys(pat->pat_row.size());
      for (size_t k = 0; k < keys.size(); ++k) keys[k] = (int64_t)pat->pat_col[k] * n + pat->pat_row[k];
      for (int64_t k = 0; k < nnz; ++k) {
        const int32_t r = std::max(row[k], col[k]), c = std::min(row[k], col[k]);
        if (r < 0 || r >= n || c < 0) throw PatternError(SDP_ERR_ARG, "coordinate out of range");
        const int64_t key = (int64_t)c * n + r;
        const auto it = std::lower_bound(keys.begin(), keys.end(), key);
        index_out[k] = (it != keys.end() && *it == key) ? (int64_t)(it - keys.begin()) : -1;
      }
    }
  });
}

void sdp_pattern_destroy(sdp_pattern *pat) { delete pat; }

}  // extern "C"
