// Host side of libsdp: validation, index construction, device layout, the
// iteration driver (HIP graphs) and the C ABI of include/sdp.h.
//
// Everything numerical runs in the HIP kernels of k_project.hip, k_affine.hip
// and k_factor.hip; this file only builds integer index structures, moves
// data and launches work.
#include "../../include/sdp.h"
#include "sdp_host.h"
#include "sdp_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

namespace {

thread_local std::string g_last_error;

using sdp_host::SdpError;
using sdp_host::fail;

void hip_check(hipError_t e, const char *what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(SDP_ERR_OOM, std::string(what) + ": " + hipGetErrorString(e));
  fail(SDP_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(x) hip_check((x), #x)

using sdp_host::HostInst;
using sdp_host::round_up;

template <typename T>
T *dev_upload(const std::vector<T> &v, std::vector<void *> &owned) {
  T *p = nullptr;
  const size_t bytes = std::max<size_t>(v.size(), 1) * sizeof(T);
  HIPCHK(hipMalloc((void **)&p, bytes));
  owned.push_back(p);
  if (!v.empty()) HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  // the copy runs on the null stream, which does not order work on the
  // handle's non-blocking stream: wait for it before anything can read p
  HIPCHK(hipDeviceSynchronize());
  return p;
}

template <typename T>
T *dev_zeros(size_t count, std::vector<void *> &owned) {
  T *p = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  HIPCHK(hipMalloc((void **)&p, bytes));
  owned.push_back(p);
  HIPCHK(hipMemset(p, 0, bytes));
  HIPCHK(hipDeviceSynchronize());   // null-stream fill: see dev_upload
  return p;
}

// ---------------------------------------------------------------------------
// Autotuner: for one clique size, time every kernel variant that fits on
// synthetic symmetric blocks (min(count, 4096) of them, as many as the
// projection will see) and keep the fastest.  Decisions are cached per
// (precision, size, power-of-two count) for the life of the process.
// ---------------------------------------------------------------------------
std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int, int>, int> g_tune_cache;

// Times the candidate variants on synthetic blocks: nearly diagonal ones
// (off-diagonal entries scaled by 1e-3) when the solves are warm-started,
// which is the matrix such a solve diagonalises, else cold random ones.
// Variants that hold cliques of size s under projection method `method` (0
// any, 1 scalar only, 2 two-level when one fits, else scalar).
std::vector<int> fitting_variants(int precision, int s, int method) {
  const int n = s + (s & 1);
  std::vector<int> any, scalar, two;
  for (int v = 0; v < projection_variant_count(precision); ++v) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (N < n) continue;
    if (projection_variant_kind(precision, v) == 2) continue;   // no eigenvectors
    any.push_back(v);
    (projection_variant_two_level(precision, v) ? two : scalar).push_back(v);
  }
  if (method == 1) return scalar;
  if (method == 2 && !two.empty()) return two;
  if (method == 2) return scalar;
  return any;
}

// The untuned choice: the first listed variant of the smallest fitting N.
int default_variant(int precision, int s, int method) {
  const std::vector<int> c = fitting_variants(precision, s, method);
  int best = -1, bestN = 1 << 30;
  for (int v : c) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (N < bestN) {
      best = v;
      bestN = N;
    }
  }
  return best;
}

// The sign-function variant the solver's plan takes for cliques of s
// vertices: the register-resident kernels (one wave, N = 16 or 32) for
// s <= 32; in FP64 also the one-block LDS kernel (NT = 4N) of the smallest
// fitting N for 33-128 (measured against the warm-started Jacobi kernels:
// nonchordal workload FP64 1046 -> 1439 iter/s, batched 72.3 -> 75.8; in
// FP32 the Jacobi kernels and the decoupling stay faster, batched 93.4 ->
// 92.2 with the sign function for blocks of 48).  -1 otherwise.
int sign_variant(int precision, int s) {
  const bool big = precision == 0 && s > 32;
  if (s > 32 && !big) return -1;
  const int n = s + (s & 1);
  int best = -1, bestN = 1 << 30;
  for (int v = 0; v < projection_variant_count(precision); ++v) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (projection_variant_kind(precision, v) != 2 || N < n) continue;
    const bool ok = big ? (N >= 48 && NT == 4 * N) : (NT == 64 && (N == 16 || N == 32));
    if (ok && N < bestN) {
      best = v;
      bestN = N;
    }
  }
  return best;
}

// The sign-function variant that Algorithms 1 and 2 take for cliques of s
// vertices that no Jacobi variant holds (FP64, 97-128), -1 if none.
int big_sign_variant(int precision, int s) {
  for (int v = 0; v < projection_variant_count(precision); ++v) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (projection_variant_kind(precision, v) == 2 && precision == 0 && N == 128 && NT == 512 &&
        s <= N)
      return v;
  }
  return -1;
}

// Whether projection_method 0 takes the sign-function variants for
// Algorithm 1's cliques of up to 32 vertices: yes in both precisions (one
// MI355X: banded workload projection 22.0 -> 13.8 us FP32, 52.9 -> 36.4 us
// FP64; the batched workload's cliques of 10-50 1.27 -> 1.21 ms and 4.30 ->
// 4.23 ms).
bool sign_by_default(int) { return true; }

int tune_variant(int precision, int s, int64_t count, int max_sweeps, double tol, bool warm,
                 int method, hipStream_t st) {
  std::vector<int> cand = fitting_variants(precision, s, method);
  if (cand.empty()) fail(SDP_ERR_UNSUPPORTED, "clique too large");
  // variants beyond the next-larger block size are never faster
  int nmin = 1 << 30;
  for (int v : cand) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    nmin = std::min(nmin, N);
  }
  std::vector<int> keep;
  for (int v : cand) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (N <= 2 * nmin) keep.push_back(v);
  }
  cand.swap(keep);
  if (cand.size() == 1) return cand[0];
  const int test = (int)std::min<int64_t>(count, 4096);
  int lg = 0;
  while ((1 << (lg + 1)) <= test) ++lg;
  const auto key = std::make_tuple(precision, s, lg, (warm ? 1 : 0) + 2 * method);
  {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) return it->second;
  }
  const size_t esz = precision == 1 ? sizeof(float) : sizeof(double);
  std::vector<int32_t> sizes(test, s);
  std::vector<int64_t> offs(test);
  for (int i = 0; i < test; ++i) offs[i] = (int64_t)i * s * s;
  std::vector<void *> tmp;
  int best = cand[0];
  try {
    void *in = nullptr, *out = nullptr;
    HIPCHK(hipMalloc(&in, esz * (size_t)test * s * s));
    tmp.push_back(in);
    HIPCHK(hipMalloc(&out, esz * (size_t)test * s * s));
    tmp.push_back(out);
    int32_t *d_sizes = dev_upload(sizes, tmp);
    int64_t *d_offs = dev_upload(offs, tmp);
    HIPCHK(fill_random_blocks(precision, in, s, test, 0x5eedu + (uint32_t)s, warm ? 1e-3 : 1.0,
                              st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // best of three timings of three launches each; a variant replaces the
    // default only when it is at least 5% faster (keeps the choice stable)
    const int def = default_variant(precision, s, method);
    float def_ms = 1e30f, best_ms = 1e30f;
    for (int v : cand) {
      HIPCHK(launch_standalone_projection(precision, v, test, d_sizes, d_offs, in, out, max_sweeps,
                                          tol, st));
      float vms = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r)
          HIPCHK(launch_standalone_projection(precision, v, test, d_sizes, d_offs, in, out,
                                              max_sweeps, tol, st));
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        vms = std::min(vms, ms);
      }
      if (v == def) def_ms = vms;
      if (vms < best_ms) {
        best_ms = vms;
        best = v;
      }
    }
    if (def_ms < 1e30f && best != def && best_ms > 0.95f * def_ms) best = def;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } catch (...) {
    for (void *q : tmp) (void)hipFree(q);
    throw;
  }
  for (void *q : tmp) (void)hipFree(q);
  std::lock_guard<std::mutex> g(g_tune_mutex);
  g_tune_cache[key] = best;
  return best;
}

}  // namespace

struct sdp_handle {
  int B = 0;
  sdp_options opt{};
  int precision = 0;
  int max_sweeps = 30;
  double jac_tol = 1e-6;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t cap_stream = nullptr;
  std::vector<void *> owned;
  std::vector<InstDesc> desc;
  std::vector<int64_t> npk_off;          // per instance, packed offset of its first clique
  std::vector<int64_t> inst_npk;
  std::vector<int32_t> inst_p;
  int64_t ncoord = 0, nrow = 0, npk = 0, ncl = 0;
  InstDesc *d_desc = nullptr;
  InstState *d_state = nullptr;
  InstState *h_state = nullptr;          // pinned
  double *d_obj = nullptr;
  double *h_obj = nullptr;               // pinned
  AffineArgs aff{};
  ProjArgs proj{};
  std::vector<int> bucket_size;          // kernel variant of each launch list
  std::vector<int> bucket_N;             // its padded block size
  std::vector<int> clique_N;             // padded block size of every clique
  std::vector<int64_t> cl_first;         // per instance, first global clique (B + 1)
  int32_t *d_clique_N = nullptr;
  int64_t *d_vw_off = nullptr;
  void *d_vw = nullptr;                  // warm-start bases (precision of the eigen-solve)
  int32_t *d_t_rows_all = nullptr;       // (inst, row) over every row
  int n_t_rows_all = 0;
  double *d_ytmp = nullptr;              // row-space scratch for the scaled multiplier
  double *d_utmp = nullptr;              // coordinate scratch (Algorithm 2: -rho x)
  // affine step by conjugate gradients (no factor)
  bool cg = false;
  std::vector<double> cg_tol2;           // per instance (cg_tol (1 + ||b||))^2
  // Algorithm 3
  bool hsde = false;
  HsdeArgs hsa{};
  HsdeState *d_hs = nullptr;
  std::vector<HsdeState> h_hs;
  std::vector<int32_t *> bucket_list;
  std::vector<int> bucket_count;
  // per bucket: the workspace of the split sign iteration (a few large FP64
  // cliques, split_projection), else nullptr
  std::vector<double *> bucket_ws;
  // Buckets of different block sizes run concurrently: bucket_order[0] (the
  // largest block size, the longest per-clique latency) is enqueued first on
  // an auxiliary stream forked from the iteration's stream, the others after
  // it, the last on the iteration's stream itself; then everything joins.
  std::vector<int> bucket_order;
  std::vector<hipStream_t> aux_stream;   // bucket_order.size() - 1 of them
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  hipGraphExec_t graph = nullptr;
  int graph_iters = 0;
  int hist_cap = 0;
  bool have_diag = false;
  std::vector<double> diag;              // 4 per instance
  double *d_diag = nullptr;
  DiagScratch dscr{};
  int64_t iters_enqueued = 0;
  // unrolled differentiation
  std::vector<int64_t> user_coord_off, user_row_off;   // caller's concatenated layout
  int64_t user_ncoord = 0, user_nrow = 0;
  int64_t *d_user_coord_off = nullptr, *d_user_row_off = nullptr;
  int32_t *d_row_inst = nullptr;
  int64_t *d_eig_off = nullptr;
  int64_t eig_total = 0;                 // elements of one iteration's (V, theta) records
  bool adj_ready = false;                // every bucket has an adjoint kernel
  int adj_T = 0, adj_ckpt = 0;
  double *d_ckpt = nullptr;              // [nseg][2][npk]: X, Lambda at segment starts
  int64_t ckpt_cap = 0;
  void *d_eigbuf = nullptr;              // [ckpt][eig_total]
  int64_t eigbuf_cap = 0;
  double *d_Xb = nullptr, *d_Lb = nullptr, *d_Ub = nullptr;
  double *d_bhat_bar = nullptr, *d_v_bar = nullptr, *d_bhb = nullptr;
  double *d_r_bar = nullptr, *d_y1_bar = nullptr, *d_y_bar = nullptr, *d_zero_rows = nullptr;
};

namespace {

void enqueue_projections(sdp_handle *h, const ProjArgs &p, hipStream_t st) {
  const size_t nb = h->bucket_order.size();
  if (nb <= 1 || h->aux_stream.size() + 1 != nb) {
    for (size_t b = 0; b < h->bucket_size.size(); ++b)
      HIPCHK(launch_admm_projection(h->precision, h->bucket_size[b], h->bucket_list[b],
                                    h->bucket_count[b], p, st, h->bucket_ws[b]));
    return;
  }
  // fork: every bucket but the last on its own stream, ordered after st
  HIPCHK(hipEventRecord(h->ev_fork, st));
  for (size_t i = 0; i + 1 < nb; ++i) {
    const int b = h->bucket_order[i];
    HIPCHK(hipStreamWaitEvent(h->aux_stream[i], h->ev_fork, 0));
    HIPCHK(launch_admm_projection(h->precision, h->bucket_size[b], h->bucket_list[b],
                                  h->bucket_count[b], p, h->aux_stream[i], h->bucket_ws[b]));
    HIPCHK(hipEventRecord(h->ev_join[i], h->aux_stream[i]));
  }
  const int last = h->bucket_order[nb - 1];
  HIPCHK(launch_admm_projection(h->precision, h->bucket_size[last], h->bucket_list[last],
                                h->bucket_count[last], p, st, h->bucket_ws[last]));
  // join: st continues only after every bucket
  for (size_t i = 0; i + 1 < nb; ++i) HIPCHK(hipStreamWaitEvent(st, h->ev_join[i], 0));
}

// Algorithm 1: x-update (affine), projections with the multiplier update,
// residuals.  Algorithm 2: z-update (projections), (y, x) from the KKT
// system, v and multiplier updates, residuals.
void enqueue_hsde_iteration(sdp_handle *h, hipStream_t st);

// Algorithm 1 with a fixed penalty: the scatter kernel of an iteration can
// also finish the previous one (the penalty it reads cannot change).
bool can_fold_residual(const sdp_handle *h) {
  return !h->hsde && !h->proj.dual && !h->opt.adaptive_rho;
}

// fold_prev: this iteration's scatter kernel also finishes the previous
// iteration (whose residual kernel was left out); defer: leave this
// iteration's residual kernel out (the next iteration folds it).  A sequence
// of iterations is enqueued with fold_prev = (not first), defer = (not last),
// so the state is complete after it.
void enqueue_iteration(sdp_handle *h, hipStream_t st, bool fold_prev = false, bool defer = false) {
  if (h->hsde) {
    enqueue_hsde_iteration(h, st);
    return;
  }
  if (h->proj.dual) {
    enqueue_projections(h, h->proj, st);
    HIPCHK(launch_iteration_affine(h->aff, st));
    HIPCHK(launch_dual_update(h->proj, h->ncl, st));
  } else {
    AffineArgs a = h->aff;
    if (fold_prev) a.res_blocks = (h->B + 7) / 8 * 8;
    if (h->cg) HIPCHK(launch_cg_affine(a, st));
    else HIPCHK(launch_iteration_affine(a, st));
    enqueue_projections(h, h->proj, st);
  }
  if (!defer) HIPCHK(launch_residual_reduce(h->aff, st));
}

// n iterations, the residual kernels folded into the next scatter where allowed
void enqueue_sequence(sdp_handle *h, hipStream_t st, int64_t n) {
  const bool fold = can_fold_residual(h);
  for (int64_t i = 0; i < n; ++i) enqueue_iteration(h, st, fold && i > 0, fold && i + 1 < n);
}

// One unrolled iteration (no stopping test); optionally stores (V, theta).
void enqueue_unrolled_iteration(sdp_handle *h, hipStream_t st, void *eig) {
  AffineArgs a = h->aff;
  a.params.no_stop = 1;
  a.ignore_done = 1;
  ProjArgs p = h->proj;
  p.eig = eig;
  p.eig_off = h->d_eig_off;
  p.vw = nullptr;          // the reverse sweep recomputes segments: no cross-iteration state
  HIPCHK(launch_iteration_affine(a, st));
  // always the Jacobi kernels (the sign-function lists of the plan take the
  // Jacobi default of their block size): the recomputed segments record
  // eigenvectors, and the first pass must compute the same iterates bit for
  // bit, or the checkpoint spacing would change the result
  for (size_t b = 0; b < h->bucket_size.size(); ++b) {
    int v = h->bucket_size[b];
    if (projection_variant_kind(h->precision, v) == 2)
      v = projection_default_variant(h->precision, h->bucket_N[b]);
    if (v < 0) fail(SDP_ERR_UNSUPPORTED, "no eigenvector kernel for this block size");
    HIPCHK(launch_admm_projection(h->precision, v, h->bucket_list[b], h->bucket_count[b], p, st));
  }
  HIPCHK(launch_residual_reduce(a, st));
}

// y = L^-T y1 for every row (with B = L^-1 A formed, the iteration keeps only y1).
void ensure_y(sdp_handle *h) {
  if (h->cg) return;          // the solve keeps y itself
  AffineArgs a = h->aff;
  a.t3_rows = h->d_t_rows_all;
  a.n_t3_rows = h->n_t_rows_all;
  a.ignore_done = 1;
  HIPCHK(launch_affine_stage(a, 3, h->stream));
}

// bp = L^-1 b (needed with B = L^-1 A)
void compute_bp(sdp_handle *h) {
  if (!h->aff.Bm) return;
  AffineArgs a = h->aff;
  a.r = const_cast<double *>(h->aff.b);
  a.y1 = const_cast<double *>(h->aff.bp);
  a.t_rows = h->d_t_rows_all;
  a.n_t_rows = h->n_t_rows_all;
  a.ignore_done = 1;
  HIPCHK(launch_affine_stage(a, 2, h->stream));
}

// Algorithm 3 set-up: buffers, then M^-1 zeta by one inner solve of nu = zeta
// = (c, 0, -b, 0) through the same kernels as the iteration.
void setup_hsde(sdp_handle *h, const std::vector<double> &D) {
  auto &own = h->owned;
  HsdeArgs &g = h->hsa;
  AffineArgs &a = h->aff;
  ProjArgs &p = h->proj;
  h->hsde = true;
  g.inst = h->d_desc;
  g.state = h->d_state;
  g.params = a.params;
  g.batch = h->B;
  g.ncoord = h->ncoord;
  g.coord_inst = a.coord_inst;
  g.c = a.c;
  g.w = a.w;
  std::vector<double> P(D.size());
  for (size_t j = 0; j < D.size(); ++j) P[j] = 1.0 + 0.5 * D[j];
  g.P = dev_upload(P, own);
  g.contrib_ptr = a.contrib_ptr;
  g.contrib_idx = a.contrib_idx;
  g.ux = dev_zeros<double>(h->ncoord, own);
  g.nx = dev_zeros<double>(h->ncoord, own);
  g.xp = a.bhat;
  g.v = a.v;
  g.sx = a.u;
  g.mzx = dev_zeros<double>(h->ncoord, own);
  g.atmz = dev_zeros<double>(h->ncoord, own);
  g.nrow = h->nrow;
  g.row_inst = h->d_row_inst;
  g.b = a.b;
  g.uy = dev_zeros<double>(h->nrow, own);
  g.ny = dev_zeros<double>(h->nrow, own);
  g.g = a.y;
  g.mzy = dev_zeros<double>(h->nrow, own);
  g.az = dev_zeros<double>(h->nrow, own);
  g.npk = h->npk;
  g.blk_loc = p.blk_loc;
  g.us = p.X;
  g.vz = p.Lam;
  const int64_t pk = std::max<int64_t>(h->npk, 1);
  g.ut = dev_zeros<double>(pk, own);
  g.ns = dev_zeros<double>(pk, own);
  g.nt = dev_zeros<double>(pk, own);
  g.mzs = dev_zeros<double>(pk, own);
  g.mzt = dev_zeros<double>(pk, own);
  g.cw_part = dev_zeros<double>((size_t)(h->ncoord / 64 + 1) * 4, own);
  g.rw_part = dev_zeros<double>((size_t)(h->nrow / 64 + 1) * 4, own);
  g.part = p.part;
  g.inst_cl_first = a.inst_cl_first;
  g.hist = a.hist;
  h->d_hs = dev_zeros<HsdeState>(h->B, own);
  h->h_hs.assign(h->B, HsdeState{});
  g.hs = h->d_hs;
  // the affine stages of the inner solve: r = A (w x'/P) - nu_y, g = L^-T L^-1 r,
  // sigma_x = (x' - A^T g) / P
  a.b = g.ny;
  a.D = g.P;
  // the projection in embedding mode
  p.hsde = 1;
  p.hs = h->d_hs;
  p.h_ns = g.ns;
  p.h_nt = g.nt;
  p.h_sx = g.sx;
  p.h_ux = g.ux;
  p.h_mzs = g.mzs;
  p.h_mzt = g.mzt;
  p.h_ut = g.ut;
  // M^-1 zeta
  g.ignore_done = 1;
  AffineArgs as = a;
  as.ignore_done = 1;
  HIPCHK(launch_hsde_setup_nu(g, h->stream));
  HIPCHK(launch_hsde_xprime(g, g.nx, g.ns, g.nt, h->stream));
  for (int stg = 1; stg <= 4; ++stg) HIPCHK(launch_affine_stage(as, stg, h->stream));
  HIPCHK(launch_hsde_setup_finish(g, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  g.ignore_done = 0;
}

void enqueue_hsde_iteration(sdp_handle *h, hipStream_t st) {
  const HsdeArgs &g = h->hsa;
  HIPCHK(launch_hsde_form_nu(g, st));
  HIPCHK(launch_hsde_xprime(g, g.nx, g.ns, g.nt, st));
  for (int stg = 1; stg <= 4; ++stg) HIPCHK(launch_affine_stage(h->aff, stg, st));
  HIPCHK(launch_hsde_update(g, st));
  enqueue_projections(h, h->proj, st);
  HIPCHK(launch_hsde_finish(g, st));
}

void build_graph(sdp_handle *h) {
  if (h->graph || h->opt.graph_chunk <= 0) return;
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue_sequence(h, h->cap_stream, h->opt.graph_chunk);
  } catch (...) {
    hipGraph_t dummy;
    (void)hipStreamEndCapture(h->cap_stream, &dummy);
    if (dummy) (void)hipGraphDestroy(dummy);
    throw;
  }
  HIPCHK(hipStreamEndCapture(h->cap_stream, &g));
  HIPCHK(hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0));
  HIPCHK(hipGraphDestroy(g));
  h->graph_iters = h->opt.graph_chunk;
}

void enqueue_steps(sdp_handle *h, int64_t n) {
  if (h->opt.graph_chunk > 0 && n >= h->opt.graph_chunk) {
    build_graph(h);
    while (n >= h->graph_iters) {
      HIPCHK(hipGraphLaunch(h->graph, h->stream));
      n -= h->graph_iters;
    }
  }
  enqueue_sequence(h, h->stream, n);
}

void pull_state(sdp_handle *h) {
  HIPCHK(hipMemcpyAsync(h->h_state, h->d_state, sizeof(InstState) * h->B, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
}

void ensure_y(sdp_handle *h);

void fill_results(sdp_handle *h, sdp_result *res) {
  if (h->hsde) {
    HIPCHK(hipMemcpyAsync(h->h_hs.data(), h->d_hs, sizeof(HsdeState) * h->B,
                          hipMemcpyDeviceToHost, h->stream));
    pull_state(h);
    for (int i = 0; i < h->B; ++i) {
      const InstState &s = h->h_state[i];
      const HsdeState &q = h->h_hs[i];
      sdp_result &r = res[i];
      r.iters = s.iter;
      r.status = s.done == 1 ? SDP_OK
                 : s.done == 3 ? SDP_PRIMAL_INFEASIBLE
                 : s.done == 4 ? SDP_DUAL_INFEASIBLE : SDP_MAX_ITER;
      r.eps_c = s.eps_c;
      r.eps_lambda = s.eps_l;
      r.objective = q.tau > 0 ? q.ctx / q.tau : NAN;
      r.rho = q.tau;
      r.eps_p = q.eps_p;
      r.eps_d = q.eps_d;
      r.eps_g = q.eps_g;
      r.eps_alpha = NAN;
    }
    return;
  }
  if (h->aff.dual) ensure_y(h);   // the dual objective b^T y
  HIPCHK(launch_objective(h->aff, h->d_obj, h->stream));
  HIPCHK(hipMemcpyAsync(h->h_obj, h->d_obj, sizeof(double) * h->B, hipMemcpyDeviceToHost,
                        h->stream));
  pull_state(h);
  for (int i = 0; i < h->B; ++i) {
    const InstState &s = h->h_state[i];
    sdp_result &r = res[i];
    r.iters = s.iter;
    r.status = s.done == 1 ? SDP_OK : SDP_MAX_ITER;
    r.eps_c = s.eps_c;
    r.eps_lambda = s.eps_l;
    r.objective = h->h_obj[i];
    r.rho = s.rho;
    if (h->have_diag) {
      r.eps_p = h->diag[4 * i + 0];
      r.eps_d = h->diag[4 * i + 1];
      r.eps_g = h->diag[4 * i + 2];
      r.eps_alpha = h->diag[4 * i + 3];
    } else {
      r.eps_p = r.eps_d = r.eps_g = r.eps_alpha = NAN;
    }
  }
}

void reset_state(sdp_handle *h) {
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<InstState> st(h->B);
  for (auto &s : st) {
    std::memset(&s, 0, sizeof(s));
    s.rho = h->opt.rho;
    s.eps_c = s.eps_l = INFINITY;
  }
  // every fill below is ordered on the handle's stream (a null-stream fill
  // would not be ordered with the non-blocking stream's kernels)
  HIPCHK(hipMemcpyAsync(h->d_state, st.data(), sizeof(InstState) * h->B, hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(hipMemsetAsync(h->proj.X, 0, sizeof(double) * std::max<int64_t>(h->npk, 1), h->stream));
  HIPCHK(hipMemsetAsync(h->proj.Lam, 0, sizeof(double) * std::max<int64_t>(h->npk, 1), h->stream));
  // the per-clique partial-sum records, including the decoupling's back-off
  // counter (slot 7), start from zero as in a fresh handle
  HIPCHK(hipMemsetAsync(h->proj.part, 0, sizeof(double) * NPART * std::max<int64_t>(h->ncl, 1),
                        h->stream));
  HIPCHK(hipMemsetAsync(h->aff.u, 0, sizeof(double) * h->ncoord, h->stream));
  HIPCHK(hipMemsetAsync(h->aff.y, 0, sizeof(double) * h->nrow, h->stream));
  if (h->cg) {
    HIPCHK(hipMemsetAsync(h->aff.cg_g, 0, sizeof(double) * h->ncoord, h->stream));
    HIPCHK(hipMemsetAsync(h->aff.cg, 0, sizeof(CgState) * h->B, h->stream));
  }
  if (h->proj.Vd)
    HIPCHK(hipMemsetAsync(h->proj.Vd, 0, sizeof(double) * std::max<int64_t>(h->npk, 1), h->stream));
  if (h->hsde) {
    HIPCHK(hipMemsetAsync(h->hsa.ux, 0, sizeof(double) * h->ncoord, h->stream));
    HIPCHK(hipMemsetAsync(h->hsa.uy, 0, sizeof(double) * h->nrow, h->stream));
    HIPCHK(hipMemsetAsync(h->hsa.ut, 0, sizeof(double) * std::max<int64_t>(h->npk, 1), h->stream));
    HIPCHK(launch_hsde_reset(h->hsa, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->d_vw) {
    HIPCHK(launch_identity_bases(h->precision, h->d_vw, h->d_vw_off, h->d_clique_N, 0, h->ncl,
                                 h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
  }
  h->have_diag = false;
  h->iters_enqueued = 0;
}

void destroy_handle(sdp_handle *h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  for (hipStream_t a : h->aux_stream) (void)hipStreamSynchronize(a);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  for (void *p : h->owned) (void)hipFree(p);
  if (h->d_ckpt) (void)hipFree(h->d_ckpt);
  if (h->d_eigbuf) (void)hipFree(h->d_eigbuf);
  if (h->h_state) (void)hipHostFree(h->h_state);
  if (h->h_obj) (void)hipHostFree(h->h_obj);
  for (hipStream_t a : h->aux_stream) (void)hipStreamDestroy(a);
  for (hipEvent_t e : h->ev_join) (void)hipEventDestroy(e);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
}

void setup_impl(int32_t batch, const sdp_instance *inst, const sdp_options *opt_in,
                sdp_handle **out) {
  if (!out) fail(SDP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (batch <= 0 || !inst) fail(SDP_ERR_ARG, "batch must be positive");
  sdp_options opt;
  sdp_default_options(&opt);
  if (opt_in) opt = *opt_in;
  if (!(opt.rho > 0) || !(opt.tol >= 0) || opt.max_iter <= 0 ||
      (opt.precision != SDP_FP64 && opt.precision != SDP_FP32_EIG) ||
      (opt.algorithm != SDP_ALG_PRIMAL && opt.algorithm != SDP_ALG_DUAL &&
       opt.algorithm != SDP_ALG_HSDE) ||
      (opt.algorithm == SDP_ALG_HSDE && opt.adaptive_rho) ||
      (opt.adaptive_rho && (!(opt.mu >= 1) || !(opt.nu >= 1) || opt.rho_period <= 0)) ||
      opt.graph_chunk < 0 || opt.cg_max_iter < 0 || !(opt.cg_tol >= 0) ||
      opt.projection_method < 0 || opt.projection_method > 3 || opt.decouple < 0 ||
      opt.decouple > 1)
    fail(SDP_ERR_ARG, "invalid options");
  if (opt.cg_max_iter > 0 && opt.algorithm != SDP_ALG_PRIMAL)
    fail(SDP_ERR_UNSUPPORTED, "the conjugate-gradient affine step is built for Algorithm 1 only");

  // ---- validation and host indices (nothing touches the GPU before this) ----
  std::vector<HostInst> H(batch);
  for (int i = 0; i < batch; ++i) {
    try {
      sdp_host::validate_and_index(inst[i], projection_max_size(opt.precision), H[i]);
    } catch (SdpError &e) {
      throw SdpError(e.code, "instance " + std::to_string(i) + ": " + e.what());
    }
  }

  sdp_handle *h = new sdp_handle();
  try {
    h->B = batch;
    h->opt = opt;
    h->precision = opt.precision;
    h->max_sweeps = opt.jacobi_max_sweeps > 0 ? opt.jacobi_max_sweeps
                                              : (opt.precision == SDP_FP32_EIG ? 30 : 40);
    h->jac_tol = opt.jacobi_tol > 0 ? opt.jacobi_tol : (opt.precision == SDP_FP32_EIG ? 1e-6 : 1e-14);
    if (opt.stream) {
      h->stream = (hipStream_t)opt.stream;
    } else {
      HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
      h->own_stream = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));

    // ---- global layout ----
    h->desc.resize(batch);
    int64_t coord = 0, row = 0, aoff = 0, toff = 0, cl = 0, pk = 0, csr_ptr_off = 0;
    int max_ldm = 0;
    for (int i = 0; i < batch; ++i) {
      InstDesc &d = h->desc[i];
      const HostInst &hi = H[i];
      d.n = hi.n; d.m = hi.m; d.p = hi.p; d.a_format = hi.fmt;
      d.ld = hi.ld; d.ldm = hi.ldm; d.nnz = hi.nnz;
      d.coord_off = coord; d.row_off = row; d.t_off = toff; d.clique_off = cl;
      if (hi.fmt == SDP_A_DENSE) {
        d.a_off = aoff;
        aoff += (int64_t)hi.m * hi.ld;
      } else {
        d.a_off = csr_ptr_off;          // row pointer block of m+1 entries
        csr_ptr_off += hi.m + 1;
      }
      coord += hi.ld;
      row += hi.ldm;
      toff += (int64_t)hi.ldm * hi.ldm;
      cl += hi.p;
      h->npk_off.push_back(pk);
      h->inst_npk.push_back(hi.npk);
      h->inst_p.push_back(hi.p);
      pk += hi.npk;
      max_ldm = std::max(max_ldm, hi.ldm);
    }
    h->ncoord = coord; h->nrow = row; h->npk = pk; h->ncl = cl;
    if (pk >= ((int64_t)1 << 31)) fail(SDP_ERR_UNSUPPORTED, "too many packed clique entries");

    // ---- coordinate-space arrays ----
    std::vector<int32_t> coord_inst(coord);
    std::vector<double> c(coord, 0.0), D(coord, 1.0), w(coord, 0.0), wd(coord, 0.0);
    std::vector<int64_t> cptr(coord + 1, 0);
    for (int i = 0; i < batch; ++i) {
      const InstDesc &d = h->desc[i];
      const HostInst &hi = H[i];
      for (int64_t j = 0; j < d.ld; ++j) coord_inst[d.coord_off + j] = i;
      for (int64_t j = 0; j < hi.nnz; ++j) {
        const int64_t g = d.coord_off + j;
        c[g] = inst[i].c[j];
        D[g] = (double)hi.D[j];
        w[g] = inst[i].pat_row[j] == inst[i].pat_col[j] ? 1.0 : 2.0;
        // Algorithm 3 factors I + A W P^-1 A^T with P = I + D/2
        wd[g] = opt.algorithm == SDP_ALG_HSDE ? w[g] / (1.0 + 0.5 * D[g]) : w[g] / D[g];
        cptr[g + 1] = hi.D[j];
      }
    }
    for (int64_t g = 0; g < coord; ++g) cptr[g + 1] += cptr[g];
    std::vector<int32_t> cidx(cptr[coord]);
    {
      std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
      for (int i = 0; i < batch; ++i)
        for (int64_t e = 0; e < H[i].npk; ++e) {
          const int64_t g = h->desc[i].coord_off + H[i].blk_loc[e];
          cidx[fill[g]++] = (int32_t)(h->npk_off[i] + e);
        }
    }
    // ---- clique arrays ----
    std::vector<int32_t> cl_inst(cl), cl_size(cl), blk_loc(pk);
    std::vector<int64_t> cl_off(cl), cl_first(batch + 1);
    {
      int64_t k = 0;
      for (int i = 0; i < batch; ++i) {
        cl_first[i] = k;
        for (int q = 0; q < H[i].p; ++q, ++k) {
          cl_inst[k] = i;
          cl_size[k] = inst[i].clique_ptr[q + 1] - inst[i].clique_ptr[q];
          cl_off[k] = h->npk_off[i] + H[i].cl_off[q];
        }
        for (int64_t e = 0; e < H[i].npk; ++e)
          blk_loc[h->npk_off[i] + e] = (int32_t)(h->desc[i].coord_off + H[i].blk_loc[e]);
      }
      cl_first[batch] = k;
    }
    // kernel variant per clique size (autotuned or default), one launch list
    // per variant
    std::vector<std::vector<int32_t>> lists;
    {
      std::map<int, int64_t> count_of_size;
      for (int64_t k = 0; k < cl; ++k) count_of_size[cl_size[k]]++;
      std::map<int, int> var_of_size;
      // cliques of up to 32 vertices (FP64: all): the sign-function
      // variants (no eigenvectors) where selected
      const bool sign_lists = opt.projection_method == 3 ||
                              (opt.projection_method == 0 && sign_by_default(h->precision));
      // with the decoupling (FP32, warm start) the large blocks take the
      // scalar variants, which carry it
      const int pm = opt.projection_method == 3 ? 0 : opt.projection_method;
      const int method = (opt.decouple && opt.warm_start && h->precision == SDP_FP32_EIG &&
                          pm == 0)
                             ? 1
                             : pm;
      for (auto &kv : count_of_size) {
        int sv = sign_lists ? sign_variant(h->precision, kv.first) : -1;
        if (fitting_variants(h->precision, kv.first, 0).empty()) {
          // FP64 cliques of 97-128: the sign-function kernel is the only one
          sv = big_sign_variant(h->precision, kv.first);
          if (sv < 0) fail(SDP_ERR_UNSUPPORTED, "clique too large");
        }
        var_of_size[kv.first] =
            sv >= 0 ? sv
            : opt.autotune ? tune_variant(h->precision, kv.first, kv.second, h->max_sweeps,
                                          h->jac_tol, opt.warm_start != 0, method, h->stream)
                           : default_variant(h->precision, kv.first, method);
      }
      for (int64_t k = 0; k < cl; ++k) {
        const int v = var_of_size[cl_size[k]];
        auto it = std::find(h->bucket_size.begin(), h->bucket_size.end(), v);
        size_t bi;
        if (it == h->bucket_size.end()) {
          h->bucket_size.push_back(v);
          int N, NT;
          projection_variant_info(h->precision, v, &N, &NT);
          h->bucket_N.push_back(N);
          lists.emplace_back();
          bi = lists.size() - 1;
        } else {
          bi = it - h->bucket_size.begin();
        }
        lists[bi].push_back((int32_t)k);
      }
      h->clique_N.resize(cl);
      for (int64_t k = 0; k < cl; ++k) {
        int N, NT;
        projection_variant_info(h->precision, var_of_size[cl_size[k]], &N, &NT);
        h->clique_N[k] = N;
      }
    }
    // ---- row-space arrays ----
    std::vector<double> b(row, 0.0);
    for (int i = 0; i < batch; ++i)
      for (int r = 0; r < H[i].m; ++r) b[h->desc[i].row_off + r] = inst[i].b[r];

    // ---- tiles ----
    int64_t dense_rows = 0;
    for (int i = 0; i < batch; ++i)
      if (H[i].fmt == SDP_A_DENSE) dense_rows += H[i].m;
    auto pick_r = [](int64_t rows) {
      int r = 1;
      while (r < affine_max_rows_per_tile() && rows / (2 * r) >= 2048) r *= 2;
      return r;
    };
    const int R = pick_r(dense_rows);
    const int CW = affine_col_tile_width();
    std::vector<int32_t> row_tiles, col_tiles, t_rows, csr_rows, csc_cols, syrk_tiles, syrk_rows;
    std::vector<int32_t> t_rows_all, b_tiles;
    for (int i = 0; i < batch; ++i) {
      const HostInst &hi = H[i];
      for (int r = 0; r < hi.m; ++r) { t_rows_all.push_back(i); t_rows_all.push_back(r); }
      if (hi.fmt != SDP_A_DENSE)
        for (int r = 0; r < hi.m; ++r) { t_rows.push_back(i); t_rows.push_back(r); }
      if (hi.fmt == SDP_A_DENSE) {
        for (int ti = 0; ti < (hi.m + 63) / 64; ++ti)
          for (int tj = 0; tj < hi.ld / 64; ++tj) {
            b_tiles.push_back(i); b_tiles.push_back(ti); b_tiles.push_back(tj);
          }
        for (int r = 0; r < hi.m; r += R) { row_tiles.push_back(i); row_tiles.push_back(r); }
        for (int cc = 0; cc < hi.ld; cc += CW) { col_tiles.push_back(i); col_tiles.push_back(cc); }
        for (int ti = 0; ti < hi.ldm / 64; ++ti)
          for (int tj = 0; tj <= ti; ++tj) {
            syrk_tiles.push_back(i); syrk_tiles.push_back(ti); syrk_tiles.push_back(tj);
          }
      } else {
        for (int r = 0; r < hi.m; ++r) {
          csr_rows.push_back(i); csr_rows.push_back(r);
          syrk_rows.push_back(i); syrk_rows.push_back(r);
        }
        for (int cc = 0; cc < hi.ld; cc += affine_csc_tile_width()) {
          csc_cols.push_back(i);
          csc_cols.push_back(cc);
        }
      }
    }
    const bool cg = opt.cg_max_iter > 0;
    if (!cg && max_ldm * sizeof(double) > 160 * 1024 && !syrk_rows.empty())
      fail(SDP_ERR_UNSUPPORTED, "sparse A with m > 20480 needs the conjugate-gradient affine step");

    // ---- CSR and CSC of sparse A ----
    std::vector<int64_t> a_rowptr, a_colptr;
    std::vector<int32_t> a_col, a_row;
    std::vector<double> a_val, a_cval;
    bool any_csr = !csr_rows.empty();
    if (any_csr) {
      a_colptr.assign(coord + 1, 0);
      for (int i = 0; i < batch; ++i) {
        if (H[i].fmt != SDP_A_CSR) continue;
        const sdp_instance &I = inst[i];
        const int64_t base = (int64_t)a_val.size();
        for (int r = 0; r <= I.m; ++r) a_rowptr.push_back(base + I.a_rowptr[r]);
        const int64_t annz = I.a_rowptr[I.m];
        a_col.insert(a_col.end(), I.a_col, I.a_col + annz);
        a_val.insert(a_val.end(), I.a_val, I.a_val + annz);
        for (int64_t t = 0; t < annz; ++t) a_colptr[h->desc[i].coord_off + I.a_col[t] + 1]++;
      }
      for (int64_t g = 0; g < coord; ++g) a_colptr[g + 1] += a_colptr[g];
      a_row.resize(a_colptr[coord]);
      a_cval.resize(a_colptr[coord]);
      std::vector<int64_t> fill(a_colptr.begin(), a_colptr.end() - 1);
      for (int i = 0; i < batch; ++i) {
        if (H[i].fmt != SDP_A_CSR) continue;
        const sdp_instance &I = inst[i];
        for (int r = 0; r < I.m; ++r)
          for (int64_t t = I.a_rowptr[r]; t < I.a_rowptr[r + 1]; ++t) {
            const int64_t pos = fill[h->desc[i].coord_off + I.a_col[t]]++;
            a_row[pos] = r;
            a_cval[pos] = I.a_val[t];
          }
      }
    }

    // ---- device allocation and upload ----
    auto &own = h->owned;
    h->d_desc = dev_upload(h->desc, own);
    h->d_state = dev_zeros<InstState>(batch, own);
    HIPCHK(hipHostMalloc((void **)&h->h_state, sizeof(InstState) * batch, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&h->h_obj, sizeof(double) * batch, hipHostMallocDefault));
    h->d_obj = dev_zeros<double>(batch, own);
    double *d_A = nullptr;
    if (aoff > 0) {
      d_A = dev_zeros<double>(aoff, own);
      for (int i = 0; i < batch; ++i) {
        if (H[i].fmt != SDP_A_DENSE) continue;
        const InstDesc &d = h->desc[i];
        HIPCHK(hipMemcpy2D(d_A + d.a_off, sizeof(double) * d.ld, inst[i].a_val,
                           sizeof(double) * d.nnz, sizeof(double) * d.nnz, d.m,
                           hipMemcpyHostToDevice));
      }
    }
    // the factor's inverse triangles (none with conjugate gradients)
    double *d_T = cg ? nullptr : dev_zeros<double>(toff, own);
    double *d_U = cg ? nullptr : dev_zeros<double>(toff, own);
    double *d_wd = dev_upload(wd, own);

    AffineArgs &a = h->aff;
    a.inst = h->d_desc;
    a.state = h->d_state;
    a.params.tol = opt.tol;
    a.params.mu = opt.mu;
    a.params.nu = opt.nu;
    a.params.max_iter = opt.max_iter;
    a.params.adaptive = opt.adaptive_rho;
    a.params.rho_period = opt.rho_period;
    h->hist_cap = std::min(opt.max_iter, 100000);
    a.params.hist_cap = h->hist_cap;
    a.coord_inst = dev_upload(coord_inst, own);
    a.c = dev_upload(c, own);
    a.D = dev_upload(D, own);
    a.w = dev_upload(w, own);
    a.bhat = dev_zeros<double>(coord, own);
    a.v = dev_zeros<double>(coord, own);
    a.u = dev_zeros<double>(coord, own);
    a.contrib_ptr = dev_upload(cptr, own);
    a.contrib_idx = dev_upload(cidx, own);
    a.ncoord = coord;
    a.b = dev_upload(b, own);
    a.r = dev_zeros<double>(row, own);
    a.y1 = dev_zeros<double>(row, own);
    a.y = dev_zeros<double>(row, own);
    a.A = d_A;
    // dense matrices beyond the 256 MB last-level cache stream with
    // non-temporal loads (each pass reads them once)
    a.stream_nt = (double)aoff * sizeof(double) > 256.0 * 1024 * 1024 ? 1 : 0;
    if (any_csr) {
      a.a_rowptr = dev_upload(a_rowptr, own);
      a.a_col = dev_upload(a_col, own);
      a.a_val = dev_upload(a_val, own);
      a.a_colptr = dev_upload(a_colptr, own);
      a.a_row = dev_upload(a_row, own);
      a.a_cval = dev_upload(a_cval, own);
    }
    a.T = d_T;
    a.U = d_U;
    a.row_tiles = dev_upload(row_tiles, own);
    a.n_row_tiles = (int)(row_tiles.size() / 2);
    a.rows_per_tile = R;
    a.col_tiles = dev_upload(col_tiles, own);
    a.n_col_tiles = (int)(col_tiles.size() / 2);
    a.t_rows = dev_upload(t_rows, own);
    a.n_t_rows = (int)(t_rows.size() / 2);
    a.t3_rows = a.t_rows;
    a.n_t3_rows = a.n_t_rows;
    h->d_t_rows_all = dev_upload(t_rows_all, own);
    h->n_t_rows_all = (int)(t_rows_all.size() / 2);
    h->d_ytmp = dev_zeros<double>(row, own);
    if (opt.algorithm == SDP_ALG_HSDE) {
      // the embedding solves with right-hand sides that change every
      // iteration on both sides of the factor: keep A and both triangular passes
      a.t_rows = a.t3_rows = h->d_t_rows_all;
      a.n_t_rows = a.n_t3_rows = h->n_t_rows_all;
    } else if (d_A && !cg) {
      a.Bm = dev_zeros<double>(aoff, own);
      a.bp = dev_zeros<double>(row, own);
    }
    a.csr_rows = dev_upload(csr_rows, own);
    a.n_csr_rows = (int)(csr_rows.size() / 2);
    a.csc_cols = dev_upload(csc_cols, own);
    a.n_csc_cols = (int)(csc_cols.size() / 2);
    double *d_part = dev_zeros<double>((size_t)cl * NPART, own);
    a.part = d_part;
    a.inst_cl_first = dev_upload(cl_first, own);
    a.hist = dev_zeros<double>((size_t)batch * h->hist_cap * 3, own);
    a.batch = batch;

    ProjArgs &p = h->proj;
    p.cl_inst = dev_upload(cl_inst, own);
    p.cl_size = dev_upload(cl_size, own);
    p.cl_off = dev_upload(cl_off, own);
    p.blk_loc = dev_upload(blk_loc, own);
    p.u = a.u;
    p.X = dev_zeros<double>(pk, own);
    p.Lam = dev_zeros<double>(pk, own);
    p.part = d_part;
    p.state = h->d_state;
    p.max_sweeps = h->max_sweeps;
    p.tol = h->jac_tol;
    p.decouple = opt.decouple && h->precision == SDP_FP32_EIG;
    p.dec_max_ref = h->precision == SDP_FP32_EIG ? 2 : 3;
    p.dec_skip = 4;
    // the sign-function fallback of cliques (of up to 96 vertices) whose
    // certificate keeps failing: P+ to the sweep tolerance
    sign_schedule(h->jac_tol, 96, &p.sign_k1, &p.sign_k2);
    // the rotation Q = I + T + T^2 / 2 has Q^T Q - I = T^4 / 4, at most
    // ||T||_F^4 / 4: with ||T||_F^2 <= sqrt(tol / 0.75) that stays below a
    // third of the sweep tolerance (the bound limits the refinements to
    // nearly decoupled blocks, where they converge quadratically)
    p.dec_tmax2 = std::sqrt(h->jac_tol / 0.75);
    p.dual = a.dual = opt.algorithm == SDP_ALG_DUAL ? 1 : 0;
    if (p.dual) {
      p.Vd = dev_zeros<double>(pk, own);
      h->d_utmp = dev_zeros<double>(coord, own);
    }

    a.X = p.X;
    a.Lam = p.Lam;
    for (size_t b = 0; b < lists.size(); ++b) {
      h->bucket_list.push_back(dev_upload(lists[b], own));
      h->bucket_count.push_back((int)lists[b].size());
      // (only as the plan's one list: beside other lists, which run
      // concurrently on their own streams, the split iteration's 95 short
      // launches wait behind their kernels; with the nonchordal workload's
      // four blocks of 80 split that way, FP64 went 1580 -> 1256 iter/s)
      const int64_t wsz = lists.size() == 1 ? split_workspace(h->precision, h->bucket_size[b],
                                                              (int)lists[b].size())
                                            : 0;
      h->bucket_ws.push_back(wsz > 0 ? dev_zeros<double>(wsz, own) : nullptr);
    }
    h->bucket_order.resize(lists.size());
    for (size_t b = 0; b < lists.size(); ++b) h->bucket_order[b] = (int)b;
    std::stable_sort(h->bucket_order.begin(), h->bucket_order.end(),
                     [&](int x, int y) { return h->bucket_N[x] > h->bucket_N[y]; });
    if (lists.size() > 1) {
      HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
      for (size_t i = 0; i + 1 < lists.size(); ++i) {
        hipStream_t a = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&a, hipStreamNonBlocking));
        h->aux_stream.push_back(a);
        hipEvent_t e = nullptr;
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->ev_join.push_back(e);
      }
    }
    h->cl_first = cl_first;
    h->d_clique_N = dev_upload(h->clique_N, own);
    if (opt.warm_start) {
      std::vector<int64_t> voff(cl);
      int64_t vo = 0;
      for (int64_t k = 0; k < cl; ++k) {
        voff[k] = vo;
        vo += (int64_t)h->clique_N[k] * h->clique_N[k];
      }
      h->d_vw_off = dev_upload(voff, own);
      const size_t esz = h->precision == SDP_FP32_EIG ? sizeof(float) : sizeof(double);
      HIPCHK(hipMalloc(&h->d_vw, esz * (size_t)std::max<int64_t>(vo, 1)));
      own.push_back(h->d_vw);
      p.vw = h->d_vw;
      p.ns_period = 2;
      p.ns_shift = 0;
      p.vw_off = h->d_vw_off;
    }
    h->d_diag = dev_zeros<double>((size_t)4 * batch, own);
    // caller layout of per-instance vectors, row -> instance map, and the
    // (V, theta) record offsets used by the reverse sweep
    {
      std::vector<int32_t> row_inst(row);
      int64_t uc = 0, ur = 0;
      for (int i = 0; i < batch; ++i) {
        h->user_coord_off.push_back(uc);
        h->user_row_off.push_back(ur);
        uc += H[i].nnz;
        ur += H[i].m;
        for (int r = 0; r < h->desc[i].ldm; ++r) row_inst[h->desc[i].row_off + r] = i;
      }
      h->user_ncoord = uc;
      h->user_nrow = ur;
      h->d_user_coord_off = dev_upload(h->user_coord_off, own);
      h->d_user_row_off = dev_upload(h->user_row_off, own);
      h->d_row_inst = dev_upload(row_inst, own);
      std::vector<int64_t> eoff(cl);
      int64_t eo = 0;
      h->adj_ready = true;
      for (int64_t k = 0; k < cl; ++k) {
        const int nb = h->clique_N[k];
        if (nb > adjoint_max_bucket(h->precision)) h->adj_ready = false;
        eoff[k] = eo;
        eo += (int64_t)cl_size[k] * nb + nb;
      }
      h->eig_total = eo;
      h->d_eig_off = dev_upload(eoff, own);
    }
    h->diag.assign(4 * batch, NAN);

    // ---- one-time factorisation: M = A W D^-1 A^T = L L^T, T = L^-1 ----
    // (with conjugate gradients: only diag(M) for the preconditioner)
    if (cg) {
      h->cg = true;
      a.cg_max_iter = opt.cg_max_iter;
      a.cg = dev_zeros<CgState>(batch, own);
      a.cg_g = dev_zeros<double>(coord, own);
      a.cg_z = dev_zeros<double>(row, own);
      a.cg_p = dev_zeros<double>(row, own);
      a.cg_Mp = dev_zeros<double>(row, own);
      std::vector<int32_t> tiles, tile_first(batch + 1, 0);
      for (int i = 0; i < batch; ++i) {
        tile_first[i] = (int32_t)(tiles.size() / 2);
        for (int r = 0; r < H[i].m; r += affine_cg_tile_rows()) {
          tiles.push_back(i);
          tiles.push_back(r);
        }
      }
      tile_first[batch] = (int32_t)(tiles.size() / 2);
      a.cg_tiles = dev_upload(tiles, own);
      a.cg_ntiles = tile_first[batch];
      a.cg_tile_first = dev_upload(tile_first, own);
      a.cg_part = dev_zeros<double>((size_t)3 * a.cg_ntiles, own);
      double *d_diagm = dev_zeros<double>(row, own);
      a.cg_diag = d_diagm;
      h->cg_tol2.resize(batch);
      for (int i = 0; i < batch; ++i) {
        double nb2 = 0.0;
        for (int r = 0; r < H[i].m; ++r) nb2 += inst[i].b[r] * inst[i].b[r];
        const double t = opt.cg_tol * (1.0 + std::sqrt(nb2));
        h->cg_tol2[i] = t * t;
      }
      a.cg_tol2 = dev_upload(h->cg_tol2, own);
      HIPCHK(launch_cg_diag(a, d_wd, h->d_t_rows_all, h->n_t_rows_all, d_diagm, h->stream));
      std::vector<double> dm(row);
      HIPCHK(hipMemcpyAsync(dm.data(), d_diagm, sizeof(double) * row, hipMemcpyDeviceToHost,
                            h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      for (int i = 0; i < batch; ++i)
        for (int r = 0; r < H[i].m; ++r)
          if (!(dm[h->desc[i].row_off + r] > 0))
            fail(SDP_ERR_RANK_DEFICIENT, "instance " + std::to_string(i) + ": row " +
                                             std::to_string(r) + " of A is zero");
    } else {
      double *d_M = nullptr;
      HIPCHK(hipMalloc((void **)&d_M, sizeof(double) * std::max<int64_t>(toff, 1)));
      HIPCHK(hipMemsetAsync(d_M, 0, sizeof(double) * std::max<int64_t>(toff, 1), h->stream));
      int32_t *d_fail = nullptr;
      HIPCHK(hipMalloc((void **)&d_fail, sizeof(int32_t) * batch));
      HIPCHK(hipMemsetAsync(d_fail, 0, sizeof(int32_t) * batch, h->stream));
      std::vector<void *> tmp;
      FactorArgs f{};
      f.inst = h->d_desc;
      f.batch = batch;
      f.A = d_A;
      f.a_rowptr = a.a_rowptr; f.a_col = a.a_col; f.a_val = a.a_val;
      f.a_colptr = a.a_colptr; f.a_row = a.a_row; f.a_cval = a.a_cval;
      f.wd = d_wd;
      f.diag_shift = opt.algorithm == SDP_ALG_HSDE ? 1.0 : 0.0;
      f.M = d_M;
      f.T = d_T;
      f.U = d_U;
      f.fail = d_fail;
      int32_t *d_syrk_tiles = dev_upload(syrk_tiles, tmp);
      int32_t *d_syrk_rows = dev_upload(syrk_rows, tmp);
      hipError_t e1 = launch_syrk_dense(f, d_syrk_tiles, (int)(syrk_tiles.size() / 3), h->stream);
      hipError_t e2 = e1 == hipSuccess
                          ? launch_syrk_csr(f, d_syrk_rows, (int)(syrk_rows.size() / 2), max_ldm,
                                            h->stream)
                          : e1;
      f.Bout = const_cast<double *>(a.Bm);
      int32_t *d_b_tiles = dev_upload(b_tiles, tmp);
      hipError_t e3 = e2 == hipSuccess
                          ? launch_cholesky_and_inverse(f, max_ldm / 64, h->stream)
                          : e2;
      if (e3 == hipSuccess && a.Bm)
        e3 = launch_form_b(f, d_b_tiles, (int)(b_tiles.size() / 3), h->stream);
      hipError_t e4 = hipStreamSynchronize(h->stream);
      std::vector<int32_t> failed(batch, 0);
      hipError_t e5 = hipMemcpy(failed.data(), d_fail, sizeof(int32_t) * batch, hipMemcpyDeviceToHost);
      (void)hipFree(d_M);
      (void)hipFree(d_fail);
      for (void *q : tmp) (void)hipFree(q);
      HIPCHK(e3);
      HIPCHK(e4);
      HIPCHK(e5);
      for (int i = 0; i < batch; ++i)
        if (failed[i])
          fail(SDP_ERR_RANK_DEFICIENT, "instance " + std::to_string(i) +
                                           ": A D^-1 A^T is not positive definite");
    }
    (void)wd;
    compute_bp(h);
    if (opt.algorithm == SDP_ALG_HSDE) setup_hsde(h, D);
    reset_state(h);
    *out = h;
  } catch (...) {
    destroy_handle(h);
    throw;
  }
}

template <typename F>
int guarded(F &&f) {
  try {
    g_last_error.clear();
    return f();
  } catch (SdpError &e) {
    g_last_error = e.what();
    return e.code;
  } catch (std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return SDP_ERR_OOM;
  } catch (std::exception &e) {
    g_last_error = e.what();
    return SDP_ERR_HIP;
  }
}

}  // namespace

// Scratch of the allocation-free diagnostics: one static array per device,
// held until the process ends (see diag_scratch_address).
constexpr int64_t kDiagScratchDoubles = int64_t(1) << 21;   // 16 MiB
static __device__ __align__(256) double scratch[kDiagScratchDoubles];

namespace {

// The diagnostics launches on a given scratch record (six vectors, every
// entry overwritten by the kernels before it is read), then the host copy.
void run_diagnostics(sdp_handle *h, const DiagScratch &s, sdp_result *res) {
  for (size_t b = 0; b < h->bucket_size.size(); ++b)
    HIPCHK(launch_min_eig(h->precision, h->bucket_size[b], h->bucket_list[b], h->bucket_count[b],
                          h->proj, s.lmin, h->stream));
  ensure_y(h);
  HIPCHK(launch_diagnostics(h->aff, s, h->aff.inst_cl_first, h->nrow, h->d_diag, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  HIPCHK(hipMemcpy(h->diag.data(), h->d_diag, sizeof(double) * 4 * h->B, hipMemcpyDeviceToHost));
  h->have_diag = true;
  if (res) fill_results(h, res);
}

// Host code never uses the name `scratch` as an address (on the host it
// names a stand-in, not device memory): it asks the runtime for the array's
// address on device `dev` once, with that device current, and keeps it.
constexpr int kMaxDevices = 64;

double *diag_scratch_address(int dev) {
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) fail(SDP_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    int cur = -1;
    HIPCHK(hipGetDevice(&cur));
    if (cur != dev) HIPCHK(hipSetDevice(dev));
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHK(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      fail(SDP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = static_cast<double *>(p);
  }
  return addr[dev];
}

}  // namespace

extern "C" {

void sdp_default_options(sdp_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->rho = 1.0;
  opt->tol = 1e-4;
  opt->max_iter = 20000;
  opt->precision = SDP_FP64;
  opt->adaptive_rho = 0;
  opt->mu = 2.0;
  opt->nu = 10.0;
  opt->rho_period = 1;
  opt->graph_chunk = 25;
  opt->stream = nullptr;
  opt->jacobi_max_sweeps = 0;
  opt->jacobi_tol = 0.0;
  opt->autotune = 1;
  opt->warm_start = 1;
  opt->algorithm = SDP_ALG_PRIMAL;
  opt->decouple = 1;
}

int sdp_setup(int32_t batch, const sdp_instance *inst, const sdp_options *opt, sdp_handle **out) {
  return guarded([&] {
    setup_impl(batch, inst, opt, out);
    return SDP_OK;
  });
}

int sdp_reset(sdp_handle *h) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    reset_state(h);
    return SDP_OK;
  });
}

int sdp_admm_step(sdp_handle *h, int32_t n_steps, sdp_result *res) {
  return guarded([&] {
    if (!h || n_steps < 0) fail(SDP_ERR_ARG, "NULL handle or negative step count");
    h->have_diag = false;
    enqueue_steps(h, n_steps);
    h->iters_enqueued += n_steps;
    if (res) fill_results(h, res);
    return SDP_OK;
  });
}

int sdp_solve(sdp_handle *h, sdp_result *res) {
  return guarded([&] {
    if (!h || !res) fail(SDP_ERR_ARG, "NULL handle or result array");
    h->have_diag = false;
    pull_state(h);
    const int chunk = h->opt.graph_chunk > 0 ? h->opt.graph_chunk : 25;
    for (;;) {
      bool all_done = true;
      int max_left = 0;
      for (int i = 0; i < h->B; ++i) {
        if (!h->h_state[i].done) {
          all_done = false;
          max_left = std::max(max_left, h->opt.max_iter - h->h_state[i].iter);
        }
      }
      if (all_done) break;
      enqueue_steps(h, std::min(chunk, std::max(max_left, 1)));
      pull_state(h);
    }
    fill_results(h, res);
    int st = SDP_OK;
    for (int i = 0; i < h->B; ++i)
      if (res[i].status == SDP_MAX_ITER) return (int)SDP_MAX_ITER;
      else if (res[i].status != SDP_OK && st == SDP_OK) st = res[i].status;
    return st;
  });
}

namespace {
int project_blocks(int variant, int32_t count, int32_t max_size, const int32_t *sizes,
                   const int64_t *offsets, const void *in, void *out, int32_t dtype,
                   void *stream) {
  if (count < 0 || (count > 0 && (!sizes || !offsets || !in || !out)))
    fail(SDP_ERR_ARG, "invalid arguments");
  if (dtype != SDP_DTYPE_FP64 && dtype != SDP_DTYPE_FP32) fail(SDP_ERR_ARG, "invalid dtype");
  const int prec = dtype == SDP_DTYPE_FP32 ? 1 : 0;
  if (max_size <= 0 || max_size > projection_max_size(prec))
    fail(SDP_ERR_UNSUPPORTED, "max_size out of range for this dtype");
  if (variant < 0) {
    variant = projection_standalone_variant(prec, max_size);
  } else {
    if (variant >= projection_variant_count(prec)) fail(SDP_ERR_ARG, "no such kernel variant");
    int N, NT;
    projection_variant_info(prec, variant, &N, &NT);
    if (max_size > N) fail(SDP_ERR_ARG, "max_size exceeds the variant's block size");
  }
  if (count == 0) return SDP_OK;
  const int msw = prec ? 30 : 40;
  const double tol = prec ? 1e-6 : 1e-14;
  HIPCHK(launch_standalone_projection(prec, variant, count, sizes, offsets, in, out, msw, tol,
                                      (hipStream_t)stream));
  return SDP_OK;
}
}  // namespace

int sdp_psd_project_batched(int32_t count, int32_t max_size, const int32_t *sizes,
                            const int64_t *offsets, const void *in, void *out, int32_t dtype,
                            void *stream) {
  return guarded([&] {
    return project_blocks(-1, count, max_size, sizes, offsets, in, out, dtype, stream);
  });
}

int sdp_psd_project_variant(int32_t variant, int32_t count, int32_t max_size,
                            const int32_t *sizes, const int64_t *offsets, const void *in,
                            void *out, int32_t dtype, void *stream) {
  return guarded([&] {
    if (variant < 0) fail(SDP_ERR_ARG, "no such kernel variant");
    return project_blocks(variant, count, max_size, sizes, offsets, in, out, dtype, stream);
  });
}

int sdp_projection_variants(int32_t dtype, int32_t cap, int32_t *block_n, int32_t *threads,
                            int32_t *count) {
  return guarded([&] {
    if (dtype != SDP_DTYPE_FP64 && dtype != SDP_DTYPE_FP32) fail(SDP_ERR_ARG, "invalid dtype");
    if (cap < 0 || !count) fail(SDP_ERR_ARG, "invalid arguments");
    const int prec = dtype == SDP_DTYPE_FP32 ? 1 : 0;
    const int nv = projection_variant_count(prec);
    for (int v = 0; v < nv && v < cap; ++v) {
      int N, NT;
      projection_variant_info(prec, v, &N, &NT);
      if (block_n) block_n[v] = N;
      if (threads) threads[v] = NT;
    }
    *count = nv;
    return SDP_OK;
  });
}

int sdp_projection_variant_kind(int32_t dtype, int32_t variant, int32_t *kind) {
  return guarded([&] {
    if (dtype != SDP_DTYPE_FP64 && dtype != SDP_DTYPE_FP32) fail(SDP_ERR_ARG, "invalid dtype");
    const int prec = dtype == SDP_DTYPE_FP32 ? 1 : 0;
    if (!kind || variant < 0 || variant >= projection_variant_count(prec))
      fail(SDP_ERR_ARG, "invalid arguments");
    *kind = projection_variant_kind(prec, variant);
    return SDP_OK;
  });
}

int sdp_sign_schedule(double tol, int32_t n, int32_t *k1, int32_t *k2) {
  return guarded([&] {
    if (!k1 || !k2 || n < 1) fail(SDP_ERR_ARG, "invalid arguments");
    int a = 0, b = 0;
    sign_schedule(tol, n, &a, &b);
    *k1 = a;
    *k2 = b;
    return SDP_OK;
  });
}

int sdp_projection_default_variant(int32_t dtype, int32_t max_size, int32_t *variant) {
  return guarded([&] {
    if (dtype != SDP_DTYPE_FP64 && dtype != SDP_DTYPE_FP32) fail(SDP_ERR_ARG, "invalid dtype");
    if (!variant) fail(SDP_ERR_ARG, "invalid arguments");
    const int prec = dtype == SDP_DTYPE_FP32 ? 1 : 0;
    if (max_size <= 0 || max_size > projection_max_size(prec))
      fail(SDP_ERR_UNSUPPORTED, "max_size out of range for this dtype");
    *variant = projection_standalone_variant(prec, max_size);
    return SDP_OK;
  });
}

int sdp_projection_plan_variants(sdp_handle *h, int32_t cap, int32_t *variant, int32_t *count) {
  return guarded([&] {
    if (!h || cap < 0 || !count) fail(SDP_ERR_ARG, "invalid arguments");
    const int nl = (int)h->bucket_size.size();
    for (int b = 0; b < nl && b < cap; ++b)
      if (variant) variant[b] = h->bucket_size[b];
    *count = nl;
    return SDP_OK;
  });
}

int sdp_get_solution(sdp_handle *h, int32_t inst, double *u, double *y_dual, double *Xk,
                     double *Lk) {
  return guarded([&] {
    if (!h || inst < 0 || inst >= h->B) fail(SDP_ERR_ARG, "invalid handle or instance");
    const InstDesc &d = h->desc[inst];
    const bool dual = h->aff.dual != 0;
    HIPCHK(hipStreamSynchronize(h->stream));
    if (h->hsde) {
      if (!h->d_utmp) h->d_utmp = dev_zeros<double>(h->ncoord, h->owned);
      HIPCHK(launch_hsde_solution(h->hsa, h->d_utmp, h->d_ytmp, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
      if (u) HIPCHK(hipMemcpy(u, h->d_utmp + d.coord_off, sizeof(double) * d.nnz, hipMemcpyDeviceToHost));
      if (y_dual) HIPCHK(hipMemcpy(y_dual, h->d_ytmp + d.row_off, sizeof(double) * d.m, hipMemcpyDeviceToHost));
      const int64_t o = h->npk_off[inst], n = h->inst_npk[inst];
      if (Xk) HIPCHK(hipMemcpy(Xk, h->proj.X + o, sizeof(double) * n, hipMemcpyDeviceToHost));
      if (Lk) HIPCHK(hipMemcpy(Lk, h->proj.Lam + o, sizeof(double) * n, hipMemcpyDeviceToHost));
      return SDP_OK;
    }
    if (u) {
      const double *src = h->aff.u + d.coord_off;
      if (dual) {   // the primal estimate -rho x
        HIPCHK(launch_scaled_copy(src, h->d_utmp + d.coord_off, d.nnz, h->d_state, inst,
                                  h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        src = h->d_utmp + d.coord_off;
      }
      HIPCHK(hipMemcpy(u, src, sizeof(double) * d.nnz, hipMemcpyDeviceToHost));
    }
    if (y_dual) {
      ensure_y(h);
      const double *src = h->aff.y + d.row_off;
      if (!dual) {  // the multipliers of <A_i, X> = b_i: -rho y
        HIPCHK(launch_scaled_copy(src, h->d_ytmp + d.row_off, d.m, h->d_state, inst, h->stream));
        src = h->d_ytmp + d.row_off;
      }
      HIPCHK(hipStreamSynchronize(h->stream));
      HIPCHK(hipMemcpy(y_dual, src, sizeof(double) * d.m, hipMemcpyDeviceToHost));
    }
    const int64_t o = h->npk_off[inst], n = h->inst_npk[inst];
    if (Xk) HIPCHK(hipMemcpy(Xk, h->proj.X + o, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (Lk) HIPCHK(hipMemcpy(Lk, h->proj.Lam + o, sizeof(double) * n, hipMemcpyDeviceToHost));
    return SDP_OK;
  });
}

int sdp_set_state(sdp_handle *h, int32_t inst, const double *Xk, const double *Lk, double rho) {
  return guarded([&] {
    if (!h || inst < 0 || inst >= h->B || !(rho > 0)) fail(SDP_ERR_ARG, "invalid arguments");
    if (h->hsde) fail(SDP_ERR_UNSUPPORTED, "warm starts are built for Algorithms 1 and 2");
    HIPCHK(hipStreamSynchronize(h->stream));
    const int64_t o = h->npk_off[inst], n = h->inst_npk[inst];
    if (Xk)
      HIPCHK(hipMemcpyAsync(h->proj.X + o, Xk, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    if (Lk)
      HIPCHK(hipMemcpyAsync(h->proj.Lam + o, Lk, sizeof(double) * n, hipMemcpyHostToDevice,
                            h->stream));
    if (h->proj.Vd)   // Algorithm 2: the slack blocks start at consensus, v_k = z_k
      HIPCHK(hipMemcpyAsync(h->proj.Vd + o, h->proj.X + o, sizeof(double) * n,
                            hipMemcpyDeviceToDevice, h->stream));
    {   // the instance's cliques start their decoupling back-off afresh (slot 7)
      const int64_t c0 = h->cl_first[inst], c1 = h->cl_first[inst + 1];
      if (c1 > c0)
        HIPCHK(hipMemsetAsync(h->proj.part + NPART * c0, 0, sizeof(double) * NPART * (c1 - c0),
                              h->stream));
    }
    if (h->d_vw) {
      HIPCHK(launch_identity_bases(h->precision, h->d_vw, h->d_vw_off, h->d_clique_N,
                                   h->cl_first[inst], h->cl_first[inst + 1] - h->cl_first[inst],
                                   h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    pull_state(h);
    InstState s = h->h_state[inst];
    s.rho = rho;
    s.done = 0;
    HIPCHK(hipMemcpyAsync(h->d_state + inst, &s, sizeof(InstState), hipMemcpyHostToDevice,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->have_diag = false;
    return SDP_OK;
  });
}

int sdp_get_history(sdp_handle *h, int32_t inst, int32_t cap, double *eps_c, double *eps_lambda,
                    double *rho, int32_t *count) {
  return guarded([&] {
    if (!h || inst < 0 || inst >= h->B || cap < 0) fail(SDP_ERR_ARG, "invalid arguments");
    pull_state(h);
    const int n = std::min({cap, h->h_state[inst].iter, h->hist_cap});
    std::vector<double> buf((size_t)std::max(n, 1) * 3);
    if (n > 0)
      HIPCHK(hipMemcpy(buf.data(), h->aff.hist + (size_t)inst * h->hist_cap * 3,
                       sizeof(double) * 3 * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
      if (eps_c) eps_c[i] = buf[3 * i];
      if (eps_lambda) eps_lambda[i] = buf[3 * i + 1];
      if (rho) rho[i] = buf[3 * i + 2];
    }
    if (count) *count = n;
    return SDP_OK;
  });
}

int sdp_diagnostics(sdp_handle *h, sdp_result *res) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    if (h->hsde) {   // Algorithm 3 evaluates eps_p, eps_d, eps_g in every iteration
      if (res) fill_results(h, res);
      return SDP_OK;
    }
    if (!h->dscr.wu) {
      h->dscr.wu = dev_zeros<double>(h->ncoord, h->owned);
      h->dscr.z = dev_zeros<double>(h->ncoord, h->owned);
      h->dscr.aty = dev_zeros<double>(h->ncoord, h->owned);
      h->dscr.ax = dev_zeros<double>(h->nrow, h->owned);
      h->dscr.yd = dev_zeros<double>(h->nrow, h->owned);
      h->dscr.lmin = dev_zeros<double>(h->ncl, h->owned);
    }
    run_diagnostics(h, h->dscr, res);
    return SDP_OK;
  });
}

int sdp_diagnostics_noalloc(sdp_handle *h, sdp_result *res) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    if (h->hsde) {
      if (res) fill_results(h, res);
      return SDP_OK;
    }
    const int64_t need = 3 * h->ncoord + 2 * h->nrow + h->ncl;
    if (need > kDiagScratchDoubles)
      fail(SDP_ERR_UNSUPPORTED,
           "sdp_diagnostics_noalloc: the handle needs " + std::to_string(need) +
               " doubles of scratch (3 per coordinate slot, 2 per row slot, 1 per clique); the "
               "static limit is " + std::to_string(kDiagScratchDoubles));
    int dev = -1;   // the device the handle's stream (and so its kernels) runs on
    HIPCHK(hipStreamGetDevice(h->stream, &dev));
    double *base = diag_scratch_address(dev);
    // ncoord and nrow are multiples of 64, so every vector starts 512-byte aligned
    DiagScratch s;
    s.wu = base;
    s.z = s.wu + h->ncoord;
    s.aty = s.z + h->ncoord;
    s.ax = s.aty + h->ncoord;
    s.yd = s.ax + h->nrow;
    s.lmin = s.yd + h->nrow;
    run_diagnostics(h, s, res);
    return SDP_OK;
  });
}

int sdp_get_projection_stats(sdp_handle *h, int64_t *jacobi_sweeps, int64_t *projections,
                             int64_t *sign_fallbacks) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    pull_state(h);
    int64_t sw = 0, pr = 0, sg = 0;
    for (int i = 0; i < h->B; ++i) {
      sw += (int64_t)h->h_state[i].total_sweeps;
      pr += (int64_t)h->h_state[i].iter * h->inst_p[i];
      sg += (int64_t)h->h_state[i].total_sign;
    }
    if (jacobi_sweeps) *jacobi_sweeps = sw;
    if (projections) *projections = pr;
    if (sign_fallbacks) *sign_fallbacks = sg;
    return SDP_OK;
  });
}

int sdp_get_stats(sdp_handle *h, int64_t *jacobi_sweeps, int64_t *projections) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    pull_state(h);
    int64_t sw = 0, pr = 0;
    for (int i = 0; i < h->B; ++i) {
      sw += (int64_t)h->h_state[i].total_sweeps;
      pr += (int64_t)h->h_state[i].iter * h->inst_p[i];
    }
    if (jacobi_sweeps) *jacobi_sweeps = sw;
    if (projections) *projections = pr;
    return SDP_OK;
  });
}

int sdp_cg_steps(sdp_handle *h, int64_t *steps) {
  return guarded([&] {
    if (!h || !steps) fail(SDP_ERR_ARG, "invalid arguments");
    *steps = 0;
    if (!h->cg) return SDP_OK;
    std::vector<CgState> cs(h->B);
    HIPCHK(hipMemcpyAsync(cs.data(), h->aff.cg, sizeof(CgState) * h->B, hipMemcpyDeviceToHost,
                          h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (const CgState &c : cs) *steps += c.total;
    return SDP_OK;
  });
}

int sdp_projection_plan(sdp_handle *h, int32_t cap, int32_t *block_n, int32_t *threads,
                        int32_t *cliques, int32_t *count) {
  return guarded([&] {
    if (!h || cap < 0 || !count) fail(SDP_ERR_ARG, "invalid arguments");
    const int nl = (int)h->bucket_size.size();
    for (int b = 0; b < nl && b < cap; ++b) {
      int N, NT;
      projection_variant_info(h->precision, h->bucket_size[b], &N, &NT);
      if (block_n) block_n[b] = N;
      if (threads) threads[b] = NT;
      if (cliques) cliques[b] = h->bucket_count[b];
    }
    *count = nl;
    return SDP_OK;
  });
}

int sdp_time_stages(sdp_handle *h, int32_t n_iter, double *ms) {
  return guarded([&] {
    if (!h || n_iter <= 0 || !ms) fail(SDP_ERR_ARG, "invalid arguments");
    constexpr int NS = 7;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    try {
      for (int s = 0; s < NS; ++s) {
        HIPCHK(hipEventRecord(e0, h->stream));
        for (int it = 0; it < n_iter; ++it) {
          if (h->hsde) {   // 0 nu and x', 1-4 the inner solve, 5 update + projections, 6 residuals
            if (s == 0) {
              HIPCHK(launch_hsde_form_nu(h->hsa, h->stream));
              HIPCHK(launch_hsde_xprime(h->hsa, h->hsa.nx, h->hsa.ns, h->hsa.nt, h->stream));
            } else if (s < 5) {
              HIPCHK(launch_affine_stage(h->aff, s, h->stream));
            } else if (s == 5) {
              HIPCHK(launch_hsde_update(h->hsa, h->stream));
              enqueue_projections(h, h->proj, h->stream);
            } else {
              HIPCHK(launch_hsde_finish(h->hsa, h->stream));
            }
            continue;
          }
          if (s < 5) {
            if (!h->cg) HIPCHK(launch_affine_stage(h->aff, s, h->stream));
            else if (s != 3) HIPCHK(launch_cg_stage(h->aff, s, h->stream));
          } else if (s == 5) {
            // (the launches step through the re-orthonormalisation period as
            // the iterations do; the iteration counter itself does not move)
            ProjArgs p = h->proj;
            p.ns_shift = it;
            enqueue_projections(h, p, h->stream);
            if (h->proj.dual) HIPCHK(launch_dual_update(h->proj, h->ncl, h->stream));
          } else {
            HIPCHK(launch_residual_reduce(h->aff, h->stream));
          }
        }
        HIPCHK(hipEventRecord(e1, h->stream));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        ms[s] = (double)t / n_iter;
      }
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->have_diag = false;
    return SDP_OK;
  });
}

int sdp_update_data(sdp_handle *h, const double *c, const double *b) {
  return guarded([&] {
    if (!h) fail(SDP_ERR_ARG, "NULL handle");
    if (h->hsde) fail(SDP_ERR_UNSUPPORTED, "data updates are built for Algorithms 1 and 2");
    if (c)
      HIPCHK(launch_copy_user(c, const_cast<double *>(h->aff.c), h->d_desc, h->aff.coord_inst,
                              h->d_user_coord_off, h->ncoord, 0, h->stream));
    if (b)
      HIPCHK(launch_copy_user_rows(b, const_cast<double *>(h->aff.b), h->d_desc, h->d_row_inst,
                                   h->d_user_row_off, h->nrow, h->stream));
    if (b) compute_bp(h);
    if (b && h->cg) {
      int64_t o = 0;
      for (int i = 0; i < h->B; ++i) {
        double nb2 = 0.0;
        for (int r = 0; r < h->desc[i].m; ++r) nb2 += b[o + r] * b[o + r];
        o += h->desc[i].m;
        const double t = h->opt.cg_tol * (1.0 + std::sqrt(nb2));
        h->cg_tol2[i] = t * t;
      }
      HIPCHK(hipMemcpyAsync(const_cast<double *>(h->aff.cg_tol2), h->cg_tol2.data(),
                            sizeof(double) * h->B, hipMemcpyHostToDevice, h->stream));
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->have_diag = false;
    return SDP_OK;
  });
}

int sdp_unrolled_forward(sdp_handle *h, int32_t T, int32_t ckpt_every, double *u_out) {
  return guarded([&] {
    if (!h || T <= 0 || ckpt_every <= 0) fail(SDP_ERR_ARG, "invalid arguments");
    if (h->opt.adaptive_rho) fail(SDP_ERR_ARG, "unrolled differentiation needs a fixed rho");
    if (h->proj.dual || h->hsde)
      fail(SDP_ERR_UNSUPPORTED, "unrolled differentiation is built for Algorithm 1 only");
    if (h->cg) fail(SDP_ERR_UNSUPPORTED, "unrolled differentiation needs the factored affine step");
    // the forward records every clique's eigenvectors for the adjoint
    if (!h->adj_ready)
      fail(SDP_ERR_UNSUPPORTED, "unrolled differentiation takes cliques of up to 128 vertices in "
                                "FP32 and 96 in FP64");
    const int nseg = (T + ckpt_every - 1) / ckpt_every;
    const int64_t need = (int64_t)nseg * 2 * std::max<int64_t>(h->npk, 1);
    if (need > h->ckpt_cap) {
      HIPCHK(hipStreamSynchronize(h->stream));
      if (h->d_ckpt) (void)hipFree(h->d_ckpt);
      h->d_ckpt = nullptr;
      h->ckpt_cap = 0;
      HIPCHK(hipMalloc((void **)&h->d_ckpt, sizeof(double) * need));
      h->ckpt_cap = need;
    }
    reset_state(h);
    const int64_t np = std::max<int64_t>(h->npk, 1);
    for (int t = 0; t < T; ++t) {
      if (t % ckpt_every == 0) {
        double *slot = h->d_ckpt + (int64_t)(t / ckpt_every) * 2 * np;
        HIPCHK(hipMemcpyAsync(slot, h->proj.X, sizeof(double) * h->npk, hipMemcpyDeviceToDevice,
                              h->stream));
        HIPCHK(hipMemcpyAsync(slot + np, h->proj.Lam, sizeof(double) * h->npk,
                              hipMemcpyDeviceToDevice, h->stream));
      }
      enqueue_unrolled_iteration(h, h->stream, nullptr);
    }
    if (u_out)
      HIPCHK(launch_copy_user(h->aff.u, u_out, h->d_desc, h->aff.coord_inst, h->d_user_coord_off,
                              h->ncoord, 1, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->adj_T = T;
    h->adj_ckpt = ckpt_every;
    h->have_diag = false;
    return SDP_OK;
  });
}

int sdp_vjp(sdp_handle *h, const double *u_bar, double *c_bar, double *b_bar, int32_t euclidean) {
  return guarded([&] {
    if (!h || !u_bar || !c_bar || !b_bar) fail(SDP_ERR_ARG, "invalid arguments");
    if (h->proj.dual || h->hsde)
      fail(SDP_ERR_UNSUPPORTED, "unrolled differentiation is built for Algorithm 1 only");
    if (h->cg) fail(SDP_ERR_UNSUPPORTED, "unrolled differentiation needs the factored affine step");
    if (h->adj_T <= 0) fail(SDP_ERR_ARG, "run sdp_unrolled_forward first");
    if (!h->adj_ready)
      fail(SDP_ERR_UNSUPPORTED, "the projection adjoint supports cliques of up to 128 vertices in "
                                     "FP32 and 96 in FP64");
    auto &own = h->owned;
    if (!h->d_Xb) {
      h->d_Xb = dev_zeros<double>(h->npk, own);
      h->d_Lb = dev_zeros<double>(h->npk, own);
      h->d_Ub = dev_zeros<double>(h->npk, own);
      h->d_bhat_bar = dev_zeros<double>(h->ncoord, own);
      h->d_v_bar = dev_zeros<double>(h->ncoord, own);
      h->d_bhb = dev_zeros<double>(h->ncoord, own);
      h->d_r_bar = dev_zeros<double>(h->nrow, own);
      h->d_y1_bar = dev_zeros<double>(h->nrow, own);
      h->d_y_bar = dev_zeros<double>(h->nrow, own);
      h->d_zero_rows = dev_zeros<double>(h->nrow, own);
    }
    const int T = h->adj_T, ck = h->adj_ckpt;
    const size_t esz = h->precision == SDP_FP32_EIG ? sizeof(float) : sizeof(double);
    const int64_t eneed = (int64_t)ck * std::max<int64_t>(h->eig_total, 1);
    if (eneed > h->eigbuf_cap) {
      HIPCHK(hipStreamSynchronize(h->stream));
      if (h->d_eigbuf) (void)hipFree(h->d_eigbuf);
      h->d_eigbuf = nullptr;
      h->eigbuf_cap = 0;
      HIPCHK(hipMalloc(&h->d_eigbuf, esz * eneed));
      h->eigbuf_cap = eneed;
    }
    HIPCHK(hipMemsetAsync(h->d_Xb, 0, sizeof(double) * h->npk, h->stream));
    HIPCHK(hipMemsetAsync(h->d_Lb, 0, sizeof(double) * h->npk, h->stream));
    HIPCHK(hipMemsetAsync(c_bar, 0, sizeof(double) * h->user_ncoord, h->stream));
    HIPCHK(hipMemsetAsync(b_bar, 0, sizeof(double) * h->user_nrow, h->stream));
    AdjArgs g{};
    g.inst = h->d_desc;
    g.state = h->d_state;
    g.cl_inst = h->proj.cl_inst;
    g.cl_size = h->proj.cl_size;
    g.cl_off = h->proj.cl_off;
    g.blk_loc = h->proj.blk_loc;
    g.eig_off = h->d_eig_off;
    g.Xb = h->d_Xb;
    g.Lb = h->d_Lb;
    g.Ub = h->d_Ub;
    g.npk = h->npk;
    g.ncoord = h->ncoord;
    g.nrow = h->nrow;
    g.coord_inst = h->aff.coord_inst;
    g.row_inst = h->d_row_inst;
    g.contrib_ptr = h->aff.contrib_ptr;
    g.contrib_idx = h->aff.contrib_idx;
    g.w = h->aff.w;
    g.D = h->aff.D;
    g.bhat_bar = h->d_bhat_bar;
    g.v_bar = h->d_v_bar;
    g.bhb = h->d_bhb;
    g.y_bar = h->d_y_bar;
    g.user_coord_off = h->d_user_coord_off;
    g.user_row_off = h->d_user_row_off;
    g.cbar = c_bar;
    g.bbar = b_bar;
    g.euclid = euclidean ? 1 : 0;
    g.batch = h->B;
    // the KKT solve of the reverse sweep: same factor, input ubar, b = 0
    AffineArgs ra = h->aff;
    ra.ignore_done = 1;
    ra.b = h->d_zero_rows;
    ra.bp = h->d_zero_rows;
    ra.t3_rows = h->d_t_rows_all;     // the multiplier cotangent is needed on every row
    ra.n_t3_rows = h->n_t_rows_all;
    ra.bhat = h->d_bhat_bar;
    ra.v = h->d_v_bar;
    ra.r = h->d_r_bar;
    ra.y1 = h->d_y1_bar;
    ra.y = h->d_y_bar;
    ra.u = h->d_bhb;
    const int64_t np = std::max<int64_t>(h->npk, 1);
    const int nseg = (T + ck - 1) / ck;
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int t0 = seg * ck, t1 = std::min(T, t0 + ck);
      const double *slot = h->d_ckpt + (int64_t)seg * 2 * np;
      HIPCHK(hipMemcpyAsync(h->proj.X, slot, sizeof(double) * h->npk, hipMemcpyDeviceToDevice,
                            h->stream));
      HIPCHK(hipMemcpyAsync(h->proj.Lam, slot + np, sizeof(double) * h->npk,
                            hipMemcpyDeviceToDevice, h->stream));
      for (int t = t0; t < t1; ++t)
        enqueue_unrolled_iteration(h, h->stream,
                                   (char *)h->d_eigbuf + esz * (size_t)(t - t0) * h->eig_total);
      for (int t = t1 - 1; t >= t0; --t) {
        g.eig = (const char *)h->d_eigbuf + esz * (size_t)(t - t0) * h->eig_total;
        g.seed = (t == T - 1) ? u_bar : nullptr;
        for (size_t b = 0; b < h->bucket_size.size(); ++b)
          HIPCHK(launch_adj_projection(h->precision, h->bucket_N[b], h->bucket_list[b],
                                       h->bucket_count[b], g, h->stream));
        HIPCHK(launch_adj_scatter(g, h->stream));
        for (int stg = 1; stg <= 4; ++stg) HIPCHK(launch_affine_stage(ra, stg, h->stream));
        HIPCHK(launch_adj_coord_and_gather(g, h->stream));
      }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    h->have_diag = false;
    return SDP_OK;
  });
}

void sdp_destroy(sdp_handle *h) { destroy_handle(h); }

const char *sdp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// Lets the pattern routines (a separate translation unit) report errors
// through the same thread-local message.
void sdp_set_last_error(const std::string &msg) { g_last_error = msg; }
