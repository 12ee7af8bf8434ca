// The X-step of Algorithm 1 on gfx950: the KKT system (OptCondMinYPrimal)
// solved by block elimination with the cached factor (the two-step form
// (KKTflops) of the proof of Proposition 1), written on the compact lower
// coordinates with weights w (1 on the diagonal, 2 off it):
//   bhat = sum_k H_k^T (x_k + lambda_k / rho) - c / rho        (k_scatter)
//   r    = A (w bhat / D) - b                                   (k_rowdot)
//   y    = L^-T (L^-1 r)   with L^-1, L^-T cached               (k_trmv_wave)
//   u    = (bhat - A^T y) / D                                   (k_coldot)
// For dense A the forward substitution is folded into B = L^-1 A at setup:
//   y1   = B (w bhat / D) - L^-1 b                              (k_rowdot)
//   u    = (bhat - B^T y1) / D       (A^T y = A^T L^-T y1)      (k_coldot)
// and y = L^-T y1 is formed only when the multiplier is asked for.
// plus the per-instance residual reduction, stopping test and adaptive
// penalty (k_residual_reduce).  Every kernel reads the instance's `done`
// flag first, so a converged instance is frozen at its stopping iterate.
//
// All of these passes stream HBM: A is read twice per iteration (row-wise,
// then column-wise) and the factor twice; vectors are small and L2-resident.
// Reductions use a fixed order, so results are bitwise reproducible.
#include "sdp_internal.h"

#include <math.h>

namespace {

constexpr int ROW_NT = 256;   // threads of a row-dot workgroup
constexpr int COL_NT = 512;   // threads of a column-dot workgroup
constexpr int COL_WAVES = COL_NT / 64;   // waves splitting the rows of a tile
constexpr int COL_W = 128;    // columns per column-dot tile (2 per lane)
constexpr int MAX_R = 8;      // max rows per row-dot tile

// Rows of dense A (or B) are read as pairs; for matrices larger than the
// 256 MB last-level cache (stream_nt) by the kernel instances with non-
// temporal loads (+10% on a 31.8 GB batch), otherwise with plain loads, which
// let a matrix that fits be served partly from that cache (non-temporal loads
// cost 25% on a 256 MB one).  The choice is a template parameter: a runtime
// select between the two loads of one address may be merged into one plain
// load.
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// bhat and v = w * bhat / D (owner-computes, no atomics).  Four consecutive
// lanes share a coordinate and split its contributors; their sums meet in a
// fixed butterfly, so the result does not depend on scheduling.
// ---------------------------------------------------------------------------
constexpr int SC_LANES = 4;

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD
// b % 8).  Renumber them so that each XCD gets one contiguous range of the
// logical index space: neighbouring coordinates share cache lines of X and
// Lambda, and each XCD has its own L2.
__device__ inline int xcd_contiguous(int b, int nb) {
  const int q = nb / 8, r = nb % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

__device__ void residual_block(const AffineArgs &a, int inst);

__global__ __launch_bounds__(256) void k_scatter(AffineArgs a) {
  if ((int)blockIdx.x < a.res_blocks) {
    // the previous iteration's residuals, stopping test (fixed penalty);
    // the `done` read below may see this iteration's update or not: either
    // way the scatter's outputs are only read by kernels that test it again
    if ((int)blockIdx.x < a.batch) residual_block(a, blockIdx.x);
    return;
  }
  // res_blocks is a multiple of 8: the XCD of a workgroup is unchanged
  const int64_t g = (int64_t)xcd_contiguous(blockIdx.x - a.res_blocks, gridDim.x - a.res_blocks) * 256 +
                    threadIdx.x;
  const int64_t j = g / SC_LANES;
  const int q = (int)(g % SC_LANES);
  if (j >= a.ncoord) return;             // whole lane groups leave together
  // the contributor range loads beside the instance index, and the done
  // test waits until the sums are formed (nothing is stored before it):
  // three dependent loads before the sums instead of five
  const int inst = a.coord_inst[j];
  const int64_t t0 = a.contrib_ptr[j], t1 = a.contrib_ptr[j + 1];
  const InstState &st = a.state[inst];
  const bool done = st.done != 0;
  // sum_k (x_k + lambda_k / rho) - c / rho = sum_k x_k + (sum_k lambda_k - c) / rho
  double sx = 0.0, sl = 0.0;
  for (int64_t t = t0 + q; t < t1; t += SC_LANES) {
    const int32_t e = a.contrib_idx[t];
    sx += a.X[e];
    sl += a.Lam[e];
  }
#pragma unroll
  for (int o = 1; o < SC_LANES; o <<= 1) {
    sx += __shfl_xor(sx, o, 64);
    sl += __shfl_xor(sl, o, 64);
  }
  if (done) return;                      // uniform per lane group (one coordinate)
  const double rho = st.rho;
  if (q == 0) {
    // Algorithm 1: sum_k (x_k + lambda_k/rho) - c/rho; Algorithm 2 (x_k = z_k):
    // c - sum_k (z_k + lambda_k/rho)
    const double bh = a.dual ? a.c[j] - (sx + sl / rho) : sx + (sl - a.c[j]) / rho;
    a.bhat[j] = bh;
    // with conjugate gradients: W D^-1 (bhat - A^T y_prev), so that the row
    // products give the solve's initial residual r0 = rhs - M y_prev
    a.v[j] = a.w[j] * (a.cg_g ? bh - a.cg_g[j] : bh) / a.D[j];
  }
}

// ---------------------------------------------------------------------------
// r = A v - b for dense A (m x ld row-major per instance).  One tile = R
// consecutive rows of one instance; lanes stride the columns with 16-byte
// loads, so every wave reads contiguous 1 KiB segments of A.
// ---------------------------------------------------------------------------
template <int R, bool NTL>
__global__ __launch_bounds__(ROW_NT) void k_rowdot(AffineArgs a) {
  const int inst = a.row_tiles[2 * blockIdx.x];
  const int row0 = a.row_tiles[2 * blockIdx.x + 1];
  // the descriptor loads beside the done flag (one latency fewer before the
  // stream starts); the empty asm takes its fields as inputs so that the
  // compiler keeps those loads ahead of the test instead of sinking them
  const InstDesc d = a.inst[inst];
  const int32_t done = a.state[inst].done;
  asm volatile("" ::"s"(d.m), "s"(d.ld), "s"(d.a_off), "s"(d.coord_off), "s"(d.row_off),
               "s"(done));
  if (!a.ignore_done && done) return;
  if (a.cg_loop && a.cg[inst].done) return;
  const int nrow = min(R, d.m - row0);
  const double *mat = (a.Bm ? a.Bm : a.A) + d.a_off + (int64_t)row0 * d.ld;
  const double2 *v2 = reinterpret_cast<const double2 *>(a.v + d.coord_off);
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  const int len2 = d.ld / 2;
  for (int c = threadIdx.x; c < len2; c += ROW_NT) {
    const double2 x = v2[c];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r < nrow) {
        const dvec2 *pm = reinterpret_cast<const dvec2 *>(mat + (int64_t)r * d.ld) + c;
        dvec2 m2;
        if constexpr (NTL) m2 = __builtin_nontemporal_load(pm);
        else m2 = *pm;
        acc[r] += m2.x * x.x + m2.y * x.y;
      }
    }
  }
  __shared__ double red[ROW_NT / 64][R];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double s = wave_sum(acc[r]);
    if (l == 0) red[w][r] = s;
  }
  __syncthreads();
  if (threadIdx.x < nrow) {
    const int r = threadIdx.x;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < ROW_NT / 64; ++i) s += red[i][r];
    const int64_t g = d.row_off + row0 + r;
    // Algorithm 2 solves with -b / rho in place of b
    const double bs = a.dual ? -1.0 / a.state[inst].rho : 1.0;
    if (a.no_b) a.r[g] = s;
    else if (a.Bm) a.y1[g] = s - bs * a.bp[g];
    else a.r[g] = s - bs * a.b[g];
  }
}

// ---------------------------------------------------------------------------
// Column-oriented (transposed) products over dense A.
//   RAW = 0:  u[j] = (bhat[j] - sum_i A[i][j] y[i]) / D[j]
//             (with conjugate gradients also cg_g[j] = sum_i A[i][j] y[i])
//   RAW = 1:  u[j] = sum_i A[i][j] y[i]            (diagnostics: A^T y)
//   RAW = 2:  u[j] = w[j] sum_i A[i][j] y[i] / D[j] (inside the CG solve)
// One tile = 128 columns of one instance; lane l owns columns 2l, 2l+1 and
// the COL_WAVES waves split the rows, so each wave reads contiguous 1 KiB
// segments.
// ---------------------------------------------------------------------------
template <int RAW, bool NTL>
__global__ __launch_bounds__(COL_NT) void k_coldot(AffineArgs a) {
  const int inst = a.col_tiles[2 * blockIdx.x];
  const int col0 = a.col_tiles[2 * blockIdx.x + 1];
  // the descriptor loads beside the done flag (one latency fewer before the
  // stream starts); the empty asm takes its fields as inputs so that the
  // compiler keeps those loads ahead of the test instead of sinking them
  const InstDesc d = a.inst[inst];
  const int32_t done = a.state[inst].done;
  asm volatile("" ::"s"(d.m), "s"(d.ld), "s"(d.a_off), "s"(d.coord_off), "s"(d.row_off),
               "s"(done));
  if (!a.ignore_done && done) return;
  if (a.cg_loop && a.cg[inst].done) return;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int col = col0 + 2 * l;
  const double *vec = (a.Bm ? a.y1 : a.y) + d.row_off;
  double ax = 0.0, ay = 0.0;
  if (col < d.ld) {
    const double *base = (a.Bm ? a.Bm : a.A) + d.a_off + col;
#pragma unroll 4
    for (int i = w; i < d.m; i += COL_WAVES) {
      const dvec2 *pm = reinterpret_cast<const dvec2 *>(base + (int64_t)i * d.ld);
      dvec2 m2;
      if constexpr (NTL) m2 = __builtin_nontemporal_load(pm);
      else m2 = *pm;
      const double yi = vec[i];
      ax += m2.x * yi;
      ay += m2.y * yi;
    }
  }
  __shared__ double2 red[COL_WAVES][64];
  red[w][l] = make_double2(ax, ay);
  __syncthreads();
  if (w == 0 && col < d.ld) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < COL_WAVES; ++k) {
      sx += red[k][l].x;
      sy += red[k][l].y;
    }
    const int64_t g = d.coord_off + col;
    if (RAW == 1) {
      a.u[g] = sx;
      a.u[g + 1] = sy;
    } else if (RAW == 2) {
      a.u[g] = a.w[g] * sx / a.D[g];
      a.u[g + 1] = a.w[g + 1] * sy / a.D[g + 1];
    } else {
      a.u[g] = (a.bhat[g] - sx) / a.D[g];
      a.u[g + 1] = (a.bhat[g + 1] - sy) / a.D[g + 1];
      if (a.cg_g) {
        a.cg_g[g] = sx;
        a.cg_g[g + 1] = sy;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The two substitutions with the cached factor, as triangular mat-vecs with
// the inverse factor (one wave per row, 16-byte loads, no LDS):
//   UPPER = 0:  y1[i] = sum_{k<=i} T[i][k] r[k]      (T = L^-1)
//   UPPER = 1:  y[i]  = sum_{k>=i} U[i][k] y1[k]     (U = L^-T)
// ---------------------------------------------------------------------------
template <int UPPER>
__global__ __launch_bounds__(256) void k_trmv_wave(AffineArgs a) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int32_t *rows = UPPER ? a.t3_rows : a.t_rows;
  if (wid >= (UPPER ? a.n_t3_rows : a.n_t_rows)) return;
  const int inst = rows[2 * wid], row = rows[2 * wid + 1];
  if (!a.ignore_done && a.state[inst].done) return;
  const InstDesc d = a.inst[inst];
  const int l = threadIdx.x & 63;
  const double *mat = (UPPER ? a.U : a.T) + d.t_off + (int64_t)row * d.ldm;
  const double *vec = (UPPER ? a.y1 : a.r) + d.row_off;
  // the matrix is zero outside [begin, end); both ends are even
  const int begin = UPPER ? (row & ~1) : 0;
  const int end = UPPER ? ((d.m + 1) & ~1) : ((row + 2) & ~1);
  const double2 *m2 = reinterpret_cast<const double2 *>(mat);
  const double2 *v2 = reinterpret_cast<const double2 *>(vec);
  double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 8
  for (int c = begin / 2 + l; c < end / 2; c += 64) {
    const double2 x = m2[c], y = v2[c];
    acc0 += x.x * y.x;
    acc1 += x.y * y.y;
  }
  const double sum = wave_sum(acc0 + acc1);
  if (l == 0) (UPPER ? a.y : a.y1)[d.row_off + row] = sum;
}

// ---------------------------------------------------------------------------
// Sparse A (CSR rows, CSC columns) for instances stored in SDP_A_CSR.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_csr_rowdot(AffineArgs a) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= a.n_csr_rows) return;
  const int inst = a.csr_rows[2 * wid], row = a.csr_rows[2 * wid + 1];
  if (!a.ignore_done && a.state[inst].done) return;
  if (a.cg_loop && a.cg[inst].done) return;
  const InstDesc d = a.inst[inst];
  const int l = threadIdx.x & 63;
  const int64_t t0 = a.a_rowptr[d.a_off + row], t1 = a.a_rowptr[d.a_off + row + 1];
  const double *v = a.v + d.coord_off;
  double acc = 0.0;
#pragma unroll 4
  for (int64_t t = t0 + l; t < t1; t += 64) acc += a.a_val[t] * v[a.a_col[t]];
  acc = wave_sum(acc);
  const double bs = a.dual ? -1.0 / a.state[inst].rho : 1.0;
  if (l == 0) a.r[d.row_off + row] = a.no_b ? acc : acc - bs * a.b[d.row_off + row];
}

// Transposed products with sparse A: CSC_G consecutive lanes share a column
// and read its nonzeros contiguously; their sums meet in a fixed butterfly.
constexpr int CSC_G = 8;
constexpr int CSC_COLS = 256 / CSC_G;   // columns per workgroup

template <int RAW>
__global__ __launch_bounds__(256) void k_csc_coldot(AffineArgs a) {
  const int inst = a.csc_cols[2 * blockIdx.x], col0 = a.csc_cols[2 * blockIdx.x + 1];
  if (!a.ignore_done && a.state[inst].done) return;
  if (a.cg_loop && a.cg[inst].done) return;
  const InstDesc d = a.inst[inst];
  const int col = col0 + (int)threadIdx.x / CSC_G, q = threadIdx.x % CSC_G;
  if (col >= d.ld) return;                 // whole lane groups leave together
  const int64_t g = d.coord_off + col;
  const double *y = a.y + d.row_off;
  double acc = 0.0;
  const int64_t t1 = a.a_colptr[g + 1];
  for (int64_t t = a.a_colptr[g] + q; t < t1; t += CSC_G) acc += a.a_cval[t] * y[a.a_row[t]];
#pragma unroll
  for (int o = 1; o < CSC_G; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (q == 0) {
    if (RAW == 1) {
      a.u[g] = acc;
    } else if (RAW == 2) {
      a.u[g] = a.w[g] * acc / a.D[g];
    } else {
      a.u[g] = (a.bhat[g] - acc) / a.D[g];
      if (a.cg_g) a.cg_g[g] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Residuals (PrimalConsensusResidual), stopping test and adaptive penalty.
// One workgroup per instance sums its cliques' partials (||X - Hx||^2,
// ||X||^2, ||Hx||^2, ||X - X_prev||^2, ||Lambda||^2, sweeps) in a fixed
// order.  The partial loads are issued before the `done` test so that the
// two memory round trips overlap.  With a fixed penalty the next iteration's
// scatter kernel runs these workgroups ahead of its own (k_scatter,
// res_blocks): the scatter needs only the penalty, and its outputs are
// scratch that the later kernels of an iteration that has stopped ignore.
// ---------------------------------------------------------------------------
__device__ inline double ratio(double num, double den) {
  if (den > 0.0) return num / den;
  return num == 0.0 ? 0.0 : INFINITY;
}

constexpr int RES_NT = 256;

__device__ void residual_block(const AffineArgs &a, int inst) {
  InstState &st = a.state[inst];
  const int64_t c0 = a.inst_cl_first[inst], c1 = a.inst_cl_first[inst + 1];
  double s[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
  for (int64_t k = c0 + threadIdx.x; k < c1; k += RES_NT) {
    const double2 *pk = reinterpret_cast<const double2 *>(a.part + NPART * k);
    const double2 q0 = pk[0], q1 = pk[1], q2 = pk[2];
    const double q6 = a.part[NPART * k + 6];   // sign-function fallback taken (0 or 1)
    s[0] += q0.x; s[1] += q0.y; s[2] += q1.x; s[3] += q1.y; s[4] += q2.x; s[5] += q2.y;
    s[6] += q6;
  }
  const int32_t done = st.done;
  __shared__ double red[RES_NT / 64][NPART];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int t = 0; t < NPART; ++t) {
    const double v = wave_sum(s[t]);
    if (l == 0) red[w][t] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0 || done) return;
  double S[NPART];
#pragma unroll
  for (int t = 0; t < NPART; ++t) {
    S[t] = 0.0;
#pragma unroll
    for (int i = 0; i < RES_NT / 64; ++i) S[t] += red[i][t];
  }
  const double rho = st.rho;
  const double nx = sqrt(S[1]), nhx = sqrt(S[2]);
  const double eps_c = ratio(sqrt(S[0]), nx > nhx ? nx : nhx);
  const double eps_l = ratio(rho * sqrt(S[3]), sqrt(S[4]));
  const int it = st.iter + 1;
  const SolverParams &P = a.params;
  if (a.hist && it - 1 < P.hist_cap) {
    double *h = a.hist + ((int64_t)inst * P.hist_cap + (it - 1)) * 3;
    h[0] = eps_c;
    h[1] = eps_l;
    h[2] = rho;
  }
  st.eps_c = eps_c;
  st.eps_l = eps_l;
  st.iter = it;
  st.total_sweeps += S[5];
  st.total_sign += S[6];
  if (P.no_stop) return;
  const double e = eps_c > eps_l ? eps_c : eps_l;
  if (e <= P.tol) {
    st.done = 1;
    return;
  }
  if (P.adaptive && P.rho_period > 0 && (it % P.rho_period) == 0) {
    if (eps_c >= P.nu * eps_l) st.rho = P.mu * rho;
    else if (eps_l >= P.nu * eps_c) st.rho = rho / P.mu;
  }
  if (it >= P.max_iter) st.done = 2;
}

__global__ __launch_bounds__(RES_NT) void k_residual_reduce(AffineArgs a) {
  residual_block(a, blockIdx.x);
}

// <C, X> = sum_j w_j c_j u_j per instance.
// Algorithm 2: b^T y per instance (the dual objective).
__global__ __launch_bounds__(256) void k_objective(AffineArgs a, double *obj) {
  const int inst = blockIdx.x;
  const InstDesc d = a.inst[inst];
  double s = 0.0;
  if (a.dual) {
    for (int64_t i = threadIdx.x; i < d.m; i += 256) s += a.b[d.row_off + i] * a.y[d.row_off + i];
  } else {
    for (int64_t j = threadIdx.x; j < d.ld; j += 256) {
      const int64_t g = d.coord_off + j;
      s += a.w[g] * a.c[g] * a.u[g];
    }
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) obj[inst] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// Diagnostics of the current iterate (the residuals eps_p, eps_d, eps_g
// (HSDEerror) with x = u, y_dual = -rho y, z = sum_k H_k^T lambda_k, and the
// PSD-completability violation eps_alpha (PSD-violation)).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_diag_coord(AffineArgs a, DiagScratch s) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= a.ncoord) return;
  // Algorithm 1: Z = sum_k H_k^T lambda_k and X = u;  Algorithm 2: Z = sum_k
  // H_k^T z_k and the primal estimate X = -rho x
  const double *zb = a.dual ? a.X : a.Lam;
  double z = 0.0;
  for (int64_t t = a.contrib_ptr[j]; t < a.contrib_ptr[j + 1]; ++t) z += zb[a.contrib_idx[t]];
  s.z[j] = z;
  const double xs = a.dual ? -a.state[a.coord_inst[j]].rho : 1.0;
  s.wu[j] = a.w[j] * xs * a.u[j];
}

__global__ __launch_bounds__(256) void k_diag_rows(AffineArgs a, DiagScratch s, int64_t nrow) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nrow) return;
  // instance of row i: rows are padded per instance, scan the descriptors
  int inst = 0;
  while (inst + 1 < a.batch && a.inst[inst + 1].row_off <= i) ++inst;
  s.yd[i] = a.dual ? a.y[i] : -a.state[inst].rho * a.y[i];   // Algorithm 2: y itself
}

__global__ __launch_bounds__(256) void k_diag_reduce(AffineArgs a, DiagScratch s,
                                                     const int64_t *cl_first, double *out) {
  const int inst = blockIdx.x;
  const InstDesc d = a.inst[inst];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t j = threadIdx.x; j < d.nnz; j += 256) {
    const int64_t g = d.coord_off + j;
    const double w = a.w[g], c = a.c[g], u = a.u[g];
    const double dd = s.aty[g] + s.z[g] - c;
    acc[0] += w * dd * dd;      // ||A^T y + z - c||^2 (full vec)
    acc[1] += w * c * c;        // ||c||^2
    acc[2] += w * c * u;        // c^T x
    acc[3] += w * u * u;        // ||X||_F^2 on the pattern
  }
  for (int i = threadIdx.x; i < d.m; i += 256) {
    const double r = s.ax[d.row_off + i], b = a.b[d.row_off + i];
    acc[4] += r * r;            // ||A x - b||^2
    acc[5] += b * b;
    acc[6] += b * s.yd[d.row_off + i];   // b^T y_dual
  }
  double mn = 0.0;
  for (int64_t k = cl_first[inst] + threadIdx.x; k < cl_first[inst + 1]; k += 256)
    mn = fmin(mn, s.lmin[k]);
  __shared__ double red[4][8];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int t = 0; t < 7; ++t) {
    const double v = wave_sum(acc[t]);
    if (l == 0) red[w][t] = v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if (l == 0) red[w][7] = mn;
  __syncthreads();
  if (threadIdx.x != 0) return;
  double S[8];
  for (int t = 0; t < 7; ++t) S[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
  S[7] = fmin(fmin(red[0][7], red[1][7]), fmin(red[2][7], red[3][7]));
  out[4 * inst + 0] = sqrt(S[4]) / (1.0 + sqrt(S[5]));
  out[4 * inst + 1] = sqrt(S[0]) / (1.0 + sqrt(S[1]));
  out[4 * inst + 2] = fabs(S[2] - S[6]) / (1.0 + fabs(S[2]) + fabs(S[6]));
  out[4 * inst + 3] = -S[7] / (1.0 + sqrt(S[3]));
}

__global__ __launch_bounds__(256) void k_scaled_copy(const double *src, double *dst, int64_t n,
                                                     const InstState *state, int inst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = -state[inst].rho * src[i];
}

// ---------------------------------------------------------------------------
// Affine step by preconditioned conjugate gradients (the iterative
// alternative to the factor, Section 4.1.1): M y = rhs with M = A W D^-1 A^T,
// Jacobi preconditioner diag(M), started from the previous iteration's y.
// The row products r0 = A W D^-1 (bhat - A^T y_prev) - b and M p =
// A (W D^-1 A^T p) reuse the row/column kernels above; the per-instance
// scalars (alpha, beta, the stopping test) live in one workgroup per
// instance; y, r, z and p are updated tile by tile over the instance's rows.
// ---------------------------------------------------------------------------
// Row vectors are split into tiles of CG_ROWS rows of one instance; the
// scalars of a step come from per-tile partial sums, which every consumer
// adds in tile order (fixed order: reproducible results).
constexpr int CG_NT = 256;
constexpr int CG_ROWS = 1024;

__device__ inline double cg_block_sum(double x, double *red) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CG_NT / 64; ++i) s += red[i];
  return s;
}

// sum of one partial over the tiles of an instance, by one whole wave (lane
// l takes tiles t0 + l, t0 + l + 64, ..., then the butterfly): every lane
// gets the same total, formed in a fixed order
__device__ inline double cg_tiles_sum(const double *part, int t0, int t1) {
  double s = 0.0;
  for (int t = t0 + (int)(threadIdx.x & 63); t < t1; t += 64) s += part[t];
  return wave_sum(s);
}

// MODE 0 (start): z = r / diag, p = z; partials r^T z, ||r||^2.
// MODE 1: partial p^T M p.
// MODE 2: alpha = r^T z / p^T M p; y += alpha p, r -= alpha M p, z = r / diag;
//         partials r^T z, ||r||^2.
// MODE 3: beta = r'^T z' / r^T z; p = z + beta p.
template <int MODE>
__global__ __launch_bounds__(CG_NT) void k_cg_rows(AffineArgs a) {
  const int inst = a.cg_tiles[2 * blockIdx.x], row0 = a.cg_tiles[2 * blockIdx.x + 1];
  if (!a.ignore_done && a.state[inst].done) return;
  const CgState c = a.cg[inst];
  if (MODE != 0 && c.done) return;
  const InstDesc d = a.inst[inst];
  const int row1 = min(d.m, row0 + CG_ROWS);
  const int t0 = a.cg_tile_first[inst], t1 = a.cg_tile_first[inst + 1];
  __shared__ double red[CG_NT / 64];
  double s0 = 0.0, s1 = 0.0;
  if (MODE == 0) {
    for (int i = row0 + threadIdx.x; i < row1; i += CG_NT) {
      const int64_t g = d.row_off + i;
      const double r = a.r[g], z = r / a.cg_diag[g];
      a.cg_z[g] = z;
      a.cg_p[g] = z;
      s0 += r * z;
      s1 += r * r;
    }
  } else if (MODE == 1) {
    for (int i = row0 + threadIdx.x; i < row1; i += CG_NT) {
      const int64_t g = d.row_off + i;
      s0 += a.cg_p[g] * a.cg_Mp[g];
    }
  } else if (MODE == 2) {
    const double alpha = c.rz / cg_tiles_sum(a.cg_part, t0, t1);
    for (int i = row0 + threadIdx.x; i < row1; i += CG_NT) {
      const int64_t g = d.row_off + i;
      a.y[g] += alpha * a.cg_p[g];
      const double r = a.r[g] - alpha * a.cg_Mp[g];
      const double z = r / a.cg_diag[g];
      a.r[g] = r;
      a.cg_z[g] = z;
      s0 += r * z;
      s1 += r * r;
    }
  } else {
    const double beta = cg_tiles_sum(a.cg_part + a.cg_ntiles, t0, t1) / c.rz;
    for (int i = row0 + threadIdx.x; i < row1; i += CG_NT) {
      const int64_t g = d.row_off + i;
      a.cg_p[g] = a.cg_z[g] + beta * a.cg_p[g];
    }
  }
  if (MODE == 3) return;
  s0 = cg_block_sum(s0, red);
  if (MODE != 1) s1 = cg_block_sum(s1, red);
  if (threadIdx.x == 0) {
    // MODE 1 writes slot 0 (p^T M p); MODES 0, 2 write slots 1, 2 (r^T z, ||r||^2)
    if (MODE == 1) {
      a.cg_part[blockIdx.x] = s0;
    } else {
      a.cg_part[a.cg_ntiles + blockIdx.x] = s0;
      a.cg_part[2 * a.cg_ntiles + blockIdx.x] = s1;
    }
  }
}

// Per instance, after MODE 0 (start = 1) or MODE 3 (start = 0): r^T z and
// ||r||^2 from the partials, step count and the stopping test.
__global__ __launch_bounds__(256) void k_cg_scalars(AffineArgs a, int start) {
  const int inst = blockIdx.x * 4 + (int)(threadIdx.x >> 6);   // one wave per instance
  if (inst >= a.batch) return;                                 // (uniform per wave)
  if (!a.ignore_done && a.state[inst].done) return;
  CgState c = a.cg[inst];
  if (!start && c.done) return;
  const int t0 = a.cg_tile_first[inst], t1 = a.cg_tile_first[inst + 1];
  c.rz = cg_tiles_sum(a.cg_part + a.cg_ntiles, t0, t1);
  c.rn2 = cg_tiles_sum(a.cg_part + 2 * a.cg_ntiles, t0, t1);
  if ((threadIdx.x & 63) != 0) return;
  if (start) {
    c.steps = 0;
    c.done = (a.cg_max_iter <= 0 || c.rn2 <= a.cg_tol2[inst]) ? 1 : 0;
  } else {
    c.steps += 1;
    c.total += 1;
    c.done = (c.steps >= a.cg_max_iter || c.rn2 <= a.cg_tol2[inst]) ? 1 : 0;
  }
  a.cg[inst] = c;
}

// diag(A W D^-1 A^T)_i = sum_j A_ij^2 w_j / D_j, one wave per row.
__global__ __launch_bounds__(256) void k_cg_diag(AffineArgs a, const double *wd,
                                                 const int32_t *rows, int nrows, double *out) {
  const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wid >= nrows) return;
  const int inst = rows[2 * wid], row = rows[2 * wid + 1];
  const InstDesc d = a.inst[inst];
  const int l = threadIdx.x & 63;
  double acc = 0.0;
  if (d.a_format == 0) {                 // dense rows (SDP_A_DENSE)
    const double *arow = a.A + d.a_off + (int64_t)row * d.ld;
    for (int j = l; j < d.nnz; j += 64) acc += arow[j] * arow[j] * wd[d.coord_off + j];
  } else {
    const int64_t t0 = a.a_rowptr[d.a_off + row], t1 = a.a_rowptr[d.a_off + row + 1];
    for (int64_t t = t0 + l; t < t1; t += 64)
      acc += a.a_val[t] * a.a_val[t] * wd[d.coord_off + a.a_col[t]];
  }
  acc = wave_sum(acc);
  if (l == 0) out[d.row_off + row] = acc;
}

// Dense row and column passes with the tile height and load kind of `a`.
template <bool NTL>
void rowdot_tiles(const AffineArgs &a, hipStream_t st) {
  const dim3 g(a.n_row_tiles), b(ROW_NT);
  switch (a.rows_per_tile) {
    case 1: hipLaunchKernelGGL((k_rowdot<1, NTL>), g, b, 0, st, a); break;
    case 2: hipLaunchKernelGGL((k_rowdot<2, NTL>), g, b, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_rowdot<4, NTL>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_rowdot<MAX_R, NTL>), g, b, 0, st, a); break;
  }
}

void launch_dense_rowdot(const AffineArgs &a, hipStream_t st) {
  if (a.n_row_tiles <= 0) return;
  if (a.stream_nt) rowdot_tiles<true>(a, st);
  else rowdot_tiles<false>(a, st);
}

template <int RAW>
void launch_dense_coldot(const AffineArgs &a, hipStream_t st) {
  if (a.n_col_tiles <= 0) return;
  if (a.stream_nt)
    hipLaunchKernelGGL((k_coldot<RAW, true>), dim3(a.n_col_tiles), dim3(COL_NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_coldot<RAW, false>), dim3(a.n_col_tiles), dim3(COL_NT), 0, st, a);
}

}  // namespace

// Stages of the X-step, launched in this order every iteration:
//   0 scatter (bhat, v)   1 A v - b (B v - T b)   2 T r   3 T^T y1   4 (bhat - A^T y)/D
// Stages 2 and 3 run over the rows in t_rows / t3_rows only (with B formed,
// the rows of sparse instances; 3 over all rows when the multiplier is needed).
hipError_t launch_affine_stage(const AffineArgs &a, int stage, hipStream_t st) {
  switch (stage) {
    case 0: {
      const int nb = (int)((a.ncoord * SC_LANES + 255) / 256) + a.res_blocks;
      hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, st, a);
      break;
    }
    case 1:
      launch_dense_rowdot(a, st);
      if (a.n_csr_rows > 0)
        hipLaunchKernelGGL(k_csr_rowdot, dim3((a.n_csr_rows + 3) / 4), dim3(256), 0, st, a);
      break;
    case 2:
      if (a.n_t_rows > 0)
        hipLaunchKernelGGL(k_trmv_wave<0>, dim3((a.n_t_rows + 3) / 4), dim3(256), 0, st, a);
      break;
    case 3:
      if (a.n_t3_rows > 0)
        hipLaunchKernelGGL(k_trmv_wave<1>, dim3((a.n_t3_rows + 3) / 4), dim3(256), 0, st, a);
      break;
    case 4:
      launch_dense_coldot<0>(a, st);
      if (a.n_csc_cols > 0)
        hipLaunchKernelGGL(k_csc_coldot<0>, dim3(a.n_csc_cols), dim3(256), 0, st, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_iteration_affine(const AffineArgs &a, hipStream_t st) {
  for (int stage = 0; stage < 5; ++stage) {
    const hipError_t e = launch_affine_stage(a, stage, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_residual_reduce(const AffineArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_residual_reduce, dim3(a.batch), dim3(RES_NT), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_objective(const AffineArgs &a, double *obj, hipStream_t st) {
  hipLaunchKernelGGL(k_objective, dim3(a.batch), dim3(256), 0, st, a, obj);
  return hipGetLastError();
}

int affine_col_tile_width() { return COL_W; }
int affine_cg_tile_rows() { return CG_ROWS; }
int affine_csc_tile_width() { return CSC_COLS; }
int affine_max_rows_per_tile() { return MAX_R; }

// Diagnostics: needs the per-clique minimum eigenvalues in s.lmin already.
hipError_t launch_diagnostics(const AffineArgs &a0, const DiagScratch &s, const int64_t *cl_first,
                              int64_t nrow, double *out, hipStream_t st) {
  AffineArgs a = a0;
  a.ignore_done = 1;
  a.Bm = nullptr;             // residuals of the original data
  const int nb = (int)((a.ncoord + 255) / 256);
  hipLaunchKernelGGL(k_diag_coord, dim3(nb), dim3(256), 0, st, a, s);
  hipLaunchKernelGGL(k_diag_rows, dim3((nrow + 255) / 256), dim3(256), 0, st, a, s, nrow);
  AffineArgs ar = a;          // A (w u) - b with the problem's b
  ar.v = s.wu;
  ar.r = s.ax;
  ar.dual = 0;
  launch_dense_rowdot(ar, st);
  if (ar.n_csr_rows > 0)
    hipLaunchKernelGGL(k_csr_rowdot, dim3((ar.n_csr_rows + 3) / 4), dim3(256), 0, st, ar);
  AffineArgs at = a;          // A^T y_dual
  at.y = s.yd;
  at.u = s.aty;
  launch_dense_coldot<1>(at, st);
  if (at.n_csc_cols > 0)
    hipLaunchKernelGGL(k_csc_coldot<1>, dim3(at.n_csc_cols), dim3(256), 0, st, at);
  hipLaunchKernelGGL(k_diag_reduce, dim3(a.batch), dim3(256), 0, st, a, s, cl_first, out);
  return hipGetLastError();
}

hipError_t launch_scaled_copy(const double *src, double *dst, int64_t n, const InstState *state,
                              int inst, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scaled_copy, dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n, state,
                     inst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The affine step with conjugate gradients.  Every launch is issued for every
// step up to cg_max_iter, so the sequence can be captured in a graph; the
// kernels of an instance whose solve has stopped return at once.
// ---------------------------------------------------------------------------
namespace {

void launch_rowdots(const AffineArgs &a, hipStream_t st) {
  launch_dense_rowdot(a, st);
  if (a.n_csr_rows > 0)
    hipLaunchKernelGGL(k_csr_rowdot, dim3((a.n_csr_rows + 3) / 4), dim3(256), 0, st, a);
}

}  // namespace

hipError_t launch_cg_stage(const AffineArgs &a, int stage, hipStream_t st) {
  if (stage != 2) return launch_affine_stage(a, stage, st);
  const dim3 tg(a.cg_ntiles), sg((a.batch + 3) / 4);
  hipLaunchKernelGGL(k_cg_rows<0>, tg, dim3(CG_NT), 0, st, a);
  hipLaunchKernelGGL(k_cg_scalars, sg, dim3(256), 0, st, a, 1);
  AffineArgs at = a;        // v = W D^-1 A^T p
  at.y = a.cg_p;
  at.u = a.v;
  at.cg_loop = 1;
  AffineArgs ar = a;        // M p = A v
  ar.r = a.cg_Mp;
  ar.no_b = 1;
  ar.cg_loop = 1;
  for (int k = 0; k < a.cg_max_iter; ++k) {
    launch_dense_coldot<2>(at, st);
    if (at.n_csc_cols > 0)
      hipLaunchKernelGGL(k_csc_coldot<2>, dim3(at.n_csc_cols), dim3(256), 0, st, at);
    launch_rowdots(ar, st);
    hipLaunchKernelGGL(k_cg_rows<1>, tg, dim3(CG_NT), 0, st, a);
    hipLaunchKernelGGL(k_cg_rows<2>, tg, dim3(CG_NT), 0, st, a);
    hipLaunchKernelGGL(k_cg_rows<3>, tg, dim3(CG_NT), 0, st, a);
    hipLaunchKernelGGL(k_cg_scalars, sg, dim3(256), 0, st, a, 0);
  }
  return hipGetLastError();
}

hipError_t launch_cg_affine(const AffineArgs &a, hipStream_t st) {
  for (int stage : {0, 1, 2, 4}) {
    const hipError_t e = launch_cg_stage(a, stage, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cg_diag(const AffineArgs &a, const double *wd, const int32_t *rows, int nrows,
                          double *out, hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_diag, dim3((nrows + 3) / 4), dim3(256), 0, st, a, wd, rows, nrows, out);
  return hipGetLastError();
}
