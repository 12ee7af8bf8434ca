// One-time factorisation of the X-step (Algorithm 1, data preprocessing):
//   M = A W D^-1 A^T    (the paper's A D^-1 A^T on compact coordinates)
//   M = L L^T           (blocked right-looking Cholesky, FP64)
//   T = L^-1            (blocked triangular inverse; the iteration then
//                        applies y = T^T (T r), i.e. the forward and backward
//                        substitutions with the cached factor, as two
//                        bandwidth-bound triangular mat-vecs)
//   B = T A             (dense A only: the forward substitution folded into
//                        A, so the iteration needs y1 = B v - T b and
//                        u = (bhat - B^T y1) / D: two passes, no substitution)
// Every instance's M lives at t_off with pitch ldm (m rounded up to 64); the
// padding is the identity, so all blocks are full 64 x 64 tiles.
#include "sdp_internal.h"

#include <math.h>

namespace {

constexpr int NB = 64;
constexpr int LP = NB + 1;   // LDS pitch

__device__ inline void load_tile(double (*dst)[LP], const double *src, int64_t pitch) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    dst[r][c] = src[(int64_t)r * pitch + c];
  }
}

__device__ inline void store_tile(double *dst, int64_t pitch, const double acc[4][4], int tx, int ty) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) dst[(int64_t)(ty * 4 + a) * pitch + tx * 4 + b] = acc[a][b];
}

// acc[a][b] += sum_k X[ty*4+a][k] * Y[tx*4+b][k]        (X Y^T)
__device__ inline void mm_abt(const double (*X)[LP], const double (*Y)[LP], double acc[4][4], int tx,
                              int ty) {
  for (int k = 0; k < NB; ++k) {
    double xa[4], yb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xa[a] = X[ty * 4 + a][k];
#pragma unroll
    for (int b = 0; b < 4; ++b) yb[b] = Y[tx * 4 + b][k];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * yb[b];
  }
}

// acc[a][b] += sum_k X[ty*4+a][k] * Y[k][tx*4+b]         (X Y)
__device__ inline void mm_ab(const double (*X)[LP], const double (*Y)[LP], double acc[4][4], int tx,
                             int ty) {
  for (int k = 0; k < NB; ++k) {
    double xa[4], yb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) xa[a] = X[ty * 4 + a][k];
#pragma unroll
    for (int b = 0; b < 4; ++b) yb[b] = Y[k][tx * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * yb[b];
  }
}

// ---------------------------------------------------------------------------
// M = A W D^-1 A^T for dense A: one workgroup per lower 64 x 64 tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_syrk_dense(FactorArgs f, const int32_t *tiles) {
  const int inst = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1],
            tj = tiles[3 * blockIdx.x + 2];
  const InstDesc d = f.inst[inst];
  const int i0 = ti * NB, j0 = tj * NB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double sa[NB][33], sb[NB][33];
  double acc[4][4] = {};
  const double *A = f.A + d.a_off;
  const double *wd = f.wd + d.coord_off;
  for (int k0 = 0; k0 < d.ld; k0 += 32) {
    for (int e = threadIdx.x; e < NB * 32; e += 256) {
      const int r = e >> 5, k = e & 31;
      const int ia = i0 + r, ja = j0 + r;
      sa[r][k] = ia < d.m ? A[(int64_t)ia * d.ld + k0 + k] * wd[k0 + k] : 0.0;
      sb[r][k] = ja < d.m ? A[(int64_t)ja * d.ld + k0 + k] : 0.0;
    }
    __syncthreads();
    for (int k = 0; k < 32; ++k) {
      double xa[4], yb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = sa[ty * 4 + a][k];
#pragma unroll
      for (int b = 0; b < 4; ++b) yb[b] = sb[tx * 4 + b][k];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += xa[a] * yb[b];
    }
    __syncthreads();
  }
  double *M = f.M + d.t_off;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = i0 + ty * 4 + a, j = j0 + tx * 4 + b;
      double v = acc[a][b];
      if (i >= d.m || j >= d.m) v = (i == j) ? 1.0 : 0.0;
      M[(int64_t)i * d.ldm + j] = v;
    }
}

// ---------------------------------------------------------------------------
// M = A W D^-1 A^T for CSR A: one wave per row i accumulates row i of M in
// LDS, visiting the nonzeros A_ij in increasing j and, for each, the entries
// A_kj (k <= i) of column j (CSC).  Lanes touch distinct k, so there are no
// conflicts and each M_ik is summed in increasing j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_syrk_csr(FactorArgs f, const int32_t *rows) {
  extern __shared__ double accrow[];
  const int inst = rows[2 * blockIdx.x], i = rows[2 * blockIdx.x + 1];
  const InstDesc d = f.inst[inst];
  const int l = threadIdx.x;
  for (int k = l; k < d.ldm; k += 64) accrow[k] = 0.0;
  __syncthreads();
  const int64_t t0 = f.a_rowptr[d.a_off + i], t1 = f.a_rowptr[d.a_off + i + 1];
  for (int64_t t = t0; t < t1; ++t) {
    const int j = f.a_col[t];
    const int64_t g = d.coord_off + j;
    const double fa = f.a_val[t] * f.wd[g];
    for (int64_t s = f.a_colptr[g] + l; s < f.a_colptr[g + 1]; s += 64) {
      const int k = f.a_row[s];
      if (k <= i) accrow[k] += fa * f.a_cval[s];
    }
    __syncthreads();
  }
  double *M = f.M + d.t_off + (int64_t)i * d.ldm;
  for (int k = l; k <= i; k += 64) M[k] = accrow[k];
}

__global__ __launch_bounds__(64) void k_pad_identity(FactorArgs f) {
  const InstDesc d = f.inst[blockIdx.x];
  for (int i = d.m + threadIdx.x; i < d.ldm; i += 64) f.M[d.t_off + (int64_t)i * d.ldm + i] = 1.0;
  if (f.diag_shift != 0.0)   // I + A P^-1 A^T of the self-dual embedding
    for (int i = threadIdx.x; i < d.m; i += 64) f.M[d.t_off + (int64_t)i * d.ldm + i] += f.diag_shift;
}

// ---------------------------------------------------------------------------
// Blocked Cholesky, step kb: factor the diagonal block ...
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_potrf_diag(FactorArgs f, int kb) {
  const int inst = blockIdx.x;
  const InstDesc d = f.inst[inst];
  if (kb >= d.ldm / NB) return;
  double *blk = f.M + d.t_off + (int64_t)kb * NB * d.ldm + kb * NB;
  __shared__ double L[NB][LP];
  load_tile(L, blk, d.ldm);
  __syncthreads();
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  for (int j = 0; j < NB; ++j) {
    if (threadIdx.x == 0) {
      double dj = L[j][j];
      if (!(dj > 0.0)) {
        bad = 1;
        dj = 1.0;
      }
      L[j][j] = sqrt(dj);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < NB; i += 256) L[i][j] /= L[j][j];
    __syncthreads();
    const int rem = NB - j - 1;
    for (int e = threadIdx.x; e < rem * rem; e += 256) {
      const int i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    blk[(int64_t)r * d.ldm + c] = c <= r ? L[r][c] : 0.0;
  }
  if (threadIdx.x == 0 && bad) f.fail[inst] = 1;
}

// ... solve the panel below it: L_ib,kb = M_ib,kb L_kb,kb^-T ...
__global__ __launch_bounds__(256) void k_trsm_panel(FactorArgs f, int kb) {
  const int inst = blockIdx.x, ib = blockIdx.y;
  const InstDesc d = f.inst[inst];
  const int nblk = d.ldm / NB;
  if (kb >= nblk || ib <= kb || ib >= nblk) return;
  __shared__ double L[NB][LP], B[NB][LP];
  const double *lkk = f.M + d.t_off + (int64_t)kb * NB * d.ldm + kb * NB;
  double *bik = f.M + d.t_off + (int64_t)ib * NB * d.ldm + kb * NB;
  load_tile(L, lkk, d.ldm);
  load_tile(B, bik, d.ldm);
  __syncthreads();
  if (threadIdx.x < NB) {
    const int r = threadIdx.x;
    for (int c = 0; c < NB; ++c) {
      double x = B[r][c];
      for (int t = 0; t < c; ++t) x -= B[r][t] * L[c][t];
      B[r][c] = x / L[c][c];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    bik[(int64_t)r * d.ldm + c] = B[r][c];
  }
}

// ... and update the trailing matrix: M_ib,jb -= L_ib,kb L_jb,kb^T.
__global__ __launch_bounds__(256) void k_syrk_update(FactorArgs f, int kb) {
  const int inst = blockIdx.x, ib = blockIdx.y, jb = blockIdx.z;
  const InstDesc d = f.inst[inst];
  const int nblk = d.ldm / NB;
  if (kb >= nblk || jb <= kb || jb > ib || ib >= nblk) return;
  __shared__ double X[NB][LP], Y[NB][LP];
  const double *base = f.M + d.t_off;
  load_tile(X, base + (int64_t)ib * NB * d.ldm + kb * NB, d.ldm);
  load_tile(Y, base + (int64_t)jb * NB * d.ldm + kb * NB, d.ldm);
  __syncthreads();
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  mm_abt(X, Y, acc, tx, ty);
  double *out = f.M + d.t_off + (int64_t)ib * NB * d.ldm + jb * NB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) out[(int64_t)(ty * 4 + a) * d.ldm + tx * 4 + b] -= acc[a][b];
}

// ---------------------------------------------------------------------------
// T = L^-1: diagonal blocks T_jj = L_jj^-1 (column-wise forward substitution),
// then block sub-diagonals T_ij = -T_ii sum_{k=j}^{i-1} L_ik T_kj, i = j + dlt.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_trtri_diag(FactorArgs f) {
  const int inst = blockIdx.x, jb = blockIdx.y;
  const InstDesc d = f.inst[inst];
  if (jb >= d.ldm / NB) return;
  __shared__ double L[NB][LP], X[NB][LP];
  load_tile(L, f.M + d.t_off + (int64_t)jb * NB * d.ldm + jb * NB, d.ldm);
  __syncthreads();
  if (threadIdx.x < NB) {
    const int c = threadIdx.x;
    for (int r = 0; r < NB; ++r) {
      double x;
      if (r < c) {
        x = 0.0;
      } else {
        x = (r == c) ? 1.0 : 0.0;
        for (int t = c; t < r; ++t) x -= L[r][t] * X[t][c];
        x /= L[r][r];
      }
      X[r][c] = x;
    }
  }
  __syncthreads();
  double *dst = f.T + d.t_off + (int64_t)jb * NB * d.ldm + jb * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    dst[(int64_t)r * d.ldm + c] = X[r][c];
  }
}

__global__ __launch_bounds__(256) void k_trtri_offdiag(FactorArgs f, int dlt) {
  const int inst = blockIdx.x, jb = blockIdx.y;
  const InstDesc d = f.inst[inst];
  const int nblk = d.ldm / NB;
  const int ib = jb + dlt;
  if (ib >= nblk) return;
  __shared__ double X[NB][LP], Y[NB][LP];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  const double *Lb = f.M + d.t_off;
  const double *Tb = f.T + d.t_off;
  for (int kb = jb; kb < ib; ++kb) {
    load_tile(X, Lb + (int64_t)ib * NB * d.ldm + kb * NB, d.ldm);
    load_tile(Y, Tb + (int64_t)kb * NB * d.ldm + jb * NB, d.ldm);
    __syncthreads();
    mm_ab(X, Y, acc, tx, ty);
    __syncthreads();
  }
  // Y <- S (the accumulated sum), X <- T_ii
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Y[ty * 4 + a][tx * 4 + b] = acc[a][b];
  load_tile(X, Tb + (int64_t)ib * NB * d.ldm + ib * NB, d.ldm);
  __syncthreads();
  double out[4][4] = {};
  mm_ab(X, Y, out, tx, ty);
  double *dst = f.T + d.t_off + (int64_t)ib * NB * d.ldm + jb * NB;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) dst[(int64_t)(ty * 4 + a) * d.ldm + tx * 4 + b] = -out[a][b];
}

// U = T^T, tile by tile through LDS.
__global__ __launch_bounds__(256) void k_transpose_factor(FactorArgs f) {
  const int inst = blockIdx.x, ib = blockIdx.y, jb = blockIdx.z;
  const InstDesc d = f.inst[inst];
  const int nblk = d.ldm / NB;
  if (ib >= nblk || jb >= nblk) return;
  __shared__ double X[NB][LP];
  load_tile(X, f.T + d.t_off + (int64_t)ib * NB * d.ldm + jb * NB, d.ldm);
  __syncthreads();
  double *dst = f.U + d.t_off + (int64_t)jb * NB * d.ldm + ib * NB;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int r = e >> 6, c = e & 63;
    dst[(int64_t)r * d.ldm + c] = X[c][r];
  }
}

}  // namespace

// The launch sequence needs host-side tile lists; it is driven from the host
// setup code through these entry points.
hipError_t launch_syrk_dense(const FactorArgs &f, const int32_t *tiles, int ntiles,
                             hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_syrk_dense, dim3(ntiles), dim3(256), 0, st, f, tiles);
  return hipGetLastError();
}

hipError_t launch_syrk_csr(const FactorArgs &f, const int32_t *rows, int nrows, int max_ldm,
                           hipStream_t st) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_syrk_csr, dim3(nrows), dim3(64), (size_t)max_ldm * sizeof(double), st, f,
                     rows);
  return hipGetLastError();
}

namespace {
// B = T A for one 64 x 64 tile of one dense instance (rows < m are stored;
// T is lower triangular, so the k-loop stops at the tile's last row).
__global__ __launch_bounds__(256) void k_form_b(FactorArgs f, const int32_t *tiles) {
  const int inst = tiles[3 * blockIdx.x], ti = tiles[3 * blockIdx.x + 1],
            tj = tiles[3 * blockIdx.x + 2];
  const InstDesc d = f.inst[inst];
  const int i0 = ti * NB, j0 = tj * NB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ double st[NB][LP], sa[NB][LP];
  double acc[4][4] = {};
  const double *T = f.T + d.t_off;
  const double *A = f.A + d.a_off;
  const int kend = min(i0 + NB, d.m);
  for (int k0 = 0; k0 < kend; k0 += NB) {
    for (int e = threadIdx.x; e < NB * NB; e += 256) {
      const int r = e >> 6, c = e & 63;
      st[r][c] = T[(int64_t)(i0 + r) * d.ldm + k0 + c];
      sa[r][c] = (k0 + r < d.m) ? A[(int64_t)(k0 + r) * d.ld + j0 + c] : 0.0;
    }
    __syncthreads();
    mm_ab(st, sa, acc, tx, ty);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = i0 + ty * 4 + a;
    if (row < d.m) {
#pragma unroll
      for (int b = 0; b < 4; ++b) f.Bout[d.a_off + (int64_t)row * d.ld + j0 + tx * 4 + b] = acc[a][b];
    }
  }
}
}  // namespace

hipError_t launch_form_b(const FactorArgs &f, const int32_t *tiles, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_form_b, dim3(ntiles), dim3(256), 0, st, f, tiles);
  return hipGetLastError();
}

hipError_t launch_cholesky_and_inverse(const FactorArgs &f, int max_nblk, hipStream_t st) {
  hipLaunchKernelGGL(k_pad_identity, dim3(f.batch), dim3(64), 0, st, f);
  for (int kb = 0; kb < max_nblk; ++kb) {
    hipLaunchKernelGGL(k_potrf_diag, dim3(f.batch), dim3(256), 0, st, f, kb);
    if (kb + 1 < max_nblk) {
      hipLaunchKernelGGL(k_trsm_panel, dim3(f.batch, max_nblk), dim3(256), 0, st, f, kb);
      hipLaunchKernelGGL(k_syrk_update, dim3(f.batch, max_nblk, max_nblk), dim3(256), 0, st, f,
                         kb);
    }
  }
  hipLaunchKernelGGL(k_trtri_diag, dim3(f.batch, max_nblk), dim3(256), 0, st, f);
  for (int dlt = 1; dlt < max_nblk; ++dlt)
    hipLaunchKernelGGL(k_trtri_offdiag, dim3(f.batch, max_nblk - dlt), dim3(256), 0, st, f, dlt);
  hipLaunchKernelGGL(k_transpose_factor, dim3(f.batch, max_nblk, max_nblk), dim3(256), 0, st, f);
  return hipGetLastError();
}
