// Reverse sweep of T unrolled iterations of Algorithm 1 (fixed rho): the
// vector-Jacobian product of u_T with respect to C and b.
//
// Forward, per iteration: bhat = sum_k H_k^T (X_k + L_k/rho) - c/rho;
// (u, y) from the KKT system (OptCondMinYPrimal); U_k = H_k u;
// W_k = U_k - L_k/rho; X_k' = P+(W_k) (XkUpdate); L_k' = L_k + rho (X_k' - U_k)
// (LambdakUpdate).  Cotangents of symmetric matrices are taken w.r.t. the
// Frobenius inner product (compact coordinates carry the weight w).  The
// reverse of one iteration, given the state cotangents (Xb, Lb):
//   k_adj_proj:    G = Xb + rho Lb;  Wb = DP+(W_k)[G];  Ub = Wb - rho Lb;
//                  Lb <- Lb - Wb / rho          (Daleckii-Krein, from V, theta)
//   k_adj_scatter: ubar = seed + sum_k H_k^T Ub  (adjoint of the gather)
//   affine stages: one KKT solve with b = 0: bhb = P ubar, ybar = multiplier
//   k_adj_coord:   cbar -= bhb / rho;  bbar += ybar
//   k_adj_gather:  Xb = H_k bhb;  Lb += H_k bhb / rho
// The eigenvectors and eigenvalues of each W_k come from a recomputation of
// the segment since the last checkpoint (k_project stores them).
#include "sdp_internal.h"
#include "mfma_tile.h"

#include <math.h>

namespace {

__device__ inline void tri_inv_a(int t, int &a, int &b) {
  int x = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  if ((x + 1) * (x + 2) / 2 <= t) ++x;
  if (x * (x + 1) / 2 > t) --x;
  a = x;
  b = t - x * (x + 1) / 2;
}

// Projection adjoint for the cliques of one size bucket: the four N x N
// products of the Daleckii-Krein form on the matrix cores (tile_product,
// 16x16x4 MFMA), V and one work block in LDS.  Each product is stored over
// its own input after the barrier inside tile_product:
//   B = V^T G;  B = (B V) o Gamma;  B = V B;  Wb = B V^T (lower tiles only,
//   written straight to the packed cotangents).
// V holds the eigenvectors as columns (rows >= s are zero), theta follows V
// in the clique's record.
template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_adj_proj(AdjArgs a, const int32_t *__restrict__ list) {
  constexpr int P = N + 1;
  __shared__ T Vs[N * P];
  __shared__ T Bs[N * P];
  __shared__ T th[N];
  const int cl = list[blockIdx.x];
  const int inst = a.cl_inst[cl];
  const int s = a.cl_size[cl];
  const int64_t off = a.cl_off[cl];
  const double rho = a.state[inst].rho;
  const T *eo = reinterpret_cast<const T *>(a.eig) + a.eig_off[cl];
  const int tid = threadIdx.x;
  for (int e = tid; e < N * N; e += NT) {
    const int i = e / N, j = e % N;
    Vs[i * P + j] = i < s ? eo[i * N + j] : T(0);
    T g = T(0);
    if (i < s && j < s) {
      const int ii = i > j ? i : j, jj = i > j ? j : i;
      const int64_t pk = off + (int64_t)ii * (ii + 1) / 2 + jj;
      g = (T)(a.Xb[pk] + rho * a.Lb[pk]);
    }
    Bs[i * P + j] = g;
  }
  for (int k = tid; k < N; k += NT) th[k] = eo[s * N + k];
  __syncthreads();
  // B = V^T G
  tile_product<T, N, NT, false>([&](int k, int q) { return Vs[k * P + q]; },
                                [&](int k, int q) { return Bs[k * P + q]; },
                                [&](int i, int j, T v) { Bs[i * P + j] = v; });
  __syncthreads();
  // B = (B V) o Gamma
  tile_product<T, N, NT, false>([&](int k, int q) { return Bs[q * P + k]; },
                                [&](int k, int q) { return Vs[k * P + q]; },
                                [&](int i, int j, T v) {
                                  const T ti = th[i], tj = th[j];
                                  T gam;
                                  if (ti > T(0) && tj > T(0)) gam = T(1);
                                  else if (!(ti > T(0)) && !(tj > T(0))) gam = T(0);
                                  else
                                    gam = ((ti > T(0) ? ti : T(0)) - (tj > T(0) ? tj : T(0))) /
                                          (ti - tj);
                                  Bs[i * P + j] = v * gam;
                                });
  __syncthreads();
  // B = V B
  tile_product<T, N, NT, false>([&](int k, int q) { return Vs[q * P + k]; },
                                [&](int k, int q) { return Bs[k * P + q]; },
                                [&](int i, int j, T v) { Bs[i * P + j] = v; });
  __syncthreads();
  // Wb = B V^T on the packed lower triangle, then the two cotangent updates
  tile_product<T, N, NT, true>([&](int k, int q) { return Bs[q * P + k]; },
                               [&](int k, int q) { return Vs[q * P + k]; },
                               [&](int i, int j, T v) {
                                 if (i < s && j <= i) {
                                   const int64_t g = off + (int64_t)i * (i + 1) / 2 + j;
                                   const double wb = (double)v;
                                   const double lb = a.Lb[g];
                                   a.Ub[g] = wb - rho * lb;
                                   a.Lb[g] = lb - wb / rho;
                                 }
                               });
}

__global__ __launch_bounds__(256) void k_adj_scatter(AdjArgs a) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= a.ncoord) return;
  const int inst = a.coord_inst[g];
  const InstDesc d = a.inst[inst];
  const int64_t j = g - d.coord_off;
  double u = 0.0;
  if (a.seed && j < d.nnz) {
    u = a.seed[a.user_coord_off[inst] + j];
    if (a.euclid) u /= a.w[g];
  }
  for (int64_t t = a.contrib_ptr[g]; t < a.contrib_ptr[g + 1]; ++t) u += a.Ub[a.contrib_idx[t]];
  a.bhat_bar[g] = u;
  a.v_bar[g] = a.w[g] * u / a.D[g];
}

__global__ __launch_bounds__(256) void k_adj_coord(AdjArgs a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < a.ncoord) {
    const int inst = a.coord_inst[t];
    const InstDesc d = a.inst[inst];
    const int64_t j = t - d.coord_off;
    if (j < d.nnz) {
      double v = -a.bhb[t] / a.state[inst].rho;
      if (a.euclid) v *= a.w[t];
      a.cbar[a.user_coord_off[inst] + j] += v;
    }
  }
  if (t < a.nrow) {
    const int inst = a.row_inst[t];
    const InstDesc d = a.inst[inst];
    const int64_t i = t - d.row_off;
    if (i < d.m) a.bbar[a.user_row_off[inst] + i] += a.y_bar[t];
  }
}

__global__ __launch_bounds__(256) void k_adj_gather(AdjArgs a) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.npk) return;
  const int64_t g = a.blk_loc[e];
  const int inst = a.coord_inst[g];
  const double v = a.bhb[g];
  a.Xb[e] = v;
  a.Lb[e] += v / a.state[inst].rho;
}

__global__ __launch_bounds__(256) void k_copy_user(const double *src, double *dst,
                                                   const InstDesc *inst, const int32_t *coord_inst,
                                                   const int64_t *user_coord_off, int64_t ncoord,
                                                   int to_user) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= ncoord) return;
  const int i = coord_inst[g];
  const InstDesc d = inst[i];
  const int64_t j = g - d.coord_off;
  if (j >= d.nnz) return;
  if (to_user) dst[user_coord_off[i] + j] = src[g];
  else dst[g] = src[user_coord_off[i] + j];
}

__global__ __launch_bounds__(256) void k_copy_user_rows(const double *src, double *dst,
                                                        const InstDesc *inst,
                                                        const int32_t *row_inst,
                                                        const int64_t *user_row_off, int64_t nrow) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= nrow) return;
  const int i = row_inst[r];
  const InstDesc d = inst[i];
  const int64_t k = r - d.row_off;
  if (k < d.m) dst[r] = src[user_row_off[i] + k];
}

}  // namespace

hipError_t launch_adj_projection(int precision, int N, const int32_t *list, int count,
                                 const AdjArgs &a, hipStream_t st) {
  if (count <= 0) return hipSuccess;
#define SDP_ADJ(T, n)                                                                          \
  case n:                                                                                      \
    hipLaunchKernelGGL((k_adj_proj<T, n, (n <= 64 ? 256 : 512)>), dim3(count),               \
                       dim3(n <= 64 ? 256 : 512), 0, st, a, list);                             \
    break;
  if (precision == 1) {
    switch (N) {
      SDP_ADJ(float, 16)
      SDP_ADJ(float, 32)
      SDP_ADJ(float, 48)
      SDP_ADJ(float, 64)
      SDP_ADJ(float, 80)
      SDP_ADJ(float, 96)
      SDP_ADJ(float, 112)
      SDP_ADJ(float, 128)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (N) {
      SDP_ADJ(double, 16)
      SDP_ADJ(double, 32)
      SDP_ADJ(double, 48)
      SDP_ADJ(double, 64)
      SDP_ADJ(double, 80)
      SDP_ADJ(double, 96)
      default: return hipErrorInvalidValue;
    }
  }
#undef SDP_ADJ
  return hipGetLastError();
}

int adjoint_max_bucket(int precision) { return precision == 1 ? 128 : 96; }

hipError_t launch_adj_scatter(const AdjArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_scatter, dim3((a.ncoord + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_adj_coord_and_gather(const AdjArgs &a, hipStream_t st) {
  const int64_t n = a.ncoord > a.nrow ? a.ncoord : a.nrow;
  hipLaunchKernelGGL(k_adj_coord, dim3((n + 255) / 256), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_adj_gather, dim3((a.npk + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_copy_user(const double *src, double *dst, const InstDesc *inst,
                            const int32_t *coord_inst, const int64_t *user_coord_off,
                            int64_t ncoord, int to_user, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_user, dim3((ncoord + 255) / 256), dim3(256), 0, st, src, dst, inst,
                     coord_inst, user_coord_off, ncoord, to_user);
  return hipGetLastError();
}

hipError_t launch_copy_user_rows(const double *src, double *dst, const InstDesc *inst,
                                 const int32_t *row_inst, const int64_t *user_row_off,
                                 int64_t nrow, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_user_rows, dim3((nrow + 255) / 256), dim3(256), 0, st, src, dst, inst,
                     row_inst, user_row_off, nrow);
  return hipGetLastError();
}
