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

#include <math.h>

namespace {

__device__ inline void tri_inv_a(int t, int &a, int &b) {
  int x = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  if ((x + 1) * (x + 2) / 2 <= t) ++x;
  if (x * (x + 1) / 2 > t) --x;
  a = x;
  b = t - x * (x + 1) / 2;
}

// Projection adjoint for the cliques of one size bucket (N <= 64).
template <typename T, int N>
__global__ __launch_bounds__(256) void k_adj_proj(AdjArgs a, const int32_t *__restrict__ list) {
  constexpr int NT = 256;
  constexpr int P = N + 1;
  __shared__ T Vs[N * P];
  __shared__ T Gs[N * P];
  __shared__ T Ts[N * P];
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
    Gs[i * P + j] = g;
  }
  for (int k = tid; k < N; k += NT) th[k] = eo[s * N + k];
  __syncthreads();
  // Ts = V^T G
  for (int e = tid; e < N * N; e += NT) {
    const int i = e / N, j = e % N;
    T acc = T(0);
    for (int k = 0; k < s; ++k) acc += Vs[k * P + i] * Gs[k * P + j];
    Ts[i * P + j] = acc;
  }
  __syncthreads();
  // Gs = (Ts V) o Gamma
  for (int e = tid; e < N * N; e += NT) {
    const int i = e / N, j = e % N;
    T acc = T(0);
    for (int k = 0; k < s; ++k) acc += Ts[i * P + k] * Vs[k * P + j];
    const T ti = th[i], tj = th[j];
    T gam;
    if (ti > T(0) && tj > T(0)) gam = T(1);
    else if (!(ti > T(0)) && !(tj > T(0))) gam = T(0);
    else gam = ((ti > T(0) ? ti : T(0)) - (tj > T(0) ? tj : T(0))) / (ti - tj);
    Gs[i * P + j] = acc * gam;
  }
  __syncthreads();
  // Ts = V Gs   (rows < s)
  for (int e = tid; e < s * N; e += NT) {
    const int i = e / N, j = e % N;
    T acc = T(0);
    for (int k = 0; k < N; ++k) acc += Vs[i * P + k] * Gs[k * P + j];
    Ts[i * P + j] = acc;
  }
  __syncthreads();
  // Wb = Ts V^T on the packed lower triangle, then the two cotangent updates
  const int npk = s * (s + 1) / 2;
  for (int e = tid; e < npk; e += NT) {
    int i, j;
    tri_inv_a(e, i, j);
    T acc = T(0);
    for (int k = 0; k < N; ++k) acc += Ts[i * P + k] * Vs[j * P + k];
    const double wb = (double)acc;
    const int64_t g = off + e;
    const double lb = a.Lb[g];
    a.Ub[g] = wb - rho * lb;
    a.Lb[g] = lb - wb / rho;
  }
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
  if (precision == 1) {
    switch (N) {
      case 16: hipLaunchKernelGGL((k_adj_proj<float, 16>), dim3(count), dim3(256), 0, st, a, list); break;
      case 32: hipLaunchKernelGGL((k_adj_proj<float, 32>), dim3(count), dim3(256), 0, st, a, list); break;
      case 48: hipLaunchKernelGGL((k_adj_proj<float, 48>), dim3(count), dim3(256), 0, st, a, list); break;
      case 64: hipLaunchKernelGGL((k_adj_proj<float, 64>), dim3(count), dim3(256), 0, st, a, list); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (N) {
      case 16: hipLaunchKernelGGL((k_adj_proj<double, 16>), dim3(count), dim3(256), 0, st, a, list); break;
      case 32: hipLaunchKernelGGL((k_adj_proj<double, 32>), dim3(count), dim3(256), 0, st, a, list); break;
      case 48: hipLaunchKernelGGL((k_adj_proj<double, 48>), dim3(count), dim3(256), 0, st, a, list); break;
      case 64: hipLaunchKernelGGL((k_adj_proj<double, 64>), dim3(count), dim3(256), 0, st, a, list); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

int adjoint_max_bucket() { return 64; }

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
