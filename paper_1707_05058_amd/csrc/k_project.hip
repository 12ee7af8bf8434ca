// PSD projection of clique blocks on gfx950 (the Y-step (XkUpdate) of
// Algorithm 1, fused with the multiplier update (LambdakUpdate) and the
// per-clique partial sums of the residuals (PrimalConsensusResidual)).
//
// One workgroup owns one clique block.  The block W_k (padded to even size N,
// zero padding is exact: a rotation whose off-diagonal entry is exactly zero
// is the identity) and its eigenvector matrix V live in LDS.  The symmetric
// eigenproblem is solved by the two-sided Jacobi method in parallel
// (round-robin) order: in each of the N-1 rounds of a sweep the N/2 disjoint
// index pairs are rotated at once, so J^T A J splits into independent 2x2
// block updates.  Rotations use the stable formulas of Rutishauser (the 2x2
// symmetric Schur decomposition).  Sweeps stop when off(A) <= tol * ||A||_F.
// The projection is rebuilt as X = V diag(max(theta, 0)) V^T.
#include "sdp_internal.h"

#include <math.h>

namespace {

enum Mode { MODE_ADMM = 0, MODE_STANDALONE = 1, MODE_MINEIG = 2 };

template <typename T> struct Big;
template <> struct Big<float> { static constexpr float v = 1e18f; };
template <> struct Big<double> { static constexpr double v = 1e150; };

__device__ inline float tsqrt(float x) { return sqrtf(x); }
__device__ inline double tsqrt(double x) { return sqrt(x); }

// (c, s) zeroing a_pq of J^T A J with J = [[c, s], [-s, c]] on (p, q); t = s/c.
template <typename T>
__device__ inline void sym_rotation(T app, T aqq, T apq, T &c, T &s, T &t) {
  if (apq == T(0)) {
    c = T(1); s = T(0); t = T(0);
    return;
  }
  const T tau = (aqq - app) / (T(2) * apq);
  const T at = fabs(tau);
  const T tt = (at > Big<T>::v) ? T(0.5) / at : T(1) / (at + tsqrt(T(1) + tau * tau));
  t = (tau >= T(0)) ? tt : -tt;
  c = T(1) / tsqrt(T(1) + t * t);
  s = t * c;
}

// Round-robin tournament: the k-th pair of round r among N (even) indices.
__device__ inline void rr_pair(int N, int r, int k, int &p, int &q) {
  int a, b;
  if (k == 0) {
    a = N - 1;
    b = r;
  } else {
    a = (r + k) % (N - 1);
    b = (r - k + N - 1) % (N - 1);
  }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// t -> (a, b) with a >= b, t = a(a+1)/2 + b.
__device__ inline void tri_inv(int t, int &a, int &b) {
  int x = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  if ((x + 1) * (x + 2) / 2 <= t) ++x;
  if (x * (x + 1) / 2 > t) --x;
  a = x;
  b = t - x * (x + 1) / 2;
}

template <int NT>
__device__ inline double block_sum(double v, double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (NT == 64) return v;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

template <typename T, int S, int NT, int MODE>
__global__ __launch_bounds__(NT) void k_project(ProjArgs a, const int32_t *__restrict__ list,
                                                const int32_t *__restrict__ sizes,
                                                const int64_t *__restrict__ offsets,
                                                const T *__restrict__ in, T *__restrict__ out,
                                                double *__restrict__ lmin_out, int max_sweeps,
                                                double tol) {
  constexpr int P = S + 1;
  __shared__ T As[S * P];
  __shared__ T Vs[S * P];
  __shared__ T rc[S / 2], rs[S / 2], rt[S / 2], th[S];
  __shared__ int rp[S / 2], rq[S / 2];
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  int s, cl = 0;
  int64_t off;
  double rho = 1.0;
  if (MODE == MODE_STANDALONE) {
    s = sizes[blockIdx.x];
    off = offsets[blockIdx.x];
    if (s <= 0 || s > S) return;   // sizes beyond max_size are left untouched
  } else {
    cl = list[blockIdx.x];
    const int inst = a.cl_inst[cl];
    if (MODE == MODE_ADMM && a.state[inst].done) return;
    s = a.cl_size[cl];
    off = a.cl_off[cl];
    rho = a.state[inst].rho;
  }
  const int N = s + (s & 1);

  // --- gather W_k = E_k U E_k^T - Lambda_k / rho (or the caller's block) ---
  double f2 = 0.0;
  for (int e = tid; e < N * N; e += NT) {
    const int i = e / N, j = e - (e / N) * N;
    T w = T(0);
    if (i < s && j < s) {
      if (MODE == MODE_STANDALONE) {
        w = T(0.5) * (in[off + (int64_t)i * s + j] + in[off + (int64_t)j * s + i]);
      } else {
        const int ii = i > j ? i : j, jj = i > j ? j : i;
        const int64_t g = off + (int64_t)ii * (ii + 1) / 2 + jj;
        double wd = a.u[a.blk_loc[g]];
        if (MODE == MODE_ADMM) wd -= a.Lam[g] / rho;
        w = (T)wd;
      }
    }
    As[i * P + j] = w;
    Vs[i * P + j] = (i == j) ? T(1) : T(0);
    f2 += (double)w * (double)w;
  }
  __syncthreads();
  const double nrm2 = block_sum<NT>(f2, red);   // includes the barrier
  const double thr = tol * tol * nrm2;
  const int K = N / 2;
  const int nA = K * (K + 1) / 2;
  const int nV = N * K;

  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double o2 = 0.0;
    for (int e = tid; e < N * N; e += NT) {
      const int i = e / N, j = e - (e / N) * N;
      if (i != j) {
        const double x = (double)As[i * P + j];
        o2 += x * x;
      }
    }
    o2 = block_sum<NT>(o2, red);
    if (!(o2 > thr)) break;
    for (int r = 0; r < N - 1; ++r) {
      if (tid < K) {
        int p, q;
        rr_pair(N, r, tid, p, q);
        T c, sn, t;
        sym_rotation<T>(As[p * P + p], As[q * P + q], As[p * P + q], c, sn, t);
        rc[tid] = c; rs[tid] = sn; rt[tid] = t; rp[tid] = p; rq[tid] = q;
      }
      __syncthreads();
      for (int it = tid; it < nA; it += NT) {
        int ia, ib;
        tri_inv(it, ia, ib);
        const int pa = rp[ia], qa = rq[ia];
        if (ia == ib) {
          const T t = rt[ia];
          const T apq = As[pa * P + qa];
          As[pa * P + pa] -= t * apq;
          As[qa * P + qa] += t * apq;
          As[pa * P + qa] = T(0);
          As[qa * P + pa] = T(0);
        } else {
          const int pb = rp[ib], qb = rq[ib];
          const T ca = rc[ia], sa = rs[ia], cb = rc[ib], sb = rs[ib];
          const T b00 = As[pa * P + pb], b01 = As[pa * P + qb];
          const T b10 = As[qa * P + pb], b11 = As[qa * P + qb];
          const T c00 = cb * b00 - sb * b01, c01 = sb * b00 + cb * b01;
          const T c10 = cb * b10 - sb * b11, c11 = sb * b10 + cb * b11;
          const T d00 = ca * c00 - sa * c10, d01 = ca * c01 - sa * c11;
          const T d10 = sa * c00 + ca * c10, d11 = sa * c01 + ca * c11;
          As[pa * P + pb] = d00; As[pa * P + qb] = d01;
          As[qa * P + pb] = d10; As[qa * P + qb] = d11;
          As[pb * P + pa] = d00; As[qb * P + pa] = d01;
          As[pb * P + qa] = d10; As[qb * P + qa] = d11;
        }
      }
      if (MODE != MODE_MINEIG) {
        for (int it = tid; it < nV; it += NT) {
          const int i = it / K, bb = it - (it / K) * K;
          const int pb = rp[bb], qb = rq[bb];
          const T cb = rc[bb], sb = rs[bb];
          const T vp = Vs[i * P + pb], vq = Vs[i * P + qb];
          Vs[i * P + pb] = cb * vp - sb * vq;
          Vs[i * P + qb] = sb * vp + cb * vq;
        }
      }
      __syncthreads();
    }
  }

  if (MODE == MODE_MINEIG) {
    double mn = 0.0;
    for (int k = 0; k < s; ++k) mn = fmin(mn, (double)As[k * P + k]);
    if (tid == 0) lmin_out[cl] = mn;
    return;
  }

  for (int k = tid; k < N; k += NT) {
    const T d = As[k * P + k];
    th[k] = d > T(0) ? d : T(0);
  }
  __syncthreads();

  // --- rebuild X = V diag(theta+) V^T on the packed lower triangle ---
  const int npk = s * (s + 1) / 2;
  double p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0;
  for (int e = tid; e < npk; e += NT) {
    int i, j;
    tri_inv(e, i, j);
    T acc = T(0);
    for (int k = 0; k < N; ++k) acc += Vs[i * P + k] * th[k] * Vs[j * P + k];
    if (MODE == MODE_STANDALONE) {
      out[off + (int64_t)i * s + j] = acc;
      out[off + (int64_t)j * s + i] = acc;
    } else {
      const int64_t g = off + e;
      const double hu = a.u[a.blk_loc[g]];
      const double xo = a.X[g], lo = a.Lam[g];
      const double xn = (double)acc;
      const double ln = lo + rho * (xn - hu);
      a.X[g] = xn;
      a.Lam[g] = ln;
      const double wt = (i == j) ? 1.0 : 2.0;
      const double dc = xn - hu, dx = xn - xo;
      p0 += wt * dc * dc;
      p1 += wt * xn * xn;
      p2 += wt * hu * hu;
      p3 += wt * dx * dx;
      p4 += wt * ln * ln;
    }
  }
  if (MODE == MODE_ADMM) {
    p0 = block_sum<NT>(p0, red);
    p1 = block_sum<NT>(p1, red);
    p2 = block_sum<NT>(p2, red);
    p3 = block_sum<NT>(p3, red);
    p4 = block_sum<NT>(p4, red);
    if (tid == 0) {
      double *pp = a.part + NPART * (int64_t)cl;
      pp[0] = p0; pp[1] = p1; pp[2] = p2; pp[3] = p3; pp[4] = p4;
      pp[5] = (double)sweep;
    }
  }
}

template <typename T, int S, int NT, int MODE>
hipError_t launch_one(int count, ProjArgs a, const int32_t *list, const int32_t *sizes,
                      const int64_t *offsets, const T *in, T *out, double *lmin, int msw,
                      double tol, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_project<T, S, NT, MODE>), dim3(count), dim3(NT), 0, st, a, list, sizes,
                     offsets, in, out, lmin, msw, tol);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t dispatch(int bucket, int count, ProjArgs a, const int32_t *list, const int32_t *sizes,
                    const int64_t *offsets, const T *in, T *out, double *lmin, int msw,
                    double tol, hipStream_t st);

template <int MODE>
hipError_t dispatch_f32(int bucket, int count, ProjArgs a, const int32_t *list,
                        const int32_t *sizes, const int64_t *offsets, const float *in, float *out,
                        double *lmin, int msw, double tol, hipStream_t st) {
  switch (bucket) {
    case 16: return launch_one<float, 16, 64, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 32: return launch_one<float, 32, 128, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 64: return launch_one<float, 64, 256, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 128: return launch_one<float, 128, 1024, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    default: return hipErrorInvalidValue;
  }
}

template <int MODE>
hipError_t dispatch_f64(int bucket, int count, ProjArgs a, const int32_t *list,
                        const int32_t *sizes, const int64_t *offsets, const double *in,
                        double *out, double *lmin, int msw, double tol, hipStream_t st) {
  switch (bucket) {
    case 16: return launch_one<double, 16, 64, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 32: return launch_one<double, 32, 128, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 64: return launch_one<double, 64, 256, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    case 96: return launch_one<double, 96, 512, MODE>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int projection_bucket(int precision, int s) {
  const int n = s + (s & 1);
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  if (precision == 1) return n <= 128 ? 128 : 0;
  return n <= 96 ? 96 : 0;
}

int projection_max_size(int precision) { return precision == 1 ? 128 : 96; }

hipError_t launch_admm_projection(int precision, int bucket, const int32_t *list, int count,
                                  const ProjArgs &a, hipStream_t st) {
  if (precision == 1)
    return dispatch_f32<MODE_ADMM>(bucket, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                   nullptr, a.max_sweeps, a.tol, st);
  return dispatch_f64<MODE_ADMM>(bucket, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                 nullptr, a.max_sweeps, a.tol, st);
}

hipError_t launch_standalone_projection(int dtype, int bucket, int count, const int32_t *sizes,
                                        const int64_t *offsets, const void *in, void *out,
                                        int max_sweeps, double tol, hipStream_t st) {
  ProjArgs a{};
  if (dtype == 1)
    return dispatch_f32<MODE_STANDALONE>(bucket, count, a, nullptr, sizes, offsets,
                                         (const float *)in, (float *)out, nullptr, max_sweeps,
                                         tol, st);
  return dispatch_f64<MODE_STANDALONE>(bucket, count, a, nullptr, sizes, offsets,
                                       (const double *)in, (double *)out, nullptr, max_sweeps,
                                       tol, st);
}

hipError_t launch_min_eig(int precision, int bucket, const int32_t *list, int count,
                          const ProjArgs &a, double *lmin_out, hipStream_t st) {
  if (precision == 1)
    return dispatch_f32<MODE_MINEIG>(bucket, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                     lmin_out, a.max_sweeps, a.tol, st);
  return dispatch_f64<MODE_MINEIG>(bucket, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                   lmin_out, a.max_sweeps, a.tol, st);
}
