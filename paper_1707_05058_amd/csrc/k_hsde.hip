// Algorithm 3 on gfx950: ADMM for the homogeneous self-dual embedding of the
// decomposed primal-dual pair (Section 5).  One iteration:
//   u_hat = (I + Q)^-1 (u + v)   (HsdeStep1) by the block eliminations of
//            Section 5.2: the outer system (LinearSystem) with the matrix
//            inversion lemma (MatrixInverseResult, FirstBlockElimination) and
//            the inner system (SecondBlockElimination) reduced to the m x m
//            factor of I + A P^-1 A^T, P = I + D/2 (HSDEFactorizationFinal)
//   u = P_K(u_hat - v)           (HsdeStep2: x, y, t free, s in the cliques'
//                                 PSD cones, tau >= 0)
//   v = v - u_hat + u            (HsdeStep3: only z and kappa are nonzero)
// then the residuals HSDEerror and the consensus residual, or the
// infeasibility tests (Infeasibility) once tau = 0.
//
// Vectors over the pattern are compact lower coordinates with weights w (1 on
// the diagonal, 2 off it): the paper's Euclidean products on vec(X) are the
// w-weighted sums here, A x is A (w .* x), and I stays the identity.  The
// inner solve, for nu = (nu_x, nu_s, nu_y, nu_t):
//   x'      = nu_x + H^T (nu_s + nu_t) / 2                 (k_hsde_xprime)
//   g       = (I + A W P^-1 A^T)^-1 (A W x'/P - nu_y)      (affine stages 1-3)
//   sigma_x = (x' - A^T g) / P,  sigma_y = -g              (affine stage 4)
//   sigma_s = (nu_s - nu_t + H sigma_x) / 2,  sigma_t = sigma_s - H sigma_x + nu_t
// and u_hat_1 = sigma - f M^-1 zeta, f = (zeta^T sigma) / (1 + zeta^T M^-1 zeta),
// u_hat_tau = omega_2 + f.  A u_x and A^T u_y for the residuals follow from
// quantities of the solve (A W sigma_x = nu_y + g, A^T g = x' - P sigma_x) and
// the set-up products A W M^-1 zeta_x, A^T M^-1 zeta_y: no extra pass over A.
#include "sdp_internal.h"

#include <math.h>

namespace {

constexpr int HS_LANES = 4;
constexpr int HS_NT = 1024;    // per-instance reductions: one workgroup per instance

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup (NT threads); every thread gets the total.
template <int NT>
__device__ inline double block_total(double v, double *red) {
  v = wsum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// NV workgroup totals at once (one pair of barriers; red holds NV * NT / 64
// doubles), each summed in block_total's order, so the totals are the same
// bit for bit.
template <int NT, int NV>
__device__ inline void block_total_n(double (&v)[NV], double *red) {
#pragma unroll
  for (int n = 0; n < NV; ++n) v[n] = wsum(v[n]);
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int n = 0; n < NV; ++n) red[n * (NT / 64) + (threadIdx.x >> 6)] = v[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[n * (NT / 64) + i];
    v[n] = s;
  }
}

__device__ inline double cratio(double num, double a, double b) {
  const double den = a > b ? a : b;
  if (den > 0.0) return num / den;
  return num == 0.0 ? 0.0 : INFINITY;
}

// nu = omega_1 - omega_2 zeta with omega = u + v; in set-up mode nu = zeta
// = (c, 0, -b, 0) (for M^-1 zeta).
__global__ __launch_bounds__(256) void k_hsde_form_nu(HsdeArgs h, int setup) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < h.ncoord) {
    const int inst = h.coord_inst[t];
    if (setup) h.nx[t] = h.c[t];
    else if (!h.state[inst].done) h.nx[t] = h.ux[t] - h.hs[inst].w2 * h.c[t];
  }
  if (t < h.npk) {
    const int inst = h.coord_inst[h.blk_loc[t]];
    if (setup) {
      h.ns[t] = 0.0;
      h.nt[t] = 0.0;
    } else if (!h.state[inst].done) {
      h.ns[t] = h.us[t] + h.vz[t];
      h.nt[t] = h.ut[t];
    }
  }
  if (t < h.nrow) {
    const int inst = h.row_inst[t];
    if (setup) h.ny[t] = -h.b[t];
    else if (!h.state[inst].done) h.ny[t] = h.uy[t] + h.hs[inst].w2 * h.b[t];
  }
}

// x' = nu_x + H^T (nu_s + nu_t) / 2 and v = w x' / P (four lanes per coordinate,
// fixed butterfly; workgroups numbered contiguously per XCD).
__global__ __launch_bounds__(256) void k_hsde_xprime(HsdeArgs h, const double *nx, const double *ns,
                                                     const double *nt) {
  const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
  const int64_t g = (int64_t)(x8 * q8 + min(x8, r8) + blockIdx.x / 8) * 256 + threadIdx.x;
  const int64_t j = g / HS_LANES;
  const int q = (int)(g % HS_LANES);
  if (j >= h.ncoord) return;
  const int inst = h.coord_inst[j];
  if (!h.ignore_done && h.state[inst].done) return;
  double acc = 0.0;
  const int64_t t1 = h.contrib_ptr[j + 1];
  for (int64_t t = h.contrib_ptr[j] + q; t < t1; t += HS_LANES) {
    const int32_t e = h.contrib_idx[t];
    acc += ns[e] + nt[e];
  }
#pragma unroll
  for (int o = 1; o < HS_LANES; o <<= 1) acc += __shfl_xor(acc, o, 64);
  if (q == 0) {
    const double x = nx[j] + 0.5 * acc;
    h.xp[j] = x;
    h.v[j] = h.w[j] * x / h.P[j];
  }
}

// Set-up, after the inner solve of nu = zeta: the blocks of M^-1 zeta.
__global__ __launch_bounds__(256) void k_hsde_zeta_blocks(HsdeArgs h) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= h.npk) return;
  const double hx = h.sx[h.blk_loc[e]];
  h.mzs[e] = 0.5 * hx;          // (0 - 0 + H sigma_x) / 2
  h.mzt[e] = -0.5 * hx;         // sigma_s - H sigma_x + 0
}

// Set-up, one workgroup per instance: M^-1 zeta on coordinates and rows,
// A W (M^-1 zeta)_x = -b + g, A^T (M^-1 zeta)_y = -(x' - P sigma_x), kz and
// the norms of b and c; tau = kappa = 1.
__global__ __launch_bounds__(HS_NT) void k_hsde_setup_finish(HsdeArgs h) {
  const int inst = blockIdx.x;
  const InstDesc d = h.inst[inst];
  __shared__ double red[HS_NT / 64];
  double zc = 0.0, nc2 = 0.0, zb = 0.0, nb2 = 0.0;
  for (int64_t j = d.coord_off + threadIdx.x; j < d.coord_off + d.ld; j += HS_NT) {
    const double sx = h.sx[j];
    h.mzx[j] = sx;
    h.atmz[j] = -(h.xp[j] - h.P[j] * sx);
    zc += h.w[j] * h.c[j] * sx;
    nc2 += h.w[j] * h.c[j] * h.c[j];
  }
  for (int64_t i = d.row_off + threadIdx.x; i < d.row_off + d.ldm; i += HS_NT) {
    const double g = h.g[i];
    h.mzy[i] = -g;
    h.az[i] = g - h.b[i];
    zb += h.b[i] * (-g);
    nb2 += h.b[i] * h.b[i];
  }
  zc = block_total<HS_NT>(zc, red);
  nc2 = block_total<HS_NT>(nc2, red);
  zb = block_total<HS_NT>(zb, red);
  nb2 = block_total<HS_NT>(nb2, red);
  if (threadIdx.x == 0) {
    HsdeState &s = h.hs[inst];
    s.kz = 1.0 / (1.0 + zc - zb);   // zeta^T M^-1 zeta = c^T mz_x - b^T mz_y
    s.nrm_b = sqrt(nb2);
    s.nrm_c = sqrt(nc2);
    s.tau = 1.0;
    s.kappa = 1.0;
    s.w2 = 2.0;
    s.f = 0.0;
  }
}

__global__ __launch_bounds__(256) void k_hsde_reset(HsdeArgs h) {
  const int inst = blockIdx.x * 256 + threadIdx.x;
  if (inst >= h.batch) return;
  HsdeState &s = h.hs[inst];
  s.tau = 1.0;
  s.kappa = 1.0;
  s.w2 = 2.0;
  s.f = 0.0;
  s.rp2 = s.ax2 = s.bty = s.ctx = 0.0;
  s.eps_p = s.eps_d = s.eps_g = INFINITY;
}

// The per-instance sums of the iteration are formed in two steps: every wave
// of 64 consecutive coordinates (or rows) -- never shared by two instances,
// whose ranges are padded to multiples of 64 -- writes its partial sums, and
// a per-instance pass adds them in a fixed order.
//   coordinate-wave slots: 0 c^T W sigma_x, 1 c^T W u_x, 2 ||A^T u_y + H^T v_z||_W^2,
//                          3 ||(A^T u_y + H^T v_z)/tau - c||_W^2
//   row-wave slots:        0 b^T g, 1 b^T u_y, 2 ||A W u_x||^2, 3 ||A W u_x - tau b||^2
constexpr int WSLOT = 4;

__global__ __launch_bounds__(256) void k_hsde_zs_partials(HsdeArgs h) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if (t < h.ncoord) {                                  // uniform per wave
    const double v = wsum(h.w[t] * h.c[t] * h.sx[t]);
    if (lane == 0) h.cw_part[(t >> 6) * WSLOT + 0] = v;
  }
  if (t < h.nrow) {
    const double v = wsum(h.b[t] * h.g[t]);            // -b^T sigma_y
    if (lane == 0) h.rw_part[(t >> 6) * WSLOT + 0] = v;
  }
}

// One workgroup per instance: zeta^T sigma from the wave partials (each
// thread a strided share, summed over the workgroup in a fixed order), then
// f = kz zeta^T sigma, u_hat_tau = omega_2 + f, tau = max(0, u_hat_tau -
// kappa), kappa -= u_hat_tau - tau.
__global__ __launch_bounds__(256) void k_hsde_scalars(HsdeArgs h) {
  __shared__ double red[4];
  const int inst = blockIdx.x;
  if (h.state[inst].done) return;   // uniform per workgroup
  const InstDesc d = h.inst[inst];
  double zs = 0.0;
  for (int64_t q = (d.coord_off >> 6) + threadIdx.x; q < (d.coord_off + d.ld) >> 6; q += 256)
    zs += h.cw_part[q * WSLOT];
  for (int64_t q = (d.row_off >> 6) + threadIdx.x; q < (d.row_off + d.ldm) >> 6; q += 256)
    zs += h.rw_part[q * WSLOT];
  zs = block_total<256>(zs, red);
  if (threadIdx.x != 0) return;
  HsdeState &s = h.hs[inst];
  const double f = s.kz * zs;
  const double uhat_tau = s.w2 + f;
  const double tau = uhat_tau - s.kappa > 0.0 ? uhat_tau - s.kappa : 0.0;
  s.f = f;
  s.kappa = s.kappa - uhat_tau + tau;
  s.tau = tau;
  s.w2 = s.tau + s.kappa;
}

// u_x = sigma_x - f mz_x, u_y = -g - f mz_y, A W u_x = nu_y + g - f A W mz_x,
// with their wave partial sums.
__global__ __launch_bounds__(256) void k_hsde_apply(HsdeArgs h) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  if (t < h.ncoord) {
    const int inst = h.coord_inst[t];
    double ctx = 0.0;
    if (!h.state[inst].done) {
      const double ux = h.sx[t] - h.hs[inst].f * h.mzx[t];
      h.ux[t] = ux;
      ctx = h.w[t] * h.c[t] * ux;
    }
    ctx = wsum(ctx);
    if (lane == 0) h.cw_part[(t >> 6) * WSLOT + 1] = ctx;
  }
  if (t < h.nrow) {
    const int inst = h.row_inst[t];
    double bty = 0.0, ax2 = 0.0, rp2 = 0.0;
    if (!h.state[inst].done) {
      const HsdeState &s = h.hs[inst];
      const double uy = -h.g[t] - s.f * h.mzy[t];
      h.uy[t] = uy;
      bty = h.b[t] * uy;
      const double aux = h.ny[t] + h.g[t] - s.f * h.az[t];
      ax2 = aux * aux;
      const double rp = aux - s.tau * h.b[t];
      rp2 = rp * rp;
    }
    bty = wsum(bty);
    ax2 = wsum(ax2);
    rp2 = wsum(rp2);
    if (lane == 0) {
      double *q = h.rw_part + (t >> 6) * WSLOT;
      q[1] = bty;
      q[2] = ax2;
      q[3] = rp2;
    }
  }
}

// After the projections: A^T u_y + H^T v_z on the coordinates (A^T g from the
// inner solve as x' - P sigma_x) and the dual-residual sums of each group of
// 64 coordinates.  A workgroup takes one group, four lanes per coordinate
// (each lane a strided share of the coordinate's clique entries, joined by a
// fixed butterfly), so the gathers of v_z overlap.
__global__ __launch_bounds__(256) void k_hsde_dual_partials(HsdeArgs h) {
  __shared__ double red[2 * 4];
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x >> 2);   // < ncoord (padded)
  const int q4 = threadIdx.x & 3;
  const int inst = h.coord_inst[j];
  const HsdeState &s = h.hs[inst];
  double hz = 0.0;
  for (int64_t t = h.contrib_ptr[j] + q4; t < h.contrib_ptr[j + 1]; t += 4)
    hz += h.vz[h.contrib_idx[t]];
  hz += __shfl_xor(hz, 1, 64);
  hz += __shfl_xor(hz, 2, 64);
  double v[2] = {0.0, 0.0};
  if (q4 == 0) {
    const double aty = -(h.xp[j] - h.P[j] * h.sx[j]) - s.f * h.atmz[j];
    const double q = aty + hz;
    v[0] = h.w[j] * q * q;
    if (s.tau > 0.0) {
      const double dd = q / s.tau - h.c[j];
      v[1] = h.w[j] * dd * dd;
    }
  }
  block_total_n<256, 2>(v, red);
  if (threadIdx.x == 0) {
    h.cw_part[(int64_t)blockIdx.x * WSLOT + 2] = v[0];
    h.cw_part[(int64_t)blockIdx.x * WSLOT + 3] = v[1];
  }
}

// One workgroup per instance: the wave and clique partial sums in a fixed
// order, the residuals HSDEerror and the consensus residual, the stopping
// test, or the infeasibility tests when tau = 0.
__global__ __launch_bounds__(256) void k_hsde_finish(HsdeArgs h) {
  const int inst = blockIdx.x;
  InstState &st = h.state[inst];
  if (st.done) return;
  const InstDesc d = h.inst[inst];
  HsdeState &s = h.hs[inst];
  __shared__ double red[13 * 4];
  double ctx = 0.0, r2 = 0.0, rd2 = 0.0, bty = 0.0, ax2 = 0.0, rp2 = 0.0;
  for (int64_t q = (d.coord_off >> 6) + threadIdx.x; q < (d.coord_off + d.ld) >> 6; q += 256) {
    const double *p = h.cw_part + q * WSLOT;
    ctx += p[1];
    r2 += p[2];
    rd2 += p[3];
  }
  for (int64_t q = (d.row_off >> 6) + threadIdx.x; q < (d.row_off + d.ldm) >> 6; q += 256) {
    const double *p = h.rw_part + q * WSLOT;
    bty += p[1];
    ax2 += p[2];
    rp2 += p[3];
  }
  double S[7] = {0, 0, 0, 0, 0, 0, 0};
  const int64_t c0 = h.inst_cl_first[inst], c1 = h.inst_cl_first[inst + 1];
  for (int64_t k = c0 + threadIdx.x; k < c1; k += 256) {
    const double *pk = h.part + NPART * k;
#pragma unroll
    for (int q = 0; q < 7; ++q) S[q] += pk[q];
  }
  double tot[13] = {ctx, r2, rd2, bty, ax2, rp2, S[0], S[1], S[2], S[3], S[4], S[5], S[6]};
  block_total_n<256, 13>(tot, red);
  if (threadIdx.x != 0) return;
  ctx = tot[0];
  r2 = tot[1];
  rd2 = tot[2];
  bty = tot[3];
  ax2 = tot[4];
  rp2 = tot[5];
#pragma unroll
  for (int q = 0; q < 7; ++q) S[q] = tot[6 + q];
  s.ctx = ctx;
  s.bty = bty;
  const SolverParams &P = h.params;
  const int it = st.iter + 1;
  const double tau = s.tau;
  double crit_e = INFINITY, eps_c = INFINITY;
  if (tau > 0.0) {
    const double cx = ctx / tau, by = bty / tau;
    s.eps_p = sqrt(rp2) / tau / (1.0 + s.nrm_b);
    s.eps_d = sqrt(rd2) / (1.0 + s.nrm_c);
    s.eps_g = fabs(cx - by) / (1.0 + fabs(cx) + fabs(by));
    const double e1 = cratio(sqrt(S[0]), sqrt(S[1]), sqrt(S[2]));
    const double e2 = cratio(sqrt(S[3]), sqrt(S[4]), sqrt(S[6]));
    eps_c = e1 > e2 ? e1 : e2;
    crit_e = s.eps_p;
    if (s.eps_d > crit_e) crit_e = s.eps_d;
    if (s.eps_g > crit_e) crit_e = s.eps_g;
  }
  if (h.hist && it - 1 < P.hist_cap) {
    double *hh = h.hist + ((int64_t)inst * P.hist_cap + (it - 1)) * 3;
    hh[0] = eps_c;
    hh[1] = crit_e;
    hh[2] = tau;
  }
  st.eps_c = eps_c;
  st.eps_l = crit_e;
  st.iter = it;
  st.total_sweeps += S[5];
  if (tau > 0.0) {
    const double crit = crit_e > eps_c ? crit_e : eps_c;
    if (crit <= P.tol) {
      st.done = 1;
      return;
    }
  } else {
    const double tp = sqrt(r2) - (s.nrm_b > 0.0 ? bty / s.nrm_b : 0.0) * P.tol;
    const double td = sqrt(ax2) + (s.nrm_c > 0.0 ? ctx / s.nrm_c : 0.0) * P.tol;
    if (tp <= 0.0 && bty > 0.0) {
      st.done = 3;
      return;
    }
    if (td <= 0.0 && ctx < 0.0) {
      st.done = 4;
      return;
    }
  }
  if (it >= P.max_iter) st.done = 2;
}

// x = u_x / tau and y = u_y / tau (the raw u_x, u_y when tau = 0).
__global__ __launch_bounds__(256) void k_hsde_solution(HsdeArgs h, double *x_out, double *y_out) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < h.ncoord) {
    const double tau = h.hs[h.coord_inst[t]].tau;
    x_out[t] = tau > 0.0 ? h.ux[t] / tau : h.ux[t];
  }
  if (t < h.nrow) {
    const double tau = h.hs[h.row_inst[t]].tau;
    y_out[t] = tau > 0.0 ? h.uy[t] / tau : h.uy[t];
  }
}

int64_t max3(int64_t a, int64_t b, int64_t c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }

}  // namespace

hipError_t launch_hsde_form_nu(const HsdeArgs &h, hipStream_t st) {
  const int64_t n = max3(h.ncoord, h.npk, h.nrow);
  hipLaunchKernelGGL(k_hsde_form_nu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, 0);
  return hipGetLastError();
}

hipError_t launch_hsde_xprime(const HsdeArgs &h, const double *nx, const double *ns,
                              const double *nt, hipStream_t st) {
  const int64_t n = h.ncoord * HS_LANES;
  hipLaunchKernelGGL(k_hsde_xprime, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, nx, ns,
                     nt);
  return hipGetLastError();
}

hipError_t launch_hsde_setup_finish(const HsdeArgs &h, hipStream_t st) {
  // the set-up inner solve runs between these two: form nu = zeta first
  if (h.npk > 0)
    hipLaunchKernelGGL(k_hsde_zeta_blocks, dim3((unsigned)((h.npk + 255) / 256)), dim3(256), 0, st,
                       h);
  hipLaunchKernelGGL(k_hsde_setup_finish, dim3(h.batch), dim3(HS_NT), 0, st, h);
  return hipGetLastError();
}

hipError_t launch_hsde_setup_nu(const HsdeArgs &h, hipStream_t st) {
  const int64_t n = max3(h.ncoord, h.npk, h.nrow);
  hipLaunchKernelGGL(k_hsde_form_nu, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, 1);
  return hipGetLastError();
}

hipError_t launch_hsde_update(const HsdeArgs &h, hipStream_t st) {
  const int64_t n = h.ncoord > h.nrow ? h.ncoord : h.nrow;
  const unsigned nb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_hsde_zs_partials, dim3(nb), dim3(256), 0, st, h);
  hipLaunchKernelGGL(k_hsde_scalars, dim3(h.batch), dim3(256), 0, st, h);
  hipLaunchKernelGGL(k_hsde_apply, dim3(nb), dim3(256), 0, st, h);
  return hipGetLastError();
}

hipError_t launch_hsde_finish(const HsdeArgs &h, hipStream_t st) {
  hipLaunchKernelGGL(k_hsde_dual_partials, dim3((unsigned)(h.ncoord / 64)), dim3(256), 0,
                     st, h);
  hipLaunchKernelGGL(k_hsde_finish, dim3(h.batch), dim3(256), 0, st, h);
  return hipGetLastError();
}

hipError_t launch_hsde_reset(const HsdeArgs &h, hipStream_t st) {
  hipLaunchKernelGGL(k_hsde_reset, dim3((h.batch + 255) / 256), dim3(256), 0, st, h);
  return hipGetLastError();
}

hipError_t launch_hsde_solution(const HsdeArgs &h, double *x_out, double *y_out, hipStream_t st) {
  const int64_t n = h.ncoord > h.nrow ? h.ncoord : h.nrow;
  hipLaunchKernelGGL(k_hsde_solution, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, h, x_out,
                     y_out);
  return hipGetLastError();
}
