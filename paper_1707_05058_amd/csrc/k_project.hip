// PSD projection of clique blocks on gfx950 (the Y-step (XkUpdate) of
// Algorithm 1, fused with the multiplier update (LambdakUpdate) and the
// per-clique partial sums of the residuals (PrimalConsensusResidual)).
//
// One workgroup owns one clique block W_k, zero-padded to the bucket size N
// (padding is exact: a rotation whose off-diagonal entry is exactly zero is
// the identity, so padded rows/columns never mix with real ones).  The
// symmetric eigenproblem is solved by the two-sided Jacobi method in parallel
// order.  The N indices sit in N "slots"; in every round the K = N/2 slot
// pairs (2k, 2k+1) are rotated at once, so J^T A J splits into independent
// 2x2 block updates.  Between rounds a fixed slot permutation moves the
// indices (one index stays, the others advance around a circle), which makes
// every pair of indices meet exactly once per sweep of N-1 rounds.
//
// Work split: thread t owns the 2x2 blocks (row pair a_j, column pair b) of A
// and of V in registers, b = t mod K, a_j = t / K + (NT/K) j.  A round is:
// owners of diagonal blocks compute the rotation (Rutishauser's stable 2x2
// Schur formulas) and publish (c, s) in LDS; every thread applies
// R_a^T B R_b to its A blocks and B R_b to its V blocks; then A and V are
// written to LDS at their permuted positions and read back.  V's rows keep
// the original index order, so X = V diag(max(theta, 0)) V^T needs no
// un-permutation.  Sweeps stop when off(A) <= tol * ||A||_F.
#include "sdp_internal.h"
#include "mfma_tile.h"

#include <math.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

namespace {

// MODE_ADMM_DEC: MODE_ADMM with the positive/negative decoupling compiled in
// (FP32 scalar variants with N >= DEC_MIN_N; separate instances keep the
// register use of the others).  For smaller blocks a sweep costs less than
// the refinements, and FP64's tolerance leaves one Newton-Schulz step too
// little room (||T||_F <= 3.4e-4).
enum Mode { MODE_ADMM = 0, MODE_STANDALONE = 1, MODE_MINEIG = 2, MODE_ADMM_DEC = 3 };
constexpr int DEC_MIN_N = 64;

template <typename T> struct Num;
template <> struct Num<float> {
  static constexpr float big = 1e18f;
  static constexpr float tiny = 1.17549435e-38f;
  __device__ static float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  __device__ static float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
  __device__ static float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
};
template <> struct Num<double> {
  static constexpr double big = 1e150;
  static constexpr double tiny = 2.2250738585072014e-308;
  __device__ static double rcp(double x) { return 1.0 / x; }
  __device__ static double rsq(double x) { return 1.0 / sqrt(x); }
  __device__ static double sqrt_(double x) { return sqrt(x); }
};

// (c, s, t) zeroing a_pq of J^T A J with J = [[c, s], [-s, c]] on (p, q),
// written without branches (both alternatives are evaluated and selected).
// |a_pq| below the smallest normal number counts as zero: no rotation.
template <typename T>
__device__ inline void sym_rotation(T app, T aqq, T apq, T &c, T &s, T &t) {
  const bool z = !(fabs(apq) >= Num<T>::tiny);
  const T tau = (aqq - app) * T(0.5) * Num<T>::rcp(z ? T(1) : apq);
  const T at = fabs(tau);
  const T t_big = T(0.5) * Num<T>::rcp(at);
  const T t_std = Num<T>::rcp(at + Num<T>::sqrt_(T(1) + tau * tau));
  const T tt = (at > Num<T>::big) ? t_big : t_std;
  t = z ? T(0) : ((tau >= T(0)) ? tt : -tt);
  c = z ? T(1) : Num<T>::rsq(T(1) + t * t);
  s = t * c;
}

// Slot permutation applied after every round (see the file comment):
// even slots advance one pair, odd slots move back one pair, slot 1 stays.
__host__ __device__ constexpr int sigma_slot(int s, int N) {
  return (s & 1) ? ((s >> 1) == 0 ? 1 : ((s >> 1) == 1 ? 0 : 2 * ((s >> 1) - 1) + 1))
                 : ((s >> 1) < N / 2 - 1 ? 2 * ((s >> 1) + 1) : N - 1);
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

// NV block sums at once (one pair of barriers); each value is summed in the
// order block_sum uses, so the results are the same bit for bit.
template <int NT, int NV>
__device__ inline void block_sum_n(double (&v)[NV], double *red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int n = 0; n < NV; ++n) v[n] += __shfl_xor(v[n], o, 64);
  if (NT == 64) return;
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int n = 0; n < NV; ++n) red[n * (NT / 64) + w] = v[n];
  __syncthreads();
#pragma unroll
  for (int n = 0; n < NV; ++n) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[n * (NT / 64) + i];
    v[n] = s;
  }
}

// Row pitch of the LDS blocks (in elements).  FP32, N <= 48: P = N/4
// (mod 32), so the row pairs that the 64 / K row groups of a wave read in a
// Jacobi round sit on disjoint banks.  FP32, N >= 64 (one or two row groups
// per wave): P = 16 (mod 32), so the matrix-core operand reads (4 rows x 16
// consecutive stored columns per wave) are free of bank conflicts.  FP64:
// an odd pitch (its blocks must fit the LDS).
template <typename T>
__host__ __device__ constexpr int lds_pitch(int N, bool two_level) {
  if (sizeof(T) == 8 || two_level) return N + 1;
  const int target = N <= 48 ? (N / 4) % 32 : 16;
  int p = N;
  while (p % 32 != target) ++p;
  return p;
}


// ---------------------------------------------------------------------------
// Two-level (block) Jacobi for large blocks.  The N indices form N/8 groups of
// 8; in each round of a sweep the groups are paired by the circle method (N/8
// - 1 rounds meet every pair of groups once).  Each pair's 16 x 16 principal
// submatrix S is diagonalised by one wave (the parallel-order Jacobi above on
// 16 indices, its exchanges in wave-private LDS), giving S = Q diag(lambda)
// Q^T; then every 16 x 16 submatrix A[P1, P2] of two pairs becomes
// Q1^T A[P1, P2] Q2 (lambda on the pair's own diagonal block) and every 16-row
// panel of V[:, P] becomes V[:, P] Q, both on the matrix cores.  A and V stay
// in place in LDS (row-major, pitch N + 1); only 16 x 16 submatrices move.
// ---------------------------------------------------------------------------
constexpr int QP = 17;                        // pitch of the per-wave 16 x 16 scratch

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// orders this wave's LDS accesses: what a lane wrote is visible to every lane
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_s_waitcnt(0xc07f);         // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// groups of pair w in round r (nb groups, circle method)
__device__ inline void round_pair(int r, int w, int nb, int &gi, int &gj) {
  const int m = nb - 1;
  if (w == 0) {
    gi = nb - 1;
    gj = r % m;
  } else {
    gi = (r + w) % m;
    gj = (r - w + m) % m;
  }
}

// index of entry k (0..15) of a pair made of groups gi, gj
__device__ inline int pair_index(int gi, int gj, int k) { return k < 8 ? 8 * gi + k : 8 * gj + k - 8; }

// One wave: diagonalise S = A[idx, idx] (idx from groups gi, gj) by at most
// max_sweeps sweeps of the parallel-order Jacobi; Q (16 x 16, row-major,
// pitch QP: entry (i, slot k)) into q, Q^T S Q into sa (16 x QP, also the
// exchange scratch), its diagonal into lam; prm is scratch of 16.
template <typename T, int P>
__device__ void pair_eig16(const T *Abuf, int gi, int gj, T *sa, T *q, T *prm, T *lam,
                           double tol, int max_sweeps) {
  const int l = threadIdx.x & 63, a0 = l >> 3, b = l & 7;   // 2x2 block (a0, b) of 8x8
  T A[2][2], V[2][2];
  double f2 = 0.0;
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = pair_index(gi, gj, 2 * a0 + d), k = pair_index(gi, gj, 2 * b + e);
      A[d][e] = Abuf[i * P + k];
      V[d][e] = (2 * a0 + d == 2 * b + e) ? T(1) : T(0);
      f2 += (double)A[d][e] * (double)A[d][e];
    }
  const bool diag = a0 == b;
  const double thr = tol * tol * wave_sum(f2);
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    double o2 = (double)A[0][1] * A[0][1] + (double)A[1][0] * A[1][0];
    if (!diag) o2 += (double)A[0][0] * A[0][0] + (double)A[1][1] * A[1][1];
    if (!(wave_sum(o2) > thr)) break;
    for (int r = 0; r < 15; ++r) {
      if (diag) {
        T c, sn, t;
        const T apq = A[0][1];
        sym_rotation<T>(A[0][0], A[1][1], apq, c, sn, t);
        A[0][0] -= t * apq;
        A[1][1] += t * apq;
        A[0][1] = T(0);
        A[1][0] = T(0);
        prm[b] = c;
        prm[8 + b] = sn;
      }
      wave_lds_sync();
      const T cb = prm[b], sb = prm[8 + b];
      if (!diag) {
        const T ca = prm[a0], s_a = prm[8 + a0];
        const T b00 = A[0][0], b01 = A[0][1], b10 = A[1][0], b11 = A[1][1];
        const T c00 = cb * b00 - sb * b01, c01 = sb * b00 + cb * b01;
        const T c10 = cb * b10 - sb * b11, c11 = sb * b10 + cb * b11;
        A[0][0] = ca * c00 - s_a * c10;
        A[0][1] = ca * c01 - s_a * c11;
        A[1][0] = s_a * c00 + ca * c10;
        A[1][1] = s_a * c01 + ca * c11;
      }
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const T vp = V[d][0], vq = V[d][1];
        V[d][0] = cb * vp - sb * vq;
        V[d][1] = sb * vp + cb * vq;
      }
      const int sa0 = sigma_slot(2 * a0, 16), sa1 = sigma_slot(2 * a0 + 1, 16);
      const int sb0 = sigma_slot(2 * b, 16), sb1 = sigma_slot(2 * b + 1, 16);
      sa[sa0 * QP + sb0] = A[0][0];
      sa[sa0 * QP + sb1] = A[0][1];
      sa[sa1 * QP + sb0] = A[1][0];
      sa[sa1 * QP + sb1] = A[1][1];
      q[(2 * a0) * QP + sb0] = V[0][0];
      q[(2 * a0) * QP + sb1] = V[0][1];
      q[(2 * a0 + 1) * QP + sb0] = V[1][0];
      q[(2 * a0 + 1) * QP + sb1] = V[1][1];
      wave_lds_sync();
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          A[d][e] = sa[(2 * a0 + d) * QP + 2 * b + e];
          V[d][e] = q[(2 * a0 + d) * QP + 2 * b + e];
        }
      wave_lds_sync();
    }
  }
  if (diag) {
    lam[2 * b] = A[0][0];
    lam[2 * b + 1] = A[1][1];
  }
  // Q, and Q^T S Q itself (diagonal only to the inner tolerance)
#pragma unroll
  for (int d = 0; d < 2; ++d)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      q[(2 * a0 + d) * QP + 2 * b + e] = V[d][e];
      sa[(2 * a0 + d) * QP + 2 * b + e] = A[d][e];
    }
  wave_lds_sync();
}

// Sweeps of the two-level Jacobi over A and V in LDS (row-major, pitch P).
// ws holds per-wave scratch: 16 x QP for S / intermediate products, 16 x QP
// for Q, 16 rotation parameters, 16 eigenvalues.  Returns the sweeps done.
template <typename T, int N, int NT, int P, bool WANT_V>
__device__ int two_level_sweeps(T *Abuf, T *Vbuf, T *ws, double *red, double thr, double tol,
                                int max_sweeps) {
  constexpr int NG = N / 8;                   // groups of 8
  constexpr int NP = N / 16;                  // pairs per round
  constexpr int NW = NT / 64;
  constexpr int WS = 2 * 16 * QP + 32;        // scratch per wave
  static_assert(NW >= NP, "one wave per pair");
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  T *sa = ws + w * WS, *q = sa + 16 * QP, *prm = q + 16 * QP, *lam = prm + 16;
  const auto wsq = [&](int pw) { return ws + pw * WS + 16 * QP; };        // Q of pair pw
  const auto wss = [&](int pw) { return ws + pw * WS; };                   // Q^T S Q of pair pw
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    double o2 = 0.0;
    for (int e = tid; e < N * N; e += NT) {
      const int i = e / N, k = e % N;
      if (i != k) o2 += (double)Abuf[i * P + k] * (double)Abuf[i * P + k];
    }
    o2 = block_sum<NT>(o2, red);
    if (!(o2 > thr)) break;
    for (int r = 0; r < NG - 1; ++r) {
      if (w < NP) {
        int gi, gj;
        round_pair(r, w, NG, gi, gj);
        pair_eig16<T, P>(Abuf, gi, gj, sa, q, prm, lam, tol, max_sweeps);
      }
      __syncthreads();
      // A[P1, P2] <- Q1^T A[P1, P2] Q2: tiles (p1, p2) dealt to the waves
      for (int t = w; t < NP * NP; t += NW) {
        const int p1 = t / NP, p2 = t % NP;
        int g1i, g1j, g2i, g2j;
        round_pair(r, p1, NG, g1i, g1j);
        round_pair(r, p2, NG, g2i, g2j);
        if (p1 == p2) {
          const T *sd = wss(p1);
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int i = Mma<T>::row(l, rr), k = l & 15;
            Abuf[pair_index(g1i, g1j, i) * P + pair_index(g1i, g1j, k)] = sd[i * QP + k];
          }
          continue;
        }
        const T *q1 = wsq(p1), *q2 = wsq(p2);
        // T = A[P1, P2] Q2 (in registers: T(row(l, r), l % 16) in acc[r])
        typename Mma<T>::v4 acc = {0, 0, 0, 0};
        const int ia = pair_index(g1i, g1j, l & 15);
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const int k = k0 + (l >> 4);
          acc = Mma<T>::step(Abuf[ia * P + pair_index(g2i, g2j, k)], q2[k * QP + (l & 15)], acc);
        }
        // Q1^T T straight from those registers: step r sums over the rows
        // k = row(l, r) that lane l holds, so the b operand is acc[r]
        typename Mma<T>::v4 acc2 = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc2 = Mma<T>::step(q1[Mma<T>::row(l, r) * QP + (l & 15)], acc[r], acc2);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          Abuf[pair_index(g1i, g1j, Mma<T>::row(l, rr)) * P + pair_index(g2i, g2j, l & 15)] =
              acc2[rr];
      }
      if (WANT_V) {
        // V[:, P] <- V[:, P] Q: 16-row panels x pairs
        for (int t = w; t < NP * (N / 16); t += NW) {
          const int pc = t % NP, rt = t / NP;
          int gi, gj;
          round_pair(r, pc, NG, gi, gj);
          const T *qc = wsq(pc);
          typename Mma<T>::v4 acc = {0, 0, 0, 0};
          const int row = 16 * rt + (l & 15);
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4) {
            const int k = k0 + (l >> 4);
            acc = Mma<T>::step(Vbuf[row * P + pair_index(gi, gj, k)], qc[k * QP + (l & 15)], acc);
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            Vbuf[(16 * rt + Mma<T>::row(l, rr)) * P + pair_index(gi, gj, l & 15)] = acc[rr];
        }
      }
      __syncthreads();
    }
  }
  return sweep;
}

// ---------------------------------------------------------------------------
// Positive/negative decoupling of a warm-started block (scalar-round
// variants).  P_+(W) depends only on the split of R^N into the invariant
// subspaces of the positive and of the non-positive eigenvalues, not on a
// full diagonalisation.  In the warm-started basis A = V^T W V is nearly
// diagonal; with P = {i : a_ii > 0} and N the rest, one refinement applies
// the Jacobi rotations of all opposite-sign pairs (p, q) at once:
// T(p, q) = tan of the angle that zeroes a_pq in its own 2x2 problem (T skew,
// |T(p, q)| <= 1; the same-sign pairs are left alone), Q = I + T - T^T T / 2
// (= I + T + T^2 / 2 for skew T, the exponential of T to second order; then
// Q^T Q = I + T^4 / 4 exactly), A <- Q^T A Q, V <- V Q: four products on the
// matrix cores (T^T T, A Q, Q^T (A Q), V Q).  Near the
// decoupled state the opposite-sign mass falls quadratically.  The block is
// accepted when
//   * sum over opposite-sign pairs of a_pq^2 <= thr (= tol^2 ||W||_F^2), and
//   * Gershgorin certifies A_PP >= -eps and A_NN <= eps (eps = sqrt(thr)):
//     |a_ii| - sum_{j != i, same sign} |a_ij| >= -eps for every i,
// and then P_+(W) = V [A_PP 0; 0 0] V^T up to O(eps) (P_+ is 1-Lipschitz, so
// the dropped coupling costs at most sqrt(2) sqrt(thr); the certified blocks
// add at most eps per eigenvalue).  The refinement is only taken while
// ||T||_F <= tmax, so that Q is orthogonal to
// O(||T||^4) below the tolerance.  Returns true when accepted; otherwise A, V
// are still V^T W V and an orthonormal basis and the sweeps continue.
// Layout as in k_project's scalar path: A and V in registers (2x2 blocks),
// LDS blocks with de-interleaved slot columns; Abuf, Vbuf are scratch here.
// ---------------------------------------------------------------------------
template <typename T, int N, int NT, int P>
__device__ bool decouple_blocks(T (&A)[(N / 2) * (N / 2) / NT][2][2],
                                T (&V)[(N / 2) * (N / 2) / NT][2][2], T *Abuf, T *Vbuf, T *th,
                                double *red, double thr, double tmax2, int max_ref) {
  constexpr int K = N / 2;
  constexpr int BPT = K * K / NT;
  constexpr int AS = NT / K;
  const auto ix = [](int r, int c) { return r * P + (c & 1) * K + (c >> 1); };
  const auto slot = [](int q) { return q < K ? 2 * q : 2 * (q - K) + 1; };
  const double eps = sqrt(thr);
  for (int ref = 0;; ++ref) {
    // thread coordinates through an empty asm statement: the addresses of
    // this pass are computed in it, not kept live across the refinements
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int b = tid % K, a0 = tid / K;
    // diagonal (its signs define P and N)
#pragma unroll
    for (int j = 0; j < BPT; ++j)
      if (a0 + AS * j == b) {
        th[2 * b] = A[j][0][0];
        th[2 * b + 1] = A[j][1][1];
      }
    __syncthreads();
    // opposite-sign mass; same-sign absolute row sums, per thread into Abuf
    double o2 = 0.0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        const int r = 2 * aj + d;
        const bool pr = th[r] > T(0);
        double rs = 0.0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int c = 2 * b + e;
          const double v = (double)A[j][d][e];
          if (r == c) continue;
          if (pr != (th[c] > T(0))) o2 += v * v;
          else rs += fabs(v);
        }
        Abuf[r * P + b] = (T)rs;
      }
    }
    o2 = block_sum<NT>(o2, red);   // (its barriers also order the row sums)
    __syncthreads();
    double bad = 0.0;
    for (int r = tid; r < N; r += NT) {
      double rs = 0.0;
      for (int k = 0; k < K; ++k) rs += (double)Abuf[r * P + k];
      if (fabs((double)th[r]) - rs < -eps) bad += 1.0;
    }
    bad = block_sum<NT>(bad, red);
    if (o2 <= thr && bad == 0.0) return true;
    if (ref >= max_ref) return false;
    // generator T of the opposite-sign rotations (skew), into Abuf
    double t2 = 0.0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = 2 * aj + d, c = 2 * b + e;
          T t = T(0);
          if (r != c && ((th[r] > T(0)) != (th[c] > T(0)))) {
            T cs, sn;
            sym_rotation<T>(th[r], th[c], A[j][d][e], cs, sn, t);
          }
          t2 += (double)t * (double)t;
          Abuf[ix(r, c)] = t;
        }
    }
    t2 = block_sum<NT>(t2, red);
    if (!(t2 <= tmax2)) return false;
    __syncthreads();
    // Z = T^T T (symmetric: tiles on or below the diagonal, mirrored)
    tile_product<T, N, NT, true>([&](int k, int q) { return Abuf[k * P + q]; },
                                 [&](int k, int q) { return Abuf[k * P + q]; },
                                 [&](int qi, int qj, T v) {
                                   if (qi >= qj) {
                                     Vbuf[slot(qi) * P + qj] = v;
                                     Vbuf[slot(qj) * P + qi] = v;
                                   }
                                 });
    __syncthreads();
    // Q = I + T - Z / 2 over T in Abuf, and A over Z in Vbuf: each thread
    // reads and writes only its own entries; then A Q and Q^T (A Q)
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = 2 * aj + d, c = 2 * b + e, x = ix(r, c);
          Abuf[x] = (r == c ? T(1) : T(0)) + Abuf[x] - T(0.5) * Vbuf[x];
          Vbuf[x] = A[j][d][e];
        }
    }
    __syncthreads();
    tile_product<T, N, NT, false>([&](int k, int q) { return Vbuf[k * P + q]; },
                                  [&](int k, int q) { return Abuf[k * P + q]; },
                                  [&](int qi, int qj, T v) { Vbuf[slot(qi) * P + qj] = v; });
    __syncthreads();
    // Q^T (A Q), symmetric
    tile_product<T, N, NT, true>([&](int k, int q) { return Abuf[k * P + q]; },
                                 [&](int k, int q) { return Vbuf[k * P + q]; },
                                 [&](int qi, int qj, T v) {
                                   if (qi >= qj) {
                                     Vbuf[slot(qi) * P + qj] = v;
                                     Vbuf[slot(qj) * P + qi] = v;
                                   }
                                 });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = 2 * aj + d, c = 2 * b + e;
          // exactly symmetric: the lower-tile product stored both
          // triangles from one value (no transposed, bank-conflicted read)
          A[j][d][e] = Vbuf[ix(r, c)];
        }
    }
    __syncthreads();
    // V <- V Q: x(k, i) = V(i, k) from V^T in Vbuf
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) Vbuf[ix(2 * b + e, 2 * aj + d)] = V[j][d][e];
    }
    __syncthreads();
    tile_product<T, N, NT, false>([&](int k, int q) { return Vbuf[k * P + q]; },
                                  [&](int k, int q) { return Abuf[k * P + q]; },
                                  [&](int qi, int qj, T v) { Vbuf[slot(qi) * P + qj] = v; });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) V[j][d][e] = Vbuf[ix(2 * aj + d, 2 * b + e)];
    }
    __syncthreads();
  }
}

// P+(A) for a block held in registers (the scalar variants' 2 x 2 layout),
// by the matrix sign function on the matrix cores: X0 = A / ||A||_F, k1
// steps X <- X (3 I - 3.2 X^2 + 1.2 X^4), k2 steps X <- X (3 I - X^2) / 2,
// then P+(A) = (A + A sign(A)) / 2, which replaces A in the registers.  The
// products are the lower-tile ones (every iterate exactly symmetric); Abuf
// and Vbuf are scratch.  For blocks whose eigenvalue groups both reach zero,
// where the decoupling's certificate fails and the sweeps would need several
// passes of N - 1 rounds.
template <typename T, int N, int NT, int P>
__device__ void sign_project_regs(T (&A)[(N / 2) * (N / 2) / NT][2][2], T *Abuf, T *Vbuf,
                                  double *red, int k1, int k2) {
  constexpr int K = N / 2;
  constexpr int BPT = K * K / NT;
  constexpr int AS = NT / K;
  const auto ix = [](int r, int c) { return r * P + (c & 1) * K + (c >> 1); };
  const auto slot = [](int q) { return q < K ? 2 * q : 2 * (q - K) + 1; };
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int b = tid % K, a0 = tid / K;
  double f2 = 0.0;
#pragma unroll
  for (int j = 0; j < BPT; ++j)
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) f2 += (double)A[j][d][e] * (double)A[j][d][e];
  f2 = block_sum<NT>(f2, red);
  const T scale = f2 > 0.0 ? (T)(1.0 / sqrt(f2)) : T(0);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) Abuf[ix(2 * aj + d, 2 * b + e)] = A[j][d][e] * scale;
  }
  __syncthreads();
  const auto mirror_to = [&](T *buf) {
    return [=](int qi, int qj, T v) {
      if (qi >= qj) {
        buf[slot(qi) * P + qj] = v;
        buf[slot(qj) * P + qi] = v;
      }
    };
  };
  for (int it = 0; it < k1 + k2; ++it) {
    // Y = X^2 into Vbuf
    tile_product<T, N, NT, true>([&](int k, int q) { return Abuf[k * P + q]; },
                                 [&](int k, int q) { return Abuf[k * P + q]; }, mirror_to(Vbuf));
    __syncthreads();
    if (it < k1) {
      // Y (-3.2 I + 1.2 Y) over Y, then X (3 I + that) over X
      tile_product<T, N, NT, true>(
          [&](int k, int q) { return Vbuf[k * P + q]; },
          [&](int k, int q) { return (k == slot(q) ? T(-3.2) : T(0)) + T(1.2) * Vbuf[k * P + q]; },
          mirror_to(Vbuf));
      __syncthreads();
      tile_product<T, N, NT, true>(
          [&](int k, int q) { return Abuf[k * P + q]; },
          [&](int k, int q) { return (k == slot(q) ? T(3) : T(0)) + Vbuf[k * P + q]; },
          mirror_to(Abuf));
    } else {
      tile_product<T, N, NT, true>(
          [&](int k, int q) { return Abuf[k * P + q]; },
          [&](int k, int q) { return (k == slot(q) ? T(1.5) : T(0)) - T(0.5) * Vbuf[k * P + q]; },
          mirror_to(Abuf));
    }
    __syncthreads();
  }
  // A sign(A) with A into Vbuf, then P+(A) = (A + A sign(A)) / 2
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) Vbuf[ix(2 * aj + d, 2 * b + e)] = A[j][d][e];
  }
  __syncthreads();
  tile_product<T, N, NT, true>([&](int k, int q) { return Vbuf[k * P + q]; },
                               [&](int k, int q) { return Abuf[k * P + q]; }, mirror_to(Abuf));
  __syncthreads();
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        A[j][d][e] = T(0.5) * (A[j][d][e] + Abuf[ix(2 * aj + d, 2 * b + e)]);
  }
  __syncthreads();
}

template <typename T, int N, int NT, int MODE, bool BLK>
__global__ __launch_bounds__(NT) void k_project(ProjArgs a, const int32_t *__restrict__ list,
                                                const int32_t *__restrict__ sizes,
                                                const int64_t *__restrict__ offsets,
                                                const T *__restrict__ in, T *__restrict__ out,
                                                double *__restrict__ lmin_out, int max_sweeps,
                                                double tol) {
  constexpr int K = N / 2;
  static_assert(NT % K == 0 && (K * K) % NT == 0, "block ownership must tile the matrix");
  constexpr int BPT = K * K / NT;     // 2x2 blocks per thread
  constexpr int AS = NT / K;          // row-pair stride between a thread's blocks
  // LDS layout: row r at r * P, column (slot) c at position
  // (c & 1) * K + c / 2 (even slots first, then odd), so the K lanes that read
  // a row's column pairs, and the lanes that write the advancing even /
  // retreating odd slots, touch consecutive words.  slot(q) inverts the
  // position map.
  // (two-level mode: plain row-major, pitch N + 1)
  constexpr int P = lds_pitch<T>(N, BLK);
  const auto ix = [](int r, int c) { return BLK ? r * P + c : r * P + (c & 1) * K + (c >> 1); };
  const auto slot = [](int q) { return BLK ? q : (q < K ? 2 * q : 2 * (q - K) + 1); };
  constexpr bool WANT_V = MODE != MODE_MINEIG;
  constexpr bool ADMM = MODE == MODE_ADMM || MODE == MODE_ADMM_DEC;
  constexpr bool DEC = MODE == MODE_ADMM_DEC && !BLK;
  // the rebuild of larger blocks sums over the positive slots only (listed)
  constexpr bool COMPACT = WANT_V && N >= 64 && NT >= N;

  __shared__ T Abuf[N * P];
  __shared__ int plist[COMPACT ? N : 1];
  __shared__ int pwc[COMPACT ? (N + 63) / 64 : 1];
  __shared__ T Vbuf[WANT_V ? N * P : 1];
  __shared__ T prm_c[K], prm_s[K];
  __shared__ T th[N], thp[N];
  __shared__ double red[NT / 64];
  __shared__ double red6[ADMM ? 6 * (NT / 64) : 1];
  __shared__ T ws[BLK ? (NT / 64) * (2 * 16 * QP + 32) : 1];

  const int tid = threadIdx.x;
  int s, cl = 0;
  bool inst_done = false;
  int64_t off;
  double rho = 1.0;
  int iter = 0;
  if (MODE == MODE_STANDALONE) {
    s = sizes[blockIdx.x];
    off = offsets[blockIdx.x];
    if (s <= 0 || s > N) return;   // sizes beyond max_size are left untouched
  } else {
    // neighbouring cliques share coordinates of u: keep them on one XCD
    // (workgroups are dealt to the 8 XCDs round-robin)
    const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
    cl = list[x8 * q8 + min(x8, r8) + blockIdx.x / 8];
    const int inst = a.cl_inst[cl];
    // the clique record is loaded beside the instance index, and the
    // instance's done flag is tested only after the gather (below) has its
    // loads in flight: two memory latencies fewer before the first use of u
    s = a.cl_size[cl];
    off = a.cl_off[cl];
    if (ADMM) inst_done = a.state[inst].done != 0;
    rho = a.state[inst].rho;
    if (ADMM) iter = a.state[inst].iter;
  }

  // small variants: the loads of the warm-start basis and of the epilogue's
  // old X, Lambda and H_k x are issued here, so that their latency overlaps
  // the gather and the sweeps instead of adding to the chain after them
  constexpr int VPT = N * N / NT;                       // basis entries per thread
  constexpr int EPT = (N * (N + 1) / 2 + NT - 1) / NT;  // packed entries per thread
  constexpr bool PRE = ADMM && VPT <= 4 && EPT <= 4;
  static_assert(!PRE || (N * N) % NT == 0, "whole basis rows per thread");
  T pre_v[PRE ? VPT : 1];
  double pre_x[PRE ? EPT : 1], pre_l[PRE ? EPT : 1], pre_u[PRE ? EPT : 1];
  if constexpr (PRE) {
    if (a.vw) {
      const T *vp = reinterpret_cast<const T *>(a.vw) + a.vw_off[cl];
#pragma unroll
      for (int i = 0; i < VPT; ++i) pre_v[i] = vp[tid + NT * i];
    }
    if (!a.hsde && !a.dual) {
      const int npk0 = s * (s + 1) / 2;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + NT * i;
        pre_x[i] = pre_l[i] = pre_u[i] = 0.0;
        if (e < npk0) {
          const int64_t g = off + e;
          pre_x[i] = a.X[g];
          pre_l[i] = a.Lam[g];
          pre_u[i] = a.u[a.blk_loc[g]];
        }
      }
    }
  }

  const int b = tid % K;
  const int a0 = tid / K;
  T A[BPT][2][2];
  T V[BPT][2][2];
  // decoupling: iterations this clique still skips it (loaded early)
  double dec_skip_left = 0.0;
  if constexpr (DEC) dec_skip_left = a.part[NPART * (int64_t)cl + 7];

  // --- gather W_k = E_k U E_k^T - Lambda_k / rho (or the caller's block) ---
  double f2 = 0.0;
  // Algorithm 1 (the uniform common case): every entry's index and
  // multiplier loads are issued before any is used, then the loads of u
  // they index, so the thread waits for two memory latencies rather than
  // two per entry (entries outside the clique load its first entry and
  // are masked)
  const bool primal = ADMM && !a.hsde && !a.dual;
  if (primal) {
    int32_t loc[BPT][2][2];
    double lam[BPT][2][2];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int i = 2 * aj + d, k = 2 * b + e;
          const int ii = i > k ? i : k, kk = i > k ? k : i;
          const int64_t g = (i < s && k < s) ? off + (int64_t)ii * (ii + 1) / 2 + kk : off;
          loc[j][d][e] = a.blk_loc[g];
          lam[j][d][e] = a.Lam[g];
        }
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int i = 2 * aj + d, k = 2 * b + e;
          const double wd = a.u[loc[j][d][e]] - lam[j][d][e] / rho;
          const T w = (i < s && k < s) ? (T)wd : T(0);
          A[j][d][e] = w;
          V[j][d][e] = (i == k) ? T(1) : T(0);
          f2 += (double)w * (double)w;
        }
    }
  } else {
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const int i = 2 * aj + d, k = 2 * b + e;
        T w = T(0);
        if (i < s && k < s) {
          if (MODE == MODE_STANDALONE) {
            w = T(0.5) * (in[off + (int64_t)i * s + k] + in[off + (int64_t)k * s + i]);
          } else {
            const int ii = i > k ? i : k, kk = i > k ? k : i;
            const int64_t g = off + (int64_t)ii * (ii + 1) / 2 + kk;
            double wd;
            if (ADMM && a.hsde) {
              // u_hat_s - v_z
              const double hx = a.h_sx[a.blk_loc[g]];
              const double ss = 0.5 * (a.h_ns[g] - a.h_nt[g] + hx);
              wd = ss - a.hs[a.cl_inst[cl]].f * a.h_mzs[g] - a.Lam[g];
            } else if (ADMM && a.dual) {
              wd = a.Vd[g] - a.Lam[g] / rho;                 // v_k - lambda_k / rho
            } else {
              wd = a.u[a.blk_loc[g]];
              if (ADMM) wd -= a.Lam[g] / rho;   // H_k x - lambda_k / rho
              if (MODE == MODE_MINEIG && a.dual) wd *= -rho; // primal estimate -rho x
            }
            w = (T)wd;
          }
        }
        A[j][d][e] = w;
        V[j][d][e] = (i == k) ? T(1) : T(0);
        f2 += (double)w * (double)w;
      }
  }
  }
  // a finished instance writes nothing (uniform per workgroup; the gather's
  // loads feed f2, so they are issued before this test)
  if (ADMM && inst_done) return;
  const double thr = tol * tol * block_sum<NT>(f2, red);
  if (MODE == MODE_STANDALONE && !(thr < INFINITY)) {
    // a NaN or infinite entry: NaN throughout, never a finite result
    for (int e = tid; e < s * s; e += NT) out[off + e] = T(NAN);
    return;
  }

  // --- warm start: rotate W into the basis V0 the clique ended with last
  // iteration, A = V0^T W V0 (symmetrised), and let the rotations accumulate
  // onto V0.  The basis is orthonormal to rounding (re-orthonormalised when
  // it is stored), so A has the eigenvalues of W and is nearly diagonal once
  // the iteration settles: one or two sweeps instead of five or more. ---
  T *vw = nullptr;
  if (ADMM && a.vw) {
    vw = reinterpret_cast<T *>(a.vw) + a.vw_off[cl];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) Abuf[ix(2 * aj + d, 2 * b + e)] = A[j][d][e];
    }
    if constexpr (PRE) {
#pragma unroll
      for (int i = 0; i < VPT; ++i) {
        const int e = tid + NT * i;
        Vbuf[ix(e / N, e % N)] = pre_v[i];
      }
    } else {
      for (int e = tid; e < N * N; e += NT) Vbuf[ix(e / N, e % N)] = vw[e];
    }
    __syncthreads();
    // W V0 (W is symmetric: W(i, k) = W(k, i)), then V0^T (W V0), both into Abuf
    tile_product<T, N, NT, false>([&](int k, int q) { return Abuf[k * P + q]; },
                                  [&](int k, int q) { return Vbuf[k * P + q]; },
                                  [&](int qi, int qj, T v) { Abuf[slot(qi) * P + qj] = v; });
    __syncthreads();
    // (symmetric: tiles on or below the diagonal, mirrored)
    tile_product<T, N, NT, true>([&](int k, int q) { return Vbuf[k * P + q]; },
                                 [&](int k, int q) { return Abuf[k * P + q]; },
                                 [&](int qi, int qj, T v) {
                                   if (qi >= qj) {
                                     Abuf[slot(qi) * P + qj] = v;
                                     Abuf[slot(qj) * P + qi] = v;
                                   }
                                 });
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = 2 * aj + d, c = 2 * b + e;
          // exactly symmetric: the lower-tile product stored both
          // triangles from one value (no transposed, bank-conflicted read)
          A[j][d][e] = Abuf[ix(r, c)];
          V[j][d][e] = Vbuf[ix(r, c)];
        }
    }
  }

  // positive/negative decoupling instead of sweeps (warm-started ADMM blocks
  // whose eigenvectors are not recorded).  After a failed attempt the clique
  // skips it for a while, doubling the wait with every further failure in a
  // row: dec_skip, 2 dec_skip, ... 16 dec_skip iterations (blocks whose two
  // eigenvalue groups both reach zero fail the certificate every time); a
  // success starts over.  Its partial-sum slot 7 keeps 256 level + wait.
  bool dec = false, sgn = false;
  if constexpr (DEC) {
    if (vw && !a.eig) {
      double *flag = a.part + NPART * (int64_t)cl + 7;
      const double v = dec_skip_left;
      const int level = (int)(v * (1.0 / 256.0));
      __syncthreads();   // every thread has read the counter before it changes
      if (v - 256.0 * level > 0.0) {
        if (tid == 0) *flag = v - 1.0;
        // blocks of up to 96 with two or more failures in a row: the sign
        // function instead of sweeps (for larger blocks its ~46 products
        // cost more than the sweeps from the refined basis, which are few
        // where failures are rare, as on the large workload's blocks of 128)
        if (N <= 96 && level >= 2) {
          sign_project_regs<T, N, NT, P>(A, Abuf, Vbuf, red, a.sign_k1, a.sign_k2);
          sgn = true;
        }
      } else {
        dec = decouple_blocks<T, N, NT, P>(A, V, Abuf, Vbuf, th, red, thr, a.dec_tmax2,
                                           a.dec_max_ref);
        const int nl = level < 5 ? level + 1 : 5;
        if (tid == 0) *flag = dec ? 0.0 : 256.0 * nl + (double)(a.dec_skip << (nl - 1));
      }
    }
  }

  int sweep = 0;
  if constexpr (BLK) {
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          Abuf[ix(2 * aj + d, 2 * b + e)] = A[j][d][e];
          if (WANT_V) Vbuf[ix(2 * aj + d, 2 * b + e)] = V[j][d][e];
        }
    }
    __syncthreads();
    sweep = two_level_sweeps<T, N, NT, P, WANT_V>(Abuf, Vbuf, ws, red, thr, tol, max_sweeps);
    for (int k = tid; k < N; k += NT) th[k] = Abuf[k * P + k];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e)
          if (WANT_V) V[j][d][e] = Vbuf[ix(2 * aj + d, 2 * b + e)];
    }
  }
  for (; !BLK && !dec && !sgn && sweep < max_sweeps; ++sweep) {
    double o2 = 0.0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const bool diag = (a0 + AS * j) == b;
      o2 += (double)A[j][0][1] * A[j][0][1] + (double)A[j][1][0] * A[j][1][0];
      if (!diag) o2 += (double)A[j][0][0] * A[j][0][0] + (double)A[j][1][1] * A[j][1][1];
    }
    o2 = block_sum<NT>(o2, red);
    if (!(o2 > thr)) break;

    for (int r = 0; r < N - 1; ++r) {
      T cb, sb;
      {
        // 1. rotations of the diagonal blocks, published in LDS
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
          if (a0 + AS * j == b) {
            T c, sn, t;
            const T apq = A[j][0][1];
            sym_rotation<T>(A[j][0][0], A[j][1][1], apq, c, sn, t);
            A[j][0][0] -= t * apq;
            A[j][1][1] += t * apq;
            A[j][0][1] = T(0);
            A[j][1][0] = T(0);
            prm_c[b] = c;
            prm_s[b] = sn;
          }
        }
        __syncthreads();
        cb = prm_c[b];
        sb = prm_s[b];
      }
      // 2. two-sided update of the off-diagonal blocks, column update of V
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int aj = a0 + AS * j;
        if (aj != b) {
          const T ca = prm_c[aj], sa = prm_s[aj];
          const T b00 = A[j][0][0], b01 = A[j][0][1], b10 = A[j][1][0], b11 = A[j][1][1];
          const T c00 = cb * b00 - sb * b01, c01 = sb * b00 + cb * b01;
          const T c10 = cb * b10 - sb * b11, c11 = sb * b10 + cb * b11;
          A[j][0][0] = ca * c00 - sa * c10;
          A[j][0][1] = ca * c01 - sa * c11;
          A[j][1][0] = sa * c00 + ca * c10;
          A[j][1][1] = sa * c01 + ca * c11;
        }
        if (WANT_V) {
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            const T vp = V[j][d][0], vq = V[j][d][1];
            V[j][d][0] = cb * vp - sb * vq;
            V[j][d][1] = sb * vp + cb * vq;
          }
        }
      }
      // 3. move to the next round's slots: A' = P A P^T, V' = V P^T
      T *An = Abuf;
      T *Vn = Vbuf;
      const int sb0 = sigma_slot(2 * b, N), sb1 = sigma_slot(2 * b + 1, N);
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int aj = a0 + AS * j;
        const int sa0 = sigma_slot(2 * aj, N), sa1 = sigma_slot(2 * aj + 1, N);
        An[ix(sa0, sb0)] = A[j][0][0];
        An[ix(sa0, sb1)] = A[j][0][1];
        An[ix(sa1, sb0)] = A[j][1][0];
        An[ix(sa1, sb1)] = A[j][1][1];
        if (WANT_V) {
          Vn[ix(2 * aj, sb0)] = V[j][0][0];
          Vn[ix(2 * aj, sb1)] = V[j][0][1];
          Vn[ix(2 * aj + 1, sb0)] = V[j][1][0];
          Vn[ix(2 * aj + 1, sb1)] = V[j][1][1];
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int aj = a0 + AS * j;
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            A[j][d][e] = An[ix(2 * aj + d, 2 * b + e)];
            if (WANT_V) V[j][d][e] = Vn[ix(2 * aj + d, 2 * b + e)];
          }
      }
    }
  }

  // eigenvalues sit on the diagonal slots
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (!BLK && a0 + AS * j == b) {
      th[2 * b] = A[j][0][0];
      th[2 * b + 1] = A[j][1][1];
    }
  }
  if (MODE == MODE_MINEIG) {
    __syncthreads();
    if (tid == 0) {
      double mn = 0.0;
      for (int k = 0; k < N; ++k) mn = fmin(mn, (double)th[k]);
      lmin_out[cl] = mn;
    }
    return;
  }
  __syncthreads();   // every thread has read Vbuf of the last round
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) Vbuf[ix(2 * aj + d, 2 * b + e)] = V[j][d][e];
  }
  for (int k = tid; k < N; k += NT) thp[k] = th[k] > T(0) ? th[k] : T(0);
  // the positive slots in increasing order, plist[0 .. npos): wave ballots
  int npos = N;
  if constexpr (COMPACT) {
    const bool ispos = tid < N && th[tid] > T(0);
    const unsigned long long bal = __ballot(ispos);
    if ((tid & 63) == 0 && tid < N) pwc[tid >> 6] = __popcll(bal);
    __syncthreads();
    int base = 0;
    npos = 0;
#pragma unroll
    for (int w2 = 0; w2 < (N + 63) / 64; ++w2) {
      const int c = pwc[w2];
      if (w2 < (tid >> 6)) base += c;
      npos += c;
    }
    if (ispos) plist[base + __popcll(bal & ((1ull << (tid & 63)) - 1ull))] = tid;
  }
  __syncthreads();
  // the basis is re-orthonormalised by a Newton-Schulz step on every
  // ns_period-th iteration of the instance: it departs from orthonormality
  // by rounding only (about N eps per iteration), and one step squares the
  // departure, so every second iteration keeps it at the level of a few eps
  const bool ns = ADMM && vw && (a.ns_period <= 1 || (iter + a.ns_shift) % a.ns_period == 0);
  // the Gram matrix V^T V of the Newton-Schulz step reads V by rows; the
  // products after it read V^T, written over V from the registers
  if (ns) {
    // (symmetric: tiles on or below the diagonal, mirrored)
    tile_product<T, N, NT, true>([&](int k, int q) { return Vbuf[k * P + q]; },
                                 [&](int k, int q) { return Vbuf[k * P + q]; },
                                 [&](int qi, int qj, T v) {
                                   if (qi >= qj) {
                                     Abuf[slot(qi) * P + qj] = v;
                                     Abuf[slot(qj) * P + qi] = v;
                                   }
                                 });
  }
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int aj = a0 + AS * j;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) Vbuf[ix(2 * b + e, 2 * aj + d)] = V[j][d][e];
  }
  __syncthreads();
  if (ns) {
    // store the basis for the next iteration after one Newton-Schulz step,
    // V <- V (3I - V^T V) / 2, which squares its departure from orthonormality:
    // (V G)(i, j) = sum_k V^T(k, i) G(k, j), V(i, j) = V^T(j, i)
    tile_product<T, N, NT, false>(
        [&](int k, int q) { return Vbuf[k * P + q]; },
        [&](int k, int q) { return Abuf[k * P + q]; },
        [&](int qi, int qj, T v) {
          vw[(int64_t)slot(qi) * N + slot(qj)] = T(1.5) * Vbuf[slot(qj) * P + qi] - T(0.5) * v;
        });
  } else if (ADMM && vw) {
    // store the basis as it is
    for (int e = tid; e < N * N; e += NT) {
      const int qi = e / N, qj = e % N;
      vw[(int64_t)slot(qi) * N + slot(qj)] = Vbuf[slot(qj) * P + qi];
    }
  }
  if (ADMM && a.eig) {
    // keep V (rows < s, all N slots) and the eigenvalues for the reverse sweep
    T *eo = reinterpret_cast<T *>(a.eig) + a.eig_off[cl];
    for (int e = tid; e < s * N; e += NT) eo[e] = Vbuf[ix(e % N, e / N)];
    for (int k = tid; k < N; k += NT) eo[s * N + k] = th[k];
  }

  // --- rebuild X = V diag(theta+) V^T = sum_k V^T(k, i) theta+_k V^T(k, j):
  // tiles on or below the diagonal, each result stored at (i, j) and (j, i);
  // after a decoupling X = V M V^T with M = A on the positive slots, zero
  // elsewhere (Y = M V^T first; Abuf is free once the Newton-Schulz product
  // has passed its barrier).  Blocks of 64 and more sum over the npos
  // positive slots p_a = plist[a] only (X has rank npos): after a decoupling
  // Y(a, j) = sum_b A(p_a, p_b) V(j, p_b) for a < npos, then
  // X = sum_a V(i, p_a) Y(a, j); otherwise X = sum_a V(i, p_a) theta_{p_a} V(j, p_a).
  // Then the epilogue over the packed lower triangle ---
  const auto mirror = [&](int qi, int qj, T v) {
    Abuf[slot(qi) * P + qj] = v;
    Abuf[slot(qj) * P + qi] = v;
  };
  if (!BLK && (dec || sgn)) {
    // (after the sign function M is P+(A) itself, a full matrix)
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int aj = a0 + AS * j;
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = 2 * aj + d, c = 2 * b + e;
          Abuf[ix(r, c)] = (sgn || (th[r] > T(0) && th[c] > T(0))) ? A[j][d][e] : T(0);
        }
    }
    __syncthreads();
    if (COMPACT && !sgn) {
      const int kend = (npos + 3) & ~3;
      tile_product_part<T, N, NT, false>(
          npos, kend,
          [&](int k, int q) {
            return (k < npos && q < npos) ? Abuf[plist[k] * P + ix(0, plist[q])] : T(0);
          },
          [&](int k, int q) { return k < npos ? Vbuf[plist[k] * P + q] : T(0); },
          [&](int qi, int qj, T v) {
            if (qi < npos) Abuf[qi * P + qj] = v;
          });
      __syncthreads();
      tile_product_part<T, N, NT, true>(
          N, kend, [&](int k, int q) { return k < npos ? Vbuf[plist[k] * P + q] : T(0); },
          [&](int k, int q) { return k < npos ? Abuf[k * P + q] : T(0); }, mirror);
    } else {
      tile_product<T, N, NT, false>([&](int k, int q) { return Abuf[k * P + q]; },
                                    [&](int k, int q) { return Vbuf[k * P + q]; },
                                    [&](int qi, int qj, T v) { Abuf[slot(qi) * P + qj] = v; });
      __syncthreads();
      tile_product<T, N, NT, true>([&](int k, int q) { return Vbuf[k * P + q]; },
                                   [&](int k, int q) { return Abuf[k * P + q]; }, mirror);
    }
  } else if constexpr (COMPACT) {
    tile_product_part<T, N, NT, true>(
        N, (npos + 3) & ~3,
        [&](int k, int q) {
          if (k >= npos) return T(0);
          const int pk = plist[k];
          return Vbuf[pk * P + q] * thp[pk];
        },
        [&](int k, int q) { return k < npos ? Vbuf[plist[k] * P + q] : T(0); }, mirror);
  } else {
    tile_product<T, N, NT, true>([&](int k, int q) { return Vbuf[k * P + q] * thp[k]; },
                                 [&](int k, int q) { return Vbuf[k * P + q]; }, mirror);
  }
  __syncthreads();
  const int npk = s * (s + 1) / 2;
  double p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0, p6 = 0;
  // Algorithm 1 at packed entry e, given H_k x (hu) and the old X (xo) and
  // Lambda (lo) there: X, Lambda and the residual partials
  auto primal_step = [&](int e, double hu, double xo, double lo) {
    int i, j;
    tri_inv(e, i, j);
    const int64_t g = off + e;
    const double xn = (double)Abuf[ix(i, j)];
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
  };
  // packed entry e (the it-th of this thread)
  auto epilogue = [&](int e, int it) {
    int i, j;
    tri_inv(e, i, j);
    const T acc = Abuf[ix(i, j)];
    if (MODE == MODE_STANDALONE) {
      out[off + (int64_t)i * s + j] = acc;
      out[off + (int64_t)j * s + i] = acc;
    } else if (a.hsde) {
      // Algorithm 3: u_s = P+(u_hat_s - v_z), v_z += u_s - u_hat_s, u_t = u_hat_t;
      // partials of the consensus residuals on (u_s, H u_x) and (v_z, u_t)
      const int64_t g = off + e;
      const double f = a.hs[a.cl_inst[cl]].f;
      const int32_t loc = a.blk_loc[g];
      const double hx = a.h_sx[loc], nt = a.h_nt[g];
      const double ss = 0.5 * (a.h_ns[g] - nt + hx);
      const double us_hat = ss - f * a.h_mzs[g];
      const double ut = ss - hx + nt - f * a.h_mzt[g];
      const double usn = (double)acc;
      const double vzn = a.Lam[g] - us_hat + usn;
      a.X[g] = usn;
      a.Lam[g] = vzn;
      a.h_ut[g] = ut;
      const double hux = a.h_ux[loc];
      const double wt = (i == j) ? 1.0 : 2.0;
      p0 += wt * (usn - hux) * (usn - hux);
      p1 += wt * usn * usn;
      p2 += wt * hux * hux;
      p3 += wt * (vzn - ut) * (vzn - ut);
      p4 += wt * vzn * vzn;
      p6 += wt * ut * ut;
    } else if (a.dual) {
      // Algorithm 2: z_k only; the multiplier and the other partials follow
      // the affine step (launch_dual_update)
      const int64_t g = off + e;
      const double zo = a.X[g], zn = (double)acc;
      a.X[g] = zn;
      const double wt = (i == j) ? 1.0 : 2.0;
      p3 += wt * (zn - zo) * (zn - zo);
    } else {
      const int64_t g = off + e;
      if constexpr (PRE) primal_step(e, pre_u[it], pre_x[it], pre_l[it]);
      else primal_step(e, a.u[a.blk_loc[g]], a.X[g], a.Lam[g]);
    }
  };
  if constexpr (PRE) {
#pragma unroll
    for (int it = 0; it < EPT; ++it) {
      const int e = tid + NT * it;
      if (e < npk) epilogue(e, it);
    }
  } else if (primal) {
    // chunks of CH entries: all their loads are issued before any is used
    // (entries past the end load the first entry and are skipped)
    constexpr int CH = 8;
    for (int e0 = tid; e0 < npk; e0 += CH * NT) {
      int32_t lc[CH];
      double cx[CH], cm[CH], cu[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int e = e0 + c * NT;
        const int64_t g = off + (e < npk ? e : 0);
        lc[c] = a.blk_loc[g];
        cx[c] = a.X[g];
        cm[c] = a.Lam[g];
      }
#pragma unroll
      for (int c = 0; c < CH; ++c) cu[c] = a.u[lc[c]];
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int e = e0 + c * NT;
        if (e < npk) primal_step(e, cu[c], cx[c], cm[c]);
      }
    }
  } else {
    for (int e = tid; e < npk; e += NT) epilogue(e, 0);
  }
  if (ADMM) {
    if (a.hsde) {
      double pv[6] = {p0, p1, p2, p3, p4, p6};
      block_sum_n<NT, 6>(pv, red6);
      p0 = pv[0]; p1 = pv[1]; p2 = pv[2]; p3 = pv[3]; p4 = pv[4]; p6 = pv[5];
    } else {
      double pv[5] = {p0, p1, p2, p3, p4};
      block_sum_n<NT, 5>(pv, red6);
      p0 = pv[0]; p1 = pv[1]; p2 = pv[2]; p3 = pv[3]; p4 = pv[4];
    }
    if (tid == 0) {
      double *pp = a.part + NPART * (int64_t)cl;
      if (!a.dual) {
        pp[0] = p0; pp[1] = p1; pp[2] = p2; pp[4] = p4;
      }
      pp[3] = p3;
      pp[5] = (double)sweep;
      pp[6] = a.hsde ? p6 : (sgn ? 1.0 : 0.0);   // Algorithms 1, 2: sign fallback taken
    }
  }
}

// ---------------------------------------------------------------------------
// Standalone projection by the matrix sign function (no eigenvectors):
// P+(W) = (W + W sign(W)) / 2.  sign(W) is the limit of polynomial
// iterations on X0 = W / ||W||_F (all eigenvalues in [-1, 1]):
//   k1 steps  X <- X (3 I - 3.2 X^2 + 1.2 X^4)  (p(x) = 3x - 3.2x^3 + 1.2x^5:
//             slope 3 at 0, fixed point 1 with |p'(1)| = 0.6, p([0,1]) within
//             [0, 1.21], inside the basin of the next phase)
//   k2 steps  X <- X (3 I - X^2) / 2            (quadratic convergence to +-1)
// Small eigenvalues triple in each fast step; one that stays below 1 adds at
// most |lambda| (1 - s(lambda)) / 2 to the error of P+.  (k1, k2) come from
// sign_schedule: the fewest products that keep the Frobenius error below
// the tolerance (relative to ||W||_F) of the Jacobi variants.  Each
// product is a polynomial in W, symmetric in exact arithmetic: only the tiles
// on or below the diagonal are computed, and only the lanes on or below the
// diagonal store (both triangles), so every iterate is exactly symmetric.
// The products run on the matrix cores from two N x N LDS buffers (natural
// layout, odd pitch N + 1: the mirrored stores run down columns).
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ constexpr int sign_pitch(int N) {
  return N + 1;
}

template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_project_sign(const int32_t *__restrict__ sizes,
                                                     const int64_t *__restrict__ offsets,
                                                     const T *__restrict__ in, T *__restrict__ out,
                                                     int k1, int k2) {
  constexpr int P = sign_pitch<T>(N);
  constexpr int VPT = N * N / NT;
  static_assert((N * N) % NT == 0, "whole entries per thread");
  __shared__ T X[N * P];
  __shared__ T Y[N * P];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int s = sizes[blockIdx.x];
  const int64_t off = offsets[blockIdx.x];
  if (s <= 0 || s > N) return;   // sizes beyond max_size are left untouched
  // W (symmetrised, zero-padded): entry e = tid + NT i is (e / N, e % N)
  T w[VPT];
  double f2 = 0.0;
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int e = tid + NT * i, r = e / N, c = e % N;
    T v = T(0);
    if (r < s && c < s) v = T(0.5) * (in[off + (int64_t)r * s + c] + in[off + (int64_t)c * s + r]);
    w[i] = v;
    f2 += (double)v * (double)v;
  }
  f2 = block_sum<NT>(f2, red);
  if (!(f2 > 0.0 && f2 < INFINITY)) {
    // W = 0: P+(W) = 0; a NaN or infinite entry: NaN throughout (as the
    // Jacobi variants give), never a finite result
    const T fill = f2 == 0.0 ? T(0) : T(NAN);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      const int e = tid + NT * i, r = e / N, c = e % N;
      if (r < s && c < s) out[off + (int64_t)r * s + c] = fill;
    }
    return;
  }
  const T scale = (T)(1.0 / sqrt(f2));
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int e = tid + NT * i;
    X[(e / N) * P + e % N] = w[i] * scale;
  }
  __syncthreads();
  const auto eye = [](int k, int q) { return k == q ? T(1) : T(0); };
  const auto sym_x = [&](int qi, int qj, T v) {
    if (qi >= qj) {
      X[qi * P + qj] = v;
      X[qj * P + qi] = v;
    }
  };
  const auto sym_y = [&](int qi, int qj, T v) {
    if (qi >= qj) {
      Y[qi * P + qj] = v;
      Y[qj * P + qi] = v;
    }
  };
  for (int it = 0; it < k1 + k2; ++it) {
    // Y = X^2
    tile_product<T, N, NT, true>([&](int k, int q) { return X[k * P + q]; },
                                 [&](int k, int q) { return X[k * P + q]; }, sym_y);
    __syncthreads();
    if (it < k1) {
      // Y = X^2 (-3.2 I + 1.2 X^2), then X = X (3 I + Y)
      tile_product<T, N, NT, true>(
          [&](int k, int q) { return Y[k * P + q]; },
          [&](int k, int q) { return T(-3.2) * eye(k, q) + T(1.2) * Y[k * P + q]; }, sym_y);
      __syncthreads();
      tile_product<T, N, NT, true>([&](int k, int q) { return X[k * P + q]; },
                                   [&](int k, int q) { return T(3) * eye(k, q) + Y[k * P + q]; },
                                   sym_x);
    } else {
      // X = X (1.5 I - 0.5 X^2)
      tile_product<T, N, NT, true>(
          [&](int k, int q) { return X[k * P + q]; },
          [&](int k, int q) { return T(1.5) * eye(k, q) - T(0.5) * Y[k * P + q]; }, sym_x);
    }
    __syncthreads();
  }
  // C = W S (W into Y), then P+(W) = (W + C) / 2
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int e = tid + NT * i;
    Y[(e / N) * P + e % N] = w[i];
  }
  __syncthreads();
  tile_product<T, N, NT, true>([&](int k, int q) { return Y[k * P + q]; },
                               [&](int k, int q) { return X[k * P + q]; }, sym_x);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int e = tid + NT * i, r = e / N, c = e % N;
    if (r < s && c < s) out[off + (int64_t)r * s + c] = T(0.5) * (w[i] + X[r * P + c]);
  }
}

// Algorithm 2, after the affine step: v_k and lambda_k on the packed lower
// triangle of every clique, one workgroup per clique, with the partial sums
// of DualConsensusResidual (full Frobenius norms: off-diagonal entries count
// twice).
__global__ __launch_bounds__(256) void k_dual_update(ProjArgs a) {
  const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
  const int cl = x8 * q8 + min(x8, r8) + blockIdx.x / 8;
  const int inst = a.cl_inst[cl];
  if (a.state[inst].done) return;
  const double rho = a.state[inst].rho;
  const int s = a.cl_size[cl];
  const int64_t off = a.cl_off[cl];
  const int npk = s * (s + 1) / 2;
  double p0 = 0, p1 = 0, p2 = 0, p4 = 0;
  for (int e = threadIdx.x; e < npk; e += 256) {
    int i, j;
    tri_inv(e, i, j);
    const int64_t g = off + e;
    const double z = a.X[g], lo = a.Lam[g];
    const double v = z + lo / rho + a.u[a.blk_loc[g]];
    const double ln = lo + rho * (z - v);
    a.Vd[g] = v;
    a.Lam[g] = ln;
    const double wt = (i == j) ? 1.0 : 2.0;
    p0 += wt * (z - v) * (z - v);
    p1 += wt * z * z;
    p2 += wt * v * v;
    p4 += wt * ln * ln;
  }
  // (the four sums in one barrier pair, each in block_sum's order)
  __shared__ double red[4 * 4];
  double pv[4] = {p0, p1, p2, p4};
  block_sum_n<256, 4>(pv, red);
  if (threadIdx.x == 0) {
    double *pp = a.part + NPART * (int64_t)cl;
    pp[0] = pv[0]; pp[1] = pv[1]; pp[2] = pv[2]; pp[4] = pv[3];
  }
}

template <typename T, int N, int NT, int MODE, bool BLK>
hipError_t launch_one(int count, ProjArgs a, const int32_t *list, const int32_t *sizes,
                      const int64_t *offsets, const T *in, T *out, double *lmin, int msw,
                      double tol, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_project<T, N, NT, MODE, BLK>), dim3(count), dim3(NT), 0, st, a, list,
                     sizes, offsets, in, out, lmin, msw, tol);
  return hipGetLastError();
}

// Kernel variants: padded block size N, threads per workgroup NT and kind
// (0 scalar Jacobi: each thread owns K*K/NT 2x2 blocks, K = N/2; 1 two-level
// Jacobi; 2 sign function: it yields no eigenvectors).  The autotuner picks,
// per clique size, the Jacobi variant that runs fastest; without it the
// smallest N and the first NT listed for that N are used.  FP64 blocks of
// 97-128 have the sign function only (k_sign_big: two FP64 blocks of 128 do
// not fit in LDS, which every Jacobi variant with eigenvectors needs).
struct Variant { int N, NT, kind; };
constexpr Variant kVar32[] = {
    {16, 64, 0},   {32, 64, 0},    {32, 128, 0},  {32, 256, 0}, {48, 192, 0},
    {64, 256, 0},  {64, 128, 0},   {64, 512, 0},  {80, 320, 0}, {96, 576, 0},
    {112, 448, 0}, {128, 1024, 0}, {128, 512, 0}, {64, 256, 1}, {80, 320, 1},
    {96, 384, 1},  {112, 448, 1},  {128, 512, 1}, {16, 64, 2},  {32, 256, 2},
    {32, 64, 2},   {48, 192, 2},   {64, 256, 2},  {80, 320, 2}, {96, 384, 2},
    {112, 448, 2}, {128, 512, 2}};
constexpr Variant kVar64[] = {{16, 64, 0},  {32, 64, 0},  {32, 128, 0}, {32, 256, 0},
                              {48, 192, 0}, {64, 256, 0}, {64, 128, 0}, {64, 512, 0},
                              {80, 320, 0}, {96, 576, 0}, {64, 256, 1}, {80, 320, 1},
                              {16, 64, 2},  {32, 64, 2},  {48, 192, 2}, {64, 256, 2},
                              {80, 320, 2}, {96, 384, 2}, {128, 512, 2}};
constexpr int kNVar32 = sizeof(kVar32) / sizeof(kVar32[0]);
constexpr int kNVar64 = sizeof(kVar64) / sizeof(kVar64[0]);

template <typename T, int MODE>
hipError_t dispatch(int N, int NT, int blk, int count, ProjArgs a, const int32_t *list,
                    const int32_t *sizes, const int64_t *offsets, const T *in, T *out,
                    double *lmin, int msw, double tol, hipStream_t st) {
#define SDP_VARIANT(n, nt, bl)                                                                 \
  if (N == n && NT == nt && blk == bl)                                                         \
    return launch_one<T, n, nt,                                                                \
                      (MODE == MODE_ADMM_DEC && (bl || n < DEC_MIN_N || sizeof(T) == 8))       \
                          ? MODE_ADMM                                                          \
                          : MODE,                                                              \
                      bl>(count, a, list, sizes, offsets, in, out, lmin, msw, tol, st);
  SDP_VARIANT(16, 64, 0)
  SDP_VARIANT(32, 64, 0)
  SDP_VARIANT(32, 128, 0)
  SDP_VARIANT(32, 256, 0)
  SDP_VARIANT(48, 192, 0)
  SDP_VARIANT(64, 128, 0)
  SDP_VARIANT(64, 256, 0)
  SDP_VARIANT(64, 512, 0)
  SDP_VARIANT(80, 320, 0)
  SDP_VARIANT(96, 576, 0)
  SDP_VARIANT(64, 256, 1)
  SDP_VARIANT(80, 320, 1)
  if constexpr (sizeof(T) == 4) {
    SDP_VARIANT(112, 448, 0)
    SDP_VARIANT(128, 512, 0)
    SDP_VARIANT(128, 1024, 0)
    SDP_VARIANT(96, 384, 1)
    SDP_VARIANT(112, 448, 1)
    SDP_VARIANT(128, 512, 1)
  }
#undef SDP_VARIANT
  return hipErrorInvalidValue;
}

// Fills `count` symmetric s x s blocks (row-major, contiguous) with values in
// (-1, 1) from a counter-based hash, the off-diagonal ones scaled by offdiag:
// synthetic inputs for the autotuner (offdiag = 1: a cold eigensolve;
// offdiag << 1: the nearly diagonal matrix a warm-started one sees).
template <typename T>
__global__ __launch_bounds__(256) void k_fill_blocks(T *out, int s, int count, uint32_t seed,
                                                     double offdiag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)count * s * s) return;
  const int64_t blk = e / ((int64_t)s * s);
  const int r = (int)(e % ((int64_t)s * s)) / s, c = (int)(e % ((int64_t)s * s)) % s;
  const int i = r > c ? r : c, j = r > c ? c : r;
  uint32_t x = seed ^ (uint32_t)(blk * 2654435761u) ^ (uint32_t)(i * 40503u + j * 2246822519u);
  x ^= x >> 16; x *= 0x7feb352du; x ^= x >> 15; x *= 0x846ca68bu; x ^= x >> 16;
  const double v = (double)x * (2.0 / 4294967296.0) - 1.0;
  out[e] = (T)(i == j ? v : offdiag * v);
}

template <typename T>
__global__ __launch_bounds__(256) void k_identity_bases(T *vw, const int64_t *vw_off,
                                                        const int32_t *cl_n, int64_t c0) {
  const int64_t cl = c0 + blockIdx.x;
  const int n = cl_n[cl];
  T *v = vw + vw_off[cl];
  for (int e = threadIdx.x; e < n * n; e += 256) v[e] = (e / n == e % n) ? T(1) : T(0);
}

}  // namespace

// The sign iteration's schedule.  X0 = W / ||W||_F has eigenvalues delta_i
// with sum delta_i^2 = 1; the fast map p(x) = 3x - 3.2x^3 + 1.2x^5 (three
// products) and the Newton-Schulz map x(3 - x^2)/2 (two) are odd and act on
// each eigenvalue alone, so P+ = (W + W s(X0)) / 2 is off by
// e(delta) = |delta| |1 - s(|delta|)| / 2 (in units of ||W||_F) along
// eigenvector i.  Every eigenvalue but the largest (|delta| >= 1/sqrt(n)) may
// sit at the worst delta, so the Frobenius error is at most
// sqrt(n - 1) max e.  The schedule takes the fewest products, with at least
// two Newton-Schulz steps, for which 2 sqrt(n - 1) max e <= tol on a grid
// of delta: 256 points per decade down to where delta / 2 alone meets the
// bound, and 1024 uniform points on (0, 1] (e is smooth; the factor 2 covers
// the grid and rounding).  Tolerances below 1e-16, beyond what FP64 products
// resolve, are taken as 1e-16.
void sign_schedule(double tol, int n, int *k1_out, int *k2_out) {
  static std::mutex mu;
  static std::map<std::pair<double, int>, std::pair<int, int>> cache;
  const double t = tol >= 1e-16 ? tol : 1e-16;   // (also a NaN tolerance)
  std::lock_guard<std::mutex> lock(mu);
  const std::pair<double, int> key(t, n);
  auto it = cache.find(key);
  if (it == cache.end()) {
    const double target = t / (2.0 * std::sqrt((double)std::max(n - 1, 1)));
    const int dec = std::max(1, (int)std::ceil(-std::log10(2.0 * target)));
    std::vector<double> d;
    for (int j = 0; j <= 256 * dec; ++j) d.push_back(std::pow(10.0, -dec + j / 256.0));
    for (int j = 1; j <= 1024; ++j) d.push_back(j / 1024.0);
    std::vector<double> x(d), y(d.size());
    constexpr int K1_MAX = 200, K2_MAX = 8;
    int best = INT_MAX, b1 = K1_MAX, b2 = 4;
    for (int k1 = 0; k1 <= K1_MAX && 3 * k1 + 4 < best; ++k1) {
      if (k1 > 0)
        for (double &v : x) v = v * (3.0 - 3.2 * v * v + 1.2 * v * v * v * v);
      y = x;
      for (int k2 = 1; k2 <= K2_MAX && 3 * k1 + 2 * k2 < best; ++k2) {
        double e = 0.0;
        for (size_t j = 0; j < d.size(); ++j) {
          y[j] = y[j] * (3.0 - y[j] * y[j]) / 2.0;
          e = std::max(e, d[j] * std::fabs(1.0 - y[j]) / 2.0);
        }
        if (k2 >= 2 && e <= target) {
          best = 3 * k1 + 2 * k2;
          b1 = k1;
          b2 = k2;
          break;
        }
      }
    }
    it = cache.emplace(key, std::make_pair(b1, b2)).first;
  }
  *k1_out = it->second.first;
  *k2_out = it->second.second;
}

hipError_t launch_dual_update(const ProjArgs &a, int64_t ncl, hipStream_t st) {
  if (ncl <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dual_update, dim3((unsigned)ncl), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_identity_bases(int precision, void *vw, const int64_t *vw_off,
                                 const int32_t *cl_n, int64_t c0, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (precision == 1)
    hipLaunchKernelGGL(k_identity_bases<float>, dim3((unsigned)count), dim3(256), 0, st,
                       (float *)vw, vw_off, cl_n, c0);
  else
    hipLaunchKernelGGL(k_identity_bases<double>, dim3((unsigned)count), dim3(256), 0, st,
                       (double *)vw, vw_off, cl_n, c0);
  return hipGetLastError();
}

int projection_variant_count(int precision) { return precision == 1 ? kNVar32 : kNVar64; }

void projection_variant_info(int precision, int v, int *N, int *NT) {
  const Variant &x = precision == 1 ? kVar32[v] : kVar64[v];
  *N = x.N;
  *NT = x.NT;
}

int projection_variant_kind(int precision, int v) {
  return (precision == 1 ? kVar32[v] : kVar64[v]).kind;
}

int projection_variant_two_level(int precision, int v) {
  return projection_variant_kind(precision, v) == 1;
}

int projection_default_variant(int precision, int s) {
  const int n = s + (s & 1);
  const int nv = projection_variant_count(precision);
  int best = -1, bestN = 1 << 30;
  for (int v = 0; v < nv; ++v) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (projection_variant_kind(precision, v) == 2) continue;
    if (N >= n && N < bestN) {   // first listed NT of the smallest fitting N
      best = v;
      bestN = N;
    }
  }
  return best;
}

// Standalone projections: the sign-function variant of the smallest fitting
// N with the fewest threads (fastest at every size measured: for N = 32 the
// one-wave register kernel beats the LDS one by 1.6x), else the Jacobi default.
int projection_standalone_variant(int precision, int s) {
  const int n = s + (s & 1);
  int best = -1, bestN = 1 << 30, bestNT = 1 << 30;
  for (int v = 0; v < projection_variant_count(precision); ++v) {
    int N, NT;
    projection_variant_info(precision, v, &N, &NT);
    if (projection_variant_kind(precision, v) != 2 || N < n) continue;
    if (N < bestN || (N == bestN && NT < bestNT)) {
      best = v;
      bestN = N;
      bestNT = NT;
    }
  }
  return best >= 0 ? best : projection_default_variant(precision, s);
}

hipError_t fill_random_blocks(int precision, void *out, int s, int count, uint32_t seed,
                              double offdiag, hipStream_t st) {
  const int64_t n = (int64_t)count * s * s;
  const int nb = (int)((n + 255) / 256);
  if (precision == 1)
    hipLaunchKernelGGL(k_fill_blocks<float>, dim3(nb), dim3(256), 0, st, (float *)out, s, count,
                       seed, offdiag);
  else
    hipLaunchKernelGGL(k_fill_blocks<double>, dim3(nb), dim3(256), 0, st, (double *)out, s,
                       count, seed, offdiag);
  return hipGetLastError();
}


int projection_bucket(int precision, int s) {
  const int v = projection_default_variant(precision, s);
  if (v < 0) return 0;
  int N, NT;
  projection_variant_info(precision, v, &N, &NT);
  return N;
}

int projection_max_size(int precision) { return 128; }

// The sign iteration for blocks of 16, one wave per block, entirely in
// registers.  A 16 x 16 x 16 product is four 16x16x4 matrix-core steps; the
// sum over k may be split over the steps in any order as long as both
// operands agree, and step j takes k = R(g, j) from lane group g = l / 16,
// where R(g, r) is the row of result register r (4g + r for FP32, g + 4r for
// FP64).  Lane l then keeps X(R(g, r), l mod 16) in register r, and that is
// exactly its operand of step r of the next product: the left operand
// X(l mod 16, k) = X(k, l mod 16) by symmetry, the right one M(k, l mod 16).
// So every product is four back-to-back steps on registers.  Using the
// transposed element for the left operand makes each product X^T M, equal
// to X M only while X is symmetric: without a correction the antisymmetric
// rounding grows through the iteration (errors near 1e-2 in a lane-exact
// simulation: the antisymmetric part changes sign and is scaled by up to 3
// at every step), so X <- (X + X^T) / 2 through LDS after every second step
// and after the last (the part then stays within 9 steps' rounding), and
// once more for the result.
template <typename T>
__device__ inline int sign16_row(int g, int r) {
  return sizeof(T) == 4 ? 4 * g + r : g + 4 * r;
}

template <typename T>
__global__ __launch_bounds__(64) void k_project_sign16(const int32_t *__restrict__ sizes,
                                                      const int64_t *__restrict__ offsets,
                                                      const T *__restrict__ in,
                                                      T *__restrict__ out, int k1, int k2) {
  typedef typename Mma<T>::v4 v4;
  __shared__ T C[16 * 17];
  const int l = threadIdx.x, g = l >> 4, col = l & 15;
  const int s = sizes[blockIdx.x];
  const int64_t off = offsets[blockIdx.x];
  if (s <= 0 || s > 16) return;   // sizes beyond max_size are left untouched
  T w[4];
  double f2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = sign16_row<T>(g, r);
    T v = T(0);
    if (row < s && col < s)
      v = T(0.5) * (in[off + (int64_t)row * s + col] + in[off + (int64_t)col * s + row]);
    w[r] = v;
    f2 += (double)v * (double)v;
  }
  f2 = wave_sum(f2);
  if (!(f2 > 0.0 && f2 < INFINITY)) {
    const T fill = f2 == 0.0 ? T(0) : T(NAN);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = sign16_row<T>(g, r);
      if (row < s && col < s) out[off + (int64_t)row * s + col] = fill;
    }
    return;
  }
  const T scale = (T)(1.0 / sqrt(f2));
  T x[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = w[r] * scale;
  // identity in the register layout
  T id[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) id[r] = sign16_row<T>(g, r) == col ? T(1) : T(0);
  const auto prod = [](const T (&a)[4], const T (&b)[4], T (&c)[4]) {
    v4 acc = v4{0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = Mma<T>::step(a[j], b[j], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) c[r] = acc[r];
  };
  for (int it = 0; it < k1 + k2; ++it) {
    T y[4], m[4];
    prod(x, x, y);                                              // Y = X^2
    if (it < k1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) m[r] = T(-3.2) * id[r] + T(1.2) * y[r];
      T t[4];
      prod(y, m, t);                                            // T = Y (-3.2 I + 1.2 Y)
#pragma unroll
      for (int r = 0; r < 4; ++r) m[r] = T(3) * id[r] + t[r];
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) m[r] = T(1.5) * id[r] - T(0.5) * y[r];
    }
    T xn[4];
    prod(x, m, xn);                                             // X <- X M
    if ((it & 1) || it == k1 + k2 - 1) {
      // X <- (X + X^T) / 2 (both triangles from the same two values)
#pragma unroll
      for (int r = 0; r < 4; ++r) C[sign16_row<T>(g, r) * 17 + col] = xn[r];
      __syncthreads();
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = T(0.5) * (xn[r] + C[col * 17 + sign16_row<T>(g, r)]);
      __syncthreads();
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) x[r] = xn[r];
    }
  }
  // W S, symmetrised through LDS: P+(W) = (W + (W S + S W) / 2) / 2
  T c[4];
  prod(w, x, c);
#pragma unroll
  for (int r = 0; r < 4; ++r) C[sign16_row<T>(g, r) * 17 + col] = c[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = sign16_row<T>(g, r);
    if (row < s && col < s)
      out[off + (int64_t)row * s + col] = T(0.5) * (w[r] + T(0.5) * (c[r] + C[col * 17 + row]));
  }
}

// The same for blocks of 32, one wave per block: X is held as 2 x 2 tiles
// of 16 (tile t = 2 I + J in registers 4t .. 4t + 3, rows 16 I + R(g, r),
// column 16 J + l mod 16).  Tile (I, J) of a product sums over the depth
// tiles K: its left operand X(16 I + i, 16 K + k) is, by symmetry, register
// j of tile (K, I), its right operand register j of tile (K, J), so each
// product is 32 matrix-core steps on registers (all four tiles are formed,
// both off-diagonal ones included, since each is the other's operand).
template <typename T>
__global__ __launch_bounds__(64) void k_project_sign32(const int32_t *__restrict__ sizes,
                                                      const int64_t *__restrict__ offsets,
                                                      const T *__restrict__ in,
                                                      T *__restrict__ out, int k1, int k2) {
  typedef typename Mma<T>::v4 v4;
  __shared__ T C[32 * 33];
  const int l = threadIdx.x, g = l >> 4, col = l & 15;
  const int s = sizes[blockIdx.x];
  const int64_t off = offsets[blockIdx.x];
  if (s <= 0 || s > 32) return;   // sizes beyond max_size are left untouched
  const auto rowof = [&](int t, int r) { return 16 * (t >> 1) + sign16_row<T>(g, r); };
  const auto colof = [&](int t) { return 16 * (t & 1) + col; };
  T w[4][4];
  double f2 = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rowof(t, r), cc = colof(t);
      T v = T(0);
      if (row < s && cc < s)
        v = T(0.5) * (in[off + (int64_t)row * s + cc] + in[off + (int64_t)cc * s + row]);
      w[t][r] = v;
      f2 += (double)v * (double)v;
    }
  f2 = wave_sum(f2);
  if (!(f2 > 0.0 && f2 < INFINITY)) {
    const T fill = f2 == 0.0 ? T(0) : T(NAN);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rowof(t, r), cc = colof(t);
        if (row < s && cc < s) out[off + (int64_t)row * s + cc] = fill;
      }
    return;
  }
  const T scale = (T)(1.0 / sqrt(f2));
  T x[4][4], id[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      x[t][r] = w[t][r] * scale;
      id[t][r] = rowof(t, r) == colof(t) ? T(1) : T(0);
    }
  const auto prod = [](const T (&a)[4][4], const T (&b)[4][4], T (&c)[4][4]) {
#pragma unroll
    for (int I = 0; I < 2; ++I)
#pragma unroll
      for (int J = 0; J < 2; ++J) {
        v4 acc = v4{0, 0, 0, 0};
#pragma unroll
        for (int K = 0; K < 2; ++K)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc = Mma<T>::step(a[2 * K + I][j], b[2 * K + J][j], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) c[2 * I + J][r] = acc[r];
      }
  };
  const auto symmetrise = [&](const T (&v)[4][4], T (&dst)[4][4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) C[rowof(t, r) * 33 + colof(t)] = v[t][r];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[t][r] = T(0.5) * (v[t][r] + C[colof(t) * 33 + rowof(t, r)]);
    __syncthreads();
  };
  for (int it = 0; it < k1 + k2; ++it) {
    T y[4][4], m[4][4];
    prod(x, x, y);                                              // Y = X^2
    if (it < k1) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(-3.2) * id[t][r] + T(1.2) * y[t][r];
      T u[4][4];
      prod(y, m, u);                                            // U = Y (-3.2 I + 1.2 Y)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(3) * id[t][r] + u[t][r];
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(1.5) * id[t][r] - T(0.5) * y[t][r];
    }
    T xn[4][4];
    prod(x, m, xn);                                             // X <- X M
    if ((it & 1) || it == k1 + k2 - 1) {
      symmetrise(xn, x);
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[t][r] = xn[t][r];
    }
  }
  // W S, symmetrised: P+(W) = (W + (W S + S W) / 2) / 2
  T c[4][4], cs[4][4];
  prod(w, x, c);
  symmetrise(c, cs);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = rowof(t, r), cc = colof(t);
      if (row < s && cc < s) out[off + (int64_t)row * s + cc] = T(0.5) * (w[t][r] + cs[t][r]);
    }
}

// ---------------------------------------------------------------------------
// Algorithm 1's clique step for blocks of up to 16 TB vertices (TB = 1, 2) in
// one wave's registers, with no eigenvectors: X_k = P+(W_k) by the sign
// iteration of k_project_sign16/32 on W_k = H_k x - Lambda_k / rho, then the
// multiplier update Lambda_k += rho (X_k - H_k x) (XkUpdate, LambdakUpdate)
// and the five residual partials of k_project's ADMM epilogue.  With DUAL,
// Algorithm 2's z-update instead: z_k = P+(v_k - lambda_k / rho) (zkUpdate)
// and ||z_k - z_k_prev||^2, the rest following the affine step as with the
// Jacobi kernels.  With HSDE, Algorithm 3's cone step on the PSD blocks:
// u_s = P+(u_hat_s - v_z), v_z += u_s - u_hat_s, u_t = u_hat_t and the six
// consensus partials of the Jacobi kernel's embedding mode.  The register
// layout is the sign kernels': tile t = TB I + J
// holds rows 16 I + R(g, r) at column 16 J + l mod 16.  W_k(i, k) and
// W_k(k, i) come from the same packed entry, so W_k is exactly symmetric.
// ---------------------------------------------------------------------------
template <typename T, int TB, bool DUAL, bool HSDE = false>
__global__ __launch_bounds__(64) void k_admm_sign(ProjArgs a, const int32_t *__restrict__ list,
                                                  int k1, int k2) {
  static_assert(!(DUAL && HSDE), "one algorithm per kernel");
  constexpr int NTL = TB * TB, NB = 16 * TB, CP = NB + 1;
  typedef typename Mma<T>::v4 v4;
  __shared__ T C[NB * CP];
  const int l = threadIdx.x, g = l >> 4, col = l & 15;
  // neighbouring cliques share coordinates of u: keep them on one XCD
  const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
  const int cl = list[x8 * q8 + min(x8, r8) + blockIdx.x / 8];
  const int inst = a.cl_inst[cl];
  const int s = a.cl_size[cl];
  const int64_t off = a.cl_off[cl];
  const bool inst_done = a.state[inst].done != 0;
  const double rho = a.state[inst].rho;
  const auto rowof = [&](int t, int r) { return 16 * (t / TB) + sign16_row<T>(g, r); };
  const auto colof = [&](int t) { return 16 * (t % TB) + col; };

  // gather: every index, multiplier and old-X load is issued before any is
  // used, then the loads of u they index (entries outside the clique read
  // its first entry and are masked).  Blocks of 16 keep the FP64 values for
  // the epilogue in registers; blocks of 32 (16 entries per lane) load them
  // again there, from the cache, so that the sign iteration keeps two waves
  // per SIMD.
  // (Algorithm 3 reloads its inputs in the epilogue, which needs more of
  // them: its gather keeps nothing)
  constexpr bool KEEP = TB == 1 && !HSDE;
  constexpr int KT = KEEP ? NTL : 1;
  int32_t loc[DUAL ? 1 : NTL][4];
  double lam[NTL][4], xo[KT][4], hu[DUAL ? 1 : KT][4], vd[(DUAL || HSDE) ? NTL : 1][4];
  const double hf = HSDE ? a.hs[inst].f : 0.0;
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rowof(t, r), k = colof(t);
      const int ii = i > k ? i : k, kk = i > k ? k : i;
      const int64_t e = (i < s && k < s) ? off + (int64_t)ii * (ii + 1) / 2 + kk : off;
      if constexpr (!DUAL) loc[t][r] = a.blk_loc[e];
      lam[t][r] = a.Lam[e];
      if constexpr (KEEP) xo[t][r] = a.X[e];
      if constexpr (DUAL) vd[t][r] = a.Vd[e];   // the slack block v_k
      if constexpr (HSDE) vd[t][r] = a.h_ns[e] - a.h_nt[e];   // Algorithm 3: n_s - n_t
    }
  T w[NTL][4];
  double f2 = 0.0;
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rowof(t, r), k = colof(t);
      double wd;
      if constexpr (DUAL) {
        wd = vd[t][r] - lam[t][r] / rho;
      } else if constexpr (HSDE) {
        // u_hat_s - v_z, u_hat_s = 0.5 (n_s - n_t + s_x) - f m_s (the Jacobi
        // kernel's arithmetic, term for term)
        const int ii = i > k ? i : k, kk = i > k ? k : i;
        const int64_t e = (i < s && k < s) ? off + (int64_t)ii * (ii + 1) / 2 + kk : off;
        const double ss = 0.5 * (vd[t][r] + a.h_sx[loc[t][r]]);
        wd = ss - hf * a.h_mzs[e] - lam[t][r];
      } else {
        const double h = a.u[loc[t][r]];
        if constexpr (KEEP) hu[t][r] = h;
        wd = h - lam[t][r] / rho;
      }
      const T v = (i < s && k < s) ? (T)wd : T(0);
      w[t][r] = v;
      f2 += (double)v * (double)v;
    }
  f2 = wave_sum(f2);
  // a finished instance writes nothing (uniform per workgroup)
  if (inst_done) return;

  // sign(W) from X0 = W / ||W||_F (W = 0 gives X = 0 and P+(W) = 0)
  const T scale = f2 > 0.0 ? (T)(1.0 / sqrt(f2)) : T(0);
  T x[NTL][4], id[NTL][4];
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      x[t][r] = w[t][r] * scale;
      id[t][r] = rowof(t, r) == colof(t) ? T(1) : T(0);
    }
  const auto prod = [](const T (&p)[NTL][4], const T (&q)[NTL][4], T (&z)[NTL][4]) {
#pragma unroll
    for (int I = 0; I < TB; ++I)
#pragma unroll
      for (int J = 0; J < TB; ++J) {
        v4 acc = v4{0, 0, 0, 0};
#pragma unroll
        for (int K = 0; K < TB; ++K)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc = Mma<T>::step(p[TB * K + I][j], q[TB * K + J][j], acc);
#pragma unroll
        for (int r = 0; r < 4; ++r) z[TB * I + J][r] = acc[r];
      }
  };
  const auto symmetrise = [&](const T (&v)[NTL][4], T (&dst)[NTL][4]) {
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) C[rowof(t, r) * CP + colof(t)] = v[t][r];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[t][r] = T(0.5) * (v[t][r] + C[colof(t) * CP + rowof(t, r)]);
    __syncthreads();
  };
  for (int it = 0; it < k1 + k2; ++it) {
    T y[NTL][4], m[NTL][4];
    prod(x, x, y);                                              // Y = X^2
    if (it < k1) {
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(-3.2) * id[t][r] + T(1.2) * y[t][r];
      T z[NTL][4];
      prod(y, m, z);                                            // Z = Y (-3.2 I + 1.2 Y)
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(3) * id[t][r] + z[t][r];
    } else {
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) m[t][r] = T(1.5) * id[t][r] - T(0.5) * y[t][r];
    }
    T xn[NTL][4];
    prod(x, m, xn);                                             // X <- X M
    if ((it & 1) || it == k1 + k2 - 1) {
      symmetrise(xn, x);
    } else {
#pragma unroll
      for (int t = 0; t < NTL; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) x[t][r] = xn[t][r];
    }
  }
  // X_k = P+(W) = (W + (W S + S W) / 2) / 2
  T c[NTL][4], cs[NTL][4];
  prod(w, x, c);
  symmetrise(c, cs);

  // epilogue on the lower entries: X_k, Lambda_k and the residual partials
  // (||X - Hx||^2, ||X||^2, ||Hx||^2, ||X - X_prev||^2, ||Lambda||^2, full
  // Frobenius norms: off-diagonal entries count twice)
  double p0 = 0, p1 = 0, p2 = 0, p3 = 0, p4 = 0, p6 = 0;
  if constexpr (HSDE) {
    // Algorithm 3: u_s = P+(u_hat_s - v_z), v_z += u_s - u_hat_s,
    // u_t = u_hat_t, and the partials of the consensus residuals on (u_s,
    // H u_x) and (v_z, u_t) (the Jacobi kernel's embedding epilogue)
#pragma unroll
    for (int t = 0; t < NTL; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = rowof(t, r), k = colof(t);
        if (!(i < s && k <= i)) continue;
        const int64_t e = off + (int64_t)i * (i + 1) / 2 + k;
        const int32_t lc = loc[t][r];
        const double hx = a.h_sx[lc], nt = a.h_nt[e];
        const double ss = 0.5 * (a.h_ns[e] - nt + hx);
        const double us_hat = ss - hf * a.h_mzs[e];
        const double ut = ss - hx + nt - hf * a.h_mzt[e];
        const double usn = (double)(T(0.5) * (w[t][r] + cs[t][r]));
        const double vzn = a.Lam[e] - us_hat + usn;
        a.X[e] = usn;
        a.Lam[e] = vzn;
        a.h_ut[e] = ut;
        const double hux = a.h_ux[lc];
        const double wt = (i == k) ? 1.0 : 2.0;
        p0 += wt * (usn - hux) * (usn - hux);
        p1 += wt * usn * usn;
        p2 += wt * hux * hux;
        p3 += wt * (vzn - ut) * (vzn - ut);
        p4 += wt * vzn * vzn;
        p6 += wt * ut * ut;
      }
  }
  double lo[NTL][4], xp[NTL][4], hp[NTL][4];
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rowof(t, r), k = colof(t);
      const int64_t e = off + (int64_t)i * (i + 1) / 2 + k;
      const bool lower = !HSDE && i < s && k <= i;
      if constexpr (HSDE) {
        lo[t][r] = xp[t][r] = hp[t][r] = 0.0;
      } else if constexpr (DUAL) {
        lo[t][r] = hp[t][r] = 0.0;
        if constexpr (KEEP) xp[t][r] = xo[t][r];
        else xp[t][r] = lower ? a.X[e] : 0.0;
      } else if constexpr (KEEP) {
        lo[t][r] = lam[t][r];
        xp[t][r] = xo[t][r];
        hp[t][r] = hu[t][r];
      } else {
        lo[t][r] = lower ? a.Lam[e] : 0.0;
        xp[t][r] = lower ? a.X[e] : 0.0;
        hp[t][r] = lower ? a.u[loc[t][r]] : 0.0;
      }
    }
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = rowof(t, r), k = colof(t);
      if (DUAL && i < s && k <= i) {
        // Algorithm 2: z_k and ||z_k - z_k_prev||^2 only
        const int64_t e = off + (int64_t)i * (i + 1) / 2 + k;
        const double zn = (double)(T(0.5) * (w[t][r] + cs[t][r]));
        a.X[e] = zn;
        const double wt = (i == k) ? 1.0 : 2.0;
        const double dz = zn - xp[t][r];
        p3 += wt * dz * dz;
      } else if (!DUAL && !HSDE && i < s && k <= i) {
        const int64_t e = off + (int64_t)i * (i + 1) / 2 + k;
        const double xn = (double)(T(0.5) * (w[t][r] + cs[t][r]));
        const double hx = hp[t][r];
        const double ln = lo[t][r] + rho * (xn - hx);
        a.X[e] = xn;
        a.Lam[e] = ln;
        const double wt = (i == k) ? 1.0 : 2.0;
        const double dc = xn - hx, dx = xn - xp[t][r];
        p0 += wt * dc * dc;
        p1 += wt * xn * xn;
        p2 += wt * hx * hx;
        p3 += wt * dx * dx;
        p4 += wt * ln * ln;
      }
    }
  p0 = wave_sum(p0);
  p1 = wave_sum(p1);
  p2 = wave_sum(p2);
  p3 = wave_sum(p3);
  p4 = wave_sum(p4);
  if (HSDE) p6 = wave_sum(p6);
  if (l == 0) {
    double *pp = a.part + NPART * (int64_t)cl;
    if (!DUAL) {   // (Algorithm 2: the multiplier update writes these)
      pp[0] = p0;
      pp[1] = p1;
      pp[2] = p2;
      pp[4] = p4;
    }
    pp[3] = p3;
    pp[5] = 0.0;   // no Jacobi sweeps
    pp[6] = p6;    // Algorithm 3: ||u_t||^2; else 0 (no sign fallback)
  }
}

// One pass of k_sign_big for a wave with NTL lower tiles in column block J:
// the product acc(t) = sum_k L(k, 16 (J + t) + c')^T M(k, J), M from x or
// (from_l) alpha [k == j] + beta L(k, j); then, between barriers, the lower
// tiles transformed to sa [i == j] + sb v into L on both sides of the
// diagonal.  Step (K, r) of the product takes k = 16 K + R(g, r) from lane
// group g (R the result-row map of the matrix cores: g + 4 r in FP64,
// 4 g + r in FP32), which is where register r of tile K holds row k.  The
// tile count is a template parameter, so each step's loads and matrix-core
// steps form one straight block (a run-time bound puts every load and step
// under a branch of its own), and the accumulators live only inside the
// pass.  The loads of step s + 1 are issued before the steps of s; the
// scheduling barrier keeps the compiler from hoisting all of them, which
// would need more registers than a wave has.
template <typename T, int N, int NTL>
__device__ __forceinline__ void sb_pass(T *L, const T (&x)[N / 16][4], bool from_l, T alpha,
                                        T beta, T sa, T sb, int J, int g, int c) {
  constexpr int P = N + 1, STEPS = N / 4;
  typedef typename Mma<T>::v4 v4;
  const int jc = 16 * J + c;
  const auto krow = [&](int K, int r) { return 16 * K + sign16_row<T>(g, r); };
  const auto bval = [&](int K, int r) {
    const int k = krow(K, r);
    return from_l ? (k == jc ? alpha : T(0)) + beta * L[k * P + jc] : x[K][r];
  };
  v4 acc[NTL];
#pragma unroll
  for (int t = 0; t < NTL; ++t) acc[t] = v4{0, 0, 0, 0};
  T av[NTL], b = bval(0, 0);
  {
    const int k = krow(0, 0);
#pragma unroll
    for (int t = 0; t < NTL; ++t) av[t] = L[k * P + jc + 16 * t];
  }
#pragma unroll
  for (int st = 0; st < STEPS; ++st) {
    T an[NTL], bn = T(0);
    if (st + 1 < STEPS) {
      const int K = (st + 1) >> 2, r = (st + 1) & 3, k = krow(K, r);
      bn = bval(K, r);
#pragma unroll
      for (int t = 0; t < NTL; ++t) an[t] = L[k * P + jc + 16 * t];
    }
#pragma unroll
    for (int t = 0; t < NTL; ++t) acc[t] = Mma<T>::step(av[t], b, acc[t]);
    __builtin_amdgcn_sched_barrier(0);
    if (st + 1 < STEPS) {
#pragma unroll
      for (int t = 0; t < NTL; ++t) av[t] = an[t];
      b = bn;
    }
  }
  __syncthreads();   // every wave has read L
#pragma unroll
  for (int t = 0; t < NTL; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * (J + t) + sign16_row<T>(g, r);
      if (i >= jc) {
        const T v = (i == jc ? sa : T(0)) + sb * acc[t][r];
        L[i * P + jc] = v;
        L[jc * P + i] = v;
      }
    }
  __syncthreads();
}

// Blocks of N = 48..128 by the sign iteration with one N x N matrix in LDS
// (the LDS kernels above hold two: 264 KB for FP64 blocks of 128).  One wave
// per column block of 16 (NT = 4 N); wave w owns column block J (J = w; for
// N = 128, 11 - w for w >= 4, so that the two waves that share a SIMD hold 9
// of the 36 tiles on or below the diagonal between them) and the lower tiles
// (I, J), I >= J, in it.  A product C = L M takes its left operand from the
// matrix L in LDS and its right operand M from registers: the wave's column
// block of M in the matrix cores' result layout (register r of lane l in row
// block K holds M(16K + R(g, r), 16J + c), g = l / 16, c = l % 16), which is
// exactly the right operand of step (K, r) of a product.  (Z = Y (-3.2 I +
// 1.2 Y) reads both operands from LDS.)  The lower tiles of a result go to
// LDS on both sides of the diagonal, so every iterate is exactly symmetric,
// and a wave reloads its column block of X from there after each step.  All
// factors are polynomials in W and commute, so the fast step X (3 I + Z) is
// formed as (3 I + Z) X with X the register operand, and the result as S W,
// which also goes to LDS for the epilogue.
// MODE: 0 standalone (row-major s x s blocks in `in` / `out`), 1 Algorithm
// 1's clique step (X_k, Lambda_k and the five residual partials, as
// k_admm_sign), 2 Algorithm 2's z-update (z_k and ||z_k - z_k_prev||^2), 3
// Algorithm 3's cone step on the PSD blocks (as k_admm_sign's HSDE mode).
template <typename T, int N, int MODE>
__global__ __launch_bounds__(4 * N) void k_sign_big(ProjArgs a, const int32_t *__restrict__ list,
                                                    const int32_t *__restrict__ sizes,
                                                    const int64_t *__restrict__ offsets,
                                                    const T *__restrict__ in, T *__restrict__ out,
                                                    int k1, int k2) {
  constexpr int P = N + 1, TN = N / 16, NT = 4 * N;
  static_assert(N % 16 == 0 && N >= 48 && N <= 128, "column blocks of 16");
  __shared__ T L[N * P];
  __shared__ double red[6 * (NT / 64)];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  const int J = (TN == 8 && w >= 4) ? 11 - w : w, nt = TN - J, jc = 16 * J + c;

  int s, cl = 0;
  int64_t off;
  bool inst_done = false;
  double rho = 1.0, hf = 0.0;
  if (MODE == 0) {
    s = sizes[blockIdx.x];
    off = offsets[blockIdx.x];
    if (s <= 0 || s > N) return;   // sizes beyond max_size are left untouched
  } else {
    // neighbouring cliques share coordinates of u: keep them on one XCD
    const int nb = gridDim.x, q8 = nb / 8, r8 = nb % 8, x8 = blockIdx.x % 8;
    cl = list[x8 * q8 + min(x8, r8) + blockIdx.x / 8];
    const int inst = a.cl_inst[cl];
    s = a.cl_size[cl];
    off = a.cl_off[cl];
    inst_done = a.state[inst].done != 0;
    rho = a.state[inst].rho;
    if (MODE == 3) hf = a.hs[inst].f;
  }
  // packed position of (i, j) in the clique's lower triangle (i, j < s)
  const auto packed = [&](int i, int j) {
    const int ii = i > j ? i : j, jj = i > j ? j : i;
    return off + (int64_t)ii * (ii + 1) / 2 + jj;
  };
  // W(i, j) inside the clique in the block's precision, the same arithmetic
  // at every call (MODE 3: h = n_s - n_t, sx = s_x at the entry's
  // coordinate, mz = m_s; u_hat_s - v_z as the Jacobi kernel forms it)
  const auto w_entry = [&](int i, int j, double lam, double h, double sx, double mz) {
    if (MODE == 0) return T(0.5) * (in[off + (int64_t)i * s + j] + in[off + (int64_t)j * s + i]);
    if (MODE == 3) return (T)(0.5 * (h + sx) - hf * mz - lam);
    return (T)(h - lam / rho);
  };
  // the wave's column block of W (zero outside the clique) into x; returns
  // its sum of squares
  T x[TN][4];
  const auto gather_w = [&]() {
    // the lane index passes through an empty asm statement, so that the
    // addresses are formed at each call rather than hoisted out of the
    // iteration loop and kept live across it
    int gl = g;
    asm volatile("" : "+v"(gl));
    double f2 = 0.0;
    if constexpr (MODE == 3) {
      // Algorithm 3's six operands per entry, one row of tiles at a time
      // (entries outside the clique read the clique's first entry)
#pragma unroll
      for (int K = 0; K < TN; ++K) {
        int32_t lc[4];
        double ns[4], ntv[4], lm[4], mz[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * K + sign16_row<T>(gl, r);
          const int64_t e = (i < s && jc < s) ? packed(i, jc) : off;
          lc[r] = a.blk_loc[e];
          ns[r] = a.h_ns[e];
          ntv[r] = a.h_nt[e];
          lm[r] = a.Lam[e];
          mz[r] = a.h_mzs[e];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * K + sign16_row<T>(gl, r);
          const T v = (i < s && jc < s) ? w_entry(i, jc, lm[r], ns[r] - ntv[r], a.h_sx[lc[r]], mz[r])
                                        : T(0);
          x[K][r] = v;
          f2 += (double)v * (double)v;
        }
      }
      return f2;
    }
    int32_t loc[MODE == 1 ? TN : 1][4];
    double lam[MODE == 0 ? 1 : TN][4], hv[MODE == 2 ? TN : 1][4];
#pragma unroll
    for (int K = 0; K < TN; ++K)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * K + sign16_row<T>(gl, r);
        const int64_t e = (i < s && jc < s) ? packed(i, jc) : off;
        if constexpr (MODE != 0) lam[K][r] = a.Lam[e];
        if constexpr (MODE == 1) loc[K][r] = a.blk_loc[e];
        if constexpr (MODE == 2) hv[K][r] = a.Vd[e];   // the slack block v_k
      }
#pragma unroll
    for (int K = 0; K < TN; ++K)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * K + sign16_row<T>(gl, r);
        T v = T(0);
        if (i < s && jc < s) {
          if constexpr (MODE == 0) {
            v = w_entry(i, jc, 0.0, 0.0, 0.0, 0.0);
          } else if constexpr (MODE == 1) {
            v = w_entry(i, jc, lam[K][r], a.u[loc[K][r]], 0.0, 0.0);
          } else {
            v = w_entry(i, jc, lam[K][r], hv[K][r], 0.0, 0.0);
          }
        }
        x[K][r] = v;
        f2 += (double)v * (double)v;
      }
    return f2;
  };
  double f2 = block_sum<NT>(gather_w(), red);
  if (inst_done) return;   // a finished instance writes nothing (uniform)
  if (MODE == 0 && !(f2 > 0.0 && f2 < INFINITY)) {
    // W = 0: P+(W) = 0; a NaN or infinite entry: NaN throughout
    const T fill = f2 == 0.0 ? T(0) : T(NAN);
#pragma unroll
    for (int K = 0; K < TN; ++K)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * K + sign16_row<T>(g, r);
        if (i < s && jc < s) out[off + (int64_t)i * s + jc] = fill;
      }
    return;
  }
  // X0 = W / ||W||_F into L (the column blocks partition the matrix) and x
  const T scale = f2 > 0.0 ? (T)(1.0 / sqrt(f2)) : T(0);
#pragma unroll
  for (int K = 0; K < TN; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      x[K][r] *= scale;
      L[(16 * K + sign16_row<T>(g, r)) * P + jc] = x[K][r];
    }
  __syncthreads();

  const int ntu = __builtin_amdgcn_readfirstlane(nt);   // uniform per wave
  // one pass: L <- sa I + sb (L M), M from x or alpha I + beta L (from_l)
  const auto pass = [&](bool from_l, T alpha, T beta, T sa, T sb, int gq, int cq) {
    switch (ntu) {
      case 8: if constexpr (TN >= 8) sb_pass<T, N, 8>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 7: if constexpr (TN >= 7) sb_pass<T, N, 7>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 6: if constexpr (TN >= 6) sb_pass<T, N, 6>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 5: if constexpr (TN >= 5) sb_pass<T, N, 5>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 4: if constexpr (TN >= 4) sb_pass<T, N, 4>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 3: sb_pass<T, N, 3>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      case 2: sb_pass<T, N, 2>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
      default: sb_pass<T, N, 1>(L, x, from_l, alpha, beta, sa, sb, J, gq, cq); break;
    }
  };
  // The passes of the k1 fast steps (L = X X; L = 3 I + L (-3.2 I + 1.2 L);
  // L = L X, then x = L) and of the k2 Newton-Schulz steps (L = 1.5 I -
  // 0.5 X X; L = L X, then x = L), and a last one, L = S W with W again in
  // x.  (The lane index passes through an empty asm statement at each pass,
  // so that the LDS addresses derived from it are formed in the pass instead
  // of hoisted out of the loop and kept live, which spills.)
  const int nprod = 3 * k1 + 2 * k2;
  for (int q = 0; q <= nprod; ++q) {
    int lq = l;
    asm volatile("" : "+v"(lq));
    const int gq = lq >> 4, cq = lq & 15;
    const bool fast = q < 3 * k1;
    const int ph = fast ? q % 3 : ((q - 3 * k1) % 2 == 0 ? 0 : 2);   // Y, Z, X
    if (q == nprod) gather_w();
    T sa = T(0), sb = T(1);
    if (q < nprod && ph == 1) sa = T(3);
    if (q < nprod && !fast && ph == 0) {
      sa = T(1.5);
      sb = T(-0.5);
    }
    pass(q < nprod && ph == 1, T(-3.2), T(1.2), sa, sb, gq, cq);
    if (q < nprod && ph == 2) {
#pragma unroll
      for (int K = 0; K < TN; ++K)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          x[K][r] = L[(16 * K + sign16_row<T>(gq, r)) * P + 16 * J + cq];
    }
  }

  // P+(W) = (W + C) / 2 on the lower entries of the wave's column block
  double pv[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int K = 0; K < TN; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * K + sign16_row<T>(g, r);
      if (i < jc || i >= s) continue;
      const T cv = L[i * P + jc];
      if (MODE == 0) {
        const T xn = T(0.5) * (w_entry(i, jc, 0.0, 0.0, 0.0, 0.0) + cv);
        out[off + (int64_t)i * s + jc] = xn;
        out[off + (int64_t)jc * s + i] = xn;
        continue;
      }
      const int64_t e = packed(i, jc);
      if (MODE == 3) {
        // Algorithm 3: u_s = P+(u_hat_s - v_z), v_z += u_s - u_hat_s,
        // u_t = u_hat_t and the six consensus partials
        const int32_t lc = a.blk_loc[e];
        const double lam = a.Lam[e], hx = a.h_sx[lc], ntv = a.h_nt[e], nsv = a.h_ns[e];
        const double mzs = a.h_mzs[e];
        const double ss = 0.5 * (nsv - ntv + hx);
        const double us_hat = ss - hf * mzs;
        const double ut = ss - hx + ntv - hf * a.h_mzt[e];
        const double usn = (double)(T(0.5) * (w_entry(i, jc, lam, nsv - ntv, hx, mzs) + cv));
        const double vzn = lam - us_hat + usn;
        a.X[e] = usn;
        a.Lam[e] = vzn;
        a.h_ut[e] = ut;
        const double hux = a.h_ux[lc];
        const double wt = (i == jc) ? 1.0 : 2.0;
        pv[0] += wt * (usn - hux) * (usn - hux);
        pv[1] += wt * usn * usn;
        pv[2] += wt * hux * hux;
        pv[3] += wt * (vzn - ut) * (vzn - ut);
        pv[4] += wt * vzn * vzn;
        pv[5] += wt * ut * ut;
        continue;
      }
      const double lam = a.Lam[e], xo = a.X[e];
      const double h = MODE == 1 ? a.u[a.blk_loc[e]] : a.Vd[e];
      const double xn = (double)(T(0.5) * (w_entry(i, jc, lam, h, 0.0, 0.0) + cv));
      const double wt = (i == jc) ? 1.0 : 2.0;
      a.X[e] = xn;
      const double dx = xn - xo;
      pv[3] += wt * dx * dx;
      if (MODE == 1) {
        const double ln = lam + rho * (xn - h);
        a.Lam[e] = ln;
        const double dc = xn - h;
        pv[0] += wt * dc * dc;
        pv[1] += wt * xn * xn;
        pv[2] += wt * h * h;
        pv[4] += wt * ln * ln;
      }
    }
  if (MODE == 0) return;
  block_sum_n<NT, 6>(pv, red);
  if (tid == 0) {
    double *pp = a.part + NPART * (int64_t)cl;
    if (MODE != 2) {   // (Algorithm 2: the multiplier update writes these)
      pp[0] = pv[0];
      pp[1] = pv[1];
      pp[2] = pv[2];
      pp[4] = pv[4];
    }
    pp[3] = pv[3];
    pp[5] = 0.0;     // no Jacobi sweeps
    pp[6] = pv[5];   // Algorithm 3: ||u_t||^2; else 0 (no sign fallback)
  }
}

// ---------------------------------------------------------------------------
// The same sign iteration for a few large FP64 cliques, split over
// workgroups.  k_sign_big puts one clique on one compute unit, so a handful
// of large cliques leaves most of the chip idle for all 3 k1 + 2 k2 + 1
// products.  Here every product is a launch of its own over all the
// clique's lower 16 x 16 tiles, one wave per tile (36 waves for a block of
// 128), and the iterates live in a per-clique workspace of four N x N
// row-major matrices (three that the products rotate through, and W for the
// last product).  A product reads its left operand A(i, k) as A(k, i): every
// iterate is exactly symmetric (the lower tiles are computed and mirrored),
// so each step of the matrix cores loads four rows of 16 consecutive
// entries.  The products accumulate over k in the order k_sign_big uses;
// ||W||_F is summed in another order, so the iterates agree with k_sign_big's
// to rounding, not bit for bit.
// ---------------------------------------------------------------------------
constexpr int SPLIT_GNT = 512;   // threads of the gather and epilogue launches
// After the count * 4 matrices the workspace holds SPLIT_META doubles per
// clique, written by the gather: done flag, rho, Algorithm 3's f, size s,
// packed offset and clique index (all exact in a double), so that the later
// launches read them with one load instead of three dependent ones.
constexpr int SPLIT_META = 8;

__device__ inline int split_slot(int b, int nb) {
  // consecutive slots on one XCD (a clique's tiles share its operands in L2)
  const int q8 = nb / 8, r8 = nb % 8, x8 = b % 8;
  return x8 * q8 + min(x8, r8) + b / 8;
}

// W = the projection input (zero outside the clique) into matrix 3 of the
// clique's workspace, X0 = W / ||W||_F into matrix 0.  The threads walk the
// packed lower triangle in order (coalesced loads of the clique's blocks),
// keep their values and write both triangles once ||W||_F is known; the
// padding is written too (as zeros), since the products leave other values
// there that must not reach the next iteration.
template <int N, int MODE>
__global__ __launch_bounds__(SPLIT_GNT) void k_split_gather(ProjArgs a, const int32_t *__restrict__ list,
                                                            double *__restrict__ ws) {
  constexpr int EPT = (N * (N + 1) / 2 + SPLIT_GNT - 1) / SPLIT_GNT;
  __shared__ double red[SPLIT_GNT / 64];
  const int q = split_slot(blockIdx.x, gridDim.x);
  const int cl = list[q];
  const int inst = a.cl_inst[cl];
  const int s = a.cl_size[cl];
  const int64_t off = a.cl_off[cl];
  const bool done = a.state[inst].done != 0;
  const double rho = a.state[inst].rho;
  const double hf = MODE == 3 ? a.hs[inst].f : 0.0;
  if (threadIdx.x == 0) {
    double *meta = ws + (int64_t)gridDim.x * 4 * N * N + (int64_t)q * SPLIT_META;
    meta[0] = done ? 1.0 : 0.0;
    meta[1] = rho;
    meta[2] = hf;
    meta[3] = (double)s;
    meta[4] = (double)off;
    meta[5] = (double)cl;
  }
  if (done) return;   // a finished instance: nothing (uniform)
  double *W = ws + ((int64_t)q * 4 + 3) * N * N, *X0 = ws + (int64_t)q * 4 * N * N;
  const int npk = s * (s + 1) / 2;
  // chunks of CH entries: every load of a chunk is issued before the first
  // is used (entries past the end read the clique's first entry)
  constexpr int CH = MODE == 3 ? 6 : 9;
  double v[EPT], f2 = 0.0;
#pragma unroll
  for (int t0 = 0; t0 < EPT; t0 += CH) {
    int32_t lc[CH];
    double lam[CH], h1[CH], h2[CH], h3[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int el = threadIdx.x + SPLIT_GNT * (t0 + c);
      const int64_t e = off + ((t0 + c < EPT && el < npk) ? el : 0);
      lam[c] = a.Lam[e];
      if (MODE != 2) lc[c] = a.blk_loc[e];
      if (MODE == 2) h1[c] = a.Vd[e];
      if (MODE == 3) {
        h1[c] = a.h_ns[e];
        h2[c] = a.h_nt[e];
        h3[c] = a.h_mzs[e];
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (MODE == 1) h1[c] = a.u[lc[c]];
      if (MODE == 3) h2[c] = (h1[c] - h2[c]) + a.h_sx[lc[c]];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (t0 + c >= EPT) continue;
      const int el = threadIdx.x + SPLIT_GNT * (t0 + c);
      // the arithmetic of k_sign_big's gather, term for term
      double w = MODE == 3 ? 0.5 * h2[c] - hf * h3[c] - lam[c] : h1[c] - lam[c] / rho;
      if (el >= npk) w = 0.0;
      int i, j;
      tri_inv(el < npk ? el : 0, i, j);
      v[t0 + c] = w;
      f2 += (i == j ? 1.0 : 2.0) * w * w;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  f2 = block_sum<SPLIT_GNT>(f2, red);
  const double scale = f2 > 0.0 ? 1.0 / sqrt(f2) : 0.0;
#pragma unroll
  for (int t = 0; t < EPT; ++t) {
    const int el = threadIdx.x + SPLIT_GNT * t;
    if (el < npk) {
      int i, j;
      tri_inv(el, i, j);
      const double x0 = v[t] * scale;
      W[i * N + j] = v[t];
      X0[i * N + j] = x0;
      if (i != j) {
        W[j * N + i] = v[t];
        X0[j * N + i] = x0;
      }
    }
  }
  // the padding rows and columns
  for (int idx = threadIdx.x; idx < N * N; idx += SPLIT_GNT) {
    if (idx / N >= s || idx % N >= s) {
      W[idx] = 0.0;
      X0[idx] = 0.0;
    }
  }
}

// One product of the split iteration: matrix ob = sa I + sb (A M) on the
// lower tiles, mirrored, with A = matrix lb and M = matrix mb or (from_l)
// alpha I + beta A.  A workgroup of four waves takes a 2 x 2 block of tiles
// (rows 32 I2 .. + 31, columns 32 J2 .. + 31, I2 >= J2; in a diagonal block
// the wave of the upper tile only loads): it stages the two 32-column slabs
// A(:, 32 I2 ..) and M(:, 32 J2 ..) in LDS with 16-byte loads, and each wave
// forms its tile from there, so a workgroup reads 2 N x 32 entries for four
// tiles instead of 2 N x 16 per tile.
template <int N>
__global__ __launch_bounds__(256) void k_split_pass(double *__restrict__ ws, int count, int lb,
                                                    int mb, int ob, int from_l, double alpha,
                                                    double beta, double sa, double sb) {
  constexpr int TN2 = N / 32, WPC = TN2 * (TN2 + 1) / 2, STEPS = N / 4, SP = 33;
  static_assert(N % 32 == 0, "blocks of 2 x 2 tiles");
  typedef Mma<double>::v4 v4;
  __shared__ double sA[N * SP], sM[N * SP];
  __shared__ double tr[4][16][17];
  const int lin = split_slot(blockIdx.x, gridDim.x);
  const int q = lin / WPC, blk = lin % WPC;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4, c = l & 15;
  // a finished instance's clique computes nothing (its flag loads beside
  // the operands; the workspace is the split iteration's own)
  const double done = ws[(int64_t)count * 4 * N * N + (int64_t)q * SPLIT_META];
  const double *A = ws + ((int64_t)q * 4 + lb) * N * N;
  const double *M = ws + ((int64_t)q * 4 + mb) * N * N;
  double *O = ws + ((int64_t)q * 4 + ob) * N * N;
  // block -> (I2, J2), I2 >= J2, row by row of the lower triangle
  int I2 = 0;
  while ((I2 + 1) * (I2 + 2) / 2 <= blk) ++I2;
  const int J2 = blk - I2 * (I2 + 1) / 2;
  // the slabs: row k, columns 32 I2 + 2 m, +1 (A) and 32 J2 + 2 m, +1 (M);
  // every load of the thread is issued before the first is used
  constexpr int LD = N * 16 / 256;
  const double *Ms = from_l ? A : M;
  double2 va[LD], vm[LD];
#pragma unroll
  for (int it = 0; it < LD; ++it) {
    const int f = tid + 256 * it, k = f >> 4, m = f & 15;
    va[it] = *reinterpret_cast<const double2 *>(A + k * N + 32 * I2 + 2 * m);
    vm[it] = *reinterpret_cast<const double2 *>(Ms + k * N + 32 * J2 + 2 * m);
  }
#pragma unroll
  for (int it = 0; it < LD; ++it) {
    const int f = tid + 256 * it, k = f >> 4, m = f & 15, jb = 32 * J2 + 2 * m;
    if (from_l) {
      vm[it].x = (k == jb ? alpha : 0.0) + beta * vm[it].x;
      vm[it].y = (k == jb + 1 ? alpha : 0.0) + beta * vm[it].y;
    }
    sA[k * SP + 2 * m] = va[it].x;
    sA[k * SP + 2 * m + 1] = va[it].y;
    sM[k * SP + 2 * m] = vm[it].x;
    sM[k * SP + 2 * m + 1] = vm[it].y;
  }
  __syncthreads();
  const int I = 2 * I2 + (w >> 1), J = 2 * J2 + (w & 1);
  const bool live = I >= J && done == 0.0;
  const int xa = 16 * (w >> 1) + c, xb = 16 * (w & 1) + c;   // slab columns
  v4 acc = v4{0, 0, 0, 0};
  if (live) {
#pragma unroll 8
    for (int st = 0; st < STEPS; ++st) {
      const int k = 4 * st + g;
      acc = Mma<double>::step(sA[k * SP + xa], sM[k * SP + xb], acc);
    }
  }
  // rows 16 I + g + 4 r, column 16 J + c: the lower entries directly, the
  // mirrored ones through a transpose in LDS (coalesced rows both ways)
  const int ca = 16 * I + c, cb = 16 * J + c;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int il = g + 4 * r;
    const double v = (I == J && il == c ? sa : 0.0) + sb * acc[r];
    tr[w][il][c] = v;
    if (live && (I > J || il >= c)) O[(16 * I + il) * N + cb] = v;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int il = g + 4 * r;   // target row 16 J + il, column 16 I + c
    if (live && (I > J || il < c)) O[(16 * J + il) * N + ca] = tr[w][c][il];
  }
}

// P+(W) = (W + S W) / 2 from matrices cb (S W) and 3 (W) of the workspace,
// and the clique step of each algorithm, as k_sign_big's epilogue.
template <int N, int MODE>
__global__ __launch_bounds__(SPLIT_GNT) void k_split_epilogue(ProjArgs a, const int32_t *__restrict__ list,
                                                              const double *__restrict__ ws, int cb) {
  __shared__ double red[6 * (SPLIT_GNT / 64)];
  const int q = split_slot(blockIdx.x, gridDim.x);
  const double *meta = ws + (int64_t)gridDim.x * 4 * N * N + (int64_t)q * SPLIT_META;
  if (meta[0] != 0.0) return;   // a finished instance writes nothing (uniform)
  const double rho = meta[1], hf = meta[2];
  const int s = (int)meta[3];
  const int64_t off = (int64_t)meta[4];
  const int cl = (int)meta[5];
  const double *C = ws + ((int64_t)q * 4 + cb) * N * N, *W = ws + ((int64_t)q * 4 + 3) * N * N;
  double pv[6] = {0, 0, 0, 0, 0, 0};
  // packed entries el = tid + SPLIT_GNT t of the clique, CH at a time with
  // all their loads issued first (entries past the end read the first one
  // and are skipped)
  constexpr int EPT = (N * (N + 1) / 2 + SPLIT_GNT - 1) / SPLIT_GNT;
  constexpr int CH = MODE == 3 ? 6 : 9;
  const int npk = s * (s + 1) / 2;
#pragma unroll
  for (int t0 = 0; t0 < EPT; t0 += CH) {
    int ix[CH];
    int32_t lc[CH];
    double wv[CH], cv[CH], lam[CH], xo[CH], h[CH], hx[CH], ux[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int el = threadIdx.x + SPLIT_GNT * (t0 + c);
      const bool ok = t0 + c < EPT && el < npk;
      int i, j;
      tri_inv(ok ? el : 0, i, j);
      ix[c] = i * N + j;
      const int64_t e = off + (ok ? el : 0);
      wv[c] = W[ix[c]];
      cv[c] = C[ix[c]];
      lam[c] = a.Lam[e];
      if (MODE != 3) xo[c] = a.X[e];
      if (MODE != 2) lc[c] = a.blk_loc[e];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (MODE == 1) h[c] = a.u[lc[c]];
      if (MODE == 3) {
        hx[c] = a.h_sx[lc[c]];
        ux[c] = a.h_ux[lc[c]];
      }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int el = threadIdx.x + SPLIT_GNT * (t0 + c);
      if (t0 + c >= EPT || el >= npk) continue;
      int i, j;
      tri_inv(el, i, j);
      const int64_t e = off + el;
      const double xn = 0.5 * (wv[c] + cv[c]);
      const double wt = (i == j) ? 1.0 : 2.0;
      if (MODE == 3) {
        const double ntv = a.h_nt[e];
        const double ss = 0.5 * (a.h_ns[e] - ntv + hx[c]);
        const double us_hat = ss - hf * a.h_mzs[e];
        const double ut = ss - hx[c] + ntv - hf * a.h_mzt[e];
        const double vzn = lam[c] - us_hat + xn;
        a.X[e] = xn;
        a.Lam[e] = vzn;
        a.h_ut[e] = ut;
        const double hux = ux[c];
        pv[0] += wt * (xn - hux) * (xn - hux);
        pv[1] += wt * xn * xn;
        pv[2] += wt * hux * hux;
        pv[3] += wt * (vzn - ut) * (vzn - ut);
        pv[4] += wt * vzn * vzn;
        pv[5] += wt * ut * ut;
        continue;
      }
      a.X[e] = xn;
      const double dx = xn - xo[c];
      pv[3] += wt * dx * dx;
      if (MODE == 1) {
        const double ln = lam[c] + rho * (xn - h[c]);
        a.Lam[e] = ln;
        const double dc = xn - h[c];
        pv[0] += wt * dc * dc;
        pv[1] += wt * xn * xn;
        pv[2] += wt * h[c] * h[c];
        pv[4] += wt * ln * ln;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  block_sum_n<SPLIT_GNT, 6>(pv, red);
  if (threadIdx.x == 0) {
    double *pp = a.part + NPART * (int64_t)cl;
    if (MODE != 2) {
      pp[0] = pv[0];
      pp[1] = pv[1];
      pp[2] = pv[2];
      pp[4] = pv[4];
    }
    pp[3] = pv[3];
    pp[5] = 0.0;
    pp[6] = pv[5];
  }
}

// The launches of one split projection: gather, 3 k1 + 2 k2 + 1 products,
// epilogue.  ws holds 4 N^2 + SPLIT_META doubles per clique of the list.
template <int N, int MODE>
hipError_t launch_split(const ProjArgs &a, const int32_t *list, int count, double *ws, int k1,
                        int k2, hipStream_t st) {
  constexpr int WPC = (N / 32) * (N / 32 + 1) / 2;
  hipLaunchKernelGGL((k_split_gather<N, MODE>), dim3(count), dim3(SPLIT_GNT), 0, st, a, list, ws);
  const auto pass = [&](int lb, int mb, int ob, int from_l, double alpha, double beta, double sa,
                        double sb) {
    hipLaunchKernelGGL((k_split_pass<N>), dim3(count * WPC), dim3(256), 0, st, ws, count, lb, mb,
                       ob, from_l, alpha, beta, sa, sb);
  };
  // matrices 0-2 rotate (x: the iterate; the other two: free), 3 is W
  int bx = 0;
  const auto other = [](int u, int v) { return 3 - u - v; };   // the third of 0, 1, 2
  for (int it = 0; it < k1; ++it) {
    const int by = (bx + 1) % 3, bz = other(bx, by);
    pass(bx, bx, by, 0, 0.0, 0.0, 0.0, 1.0);      // Y = X X
    pass(by, by, bz, 1, -3.2, 1.2, 3.0, 1.0);     // Z' = 3 I + Y (-3.2 I + 1.2 Y)
    pass(bz, bx, by, 0, 0.0, 0.0, 0.0, 1.0);      // X <- Z' X
    bx = by;
  }
  for (int it = 0; it < k2; ++it) {
    const int by = (bx + 1) % 3, bz = other(bx, by);
    pass(bx, bx, by, 0, 0.0, 0.0, 1.5, -0.5);     // 1.5 I - 0.5 X X
    pass(by, bx, bz, 0, 0.0, 0.0, 0.0, 1.0);      // X <- (1.5 I - 0.5 X^2) X
    bx = bz;
  }
  const int bc = (bx + 1) % 3;
  pass(bx, 3, bc, 0, 0.0, 0.0, 0.0, 1.0);         // S W
  hipLaunchKernelGGL((k_split_epilogue<N, MODE>), dim3(count), dim3(SPLIT_GNT), 0, st, a, list,
                     (const double *)ws, bc);
  return hipGetLastError();
}

template <typename T, int N, int NT>
hipError_t launch_sign(int count, const int32_t *sizes, const int64_t *offsets, const void *in,
                       void *out, int k1, int k2, hipStream_t st) {
  hipLaunchKernelGGL((k_project_sign<T, N, NT>), dim3(count), dim3(NT), 0, st, sizes, offsets,
                     (const T *)in, (T *)out, k1, k2);
  return hipGetLastError();
}

hipError_t dispatch_sign(int dtype, int N, int NT, int count, const int32_t *sizes,
                         const int64_t *offsets, const void *in, void *out, int k1, int k2,
                         hipStream_t st) {
#define SDP_SIGN(T, n, nt)                                                                     \
  if (N == n && NT == nt) return launch_sign<T, n, nt>(count, sizes, offsets, in, out, k1, k2, st);
  if (N == 16 && NT == 64) {   // blocks of 16: the register-resident kernel
    if (dtype == 1)
      hipLaunchKernelGGL(k_project_sign16<float>, dim3(count), dim3(64), 0, st, sizes, offsets,
                         (const float *)in, (float *)out, k1, k2);
    else
      hipLaunchKernelGGL(k_project_sign16<double>, dim3(count), dim3(64), 0, st, sizes, offsets,
                         (const double *)in, (double *)out, k1, k2);
    return hipGetLastError();
  }
  if (N == 32 && NT == 64) {   // blocks of 32: the register-resident kernel
    if (dtype == 1)
      hipLaunchKernelGGL(k_project_sign32<float>, dim3(count), dim3(64), 0, st, sizes, offsets,
                         (const float *)in, (float *)out, k1, k2);
    else
      hipLaunchKernelGGL(k_project_sign32<double>, dim3(count), dim3(64), 0, st, sizes, offsets,
                         (const double *)in, (double *)out, k1, k2);
    return hipGetLastError();
  }
  // blocks of 48 and more: one block in LDS, the other operand in registers
  // (1.1-1.5x the rate of the two-block LDS kernel on 4096 blocks)
#define SDP_SIGN_BIG(T, n)                                                                     \
  if (N == n && NT == 4 * n) {                                                                 \
    hipLaunchKernelGGL((k_sign_big<T, n, 0>), dim3(count), dim3(4 * n), 0, st, ProjArgs{},     \
                       nullptr, sizes, offsets, (const T *)in, (T *)out, k1, k2);              \
    return hipGetLastError();                                                                  \
  }
  if (dtype == 1) {
    SDP_SIGN(float, 32, 256)
    SDP_SIGN_BIG(float, 48)
    SDP_SIGN_BIG(float, 64)
    SDP_SIGN_BIG(float, 80)
    SDP_SIGN_BIG(float, 96)
    SDP_SIGN_BIG(float, 112)
    SDP_SIGN_BIG(float, 128)
  } else {
    SDP_SIGN_BIG(double, 48)
    SDP_SIGN_BIG(double, 64)
    SDP_SIGN_BIG(double, 80)
    SDP_SIGN_BIG(double, 96)
    SDP_SIGN_BIG(double, 128)
  }
#undef SDP_SIGN_BIG
#undef SDP_SIGN
  return hipErrorInvalidValue;
}

// A few large FP64 cliques leave most compute units idle with one workgroup
// per clique: up to SPLIT_MAX_CLIQUES cliques of blocks of 96 or 128 take
// the split iteration (a block of 128 spreads over 36 waves instead of 8).
constexpr int SPLIT_MAX_CLIQUES = 64;

int64_t split_workspace(int precision, int variant, int count) {
  int N, NT;
  projection_variant_info(precision, variant, &N, &NT);
  if (precision != 0 || projection_variant_kind(precision, variant) != 2 || NT != 4 * N ||
      (N != 96 && N != 128) || count <= 0 || count > SPLIT_MAX_CLIQUES)
    return 0;
  return (int64_t)count * (4 * N * N + SPLIT_META);
}

hipError_t launch_admm_projection(int precision, int variant, const int32_t *list, int count,
                                  const ProjArgs &a, hipStream_t st, double *split_ws) {
  int N, NT;
  projection_variant_info(precision, variant, &N, &NT);
  if (projection_variant_kind(precision, variant) == 2) {
    // sign-function lists (Algorithms 1, 2 and 3): the register kernels for
    // blocks of 16 and 32, below the one-block LDS kernel for FP64 blocks of
    // 48-128; a caller that needs eigenvectors (the unrolled forward records
    // V, theta) gets the Jacobi default of the same block size
    if (!a.eig && NT == 64 && (N == 16 || N == 32)) {
      if (count <= 0) return hipSuccess;
      int k1, k2;
      sign_schedule(a.tol, N, &k1, &k2);
#define SDP_ADMM_SIGN(T, tb)                                                                    \
  if (a.hsde)                                                                                   \
    hipLaunchKernelGGL((k_admm_sign<T, tb, false, true>), dim3(count), dim3(64), 0, st, a, list, \
                       k1, k2);                                                                 \
  else if (a.dual)                                                                              \
    hipLaunchKernelGGL((k_admm_sign<T, tb, true>), dim3(count), dim3(64), 0, st, a, list, k1,    \
                       k2);                                                                     \
  else                                                                                          \
    hipLaunchKernelGGL((k_admm_sign<T, tb, false>), dim3(count), dim3(64), 0, st, a, list, k1,   \
                       k2);
      if (precision == 1) {
        if (N == 16) {
          SDP_ADMM_SIGN(float, 1)
        } else {
          SDP_ADMM_SIGN(float, 2)
        }
      } else {
        if (N == 16) {
          SDP_ADMM_SIGN(double, 1)
        } else {
          SDP_ADMM_SIGN(double, 2)
        }
      }
#undef SDP_ADMM_SIGN
      return hipGetLastError();
    }
    // FP64 cliques of 33-128: one block in LDS, the other operand in
    // registers (cliques of 97-128 have no variant with eigenvectors: the
    // plan refuses the unrolled iterations for them)
    if (precision == 0 && N >= 48 && NT == 4 * N && !a.eig) {
      if (count <= 0) return hipSuccess;
      int k1, k2;
      sign_schedule(a.tol, N, &k1, &k2);
      if (split_ws && split_workspace(precision, variant, count) > 0) {
        const int mode = a.hsde ? 3 : a.dual ? 2 : 1;
#define SDP_SPLIT(n)                                                                           \
  if (N == n) {                                                                                \
    if (mode == 3) return launch_split<n, 3>(a, list, count, split_ws, k1, k2, st);            \
    if (mode == 2) return launch_split<n, 2>(a, list, count, split_ws, k1, k2, st);            \
    return launch_split<n, 1>(a, list, count, split_ws, k1, k2, st);                           \
  }
        SDP_SPLIT(96)
        SDP_SPLIT(128)
#undef SDP_SPLIT
        return hipErrorInvalidValue;
      }
#define SDP_ADMM_BIG(n)                                                                        \
  if (N == n) {                                                                                \
    if (a.hsde)                                                                                \
      hipLaunchKernelGGL((k_sign_big<double, n, 3>), dim3(count), dim3(4 * n), 0, st, a, list,  \
                         nullptr, nullptr, nullptr, nullptr, k1, k2);                          \
    else if (a.dual)                                                                           \
      hipLaunchKernelGGL((k_sign_big<double, n, 2>), dim3(count), dim3(4 * n), 0, st, a, list,  \
                         nullptr, nullptr, nullptr, nullptr, k1, k2);                          \
    else                                                                                       \
      hipLaunchKernelGGL((k_sign_big<double, n, 1>), dim3(count), dim3(4 * n), 0, st, a, list,  \
                         nullptr, nullptr, nullptr, nullptr, k1, k2);                          \
    return hipGetLastError();                                                                  \
  }
      SDP_ADMM_BIG(48)
      SDP_ADMM_BIG(64)
      SDP_ADMM_BIG(80)
      SDP_ADMM_BIG(96)
      SDP_ADMM_BIG(128)
#undef SDP_ADMM_BIG
      return hipErrorInvalidValue;
    }
    if (precision == 0 && N == 128) return hipErrorInvalidValue;   // needs eigenvectors
    variant = projection_default_variant(precision, N);
    projection_variant_info(precision, variant, &N, &NT);
  }
  const int blk = projection_variant_two_level(precision, variant);
  if (a.decouple && a.vw && !a.eig) {
    if (precision == 1)
      return dispatch<float, MODE_ADMM_DEC>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr,
                                            nullptr, nullptr, a.max_sweeps, a.tol, st);
    return dispatch<double, MODE_ADMM_DEC>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr,
                                           nullptr, nullptr, a.max_sweeps, a.tol, st);
  }
  if (precision == 1)
    return dispatch<float, MODE_ADMM>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                      nullptr, a.max_sweeps, a.tol, st);
  return dispatch<double, MODE_ADMM>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, a.max_sweeps, a.tol, st);
}

hipError_t launch_standalone_projection(int dtype, int variant, int count, const int32_t *sizes,
                                        const int64_t *offsets, const void *in, void *out,
                                        int max_sweeps, double tol, hipStream_t st) {
  ProjArgs a{};
  int N, NT;
  projection_variant_info(dtype, variant, &N, &NT);
  if (projection_variant_kind(dtype, variant) == 2) {
    if (count <= 0) return hipSuccess;
    int k1, k2;
    sign_schedule(tol, N, &k1, &k2);
    return dispatch_sign(dtype, N, NT, count, sizes, offsets, in, out, k1, k2, st);
  }
  const int blk = projection_variant_two_level(dtype, variant);
  if (dtype == 1)
    return dispatch<float, MODE_STANDALONE>(N, NT, blk, count, a, nullptr, sizes, offsets,
                                            (const float *)in, (float *)out, nullptr, max_sweeps,
                                            tol, st);
  return dispatch<double, MODE_STANDALONE>(N, NT, blk, count, a, nullptr, sizes, offsets,
                                           (const double *)in, (double *)out, nullptr,
                                           max_sweeps, tol, st);
}

hipError_t launch_min_eig(int precision, int variant, const int32_t *list, int count,
                          const ProjArgs &a, double *lmin_out, hipStream_t st) {
  int N, NT;
  projection_variant_info(precision, variant, &N, &NT);
  if (projection_variant_kind(precision, variant) == 2) {   // eigenvalues: Jacobi
    if (precision == 0 && N == 128)
      // eigenvalues only: the scalar Jacobi of FP64 blocks of 128 needs one
      // block in LDS (no eigenvectors), which fits
      return launch_one<double, 128, 1024, MODE_MINEIG, false>(
          count, a, list, nullptr, nullptr, nullptr, nullptr, lmin_out, a.max_sweeps, a.tol, st);
    variant = projection_default_variant(precision, N);
    projection_variant_info(precision, variant, &N, &NT);
  }
  const int blk = projection_variant_two_level(precision, variant);
  if (precision == 1)
    return dispatch<float, MODE_MINEIG>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                        lmin_out, a.max_sweeps, a.tol, st);
  return dispatch<double, MODE_MINEIG>(N, NT, blk, count, a, list, nullptr, nullptr, nullptr, nullptr,
                                       lmin_out, a.max_sweeps, a.tol, st);
}
