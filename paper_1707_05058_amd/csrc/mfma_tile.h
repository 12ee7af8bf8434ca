// Dense products of small square blocks on the matrix cores (gfx950
// 16x16x4 MFMA, FP32 and FP64), shared by the projection and adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace {

// Dense N x N products on the matrix cores, C(i, j) = sum_k x(k, i) y(k, j),
// by 16 x 16 tiles, one wave per tile (tiles dealt round-robin to the waves),
// 16x16x4 MFMA steps over k.  Tiles run over stored column positions (the
// LDS blocks keep slot c at position (c & 1) N/2 + c/2), so each operand read
// x(k, q), y(k, q) takes row k at 16 consecutive positions q; store(qi, qj, c)
// gets the result for the slots at positions qi, qj after a barrier, so a
// product may overwrite its own inputs.  Lane layouts (verified on gfx950):
// operand a lane l holds A(l % 16, k0 + l / 16), operand b lane l holds
// B(k0 + l / 16, l % 16); result register r of lane l is C(i, l % 16) with
// i = 4 (l / 16) + r (FP32) or i = l / 16 + 4 r (FP64).  LOWER = true
// computes only the tiles on or below the diagonal (in position order).
template <typename T> struct Mma;
template <> struct Mma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <typename T, int N, int NT, bool LOWER, typename FX, typename FY, typename FS>
__device__ inline void tile_product(FX fx, FY fy, FS store) {
  constexpr int TN = N / 16;
  constexpr int NW = NT / 64;
  constexpr int TILES = LOWER ? TN * (TN + 1) / 2 : TN * TN;
  constexpr int TPW = (TILES + NW - 1) / NW;
  static_assert(N % 16 == 0 && NT % 64 == 0, "tiles of 16, whole waves");
  // the lane index passes through an empty asm statement, so the addresses
  // derived from it are computed in each product rather than hoisted out of
  // the caller's loops and kept live (spilled) across them
  int lt = threadIdx.x & 63;
  asm volatile("" : "+v"(lt));
  const int l = lt, w = threadIdx.x >> 6;
  typename Mma<T>::v4 acc[TPW];
  int ti[TPW], tj[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = w + t * NW;         // uniform over the wave
    int I = 0, J = 0;
    if (LOWER) {
      I = 0;
      while ((I + 1) * (I + 2) / 2 <= tile) ++I;
      J = tile - I * (I + 1) / 2;
    } else {
      I = tile / TN;
      J = tile % TN;
    }
    ti[t] = I;
    tj[t] = J;
    acc[t] = typename Mma<T>::v4{0, 0, 0, 0};
    if (tile < TILES) {
      const int qa = 16 * I + (l & 15), qb = 16 * J + (l & 15);
#pragma unroll 4
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int k = k0 + (l >> 4);
        acc[t] = Mma<T>::step(fx(k, qa), fy(k, qb), acc[t]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (w + t * NW < TILES) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        store(16 * ti[t] + Mma<T>::row(l, r), 16 * tj[t] + (l & 15), acc[t][r]);
    }
  }
}

// The same product with a depth known only at run time: k runs over
// [0, kend) (kend a multiple of 4; fx and fy return 0 past the true depth),
// and without LOWER only the first ceil(rows / 16) rows of tiles are formed.
template <typename T, int N, int NT, bool LOWER, typename FX, typename FY, typename FS>
__device__ inline void tile_product_part(int rows, int kend, FX fx, FY fy, FS store) {
  constexpr int TN = N / 16;
  constexpr int NW = NT / 64;
  constexpr int TILES = LOWER ? TN * (TN + 1) / 2 : TN * TN;
  constexpr int TPW = (TILES + NW - 1) / NW;
  int lt = threadIdx.x & 63;
  asm volatile("" : "+v"(lt));
  const int l = lt, w = threadIdx.x >> 6;
  const int tiles = LOWER ? TILES : ((rows + 15) / 16) * TN;
  typename Mma<T>::v4 acc[TPW];
  int ti[TPW], tj[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int tile = w + t * NW;
    int I = 0, J = 0;
    if (LOWER) {
      while ((I + 1) * (I + 2) / 2 <= tile) ++I;
      J = tile - I * (I + 1) / 2;
    } else {
      I = tile / TN;
      J = tile % TN;
    }
    ti[t] = I;
    tj[t] = J;
    acc[t] = typename Mma<T>::v4{0, 0, 0, 0};
    if (tile < tiles) {
      const int qa = 16 * I + (l & 15), qb = 16 * J + (l & 15);
      for (int k0 = 0; k0 < kend; k0 += 4) {
        const int k = k0 + (l >> 4);
        acc[t] = Mma<T>::step(fx(k, qa), fy(k, qb), acc[t]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (w + t * NW < tiles) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        store(16 * ti[t] + Mma<T>::row(l, r), 16 * tj[t] + (l & 15), acc[t][r]);
    }
  }
}

}  // namespace
