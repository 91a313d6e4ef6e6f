// Device-side helpers shared by the HIP kernels of the coarse solver (gfx950,
// wave64). Reductions are written with a fixed order so that every result is
// bitwise reproducible and independent of what else runs on the device.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace coarse {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, WAVE);
  return v;
}

// Sum over a workgroup of NT threads (NT a multiple of 64, <= 1024). Result is
// valid in thread 0. `red` is LDS scratch of at least NT/64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / WAVE; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// Trilinear weight of box corner k = kx + 2ky + 4kz at local coordinates xi.
template <typename T>
__device__ __forceinline__ T trilin(int k, T x, T y, T z) {
  T fx = (k & 1) ? x : T(1) - x;
  T fy = (k & 2) ? y : T(1) - y;
  T fz = (k & 4) ? z : T(1) - z;
  return fx * fy * fz;
}

// Index of entry (a, b), a < b, among the 28 strictly upper entries of an 8x8
// matrix stored row by row.
__host__ __device__ constexpr int off8(int a, int b) { return a * 7 - (a * (a - 1)) / 2 + (b - a - 1); }

// Index of entry (a, b), a <= b, in the 36-entry upper triangle of an 8x8
// symmetric element matrix stored row by row.
__host__ __device__ constexpr int sym8(int a, int b) {
  return a <= b ? (a * 8 - (a * (a - 1)) / 2 + (b - a)) : (b * 8 - (b * (b - 1)) / 2 + (a - b));
}

}  // namespace coarse
