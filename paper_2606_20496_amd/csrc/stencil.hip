// The reduced operator A_r as a 27-point stencil on the structured box grid
// (Sec. 4, eq. (Aij)): with the centroid interpolation, A_r is the sum over the
// occupied cells of 8 x 8 cell matrices on the cell corners, so an active box
// vertex couples only with box vertices at most one step away per direction.
// The stencil holds, for each active vertex, the 27 coefficients of those
// neighbours (zero where a neighbour is inactive or shares no occupied cell),
// coefficient s = (dx+1) + 3(dy+1) + 9(dz+1) of vertex a at s * n_r + a.
//
// Uses: a sweep w = A_r y over the box grid (neighbours found from the grid
// strides, no index lists), and one step of iterative refinement of the
// reduced solve in the mixed forms: y += A_r^{-1} (r_r - A_r y), with the
// residual formed in FP64 by the sweep and the correction by the same stored
// (FP32 or FP16-stored) inverse.
#pragma once

#include "kernels.h"

namespace coarse {

// Grid of box vertices: (b+1) points per direction, vertex (i, j, k) at
// i + d0 * (j + d1 * k).
struct BoxGrid {
  int32_t d0, d1, d2, pad;
};

// Setup: the stencil from the cell matrices. Active vertex K sums, over its
// (occupied cell, corner) pairs in their stored order, the cell matrix row of
// that corner into the slots of the cell's active corners.
__global__ __launch_bounds__(256) void k_ar_stencil_build(int64_t nr, const int32_t *__restrict__ ar_ptr,
                                                          const int32_t *__restrict__ ar_src,
                                                          const int32_t *__restrict__ corner_act,
                                                          const int32_t *__restrict__ occ_cells,
                                                          const int32_t *__restrict__ act_bv, BoxGrid g, int b0,
                                                          int b1, const double *__restrict__ cellmat,
                                                          double *__restrict__ coef) {
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  const int32_t v = act_bv[K];
  const int vi = v % g.d0, vj = (v / g.d0) % g.d1, vk = v / (g.d0 * g.d1);
  for (int k = ar_ptr[K]; k < ar_ptr[K + 1]; ++k) {
    const int o = ar_src[k] >> 3, q = ar_src[k] & 7;
    const int c = occ_cells[o];
    const int ci = c % b0, cj = (c / b0) % b1, ck = c / (b0 * b1);
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      if (corner_act[8 * o + l] < 0) continue;
      const int dx = ci + (l & 1) - vi, dy = cj + ((l >> 1) & 1) - vj, dz = ck + (l >> 2) - vk;
      const int s = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
      coef[(int64_t)s * nr + K] += cellmat[(int64_t)o * 64 + q * 8 + l];
    }
  }
}

// (A_r y) at active vertex K, y given on the full box grid. Neighbours with a
// zero coefficient (inactive ones among them) do not contribute, so y may hold
// anything (NaN included) at inactive vertices.
__device__ __forceinline__ double ar_row(int64_t nr, int64_t K, const int32_t *__restrict__ act_bv,
                                         const double *__restrict__ coef, BoxGrid g,
                                         const double *__restrict__ y) {
  const int32_t v = act_bv[K];
  const int vi = v % g.d0, vj = (v / g.d0) % g.d1, vk = v / (g.d0 * g.d1);
  // all 27 coefficient and neighbour loads go out together (outside the grid
  // the address is the vertex itself, and the value is not used)
  double c[27], yv[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) c[t] = coef[(int64_t)t * nr + K];
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    const int i = vi + t % 3 - 1, j = vj + (t / 3) % 3 - 1, k = vk + t / 9 - 1;
    const bool in = i >= 0 && i < g.d0 && j >= 0 && j < g.d1 && k >= 0 && k < g.d2;
    yv[t] = y[in ? i + g.d0 * (j + g.d1 * k) : v];
  }
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 27; ++t)
    if (c[t] != 0.0) s += c[t] * yv[t];
  return s;
}

// w = A_r y on the box grid (w written at active vertices only).
__global__ __launch_bounds__(256) void k_ar_apply(int64_t nr, const int32_t *__restrict__ act_bv,
                                                  const double *__restrict__ coef, BoxGrid g,
                                                  const double *__restrict__ y, double *__restrict__ w) {
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  w[act_bv[K]] = ar_row(nr, K, act_bv, coef, g, y);
}

// Refinement, first half: res = r_r - A_r y (y the reduced solution on the box
// grid, r_r the reduced right-hand side), stored as the right-hand side of the
// correction solve.
template <typename T>
__global__ __launch_bounds__(256) void k_ar_resid(int64_t nr, const int *__restrict__ done,
                                                  const int32_t *__restrict__ act_bv,
                                                  const double *__restrict__ coef, BoxGrid g,
                                                  const double *__restrict__ y, const T *__restrict__ rr,
                                                  T *__restrict__ res) {
  if (*done) return;
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  res[K] = (T)((double)rr[K] - ar_row(nr, K, act_bv, coef, g, y));
}

// Refinement, second half: y += the correction (both on the box grid).
__global__ __launch_bounds__(256) void k_ar_add(int64_t nr, const int *__restrict__ done,
                                                const int32_t *__restrict__ act_bv, const double *__restrict__ dy,
                                                double *__restrict__ y) {
  if (*done) return;
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  const int32_t v = act_bv[K];
  y[v] += dy[v];
}

}  // namespace coarse
