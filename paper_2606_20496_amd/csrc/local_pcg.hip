// Inexact local solves: in place of the stored inverse A_p^{-1} of the additive
// preconditioner's local term (Sec. 3, eq. (asm)), each subdomain's r_p is solved
// approximately by k steps of conjugate gradients preconditioned by the diagonal
// of A_p, from a zero initial guess (the iterative inexact local solver the paper
// proposes for GPUs in its conclusions, Sec. 6.3). The corrections are summed
// over the overlap exactly as the dense ones are. Because the CG coefficients are
// formed from r_p, the preconditioner is a nonlinear function of r and the outer
// iteration must be the flexible (Polak-Ribiere) one.
//
// A_p = R_p A R_p^T is stored per subdomain in ELL form: the diagonal (FP64) and
// W off-diagonal entries per row (local column as uint16, value FP64 or FP32),
// entry (k, i) of a system at ell_off + k * npad + i, so that lane i of a
// workgroup reads its row with coalesced loads. The columns are packed two per
// 32-bit word. One workgroup solves one subdomain with one thread per row: the
// row is loaded into registers once and reused by all k steps; the search
// direction lives in LDS, where the row products gather it. Every sum has a
// fixed order, so results are bitwise reproducible. FP64 contexts run the local
// CG in FP64; the mixed forms run it in FP32.
#pragma once

#include "kernels.h"

namespace coarse {

constexpr int LOC_WMAX = 26;       // off-diagonal entries per row of A_p at most
constexpr int LOC_NT_MAX = 1024;   // rows of a subdomain at most (one thread each)

// Position of internal vertex u in the sorted list R[0..n), or -1.
__device__ __forceinline__ int loc_find(const int32_t *R, int n, int32_t u) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t x = R[mid];
    if (x == u) return mid;
    if (x < u)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// ---------------------------------------------------------------------------
// Setup, pass 1: the number of distinct off-diagonal columns of each row of A_p
// (the free vertices of R_p that share an element with the row's vertex; every
// element holding a vertex of R_p lies in the overlapping subdomain), maximised
// over all rows into *wmax. A row with more than LOC_WMAX reports LOC_WMAX + 1.
// Both setup passes search the sorted R_p in LDS (LOC_NT_MAX entries at most).
// ---------------------------------------------------------------------------
__device__ __forceinline__ const int32_t *loc_stage_R(const LocSys &S, const int32_t *__restrict__ sub_idx,
                                                      int32_t *lr) {
  for (int a = threadIdx.x; a < S.n; a += blockDim.x) lr[a] = sub_idx[S.vec_off + a];
  __syncthreads();
  return lr;
}

__global__ __launch_bounds__(512) void k_loc_count(const LocSys *__restrict__ sys, const int32_t *__restrict__ sub_idx,
                                                   const int32_t *__restrict__ vinc_ptr,
                                                   const int32_t *__restrict__ vinc, const int32_t *__restrict__ e2v,
                                                   int64_t E, int64_t nf, int *__restrict__ wmax) {
  __shared__ int32_t lr[LOC_NT_MAX];
  const LocSys S = sys[blockIdx.x];
  const int32_t *R = loc_stage_R(S, sub_idx, lr);
  for (int a = threadIdx.x; a < S.n; a += blockDim.x) {
    // the distinct columns so far, newest first (compile-time indices only, so
    // the list stays in registers); unused slots hold -1
    int32_t seen[LOC_WMAX];
#pragma unroll
    for (int j = 0; j < LOC_WMAX; ++j) seen[j] = -1;
    int cnt = 0;
    const int32_t v = R[a];
    for (int k = vinc_ptr[v]; k < vinc_ptr[v + 1] && cnt <= LOC_WMAX; ++k) {
      const int64_t e = vinc[k] >> 3;
      for (int lb = 0; lb < 8; ++lb) {
        const int32_t u = e2v[lb * E + e];
        if (u >= nf || u == v) continue;
        const int pos = loc_find(R, S.n, u);
        if (pos < 0) continue;
        bool dup = false;
#pragma unroll
        for (int j = 0; j < LOC_WMAX; ++j) dup |= (seen[j] == pos);
        if (dup) continue;
        if (cnt == LOC_WMAX) {
          cnt = LOC_WMAX + 1;
          break;
        }
#pragma unroll
        for (int j = LOC_WMAX - 1; j > 0; --j) seen[j] = seen[j - 1];
        seen[0] = pos;
        ++cnt;
      }
    }
    atomicMax(wmax, cnt);
  }
}

// ---------------------------------------------------------------------------
// Setup, pass 2: the ELL rows. Row a sums, over the elements incident to vertex
// R_p[a] in their stored order, the element-matrix row of that vertex restricted
// to the columns in R_p (the same entries the dense assembly adds); columns are
// kept in increasing order, unused slots hold column a with value 0. *bad counts
// rows whose diagonal is not positive. The row under construction is a sorted
// register list (INT32_MAX in unused slots) updated with compile-time indices
// only: a column already present takes the value, a new one is inserted by one
// downward pass that moves the larger columns up a slot.
// ---------------------------------------------------------------------------
template <typename V>
__global__ __launch_bounds__(512) void k_loc_fill(const LocSys *__restrict__ sys, int W,
                                                  const int32_t *__restrict__ sub_idx,
                                                  const int32_t *__restrict__ vinc_ptr,
                                                  const int32_t *__restrict__ vinc, const int32_t *__restrict__ e2v,
                                                  int64_t E, int64_t nf, const double *__restrict__ Ae,
                                                  double *__restrict__ diag, uint32_t *__restrict__ col,
                                                  V *__restrict__ val, int *__restrict__ bad) {
  __shared__ int32_t lr[LOC_NT_MAX];
  const LocSys S = sys[blockIdx.x];
  const int32_t *R = loc_stage_R(S, sub_idx, lr);
  for (int a = threadIdx.x; a < S.n; a += blockDim.x) {
    int32_t cs[LOC_WMAX];
    double vs[LOC_WMAX];
#pragma unroll
    for (int j = 0; j < LOC_WMAX; ++j) {
      cs[j] = INT32_MAX;
      vs[j] = 0.0;
    }
    int cnt = 0;
    double d = 0.0;
    const int32_t v = R[a];
    for (int k = vinc_ptr[v]; k < vinc_ptr[v + 1]; ++k) {
      const int64_t e = vinc[k] >> 3;
      const int la = vinc[k] & 7;
      for (int lb = 0; lb < 8; ++lb) {
        const int32_t u = e2v[lb * E + e];
        if (u >= nf) continue;
        const double x = Ae[ae_at(sym8(la, lb), e)];
        if (u == v) {
          d += x;
          continue;
        }
        const int pos = loc_find(R, S.n, u);
        if (pos < 0) continue;
        bool found = false;
#pragma unroll
        for (int j = 0; j < LOC_WMAX; ++j)
          if (cs[j] == pos) {
            vs[j] += x;
            found = true;
          }
        if (found) continue;
        if (cnt == W) continue;   // cannot happen: W is the maximum count of pass 1
#pragma unroll
        for (int j = LOC_WMAX - 1; j >= 0; --j) {
          const int32_t below = j > 0 ? cs[j - 1] : INT32_MIN;
          const double vbelow = j > 0 ? vs[j - 1] : 0.0;
          if (below > pos) {
            cs[j] = below;
            vs[j] = vbelow;
          } else if (cs[j] > pos) {
            cs[j] = pos;
            vs[j] = x;
          }
        }
        ++cnt;
      }
    }
    if (!(d > 0.0)) atomicAdd(bad, 1);
    diag[S.vec_off + a] = d;
    // (a guard, not a break: leaving the unrolled loop early would put the row
    // lists in scratch memory)
#pragma unroll
    for (int k = 0; k < LOC_WMAX; k += 2)
      if (k < W) {
        const uint32_t c0 = (uint32_t)(k < cnt ? cs[k] : a);
        const uint32_t c1 = (uint32_t)(k + 1 < cnt ? cs[k + 1] : a);
        col[S.ell_off / 2 + (int64_t)(k / 2) * S.npad + a] = c0 | (c1 << 16);
        val[S.ell_off + (int64_t)k * S.npad + a] = (V)(k < cnt ? vs[k] : 0.0);
        val[S.ell_off + (int64_t)(k + 1) * S.npad + a] = (V)(k + 1 < cnt ? vs[k + 1] : 0.0);
      }
  }
}

// Sum over the 64 lanes of a wavefront with DPP lane moves (no LDS traffic),
// in a fixed order: pairs, quads, half rows, rows, then the rows into lane 63,
// whose value every lane receives.
template <int CTRL, int ROWS>
__device__ __forceinline__ double loc_dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ float loc_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}

__device__ __forceinline__ double loc_lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ float loc_lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

template <typename C>
__device__ __forceinline__ C loc_wave_sum(C v) {
  v += loc_dpp<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += loc_dpp<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += loc_dpp<0x141, 0xF>(v);   // row_half_mirror
  v += loc_dpp<0x140, 0xF>(v);   // row_mirror
  v += loc_dpp<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += loc_dpp<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return loc_lane63(v);
}

// Sum over the workgroup, returned to every thread: per-wave sums, then each
// thread adds the wave sums in wave order. `red` must not be reused before the
// next barrier of every thread has passed.
template <typename C>
__device__ __forceinline__ C loc_block_sum(C v, C *red, int nw) {
  v = loc_wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  C s = C(0);
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// The local solves of one preconditioner application: workgroup s runs `iters`
// steps of Jacobi-preconditioned CG on A_p z_p = r_p of local system s,
//   x = 0, r = r_p, z = D^{-1} r;  step j: beta = (r,z)_j / (r,z)_{j-1} (0 for
//   j = 0), p = z + beta p, q = A_p p, alpha = (r,z)_j / (p,q), x += alpha p,
//   r -= alpha q, z = D^{-1} r (but for the last step),
// stopping early when (r, z) is exactly 0 (a zero right-hand side), and writes x
// to the packed solution zp. q = A_p p is formed as A_p z + beta q (the same
// product, split by linearity), so that the new z, not p, is what the threads
// exchange through LDS: its write goes before the barrier of the (r, z) sum,
// which then also publishes it, and a step needs two barriers instead of three.
// blockDim.x >= the largest n (a multiple of 64).
// T: the type of the packed right-hand sides. V: the stored entries of A_p and
// the arithmetic of the local CG: double in FP64 contexts; float in the mixed
// forms, whose local solves are approximations under a flexible outer iteration
// anyway (half the registers and LDS bytes, so more subdomains share a compute
// unit).
// ---------------------------------------------------------------------------
template <typename V, typename T>
__device__ __forceinline__ void local_pcg_body(const LocSys &S, int W, int iters, const T *__restrict__ rp,
                                               const double *__restrict__ diag, const uint32_t *__restrict__ col,
                                               const V *__restrict__ val, double *__restrict__ zp, V *sz,
                                               V (*red)[LOC_NT_MAX / WAVE]) {
  const int i = threadIdx.x;
  const int nw = blockDim.x / WAVE;
  const bool act = i < S.n;
  V a[LOC_WMAX];
  uint32_t c[LOC_WMAX / 2];
  V d = V(1), r = V(0);
  if (act) {
    r = (V)rp[S.vec_off + i];
    d = (V)diag[S.vec_off + i];
#pragma unroll
    for (int k = 0; k < LOC_WMAX; k += 2)
      if (k < W) {
        c[k / 2] = col[S.ell_off / 2 + (int64_t)(k / 2) * S.npad + i];
        a[k] = val[S.ell_off + (int64_t)k * S.npad + i];
        a[k + 1] = val[S.ell_off + (int64_t)(k + 1) * S.npad + i];
      }
  }
  const V dinv = V(1) / d;
  V x = V(0), p = V(0), q = V(0);
  V z = dinv * r;
  sz[i] = z;
  V rz = loc_block_sum(r * z, red[0], nw);
  V rz_old = V(1);
  for (int it = 0; it < iters; ++it) {
    if (rz == V(0)) break;
    V s = V(0);
    if (act) {
      s = d * z;
#pragma unroll
      for (int k = 0; k < LOC_WMAX; k += 2)
        if (k < W) {
          s += a[k] * sz[c[k / 2] & 0xFFFF];
          s += a[k + 1] * sz[c[k / 2] >> 16];
        }
    }
    const V beta = it == 0 ? V(0) : rz / rz_old;
    p = z + beta * p;
    q = s + beta * q;
    const V pq = loc_block_sum(p * q, red[1], nw);
    const V alpha = rz / pq;
    x += alpha * p;
    r -= alpha * q;
    if (it == iters - 1) break;
    z = dinv * r;
    sz[i] = z;
    rz_old = rz;
    rz = loc_block_sum(r * z, red[0], nw);
  }
  if (act) zp[S.vec_off + i] = (double)x;
}

template <typename V, typename T>
__global__ __launch_bounds__(LOC_NT_MAX) void k_local_pcg(const LocSys *__restrict__ sys, int W, int iters,
                                                          const int *__restrict__ done, const T *__restrict__ rp,
                                                          const double *__restrict__ diag,
                                                          const uint32_t *__restrict__ col,
                                                          const V *__restrict__ val, double *__restrict__ zp) {
  if (*done) return;
  __shared__ V sz[LOC_NT_MAX];
  __shared__ V red[2][LOC_NT_MAX / WAVE];
  local_pcg_body<V, T>(sys[blockIdx.x], W, iters, rp, diag, col, val, zp, sz, red);
}

// The same for every solve of a lock-step batch that uses inexact local solves:
// workgroup g works for the solve whose range of `off` holds g (its local system
// g - off[c]). blockDim.x >= the largest n of every such solve.
template <typename V, typename T>
__global__ __launch_bounds__(LOC_NT_MAX) void k_local_pcg_grp(const IterDev *__restrict__ ctx,
                                                              const int32_t *__restrict__ off, int n) {
  __shared__ V sz[LOC_NT_MAX];
  __shared__ V red[2][LOC_NT_MAX / WAVE];
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  if (d.sc->done) return;
  local_pcg_body<V, T>(d.loc_sys[blockIdx.x - off[c]], d.loc_w, d.loc_iters, (const T *)d.rp, d.loc_diag, d.loc_col,
                       (const V *)d.loc_val, (double *)d.zp, sz, red);
}

}  // namespace coarse
