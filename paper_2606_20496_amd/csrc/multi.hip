// Kernels of the block solve: up to MC right-hand sides on one mesh, solved by
// MC independent PCG recurrences (Sec. 1, one per column) that share every read
// of the operator's element matrices and of the stored dense inverses. Vectors
// are vertex-major, MC doubles per vertex (one 128-byte line), so every gather
// through an index list reads whole lines. The dense solves A_s^{-1} [r_1 .. r_MC]
// of the additive preconditioner (Sec. 3, eq. (asm); Sec. 4) are small matrix
// products on the matrix cores: FP64 tiles on v_mfma_f64_16x16x4f64, FP32 and
// FP16-stored tiles (widened to FP32 in LDS, the power-of-two scale applied to
// the result) on v_mfma_f32_16x16x4f32. Vectors, dots and the operator are FP64
// in every form.
//
// Every sum over the vector runs over a fixed grid in a fixed order (per
// workgroup, then one workgroup over the partials), so each column's result is
// bitwise reproducible; columns never mix.
#pragma once

#include "kernels.h"

#include <type_traits>

namespace coarse {

constexpr int MC = 16;    // columns of the block
constexpr int MCW = 4;    // columns per operator pass (LDS holds MCW values per slot)

// Solver state of the block solve (device memory, one per context).
struct MScal {
  double rho[2][MC];   // (r, z) of the last two preconditioner applications
  double alpha[MC], beta[MC], pq[MC];
  double bb[MC], rr[MC], rr0[MC], res_true[MC];
  double tol2;
  int32_t done[MC], status[MC], iters[MC];
  int32_t iter;        // completed iterations
  int32_t all_done;    // every column has finished
  int32_t max_it, ncol;
};

// One dense system for the block GEMV.
struct MSys {
  const void *tiles;     // lower tiles of A_s^{-1} (or of A_s^{-1} / scale), TILE x TILE row-major each
  int64_t voff;          // first packed entry of the system
  int32_t nb, n;
  int32_t red;           // 1: the reduced system (solution also goes to the box grid)
  float scale;           // FP16 tiles hold A_s^{-1} / scale (1 otherwise)
};

// what a k_m_scal launch forms from the column totals of its partials
enum MScalStep : int { MS_BB = 0, MS_RZ = 1, MS_PQ = 2, MS_RR = 3, MS_RES = 4 };

// Per-column sums over a workgroup of NT threads in which thread t holds a value
// of column t % MC; returned in threads 0..MC-1 (fixed order: lanes c, c^16,
// c^32, c^48 of each wave, then the waves in order). red: NT/WAVE*MC doubles.
template <int NT>
__device__ __forceinline__ double block_colsum(double v, double *red) {
  v += __shfl_xor(v, 16, WAVE);
  v += __shfl_xor(v, 32, WAVE);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  if (l < MC) red[w * MC + l] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < MC) {
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) s += red[q * MC + threadIdx.x];
  }
  __syncthreads();
  return s;
}

// The per-vertex kernels of the iteration give each vertex 4 lanes, lane q
// holding columns 4q .. 4q + 3 (two 16-byte accesses per vector), so a
// workgroup keeps 64 vertices in flight. Per-column sums over the workgroup:
// lanes with the same q in a wave (xor 4, 8, 16, 32), then the waves in order;
// returned in threads 0..MC-1 (column = thread).
template <int NT>
__device__ __forceinline__ double block_colsum4(const double v[4], double *red) {
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double x = v[j];
    x += __shfl_xor(x, 4, WAVE);
    x += __shfl_xor(x, 8, WAVE);
    x += __shfl_xor(x, 16, WAVE);
    x += __shfl_xor(x, 32, WAVE);
    if (l < 4) red[w * MC + 4 * l + j] = x;
  }
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < MC) {
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) s += red[q * MC + threadIdx.x];
  }
  __syncthreads();
  return s;
}

__device__ __forceinline__ void ld4(const double *p, double v[4]) {
  const double2 a = *(const double2 *)p, b = *(const double2 *)(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}

__device__ __forceinline__ void st4(double *p, const double v[4]) {
  *(double2 *)p = make_double2(v[0], v[1]);
  *(double2 *)(p + 2) = make_double2(v[2], v[3]);
}

// caller vectors b[c][user] (c < k; zero columns beyond) into the block R in
// internal order, x = p = z = 0, a copy of b for the final residual, and the
// partials of ||b_c||^2; workgroup 0 resets the solver state
__global__ __launch_bounds__(256) void k_m_start(int64_t nf, int64_t nv, const int32_t *__restrict__ user_of,
                                                 const double *__restrict__ b, int k, double *__restrict__ R,
                                                 double *__restrict__ X, double *__restrict__ Pa,
                                                 double *__restrict__ Pb, double *__restrict__ Z,
                                                 double *__restrict__ B, double *__restrict__ part,
                                                 MScal *__restrict__ ms, double tol2, int max_it) {
  __shared__ double red[256 / WAVE * MC];
  const int c = threadIdx.x % MC;
  double acc = 0.0;
  const int64_t n = nf * MC, G = (int64_t)gridDim.x * 256;
  for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < n; g += G) {
    const int64_t i = g / MC;
    const double v = (c < k) ? b[(int64_t)c * nv + user_of[i]] : 0.0;
    R[g] = v;
    B[g] = v;
    X[g] = 0.0;
    Pa[g] = 0.0;
    Pb[g] = 0.0;
    Z[g] = 0.0;
    acc += v * v;
  }
  const double s = block_colsum<256>(acc, red);
  if (threadIdx.x < MC) {
    part[blockIdx.x * MC + threadIdx.x] = s;
    if (blockIdx.x == 0) {
      ms->rho[0][c] = ms->rho[1][c] = 0.0;
      ms->alpha[c] = ms->beta[c] = ms->pq[c] = 0.0;
      ms->bb[c] = ms->rr[c] = ms->rr0[c] = ms->res_true[c] = 0.0;
      ms->done[c] = 0;
      ms->status[c] = 0;
      ms->iters[c] = 0;
      if (c == 0) {
        ms->tol2 = tol2;
        ms->iter = 0;
        ms->all_done = 0;
        ms->max_it = max_it;
        ms->ncol = k;
      }
    }
  }
}

// One workgroup: the column totals of part[0..n)[MC] in a fixed order, then the
// scalar step of every column (see MScalStep):
//   MS_BB  ||b||^2; a zero (or beyond k) column is finished at once
//   MS_RZ  rho_k = (r_k, z_k), beta_k = rho_k / rho_{k-1} (0 for k = 0)
//   MS_PQ  alpha_k = rho_k / p_k.A p_k (breakdown when p.Ap <= 0)
//   MS_RR  ||r_{k+1}||^2 against tol^2 ||b||^2 and the iteration cap; k + 1 done
//   MS_RES ||b - A x||^2 of the result
// A finished column keeps alpha = beta = 0, so its x and r stay as they are.
// Column totals of part[0..n)[MC] in a fixed order (rows g, g + GS, ... per
// thread group, eight loads issued together, then the groups in order); returned
// in threads 0..MC-1.
__device__ __forceinline__ double m_coltotal(const double *__restrict__ part, int n, double *red) {
  const int c = threadIdx.x % MC, g = threadIdx.x / MC;
  constexpr int GS = 256 / MC;   // partial rows per step of one thread group
  double acc = 0.0;
  for (int i0 = g; i0 < n; i0 += 8 * GS) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (i0 + u * GS < n) ? part[(int64_t)(i0 + u * GS) * MC + c] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * GS < n) acc += v[u];
  }
  return block_colsum<256>(acc, red);
}

// part2 (MS_RZ only, may be null): the partials of (r_{k+1}, z_k), for the
// Polak-Ribiere beta (rho_{k+1} - (r_{k+1}, z_k)) / rho_k of a flexible context.
__global__ __launch_bounds__(256) void k_m_scal(MScal *__restrict__ ms, const double *__restrict__ part, int n,
                                                int step, const double *__restrict__ part2) {
  __shared__ double red[256 / WAVE * MC];
  __shared__ int live[MC];
  if (step != MS_BB && step != MS_RES && ms->all_done) return;
  const int c = threadIdx.x % MC;
  const double tot = m_coltotal(part, n, red);
  const double tot2 = (step == MS_RZ && part2) ? m_coltotal(part2, n, red) : 0.0;
  const int it = ms->iter;
  if (threadIdx.x < MC) {
    bool done = ms->done[c] != 0;
    int status = ms->status[c], iters = ms->iters[c];
    switch (step) {
      case MS_BB: {
        ms->bb[c] = tot;
        ms->rr[c] = tot;
        ms->rr0[c] = tot;
        if (c >= ms->ncol || !(tot > 0.0) || !isfinite(tot)) {
          done = true;
          status = isfinite(tot) ? 0 : -6;
          iters = 0;
        }
        break;
      }
      case MS_RZ: {
        double beta = 0.0;
        if (!done) {
          if (!isfinite(tot)) {
            done = true;
            status = -6;
            iters = it;
          } else if (it > 0) {
            beta = (tot - tot2) / ms->rho[(it - 1) & 1][c];
          }
        }
        ms->rho[it & 1][c] = tot;
        ms->beta[c] = done ? 0.0 : beta;
        break;
      }
      case MS_PQ: {
        double alpha = 0.0;
        ms->pq[c] = tot;
        if (!done) {
          if (!(tot > 0.0) || !isfinite(tot)) {
            done = true;
            status = -6;
            iters = it;
          } else {
            alpha = ms->rho[it & 1][c] / tot;
          }
        }
        ms->alpha[c] = alpha;
        break;
      }
      case MS_RR: {
        if (!done) {
          ms->rr[c] = tot;
          const int nit = it + 1;
          if (!isfinite(tot)) {
            done = true;
            status = -6;
            iters = nit;
          } else if (tot <= ms->tol2 * ms->bb[c]) {
            done = true;
            status = 0;
            iters = nit;
          } else if (nit >= ms->max_it) {
            done = true;
            status = 1;
            iters = nit;
          }
        }
        break;
      }
      default:
        ms->res_true[c] = tot;
        break;
    }
    if (done) {
      ms->alpha[c] = 0.0;
      ms->beta[c] = 0.0;
    }
    ms->done[c] = done ? 1 : 0;
    ms->status[c] = status;
    ms->iters[c] = iters;
    live[c] = done ? 0 : 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && step != MS_RES) {
    int any = 0;
    for (int k = 0; k < MC; ++k) any |= live[k];
    if (step == MS_RR) ms->iter = it + 1;
    ms->all_done = any ? 0 : 1;
  }
}

// ---------------------------------------------------------------------------
// Operator on the block: q_c = A p_c for every column, with the element data
// loaded once. The workgroup stages MCW columns of its slot values at a time in
// LDS; the element products, the corner-by-corner slot sums (or the incidence
// lists) and the writes to q / the shared-vertex partials follow k_op_pass1,
// column by column, so every column sums in the same order as a single-vector
// application. fused = 1: the PCG form, p_k = z_k + beta_c p_{k-1} formed while
// staging (written once per vertex by its designated block) and the partials of
// p_c.A p_c; fused = 0: q = A p for p given in z.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(OP_BLOCK) void k_m_op(OpDev op, const double *__restrict__ z, double *__restrict__ pa,
                                                   double *__restrict__ pb, double *__restrict__ q,
                                                   double *__restrict__ partials, double *__restrict__ energy,
                                                   const MScal *__restrict__ ms, int fused) {
  extern __shared__ double lds[];
  __shared__ double red[OP_BLOCK / WAVE * MCW];
  if (fused && ms->all_done) return;
  double *out = lds;                  // [OP_BLOCK * 8], one column at a time
  double *lp = lds + OP_BLOCK * 8;    // [MCW][slots]: one column's slots contiguous (a slot-major
                                      // layout put lanes of one column 32 bytes apart: 8-way bank conflicts)
  const int blk = blockIdx.x;
  const int64_t e = (int64_t)blk * OP_BLOCK + threadIdx.x;
  const bool valid = e < op.E;
  double m[28];
  uint4 cn = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  if (valid) elem_load(op, e, m, cn);
  const int s0 = op.blk_slot_ptr[blk], ns = op.blk_slot_ptr[blk + 1] - s0;
  const int it = fused ? ms->iter : 0;
  double *pcur = (it & 1) ? pb : pa;
  const double *pprev = (it & 1) ? pa : pb;
  const bool inc = op.blk_inc[blk] != 0;
  for (int ch = 0; ch < MC / MCW; ++ch) {
    const int c0 = ch * MCW;
    double beta[MCW];
#pragma unroll
    for (int cc = 0; cc < MCW; ++cc) beta[cc] = fused ? ms->beta[c0 + cc] : 0.0;
    for (int s = threadIdx.x; s < ns; s += OP_BLOCK) {
      const int64_t v = op.slot_vid[s0 + s];
      const double2 z0 = *(const double2 *)(z + v * MC + c0);
      const double2 z1 = *(const double2 *)(z + v * MC + c0 + 2);
      double pv[MCW] = {z0.x, z0.y, z1.x, z1.y};
      if (fused) {
        const double2 q0 = *(const double2 *)(pprev + v * MC + c0);
        const double2 q1 = *(const double2 *)(pprev + v * MC + c0 + 2);
        pv[0] += beta[0] * q0.x;
        pv[1] += beta[1] * q0.y;
        pv[2] += beta[2] * q1.x;
        pv[3] += beta[3] * q1.y;
        if (op.slot_pw[s0 + s]) {
          *(double2 *)(pcur + v * MC + c0) = make_double2(pv[0], pv[1]);
          *(double2 *)(pcur + v * MC + c0 + 2) = make_double2(pv[2], pv[3]);
        }
      }
#pragma unroll
      for (int cc = 0; cc < MCW; ++cc) lp[cc * ns + s] = pv[cc];
    }
    __syncthreads();
    double y[MCW][8], en[MCW];
#pragma unroll
    for (int cc = 0; cc < MCW; ++cc) {
      en[cc] = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) y[cc][a] = 0.0;
    }
    if (valid) {
#pragma unroll
      for (int cc = 0; cc < MCW; ++cc) {
        double pe[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const unsigned sl = slot_at(cn, a);
          pe[a] = (sl == 0xFFFFu) ? 0.0 : lp[cc * ns + sl];
        }
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
          for (int b2 = a + 1; b2 < 8; ++b2) {
            const double t = m[off8(a, b2)] * (pe[b2] - pe[a]);
            y[cc][a] += t;
            y[cc][b2] -= t;
          }
#pragma unroll
        for (int a = 0; a < 8; ++a) en[cc] += pe[a] * y[cc][a];
      }
    }
    __syncthreads();
    if (inc) {
      // per slot, the element outputs of its incidences in list order
#pragma unroll
      for (int cc = 0; cc < MCW; ++cc) {
        if (valid) {
#pragma unroll
          for (int a = 0; a < 8; ++a) out[threadIdx.x * 8 + a] = y[cc][a];
        }
        __syncthreads();
        for (int s = threadIdx.x; s < ns; s += OP_BLOCK) {
          const uint4 rec = *(const uint4 *)(op.slot_inc8 + (int64_t)(s0 + s) * 8);
          const int dst = op.slot_dst[s0 + s];
          double acc = 0.0;
          if (slot_at(rec, 0) == 0xFFFEu) {
            for (int k = op.slot_inc_ptr[s0 + s]; k < op.slot_inc_ptr[s0 + s + 1]; ++k) acc += out[op.slot_inc[k]];
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const unsigned li = slot_at(rec, k);
              if (li != 0xFFFFu) acc += out[li];
            }
          }
          if (dst >= 0)
            q[(int64_t)dst * MC + c0 + cc] = acc;
          else
            partials[(int64_t)(-dst - 1) * MC + c0 + cc] = acc;
        }
        __syncthreads();
      }
    } else {
      for (int s = threadIdx.x; s < ns * MCW; s += OP_BLOCK) lp[s] = 0.0;
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        if (valid) {
          const unsigned sl = slot_at(cn, a);
          if (sl != 0xFFFFu) {
#pragma unroll
            for (int cc = 0; cc < MCW; ++cc) lp[cc * ns + sl] += y[cc][a];
          }
        }
        __syncthreads();
      }
      for (int s = threadIdx.x; s < ns; s += OP_BLOCK) {
        const int dst = op.slot_dst[s0 + s];
        double *d = (dst >= 0) ? q + (int64_t)dst * MC + c0 : partials + (int64_t)(-dst - 1) * MC + c0;
        *(double2 *)d = make_double2(lp[s], lp[ns + s]);
        *(double2 *)(d + 2) = make_double2(lp[2 * ns + s], lp[3 * ns + s]);
      }
      __syncthreads();
    }
    if (fused) {
      // the MCW column sums of p.Ap over the workgroup together: each wave's sums,
      // then the waves in order (one barrier pair for all columns)
      const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
#pragma unroll
      for (int cc = 0; cc < MCW; ++cc) {
        const double t = wave_sum(en[cc]);
        if (l == 0) red[w * MCW + cc] = t;
      }
      __syncthreads();
      if (threadIdx.x < MCW) {
        double tot = 0.0;
#pragma unroll
        for (int q = 0; q < OP_BLOCK / WAVE; ++q) tot += red[q * MCW + threadIdx.x];
        energy[blk * MC + c0 + threadIdx.x] = tot;
      }
      __syncthreads();
    }
  }
}

// q of the vertices shared between operator blocks, from their partials (the
// non-fused operator; the PCG update sums them itself)
__global__ __launch_bounds__(256) void k_m_op_pass2(OpDev op, const double *__restrict__ partials,
                                                    double *__restrict__ q) {
  const int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t i = g / MC;
  const int c = (int)(g % MC);
  if (i >= op.n_shared) return;
  double acc = 0.0;
  for (int k = op.sh_ptr[i]; k < op.sh_ptr[i + 1]; ++k) acc += partials[(int64_t)k * MC + c];
  q[(int64_t)op.sh_vid[i] * MC + c] = acc;
}

// alpha_c, x += alpha_c p, r -= alpha_c q (shared vertices summed from the
// operator's partials), partials of ||r_c||^2
__global__ __launch_bounds__(256) void k_m_update(int64_t nf, OpDev op, const double *__restrict__ partials,
                                                  const MScal *__restrict__ ms, double *__restrict__ X,
                                                  double *__restrict__ R, const double *__restrict__ pa,
                                                  const double *__restrict__ pb, const double *__restrict__ Q,
                                                  double *__restrict__ part) {
  __shared__ double red[256 / WAVE * MC];
  if (ms->all_done) return;
  const int cq = (threadIdx.x % 4) * 4;
  double alpha[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) alpha[j] = ms->alpha[cq + j];
  const double *P = (ms->iter & 1) ? pb : pa;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t n = nf * 4, G = (int64_t)gridDim.x * 256;
  for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < n; g += G) {
    const int64_t i = g / 4, o = i * MC + cq;
    const int2 vq = op.vq[i];
    double qi[4], x[4], r[4], p[4];
    ld4(X + o, x);
    ld4(R + o, r);
    ld4(P + o, p);
    if (vq.y == 0) {
      ld4(Q + o, qi);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) qi[j] = 0.0;
      for (int k = 0; k < vq.y; ++k) {
        double t[4];
        ld4(partials + (int64_t)(vq.x + k) * MC + cq, t);
#pragma unroll
        for (int j = 0; j < 4; ++j) qi[j] += t[j];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x[j] += alpha[j] * p[j];
      r[j] = r[j] - alpha[j] * qi[j];
      acc[j] += r[j] * r[j];
    }
    st4(X + o, x);
    st4(R + o, r);
  }
  const double s = block_colsum4<256>(acc, red);
  if (threadIdx.x < MC) part[blockIdx.x * MC + threadIdx.x] = s;
}

// Restriction of the block (Sec. 3 and Sec. 4): workgroups below ng gather
// r_p = R_p r for every column into the packed vectors (padding = 0); the others
// take one J^T task per wavefront, lanes (entry group g = l / MC, column l % MC),
// and write its 8 corner sums per column.
template <typename T>
__global__ __launch_bounds__(256) void k_m_pre(int ng, int64_t n_pack, const int32_t *__restrict__ idx,
                                               const double *__restrict__ R, double *__restrict__ RP, int ntask,
                                               const int32_t *__restrict__ tstart, const int32_t *__restrict__ vid,
                                               const T *__restrict__ w, const T *__restrict__ xi,
                                               int64_t nent, double *__restrict__ tpart,
                                               const MScal *__restrict__ ms) {
  if (ms->all_done) return;
  if ((int)blockIdx.x < ng) {
    // four entries per thread and step, their index and value loads issued together
    const int64_t n = n_pack * MC, G = (int64_t)ng * 256;
    for (int64_t g0 = blockIdx.x * (int64_t)256 + threadIdx.x; g0 < n; g0 += 4 * G) {
      int32_t ii[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ii[u] = (g0 + u * G < n) ? idx[(g0 + u * G) / MC] : -1;
      double vv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) vv[u] = (ii[u] >= 0) ? R[(int64_t)ii[u] * MC + (g0 + u * G) % MC] : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (g0 + u * G < n) RP[g0 + u * G] = vv[u];
    }
    return;
  }
  const int lane = threadIdx.x & 63, c = lane % MC, eg = lane / MC;
  const int nw = ((int)gridDim.x - ng) * 4;
  for (int task = ((int)blockIdx.x - ng) * 4 + (threadIdx.x >> 6); task < ntask; task += nw) {
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    const int j1 = tstart[task + 1];
    for (int j = tstart[task] + eg; j < j1; j += WAVE / MC) {
      const double v = (double)w[j] * R[(int64_t)vid[j] * MC + c];
      const double x = xi[j], y = xi[nent + j], zz = xi[2 * nent + j];
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += trilin<double>(k, x, y, zz) * v;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      acc[k] += __shfl_xor(acc[k], 16, WAVE);
      acc[k] += __shfl_xor(acc[k], 32, WAVE);
    }
    if (eg == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) tpart[((int64_t)task * 8 + k) * MC + c] = acc[k];
    }
  }
}

// Second stage of J^T: per active box vertex and column, the task sums of the
// occupied cells around it in list order.
__global__ __launch_bounds__(256) void k_m_corners(int64_t nr, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ src, const double *__restrict__ tpart,
                                                   double *__restrict__ rr, const MScal *__restrict__ ms) {
  if (ms->all_done) return;
  const int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t K = g / MC;
  const int c = (int)(g % MC);
  if (K >= nr) return;
  // the list in order, eight loads issued together
  double acc = 0.0;
  const int k1 = ptr[K + 1];
  for (int kb = ptr[K]; kb < k1; kb += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (kb + u < k1) ? tpart[(int64_t)src[kb + u] * MC + c] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (kb + u < k1) acc += v[u];
  }
  rr[K * MC + c] = acc;
}

// ---------------------------------------------------------------------------
// Dense solves of the block: Z_s = A_s^{-1} R_s for every system, one wavefront
// per tile row I of a system, on the matrix cores. Row I of the symmetric
// inverse is the stored lower tiles (I, J <= I) followed by the transposes of
// the stored tiles (J > I, I), so the wavefront owns its 32 x MC output rows
// whole: no partial sums leave it and no combine pass follows (each
// off-diagonal tile is read by two wavefronts of the same system, which run
// on one XCD, so the second read mostly hits its L2). v_mfma_f64_16x16x4f64
// takes A[16x4] (lane l holds A[l%16][l/16]) and B[4x16] (lane l holds
// B[l/16][l%16]) and accumulates D[16x16], lane l holding rows l/16 + 4r (r < 4)
// of column l%16. Output rows 0..15 and 16..31 of the tile row are two
// accumulators; the K = 32 sum of a tile takes 8 steps. A tile is read with
// 16-byte loads (one 128-byte line per four lanes), staged in the wavefront's own
// LDS region (row stride MLD doubles) and read back in the operand layout, row-
// or column-wise; the next tile's loads are in flight meanwhile.
// ---------------------------------------------------------------------------
constexpr int MLD = TILE + 2;

// loads through the global address space (not flat: a flat load also counts
// against the LDS wait below)
__device__ __forceinline__ double2 ldg2(const double2 *p) {
  const nt_d2 v = *(const __attribute__((address_space(1))) nt_d2 *)p;
  double2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}
__device__ __forceinline__ double ldg(const double *p) {
  return *(const __attribute__((address_space(1))) double *)p;
}

// LDS accesses of one wavefront in program order: the wavefront's own LDS
// operations complete (lgkmcnt 0; loads from global memory stay in flight) and
// the compiler moves no memory access across this point
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ void gemv_row_f64(const int2 *__restrict__ rows, int nrows,
                                             const MSys *__restrict__ sys, const double *__restrict__ RP,
                                             double *__restrict__ ZP, double *__restrict__ yfull,
                                             const int32_t *__restrict__ act_bv) {
  __shared__ __attribute__((aligned(16))) double stage[4][TILE * MLD];
  // consecutive rows (those of one system) go to workgroups of one XCD: the
  // grid is a multiple of 8 and workgroup b runs on XCD b % 8
  const int per = (int)gridDim.x / 8;
  const int wl = ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8;
  const int row = wl * 4 + (threadIdx.x >> 6);
  if (row >= nrows) return;   // no workgroup barrier below
  const int lane = threadIdx.x & 63, li = lane % 16, lk = lane / 16;
  const int2 sr = rows[row];
  const MSys S = sys[sr.x];
  const int I = sr.y, nb = S.nb;
  const double *__restrict__ Rs = RP + S.voff * MC;
  double *L = stage[threadIdx.x >> 6];
  const int wr = lane / 16, wc = 2 * (lane % 16);   // this lane's 16-byte pieces: rows wr + 4m, columns wc, wc + 1
  // step s visits tile column J = (s - I) mod nb: the two wavefronts that need
  // tile {I, J} (rows I and J of the system) reach it at the same step s = (I +
  // J) mod nb, so its second read comes from the L2
  auto tile_at = [&](int J) -> const double2 * {
    const int64_t toff = (J <= I) ? (int64_t)I * (I + 1) / 2 + J : (int64_t)J * (J + 1) / 2 + I;
    return (const double2 *)((const double *)S.tiles + toff * (TILE * TILE));
  };
  double2 tv[8];
  double bv[8];
  int J = (I == 0) ? 0 : nb - I;
  {
    const double2 *t = tile_at(J);
#pragma unroll
    for (int m = 0; m < 8; ++m) tv[m] = ldg2(t + m * 64 + lane);
#pragma unroll
    for (int st = 0; st < 8; ++st) bv[st] = ldg(Rs + (int64_t)(J * TILE + 4 * st + lk) * MC + li);
  }
  v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < nb; ++s) {
#pragma unroll
    for (int m = 0; m < 8; ++m) *(double2 *)(L + (wr + 4 * m) * MLD + wc) = tv[m];
    double bc[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) bc[st] = bv[st];
    const bool low = J <= I;
    // the next tile (the last step reloads its own, from the caches)
    const int J1 = (s + 1 < nb) ? ((J + 1 == nb) ? 0 : J + 1) : J;
    {
      const double2 *t = tile_at(J1);
#pragma unroll
      for (int m = 0; m < 8; ++m) tv[m] = ldg2(t + m * 64 + lane);
#pragma unroll
      for (int st = 0; st < 8; ++st) bv[st] = ldg(Rs + (int64_t)(J1 * TILE + 4 * st + lk) * MC + li);
    }
    wave_lds_sync();
    double a0[8], a1[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      // stored tile (I, J): A[i][k] = t[i][k]; stored tile (J, I): A[i][k] = t[k][i]
      const int k = 4 * st + lk;
      a0[st] = L[low ? li * MLD + k : k * MLD + li];
      a1[st] = L[low ? (16 + li) * MLD + k : k * MLD + 16 + li];
    }
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[st], bc[st], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[st], bc[st], acc1, 0, 0, 0);
    }
    wave_lds_sync();
    J = J1;
  }
  double *Zs = ZP + S.voff * MC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i0 = I * TILE + lk + 4 * r, i1 = i0 + 16;
    Zs[(int64_t)i0 * MC + li] = acc0[r];
    Zs[(int64_t)i1 * MC + li] = acc1[r];
    if (S.red) {
      if (i0 < S.n) yfull[(int64_t)act_bv[i0] * MC + li] = acc0[r];
      if (i1 < S.n) yfull[(int64_t)act_bv[i1] * MC + li] = acc1[r];
    }
  }
}

// FP32 and FP16-stored tiles: the same walk, with v_mfma_f32_16x16x4f32 (A and
// B as for the FP64 form; lane l holds rows 4(l/16) .. 4(l/16) + 3 of column l%16
// of the 16 x 16 accumulator) and FP32 arithmetic as in the single-vector mixed
// forms. A tile is loaded with 16-byte loads (four per lane for FP32, two for
// FP16), widened to FP32 and staged in the wavefront's LDS region (row stride
// MLDF floats).
constexpr int MLDF = TILE + 4;
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float nt_f4g __attribute__((ext_vector_type(4)));
typedef _Float16 nt_h8g __attribute__((ext_vector_type(8)));

template <typename TT>
struct NarrowTile;

template <>
struct NarrowTile<float> {
  static constexpr int NL = 4;   // 16-byte loads per lane
  typedef nt_f4g V;
  // piece m of lane `lane`: row, first column; 4 values
  __device__ static void place(int m, int lane, int &row, int &col) {
    const int c = m * 64 + lane;
    row = c / 8;
    col = 4 * (c % 8);
  }
  __device__ static void store(float *L, int row, int col, const V &v) {
    *(float4 *)(L + row * MLDF + col) = make_float4(v.x, v.y, v.z, v.w);
  }
};

template <>
struct NarrowTile<_Float16> {
  static constexpr int NL = 2;
  typedef nt_h8g V;
  __device__ static void place(int m, int lane, int &row, int &col) {
    const int c = m * 64 + lane;
    row = c / 4;
    col = 8 * (c % 4);
  }
  __device__ static void store(float *L, int row, int col, const V &v) {
    *(float4 *)(L + row * MLDF + col) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
    *(float4 *)(L + row * MLDF + col + 4) = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
  }
};

template <typename TT>
__device__ __forceinline__ void gemv_row_narrow(const int2 *__restrict__ rows, int nrows,
                                                const MSys *__restrict__ sys, const double *__restrict__ RP,
                                                double *__restrict__ ZP, double *__restrict__ yfull,
                                                const int32_t *__restrict__ act_bv) {
  typedef NarrowTile<TT> NT;
  __shared__ __attribute__((aligned(16))) float stage[4][TILE * MLDF];
  const int per = (int)gridDim.x / 8;
  const int wl = ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8;
  const int row = wl * 4 + (threadIdx.x >> 6);
  if (row >= nrows) return;   // no workgroup barrier below
  const int lane = threadIdx.x & 63, li = lane % 16, lk = lane / 16;
  const int2 sr = rows[row];
  const MSys S = sys[sr.x];
  const int I = sr.y, nb = S.nb;
  const double *__restrict__ Rs = RP + S.voff * MC;
  float *L = stage[threadIdx.x >> 6];
  auto tile_at = [&](int J) -> const typename NT::V * {
    const int64_t toff = (J <= I) ? (int64_t)I * (I + 1) / 2 + J : (int64_t)J * (J + 1) / 2 + I;
    return (const typename NT::V *)((const TT *)S.tiles + toff * (TILE * TILE));
  };
  auto ld = [&](const typename NT::V *p) -> typename NT::V {
    return *(const __attribute__((address_space(1))) typename NT::V *)p;
  };
  typename NT::V tv[NT::NL];
  float bv[8];
  int J = (I == 0) ? 0 : nb - I;
  {
    const typename NT::V *t = tile_at(J);
#pragma unroll
    for (int m = 0; m < NT::NL; ++m) tv[m] = ld(t + m * 64 + lane);
#pragma unroll
    for (int st = 0; st < 8; ++st) bv[st] = (float)ldg(Rs + (int64_t)(J * TILE + 4 * st + lk) * MC + li);
  }
  v4f acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  for (int s = 0; s < nb; ++s) {
#pragma unroll
    for (int m = 0; m < NT::NL; ++m) {
      int r0, c0;
      NT::place(m, lane, r0, c0);
      NT::store(L, r0, c0, tv[m]);
    }
    float bc[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) bc[st] = bv[st];
    const bool low = J <= I;
    const int J1 = (s + 1 < nb) ? ((J + 1 == nb) ? 0 : J + 1) : J;
    {
      const typename NT::V *t = tile_at(J1);
#pragma unroll
      for (int m = 0; m < NT::NL; ++m) tv[m] = ld(t + m * 64 + lane);
#pragma unroll
      for (int st = 0; st < 8; ++st) bv[st] = (float)ldg(Rs + (int64_t)(J1 * TILE + 4 * st + lk) * MC + li);
    }
    wave_lds_sync();
    float a0[8], a1[8];
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      const int k = 4 * st + lk;
      a0[st] = L[low ? li * MLDF + k : k * MLDF + li];
      a1[st] = L[low ? (16 + li) * MLDF + k : k * MLDF + 16 + li];
    }
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[st], bc[st], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[st], bc[st], acc1, 0, 0, 0);
    }
    wave_lds_sync();
    J = J1;
  }
  double *Zs = ZP + S.voff * MC;
  const double sc = (double)S.scale;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i0 = I * TILE + 4 * lk + r, i1 = i0 + 16;
    const double z0 = (double)acc0[r] * sc, z1 = (double)acc1[r] * sc;
    Zs[(int64_t)i0 * MC + li] = z0;
    Zs[(int64_t)i1 * MC + li] = z1;
    if (S.red) {
      if (i0 < S.n) yfull[(int64_t)act_bv[i0] * MC + li] = z0;
      if (i1 < S.n) yfull[(int64_t)act_bv[i1] * MC + li] = z1;
    }
  }
}

template <typename TT>
__global__ __launch_bounds__(256) void k_m_gemv(const int2 *__restrict__ rows, int nrows,
                                                const MSys *__restrict__ sys, const double *__restrict__ RP,
                                                double *__restrict__ ZP, double *__restrict__ yfull,
                                                const int32_t *__restrict__ act_bv, const MScal *__restrict__ ms) {
  if (ms->all_done) return;
  if constexpr (std::is_same<TT, double>::value)
    gemv_row_f64(rows, nrows, sys, RP, ZP, yfull, act_bv);
  else
    gemv_row_narrow<TT>(rows, nrows, sys, RP, ZP, yfull, act_bv);
}

// z = sum_p R_p^T z_p + J y_r per column (Sec. 3, Sec. 4), and the partials of
// (r_c, z_c)
template <typename T>
__global__ __launch_bounds__(256) void k_m_final(int64_t nf, const int32_t *__restrict__ cover_ptr,
                                                 const int32_t *__restrict__ cover_pos, const double *__restrict__ ZP,
                                                 const int32_t *__restrict__ jv_ptr, const int32_t *__restrict__ jv_base,
                                                 const T *__restrict__ jv_w, const T *__restrict__ jv_xi,
                                                 int64_t nent, int bx1, int bxy1, const double *__restrict__ yfull,
                                                 double *__restrict__ Z, const double *__restrict__ R,
                                                 double *__restrict__ part, double *__restrict__ part2,
                                                 const MScal *__restrict__ ms) {
  __shared__ double red[256 / WAVE * MC];
  if (ms->all_done) return;
  const int cq = (threadIdx.x % 4) * 4;
  double d[4] = {0.0, 0.0, 0.0, 0.0};
  double d2[4] = {0.0, 0.0, 0.0, 0.0};   // (r_{k+1}, z_k) for the Polak-Ribiere beta
  const int64_t n = nf * 4, G = (int64_t)gridDim.x * 256;
  for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < n; g += G) {
    const int64_t i = g / 4, o = i * MC + cq;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = cover_ptr[i]; k < cover_ptr[i + 1]; ++k) {
      double t[4];
      ld4(ZP + (int64_t)cover_pos[k] * MC + cq, t);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += t[j];
    }
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = jv_ptr[i]; k < jv_ptr[i + 1]; ++k) {
      const int64_t b0 = jv_base[k];
      const double x = jv_xi[k], y = jv_xi[nent + k], zz = jv_xi[2 * nent + k], wk = (double)jv_w[k];
      double sv[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int qq = 0; qq < 8; ++qq) {
        const int64_t bvx = b0 + (qq & 1) + ((qq >> 1) & 1) * bx1 + ((qq >> 2) & 1) * bxy1;
        const double f = trilin<double>(qq, x, y, zz);
        double yv[4];
        ld4(yfull + bvx * MC + cq, yv);
#pragma unroll
        for (int j = 0; j < 4; ++j) sv[j] += f * yv[j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) cs[j] += wk * sv[j];
    }
    double r[4];
    ld4(R + o, r);
    if (part2) {
      double zo[4];
      ld4(Z + o, zo);
#pragma unroll
      for (int j = 0; j < 4; ++j) d2[j] += r[j] * zo[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[j] += cs[j];
      d[j] += r[j] * acc[j];
    }
    st4(Z + o, acc);
  }
  const double s = block_colsum4<256>(d, red);
  if (threadIdx.x < MC) part[blockIdx.x * MC + threadIdx.x] = s;
  if (part2) {
    const double s2 = block_colsum4<256>(d2, red);
    if (threadIdx.x < MC) part2[blockIdx.x * MC + threadIdx.x] = s2;
  }
}

// partials of ||b_c - q_c||^2 (q = A x)
__global__ __launch_bounds__(256) void k_m_resnorm(int64_t nf, const double *__restrict__ B,
                                                   const double *__restrict__ Q, double *__restrict__ part) {
  __shared__ double red[256 / WAVE * MC];
  double acc = 0.0;
  const int64_t n = nf * MC, G = (int64_t)gridDim.x * 256;
  for (int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x; g < n; g += G) {
    const double t = B[g] - Q[g];
    acc += t * t;
  }
  const double s = block_colsum<256>(acc, red);
  if (threadIdx.x < MC) part[blockIdx.x * MC + threadIdx.x] = s;
}

// columns c < k of the block back to the caller's vertex order (0 on Dirichlet
// vertices)
__global__ __launch_bounds__(256) void k_m_permute_out(int64_t nv, int64_t nf, const int32_t *__restrict__ vint_of,
                                                       const double *__restrict__ X, int k, double *__restrict__ u) {
  const int64_t g = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t c = g / nv, v = g % nv;
  if (c >= k) return;
  const int32_t i = vint_of[v];
  u[g] = (i < nf) ? X[(int64_t)i * MC + c] : 0.0;
}

}  // namespace coarse
