// HIP kernels of the coarse solver for gfx950 (wave64). Every reduction has a
// fixed order (no floating-point atomics), so results are bitwise reproducible and
// do not depend on what else shares a launch.
#include "device.h"
#include "kernels.h"
#include "plan.h"

namespace coarse {

// ---------------------------------------------------------------------------
// Setup: Q1 element matrices (Sec. 3, a^e_ij = int grad l_i . grad l_j) with the
// 2x2x2 Gauss rule on the trilinear map of [-1,1]^3. One thread per element;
// the 36 distinct entries are stored per operator block (ae_at) for the setup,
// and the 28 off-diagonal ones (ae28_at) for the operator.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_elem_matrices(int64_t E, int64_t NV, const double *__restrict__ xyz,
                                                       const int32_t *__restrict__ e2v, double *__restrict__ Ae,
                                                       double *__restrict__ Ae28, int *__restrict__ bad) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= E) return;
  double X[8][3];
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int64_t u = e2v[v * E + e];
#pragma unroll
    for (int d = 0; d < 3; ++d) X[v][d] = xyz[d * NV + u];
  }
  double A[36];
#pragma unroll
  for (int k = 0; k < 36; ++k) A[k] = 0.0;
  const double g = 0.57735026918962576451;
  double detmin = 1e300;
#pragma unroll 1
  for (int q = 0; q < 8; ++q) {
    const double xq[3] = {(q & 1) ? g : -g, (q & 2) ? g : -g, (q & 4) ? g : -g};
    double dN[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const double s0 = (v & 1) ? 1.0 : -1.0, s1 = (v & 2) ? 1.0 : -1.0, s2 = (v & 4) ? 1.0 : -1.0;
      const double f0 = 1.0 + s0 * xq[0], f1 = 1.0 + s1 * xq[1], f2 = 1.0 + s2 * xq[2];
      dN[v][0] = 0.125 * s0 * f1 * f2;
      dN[v][1] = 0.125 * s1 * f0 * f2;
      dN[v][2] = 0.125 * s2 * f0 * f1;
    }
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < 8; ++v) s += X[v][i] * dN[v][j];
        J[i][j] = s;
      }
    // cofactors: inv(J)[j][i] = C[i][j] / det
    double C[3][3];
    C[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    C[0][1] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    C[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    C[1][0] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    C[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    C[1][2] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    C[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    C[2][1] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    C[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
    detmin = fmin(detmin, det);
    const double id = 1.0 / det;
    // physical gradient G[v][i] = sum_j dN[v][j] inv(J)[j][i] = sum_j dN[v][j] C[i][j] / det
    double G[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v)
#pragma unroll
      for (int i = 0; i < 3; ++i) G[v][i] = (dN[v][0] * C[i][0] + dN[v][1] * C[i][1] + dN[v][2] * C[i][2]) * id;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = a; b < 8; ++b)
        A[sym8(a, b)] += det * (G[a][0] * G[b][0] + G[a][1] * G[b][1] + G[a][2] * G[b][2]);
  }
  if (!(detmin > 0.0)) atomicAdd(bad, 1);
#pragma unroll
  for (int k = 0; k < 36; ++k) Ae[ae_at(k, e)] = A[k];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = a + 1; b < 8; ++b) Ae28[ae28_at(off8(a, b), e)] = A[sym8(a, b)];
}

// ---------------------------------------------------------------------------
// Operator q = A p (Sec. 3: A = Q^T A_L Q, the local products then the
// direct-stiffness sum). Pass 1: one workgroup per block of OP_BLOCK elements
// stages the block's vertex values in LDS, each thread applies its 8x8 element
// matrix, and the block sums the element outputs per vertex slot in a fixed
// order. Vertices entirely inside the block are written directly; vertices
// shared with other blocks go to a partial buffer that pass 2 sums. The energy
// p^T A p = sum_e p_e^T A^e p_e (the PCG denominator) comes out per block.
// ---------------------------------------------------------------------------
// An element's 8 block-local slots (one 16-byte record) and its 36 unique matrix
// entries do not depend on the vector: their loads are issued first and stay in
// flight while the block stages its vertex values.
// The element matrices are read once per application; when they are larger than
// the last-level cache (OpDev.ae_nt), the PCG operator reads them with
// non-temporal loads (NT = true), which keep them from evicting the vectors.
template <bool NT = false>
__device__ __forceinline__ void elem_load(const OpDev &op, int64_t e, double m[28], uint4 &c) {
  c = *(const uint4 *)(op.lconn + e * 8);
#pragma unroll
  for (int k = 0; k < 28; ++k) m[k] = NT ? __builtin_nontemporal_load(op.Ae + ae28_at(k, e)) : op.Ae[ae28_at(k, e)];
}

__device__ __forceinline__ unsigned slot_at(const uint4 &c, int a) {
  const unsigned w = (a < 2) ? c.x : (a < 4) ? c.y : (a < 6) ? c.z : c.w;
  return (a & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// y = A^e p_e from the staged slot values into out[0..8); returns p_e . y. The
// basis functions sum to one, so their gradients sum to zero and every row of
// A^e sums to zero: (A^e p)_a = sum_{b != a} a_ab (p_b - p_a), from the 28
// off-diagonal entries (a Dirichlet corner holds p = 0 and its row is dropped).
__device__ __forceinline__ double elem_apply(const double m[28], const uint4 &c, const double *lp, double *out) {
  double pe[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const unsigned sl = slot_at(c, a);
    pe[a] = (sl == 0xFFFFu) ? 0.0 : lp[sl];
  }
  double y[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) y[a] = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = a + 1; b < 8; ++b) {
      const double t = m[off8(a, b)] * (pe[b] - pe[a]);
      y[a] += t;
      y[b] -= t;
    }
  double en = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    out[a] = y[a];
    en += pe[a] * y[a];
  }
  return en;
}

// Per slot of the block, the element outputs of its incidences summed in list
// order (one 16-byte record holds up to 8 of them), written to q for a vertex the
// block owns or to its partial otherwise.
__device__ __forceinline__ void block_scatter(const OpDev &op, int s0, int ns, const double *out,
                                              double *__restrict__ q) {
  for (int s = threadIdx.x; s < ns; s += OP_BLOCK) {
    const uint4 rec = *(const uint4 *)(op.slot_inc8 + (int64_t)(s0 + s) * 8);
    const int dst = op.slot_dst[s0 + s];
    double acc = 0.0;
    if (slot_at(rec, 0) == 0xFFFEu) {
      // more than 8 incidences: the CSR list
      for (int k = op.slot_inc_ptr[s0 + s]; k < op.slot_inc_ptr[s0 + s + 1]; ++k) acc += out[op.slot_inc[k]];
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const unsigned li = slot_at(rec, k);
        if (li != 0xFFFFu) acc += out[li];
      }
    }
    if (dst >= 0)
      q[dst] = acc;
    else
      op.partials[-dst - 1] = acc;
  }
}

// The block's element outputs y (registers of each element's thread) summed
// into its slots, each written to q or to its partial. A block whose elements
// never hold one vertex at the same local corner adds them in LDS corner by
// corner (a = 0..7): each pass adds at most once to a slot, so no two threads
// touch a slot at once and every slot sums in corner order. A block with
// differently oriented elements sums its per-slot incidence lists instead.
// Called after the last read of the staged values in lp, which it reuses.
__device__ __forceinline__ void block_accumulate(const OpDev &op, int blk, int s0, int ns, bool valid, const uint4 &c,
                                                 const double y[8], double *lp, double *out,
                                                 double *__restrict__ q) {
  if (op.blk_inc[blk]) {
    if (valid) {
#pragma unroll
      for (int a = 0; a < 8; ++a) out[threadIdx.x * 8 + a] = y[a];
    }
    __syncthreads();
    block_scatter(op, s0, ns, out, q);
    return;
  }
  for (int s = threadIdx.x; s < ns; s += OP_BLOCK) lp[s] = 0.0;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    if (valid) {
      const unsigned sl = slot_at(c, a);
      if (sl != 0xFFFFu) lp[sl] += y[a];
    }
    __syncthreads();
  }
  for (int s = threadIdx.x; s < ns; s += OP_BLOCK) {
    const int dst = op.slot_dst[s0 + s];
    if (dst >= 0)
      q[dst] = lp[s];
    else
      op.partials[-dst - 1] = lp[s];
  }
}

__global__ __launch_bounds__(OP_BLOCK) void k_op_pass1(OpDev op, const double *__restrict__ p, double *__restrict__ q,
                                                       double *__restrict__ energy, const int *__restrict__ done) {
  extern __shared__ double lds[];
  __shared__ double red[OP_BLOCK / WAVE];
  if (done && *done) return;
  double *out = lds;                 // [OP_BLOCK*8]
  double *lp = lds + OP_BLOCK * 8;   // [slots]
  const int blk = blockIdx.x;
  const int64_t e = (int64_t)blk * OP_BLOCK + threadIdx.x;
  double m[28];
  uint4 c = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  if (e < op.E) elem_load(op, e, m, c);
  const int s0 = op.blk_slot_ptr[blk], ns = op.blk_slot_ptr[blk + 1] - s0;
  for (int s = threadIdx.x; s < ns; s += OP_BLOCK) lp[s] = p[op.slot_vid[s0 + s]];
  __syncthreads();
  double en = 0.0, y[8];
  if (e < op.E) en = elem_apply(m, c, lp, y);
  __syncthreads();
  block_accumulate(op, blk, s0, ns, e < op.E, c, y, lp, out, q);
  if (energy) {
    const double tot = block_sum<OP_BLOCK>(en, red);
    if (threadIdx.x == 0) energy[blk] = tot;
  }
}

__global__ __launch_bounds__(256) void k_op_pass2(OpDev op, double *__restrict__ q, const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= op.n_shared) return;
  double acc = 0.0;
  for (int k = op.sh_ptr[i]; k < op.sh_ptr[i + 1]; ++k) acc += op.partials[k];
  q[op.sh_vid[i]] = acc;
}

// ---------------------------------------------------------------------------
// Vector kernels of PCG. All use the same fixed grid (nblk workgroups of 256
// threads, thread t touching i = t, t + G, ...) so per-block partial sums are
// reproducible.
// ---------------------------------------------------------------------------
constexpr int VB = 256;
// The two per-vertex kernels of every iteration (update, final sum) run with
// larger workgroups: their grid is capped at 1024 workgroups (the partial sums
// that later kernels add up redundantly), so more threads per workgroup means
// more loads in flight.
constexpr int VW = 512;

// a caller vector gathered into internal order (no reduction)
__global__ __launch_bounds__(VB) void k_gather_user(int64_t nf, const int32_t *__restrict__ user_of, const double *__restrict__ b,
                                                    double *__restrict__ r) {
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) r[i] = b[user_of[i]];
}

__global__ __launch_bounds__(VB) void k_permute_out(int64_t nv, int64_t nf, const int32_t *__restrict__ vint_of,
                                                    const double *__restrict__ x, double *__restrict__ u) {
  const int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x;
  if (i >= nv) return;
  const int32_t k = vint_of[i];
  u[i] = (k < nf) ? x[k] : 0.0;
}

// t = a - q
__global__ __launch_bounds__(VB) void k_sub(int64_t nf, const int *__restrict__ done, const double *__restrict__ a,
                                            const double *__restrict__ q, double *__restrict__ t) {
  if (done && *done) return;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) t[i] = a[i] - q[i];
}

// partial sums of (a - q)^2
__global__ __launch_bounds__(VB) void k_resnorm(int64_t nf, const double *__restrict__ a, const double *__restrict__ q,
                                                double *__restrict__ part) {
  __shared__ double red[VB / WAVE];
  double acc = 0.0;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) {
    const double d = a[i] - q[i];
    acc += d * d;
  }
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ||b - A u||^2 from the partials of k_resnorm (one workgroup).
__global__ __launch_bounds__(VB) void k_res_total(Scalars *__restrict__ sc, const double *__restrict__ part, int n) {
  __shared__ double red[VB / WAVE];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += VB) acc += part[i];
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) sc->res_true = s;
}


// ---------------------------------------------------------------------------
// Fused PCG kernels. A scalar that needs a sum over workgroups of the previous
// kernel (p.Ap, ||r||^2, (r, z)) is formed by every workgroup of the consuming
// kernel from the at most 1024 partials, in the same fixed order, so all
// workgroups agree without any cross-workgroup synchronisation; workgroup 0
// records it in the solver state. Values that a kernel both reads and records
// (rho) are double-buffered by iteration parity.
// ---------------------------------------------------------------------------
constexpr int UV = 4;   // entries per thread and step in the restriction gather

// Sum of part[0..n) in a fixed order, returned to every thread (NT threads); U
// loads per thread are issued together.
template <int NT, int U = 4>
__device__ __forceinline__ double block_total(const double *__restrict__ part, int n, double *red) {
  double acc = 0.0;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * NT) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (i0 + u * NT < n) ? part[i0 + u * NT] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * NT < n) acc += v[u];
  }
  acc = wave_sum(acc);
  const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  __syncthreads();
  if (l == 0) red[w] = acc;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) s += red[i];
  return s;
}

// r = b (internal order), x = 0, both search-direction buffers and z = 0, and
// the partial sums of ||b||^2; workgroup 0 resets the solver state.
__global__ __launch_bounds__(VB) void k_start(int64_t nf, const int32_t *__restrict__ user_of, const double *__restrict__ b,
                                              double *__restrict__ r, double *__restrict__ x, double *__restrict__ pa,
                                              double *__restrict__ pb, double *__restrict__ z, double *__restrict__ bint,
                                              double *__restrict__ part, Scalars *__restrict__ sc, double tol2, int max_it,
                                              int flexible) {
  __shared__ double red[VB / WAVE];
  double acc = 0.0;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) {
    const double v = b[user_of[i]];
    r[i] = v;
    bint[i] = v;
    x[i] = 0.0;
    pa[i] = 0.0;
    pb[i] = 0.0;
    z[i] = 0.0;
    acc += v * v;
  }
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s;
    if (blockIdx.x == 0) {
      sc->tol2 = tol2;
      sc->max_it = max_it;
      sc->flexible = flexible;
      sc->iter = 0;
      sc->iters = 0;
      sc->status = 0;
      sc->done = 0;
      sc->rho[0] = sc->rho[1] = sc->alpha = sc->beta = sc->pq = 0.0;
    }
  }
}

// Operator with the direction update folded in: beta_{k-1} = rho_k / rho_{k-1}
// (or the Polak-Ribiere form) from the partials of the last preconditioner
// application, p_k = z_k + beta_{k-1} p_{k-1} formed while the block's vertex
// values are staged (p_0 = z_0), written once per vertex by its designated block,
// then q = A p_k as in k_op_pass1 with per-workgroup partials of p.Ap.
// The kernels of one PCG iteration are written as bodies that take their
// workgroup index (blk) and, where they loop over the grid, the grid size (nblk)
// explicitly, so that a launch covering several solves (a lock-step batch) runs
// each workgroup exactly as the solo launch of its own solve would.
template <bool NT = false>
__device__ __forceinline__ void op_fused_body(OpDev op, const double *__restrict__ z, double *__restrict__ pa,
                                              double *__restrict__ pb, double *__restrict__ q,
                                              double *__restrict__ energy, Scalars *__restrict__ sc,
                                              const double *__restrict__ rz1, const double *__restrict__ rz2, int nrz,
                                              int blk, double *lds, double *red) {
  if (sc->done) return;
  const int64_t e = (int64_t)blk * OP_BLOCK + threadIdx.x;
  double m[28];
  uint4 c = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  if (e < op.E) elem_load<NT>(op, e, m, c);
  const int it = sc->iter;
  const double rho = block_total<OP_BLOCK>(rz1, nrz, red);
  double beta = 0.0;
  if (it > 0) {
    const double num = sc->flexible ? rho - block_total<OP_BLOCK>(rz2, nrz, red) : rho;
    beta = num / sc->rho[(it - 1) & 1];
  }
  if (!isfinite(rho) || !isfinite(beta)) {
    if (blk == 0 && threadIdx.x == 0) {
      sc->done = 1;
      sc->status = -6;
      sc->iters = it;
    }
    return;
  }
  if (blk == 0 && threadIdx.x == 0) {
    sc->rho[it & 1] = rho;
    sc->beta = beta;
  }
  double *pcur = (it & 1) ? pb : pa;
  const double *pprev = (it & 1) ? pa : pb;
  double *out = lds;
  double *lp = lds + OP_BLOCK * 8;
  const int s0 = op.blk_slot_ptr[blk], ns = op.blk_slot_ptr[blk + 1] - s0;
  // two slots per thread and step, their loads issued together
  for (int s = threadIdx.x; s < ns; s += 2 * OP_BLOCK) {
    const int s1 = s + OP_BLOCK;
    const bool two = s1 < ns;
    const int32_t v0 = op.slot_vid[s0 + s];
    const int32_t v1 = two ? op.slot_vid[s0 + s1] : v0;
    const uint8_t w0 = op.slot_pw[s0 + s];
    const uint8_t w1 = two ? op.slot_pw[s0 + s1] : 0;
    const double z0 = z[v0], z1 = z[v1], q0 = pprev[v0], q1 = pprev[v1];
    const double pv0 = z0 + beta * q0;
    lp[s] = pv0;
    if (w0) pcur[v0] = pv0;
    if (two) {
      const double pv1 = z1 + beta * q1;
      lp[s1] = pv1;
      if (w1) pcur[v1] = pv1;
    }
  }
  __syncthreads();
  double en = 0.0, y[8];
  if (e < op.E) en = elem_apply(m, c, lp, y);
  __syncthreads();
  block_accumulate(op, blk, s0, ns, e < op.E, c, y, lp, out, q);
  const double tot = block_sum<OP_BLOCK>(en, red);
  if (threadIdx.x == 0) energy[blk] = tot;
}

template <bool NT>
__global__ __launch_bounds__(OP_BLOCK) void k_op_fused(OpDev op, const double *__restrict__ z, double *__restrict__ pa,
                                                       double *__restrict__ pb, double *__restrict__ q,
                                                       double *__restrict__ energy, Scalars *__restrict__ sc,
                                                       const double *__restrict__ rz1, const double *__restrict__ rz2,
                                                       int nrz) {
  extern __shared__ double lds[];
  __shared__ double red[OP_BLOCK / WAVE];
  op_fused_body<NT>(op, z, pa, pb, q, energy, sc, rz1, rz2, nrz, blockIdx.x, lds, red);
}

// alpha = rho / p.Ap (from the operator's partials), x += alpha p,
// r -= alpha q (q of vertices shared between operator blocks is summed here from
// the operator's partials), and partials of ||r||^2. A thread takes its vertices
// two at a time (i and i + G, then i + 2G and i + 3G, ...): their loads are
// issued together, the first pair's before the sum of the operator's partials,
// and q[i] is loaded whatever the vertex (a shared vertex then ignores it), so
// an owned vertex needs one round of loads. The squares are summed in the order
// i, i + G, i + 2G, ...
struct UpdV {
  int2 vq;
  double q, p, x, r;
};

__device__ __forceinline__ void update_load(int64_t i, int64_t nf, const OpDev &op, const double *__restrict__ q,
                                            const double *__restrict__ p, const double *__restrict__ x,
                                            const double *__restrict__ r, UpdV &v) {
  if (i < nf) {
    v.vq = op.vq[i];
    v.q = q[i];
    v.p = p[i];
    v.x = x[i];
    v.r = r[i];
  }
}

__device__ __forceinline__ void update_one(int64_t i, const OpDev &op, double alpha, const UpdV &v,
                                           double *__restrict__ x, double *__restrict__ r, double &acc) {
  double qi = v.q;
  if (v.vq.y != 0) {
    // the partials of a shared vertex are contiguous: issue the loads together
    qi = 0.0;
    for (int k0 = 0; k0 < v.vq.y; k0 += 8) {
      double pv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) pv[k] = (k0 + k < v.vq.y) ? op.partials[v.vq.x + k0 + k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k0 + k < v.vq.y) qi += pv[k];
    }
  }
  x[i] = v.x + alpha * v.p;
  const double ri = v.r - alpha * qi;
  r[i] = ri;
  acc += ri * ri;
}

__device__ __forceinline__ void update_fused_body(int64_t nf, OpDev op, Scalars *__restrict__ sc,
                                                  double *__restrict__ x, double *__restrict__ r,
                                                  const double *__restrict__ pa, const double *__restrict__ pb,
                                                  const double *__restrict__ q, const double *__restrict__ energy,
                                                  int nen, double *__restrict__ part, int blk, int nblk, double *red) {
  if (sc->done) return;
  const int it = sc->iter;
  const double *p = (it & 1) ? pb : pa;
  const int64_t G = (int64_t)nblk * VW;
  const int64_t i0 = blk * (int64_t)VW + threadIdx.x;
  UpdV a{}, b{};
  update_load(i0, nf, op, q, p, x, r, a);
  update_load(i0 + G, nf, op, q, p, x, r, b);
  const double pq = block_total<VW, 8>(energy, nen, red);
  const double rho = sc->rho[it & 1];
  if (!(pq > 0.0) || !isfinite(pq)) {
    if (blk == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->done = 1;
      sc->status = -6;
      sc->iters = it;
    }
    return;
  }
  const double alpha = rho / pq;
  if (blk == 0 && threadIdx.x == 0) {
    sc->pq = pq;
    sc->alpha = alpha;
  }
  double acc = 0.0;
  for (int64_t i = i0; i < nf; i += 2 * G) {
    update_one(i, op, alpha, a, x, r, acc);
    if (i + G < nf) update_one(i + G, op, alpha, b, x, r, acc);
    update_load(i + 2 * G, nf, op, q, p, x, r, a);
    update_load(i + 3 * G, nf, op, q, p, x, r, b);
  }
  const double s = block_sum<VW>(acc, red);
  if (threadIdx.x == 0) part[blk] = s;
}

__global__ __launch_bounds__(VW) void k_update_fused(int64_t nf, OpDev op, Scalars *__restrict__ sc, double *__restrict__ x,
                                                     double *__restrict__ r, const double *__restrict__ pa,
                                                     const double *__restrict__ pb, const double *__restrict__ q,
                                                     const double *__restrict__ energy, int nen,
                                                     double *__restrict__ part) {
  __shared__ double red[VW / WAVE];
  update_fused_body(nf, op, sc, x, r, pa, pb, q, energy, nen, part, blockIdx.x, gridDim.x, red);
}

// Convergence test at the start of a preconditioner application inside PCG.
// start = 1: the partials are those of ||b||^2 (b = 0 ends the solve at once);
// start = 2: those of the initial residual, ended at once when it already meets
// the tolerance;
// otherwise of ||r_{k+1}||^2, tested against tol^2 ||b||^2 and the iteration cap.
// Returns true when the solve is over (every workgroup reaches the same answer).
// Only workgroup blk == 0 records the outcome in the solver state. NT: threads
// of the calling workgroup (red holds NT / WAVE doubles).
template <int NT = 256>
__device__ bool pcg_check(Scalars *__restrict__ sc, const double *__restrict__ part, int n, int start, double *red,
                          int blk) {
  const double s = block_total<NT>(part, n, red);
  const bool lead = blk == 0 && threadIdx.x == 0;
  if (start) {
    // start = 2 (initial guess by projection): the partials are those of
    // ||b - A u_bar||^2 and ||b||^2 is already recorded
    const double bb = (start == 2) ? sc->bb : s;
    const bool bad = !isfinite(s) || !isfinite(bb);
    const bool stop = bad || !(bb > 0.0) || (start == 2 && s <= sc->tol2 * bb);
    if (lead) {
      sc->bb = bb;
      sc->rr = s;
      sc->rr0 = s;
      if (stop) {
        sc->done = 1;
        sc->status = bad ? -6 : 0;
        sc->iters = 0;
      }
    }
    return stop;
  }
  const int nit = sc->iter + 1;
  int status = 2;
  if (!isfinite(s))
    status = -6;
  else if (s <= sc->tol2 * sc->bb)
    status = 0;
  else if (nit >= sc->max_it)
    status = 1;
  if (lead) {
    sc->rr = s;
    if (status != 2) {
      sc->done = 1;
      sc->status = status;
      sc->iters = nit;
    }
  }
  return status != 2;
}

// The convergence test alone (used when the first kernel of a preconditioner
// variant cannot carry it).
__global__ __launch_bounds__(256) void k_check(Scalars *__restrict__ sc, const double *__restrict__ part, int n,
                                               int start) {
  __shared__ double red[256 / WAVE];
  if (sc->done) return;
  (void)pcg_check(sc, part, n, start, red, blockIdx.x);
}

// The convergence test carried by a kernel of NT threads per workgroup: true
// when the solve is over (the workgroup then does nothing else).
template <int NT>
__device__ __forceinline__ bool carried_check(const PcgCheck &ck, double *red) {
  if (!ck.sc) return false;
  return pcg_check<NT>(ck.sc, ck.part, ck.n, ck.start, red, ck.lead ? (int)blockIdx.x : 1);
}

// ---------------------------------------------------------------------------
// Initial guess by projection onto prior solutions (Sec. 5). The basis
// X_0 .. X_{n-1} is A-orthonormal and stored with AX_j = A X_j, row j at offset
// j * ld. Every sum over the vector uses the fixed grid of the PCG vector kernels
// followed by a fixed-order sum of the workgroup partials, so the basis and the
// guesses are bitwise reproducible.
// ---------------------------------------------------------------------------

// part[j][blk] (row stride gridDim.x): workgroup partials of X_j . v for the rows
// j = blockIdx.y < n, and of w . v for j = n when the grid has n + 1 rows.
__global__ __launch_bounds__(VB) void k_proj_dots(int64_t nf, int n, const double *__restrict__ X, int64_t ld,
                                                  const double *__restrict__ v, const double *__restrict__ w,
                                                  double *__restrict__ part) {
  __shared__ double red[VB / WAVE];
  const int j = blockIdx.y;
  const double *a = (j < n) ? X + (int64_t)j * ld : w;
  double acc = 0.0;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) acc += a[i] * v[i];
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = s;
}

// out[j] = sum of row j of part (nblk entries, fixed order): one workgroup per
// row. With sc given, the last workgroup records its total as ||b||^2.
__global__ __launch_bounds__(256) void k_proj_totals(const double *__restrict__ part, int nblk,
                                                     double *__restrict__ out, Scalars *__restrict__ sc) {
  __shared__ double red[256 / WAVE];
  const int j = blockIdx.x;
  const double s = block_total<256>(part + (int64_t)j * nblk, nblk, red);
  if (threadIdx.x == 0) {
    if (sc && j == (int)gridDim.x - 1)
      sc->bb = s;
    else
      out[j] = s;
  }
}

// u_bar = sum_j c_j X_j into x, r_0 = r - sum_j c_j AX_j (r holds b), and the
// partials of ||r_0||^2.
__global__ __launch_bounds__(VB) void k_proj_guess(int64_t nf, int n, const double *__restrict__ c,
                                                   const double *__restrict__ X, const double *__restrict__ AX,
                                                   int64_t ld, double *__restrict__ x, double *__restrict__ r,
                                                   double *__restrict__ part) {
  __shared__ double red[VB / WAVE];
  double acc = 0.0;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) {
    double u = 0.0, ri = r[i];
    for (int j = 0; j < n; ++j) {
      const double cj = c[j];
      u += cj * X[(int64_t)j * ld + i];
      ri -= cj * AX[(int64_t)j * ld + i];
    }
    x[i] = u;
    r[i] = ri;
    acc += ri * ri;
  }
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// A-Gram-Schmidt of a new solution u (with q = A u) against the basis, with
// e_j = X_j . (A u): w = u - sum_j e_j X_j into X_n, A w = q - sum_j e_j AX_j into
// AX_n, and the partials of w . A w.
__global__ __launch_bounds__(VB) void k_proj_orth(int64_t nf, int n, const double *__restrict__ e,
                                                  double *__restrict__ X, double *__restrict__ AX, int64_t ld,
                                                  const double *__restrict__ u, const double *__restrict__ q,
                                                  double *__restrict__ part) {
  __shared__ double red[VB / WAVE];
  double acc = 0.0;
  const int64_t G = (int64_t)gridDim.x * VB;
  double *wn = X + (int64_t)n * ld, *awn = AX + (int64_t)n * ld;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) {
    double w = u[i], aw = q[i];
    for (int j = 0; j < n; ++j) {
      const double ej = e[j];
      w -= ej * X[(int64_t)j * ld + i];
      aw -= ej * AX[(int64_t)j * ld + i];
    }
    wn[i] = w;
    awn[i] = aw;
    acc += w * aw;
  }
  const double s = block_sum<VB>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Normalise the new row n by 1/sqrt(w . A w), each workgroup forming that sum
// itself from the nblk partials; the row is kept only when its A-norm exceeds
// 1e-6 of that of u (uau = u . A u) and is finite. Workgroup 0 writes the new
// basis size to *count.
__global__ __launch_bounds__(VB) void k_proj_scale(int64_t nf, int n, const double *__restrict__ part, int nblk,
                                                   const double *__restrict__ uau, double *__restrict__ X,
                                                   double *__restrict__ AX, int64_t ld, int *__restrict__ count) {
  __shared__ double red[VB / WAVE];
  const double w2 = block_total<VB>(part, nblk, red);
  const bool keep = isfinite(w2) && w2 > 1e-12 * (*uau);
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = keep ? n + 1 : n;
  if (!keep) return;
  const double s = 1.0 / sqrt(w2);
  double *wn = X + (int64_t)n * ld, *awn = AX + (int64_t)n * ld;
  const int64_t G = (int64_t)gridDim.x * VB;
  for (int64_t i = blockIdx.x * (int64_t)VB + threadIdx.x; i < nf; i += G) {
    wn[i] *= s;
    awn[i] *= s;
  }
}

// Restriction R_p r into the packed local vectors (workgroups [0, ng), grid-
// stride) and the first stage of J^T r (the remaining workgroups, one task per
// wavefront at a time).
// One restriction task (a wavefront): the 8 corner sums of at most JT_CHUNK
// entries (i, c) of one cell, weight w_ic = n_ic/m_i times the trilinear
// weights at the local coordinates of vertex i, applied to in[i]. Each lane takes
// at most JT_CHUNK/64 entries, loaded together.
template <typename T>
__device__ __forceinline__ void jt_task(int task, const int32_t *__restrict__ tstart, const int32_t *__restrict__ vid,
                                        const T *__restrict__ w, const T *__restrict__ xi, int64_t nent,
                                        const double *__restrict__ in, T *__restrict__ tpart) {
  constexpr int PER = JT_CHUNK / 64;
  const int lane = threadIdx.x & 63;
  const int j0 = tstart[task], j1 = tstart[task + 1];
  int jj[PER];
  T v[PER], x[PER], y[PER], z[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int j = j0 + lane + 64 * m;
    jj[m] = (j < j1) ? vid[j] : -1;
    v[m] = (j < j1) ? w[j] : T(0);
    x[m] = (j < j1) ? xi[j] : T(0);
    y[m] = (j < j1) ? xi[nent + j] : T(0);
    z[m] = (j < j1) ? xi[2 * nent + j] : T(0);
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) v[m] = (jj[m] >= 0) ? v[m] * (T)in[jj[m]] : T(0);
  T acc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    acc[k] = T(0);
#pragma unroll
    for (int m = 0; m < PER; ++m) acc[k] += trilin<T>(k, x[m], y[m], z[m]) * v[m];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) tpart[task * 8 + k] = acc[k];
  }
}

template <typename T>
__device__ __forceinline__ void pre_body(int ng, int64_t n, const int *__restrict__ done,
                                         const int32_t *__restrict__ idx, const double *__restrict__ in,
                                         T *__restrict__ rp, int ntask, const int32_t *__restrict__ tstart,
                                         const int32_t *__restrict__ vid, const T *__restrict__ w,
                                         const T *__restrict__ xi, int64_t nent, T *__restrict__ tpart,
                                         Scalars *__restrict__ sc, const double *__restrict__ chk, int nchk, int start,
                                         int blk, int nblk, double *red) {
  if (*done) return;
  if (sc && pcg_check(sc, chk, nchk, start, red, blk)) return;
  if (blk < ng) {
    // UV entries per thread and step, index and value loads issued together
    const int64_t G = (int64_t)ng * 256;
    for (int64_t j0 = blk * (int64_t)256 + threadIdx.x; j0 < n; j0 += G * UV) {
      int32_t ii[UV];
#pragma unroll
      for (int u = 0; u < UV; ++u) ii[u] = (j0 + u * G < n) ? idx[j0 + u * G] : -1;
      double vv[UV];
#pragma unroll
      for (int u = 0; u < UV; ++u) vv[u] = (ii[u] >= 0) ? in[ii[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < UV; ++u)
        if (j0 + u * G < n) rp[j0 + u * G] = (ii[u] >= 0) ? (T)vv[u] : T(0);
    }
    return;
  }
  const int nw = (nblk - ng) * 4;
  for (int task = (blk - ng) * 4 + (threadIdx.x >> 6); task < ntask; task += nw)
    jt_task<T>(task, tstart, vid, w, xi, nent, in, tpart);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pre(int ng, int64_t n, const int *__restrict__ done, const int32_t *__restrict__ idx,
                                             const double *__restrict__ in, T *__restrict__ rp, int ntask,
                                             const int32_t *__restrict__ tstart, const int32_t *__restrict__ vid,
                                             const T *__restrict__ w, const T *__restrict__ xi, int64_t nent,
                                             T *__restrict__ tpart, Scalars *__restrict__ sc,
                                             const double *__restrict__ chk, int nchk, int start) {
  __shared__ double red[256 / WAVE];
  pre_body<T>(ng, n, done, idx, in, rp, ntask, tstart, vid, w, xi, nent, tpart, sc, chk, nchk, start, blockIdx.x,
              gridDim.x, red);
}

// ---------------------------------------------------------------------------
// Preconditioner, local part (Sec. 3, eq. (asm)): r_p = R_p r gathered into the
// packed vectors of all subdomains (padding = 0).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(VB) void k_gather(int64_t n, const int *__restrict__ done, const int32_t *__restrict__ idx,
                                               const double *__restrict__ in, T *__restrict__ rp) {
  if (*done) return;
  const int64_t j = blockIdx.x * (int64_t)VB + threadIdx.x;
  if (j >= n) return;
  const int32_t i = idx[j];
  rp[j] = (i >= 0) ? (T)in[i] : T(0);
}

// ---------------------------------------------------------------------------
// Reduced-space restriction J^T r (Sec. 4): J = W Q^T J_L S. Each wavefront
// handles one task (<= JT_CHUNK entries of one cell), entry (i, c) carrying the
// weight fraction n_ic/m_i and the local coordinates of vertex i in cell c; it
// accumulates the 8 corner sums and reduces them across the wave. A second
// kernel sums the tasks around each active box vertex in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_jt_tasks(int ntask, const int *__restrict__ done, const int32_t *__restrict__ tstart,
                                                  const int32_t *__restrict__ vid, const T *__restrict__ w,
                                                  const T *__restrict__ xi, int64_t nent, const double *__restrict__ in,
                                                  T *__restrict__ tpart, PcgCheck ck) {
  __shared__ double red[256 / WAVE];
  if (*done) return;
  if (carried_check<256>(ck, red)) return;
  const int task = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (task >= ntask) return;
  jt_task<T>(task, tstart, vid, w, xi, nent, in, tpart);
}

// Second stage of J^T: one wavefront per active box vertex sums the task
// partials of the occupied cells around it (lane-strided, then across the wave).
template <typename T>
__device__ __forceinline__ void corners_body(int64_t nr, const int *__restrict__ done, const int32_t *__restrict__ ptr,
                                             const int32_t *__restrict__ src, const T *__restrict__ tpart,
                                             T *__restrict__ rr, int blk) {
  if (*done) return;
  const int lane = threadIdx.x & 63;
  const int64_t K = blk * (int64_t)4 + (threadIdx.x >> 6);
  if (K >= nr) return;
  T acc = T(0);
  for (int k = ptr[K] + lane; k < ptr[K + 1]; k += 64) acc += tpart[src[k]];
  acc = wave_sum(acc);
  if (lane == 0) rr[K] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_jt_corners(int64_t nr, const int *__restrict__ done, const int32_t *__restrict__ ptr,
                                                    const int32_t *__restrict__ src, const T *__restrict__ tpart,
                                                    T *__restrict__ rr) {
  corners_body<T>(nr, done, ptr, src, tpart, rr, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Batched dense solves z_s = A_s^{-1} r_s for every system (the local A_p and the
// reduced A_r): a symmetric GEMV over the lower tiles of the stored inverse.
// Each wavefront streams up to GEMV_SEG tiles of one tile row I: it accumulates
// the row contribution (tile * r_J) in registers and emits, for off-diagonal
// tiles, the transposed contribution (tile^T * r_I) for row J. Tiles are read
// once, with 16-byte loads; the partials are summed by k_combine.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int nseg, int g) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].begin <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Streaming (non-temporal) 16-byte loads: the stored inverses are read once per
// application and should not displace the small vectors from the caches. They
// are issued as global (not flat) loads: a flat load also counts against the
// wait for LDS accesses, which would hold every LDS access of the loop until
// the prefetched tile has arrived.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
template <typename V>
__device__ __forceinline__ V ldnt_global(const V *p) {
  return __builtin_nontemporal_load((const __attribute__((address_space(1))) V *)p);
}
__device__ __forceinline__ double2 ldnt(const double2 *p) {
  const nt_d2 v = ldnt_global((const nt_d2 *)p);
  double2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}
__device__ __forceinline__ float4 ldnt(const float4 *p) {
  const nt_f4 v = ldnt_global((const nt_f4 *)p);
  float4 o;
  o.x = v.x;
  o.y = v.y;
  o.z = v.z;
  o.w = v.w;
  return o;
}

// Whole systems (nb <= WHOLE_NB_MAX): one workgroup of NW wavefronts per system
// (the context's choice, by default WHOLE_WAVES_F64 for FP64 tiles and
// WHOLE_WAVES_NARROW for the smaller FP32/FP16 tiles, so that a workgroup keeps
// as many bytes in flight), launched ahead of the work items in the same grid. Wavefront w owns the
// tile rows dealt to it in a snake order over the rows from longest to shortest
// (so the waves hold nearly equal tile counts) and streams their tiles back to
// back, the next one (across a row boundary too) loaded while the current one is
// used. A row's own contribution is summed in registers; the transposed
// contributions of its off-diagonal tiles go to the wavefront's copy of the
// solution in LDS. The copies are summed in a fixed order at the end and written
// as z_s: no partial sums leave the workgroup.
template <int NW>
__device__ __forceinline__ int snake_row(int nb, int w, int k) {
  const int p = k * NW + ((k & 1) ? NW - 1 - w : w);
  return p < nb ? nb - 1 - p : -1;
}

// the wavefront's next tile after (I, J) (its k-th row): (nI, nJ) in row nk, nI < 0 at the end
template <int NW>
__device__ __forceinline__ void whole_next(int nb, int w, int k, int I, int J, int &nk, int &nI, int &nJ) {
  nk = k;
  nI = I;
  nJ = J + 1;
  if (nJ > I) {
    nk = k + 1;
    nI = snake_row<NW>(nb, w, nk);
    nJ = 0;
  }
}

// z_s = scale times the sum of the wavefront copies, in a fixed order (the
// reduced system also goes to the full box-vertex grid)
template <int NW, typename A>
__device__ __forceinline__ void whole_finish(const SysDev &S, A *ys, double scale) {
  __syncthreads();
  const int n = S.nb * TILE;
  for (int i = threadIdx.x; i < n; i += NW * WAVE) {
    A z = A(0);
#pragma unroll
    for (int q = 0; q < NW; ++q) z += ys[q * n + i];
    const double zd = (double)z * scale;
    S.zp[i] = zd;
    if (S.yfull && i < S.n) S.yfull[S.act_bv[i]] = zd;
  }
}

// Clears the NW solution copies and stages the right-hand side r_s in LDS after
// them: gathered from the full vector gin through the system's packed indices
// (r_p = R_p r, padding 0) when gin is given and the system is a local one, else
// copied from the packed vector S.rp. Returns the wavefront's solution copy; rs
// receives the staged right-hand side.
template <int NW, typename A>
__device__ __forceinline__ A *whole_begin(const SysDev &S, A *ys, const double *__restrict__ gin, const A *&rs) {
  const int n = S.nb * TILE;
  for (int i = threadIdx.x; i < NW * n; i += NW * WAVE) ys[i] = A(0);
  A *r = ys + NW * n;
  constexpr int U = 4;   // entries per thread and step, their loads issued together
  if (gin && S.gidx) {
    for (int i0 = threadIdx.x; i0 < n; i0 += U * NW * WAVE) {
      int32_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = (i0 + u * NW * WAVE < n) ? S.gidx[i0 + u * NW * WAVE] : -1;
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = (v[u] >= 0) ? gin[v[u]] : 0.0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * NW * WAVE < n) r[i0 + u * NW * WAVE] = (v[u] >= 0) ? (A)x[u] : A(0);
    }
  } else {
    const A *__restrict__ src = (const A *)S.rp;
    for (int i = threadIdx.x; i < n; i += NW * WAVE) r[i] = src[i];
  }
  rs = r;
  __syncthreads();
  return ys + (threadIdx.x >> 6) * n;
}


// Tiles a wavefront walks in the row order: the sum over its rows I of I + 1.
template <int NW>
__device__ __forceinline__ int wave_row_tiles(int nb, int w) {
  int T = 0;
  for (int k = 0;; ++k) {
    const int I = snake_row<NW>(nb, w, k);
    if (I < 0) return T;
    T += I + 1;
  }
}

// FP64 tiles: lane layout of k_gemv_f64 below. Two register buffers take turns
// (the loop body is unrolled twice): the next tile is in flight while the
// current one is used, and the main loop issues its loads unconditionally (the
// last tiles of the walk are handled after it), so that the compiler's count of
// loads in flight stays exact and a tile's use waits for that tile alone.
template <int NW>
__device__ __forceinline__ void whole_f64(const SysDev &S, double *ys, const double *__restrict__ gin) {
  const double *r;
  double *y = whole_begin<NW>(S, ys, gin, r);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane >> 4, c2 = (lane & 15) * 2;
  const int nb = S.nb;
  const double2 *__restrict__ base = (const double2 *)S.tiles;
  const int T = wave_row_tiles<NW>(nb, w);
  if (T > 0) {
    auto load = [&](int ti, int tj, double2 *dst) {
      const double2 *t = base + ((int64_t)ti * (ti + 1) / 2 + tj) * (TILE * TILE / 2);
#pragma unroll
      for (int m = 0; m < 8; ++m) dst[m] = ldnt(t + m * 64 + lane);
    };
    // (k0, I0, J0): the tile in use; (k1, I1, J1): the next one
    int k0 = 0, I0 = snake_row<NW>(nb, w, 0), J0 = 0, k1, I1, J1;
    whole_next<NW>(nb, w, k0, I0, J0, k1, I1, J1);
    // both buffers are loaded whatever T (a walk of one tile loads it twice), so
    // that every path into the loop has issued the same loads
    double2 va[8], vb[8];
    load(I0, J0, va);
    load(T > 1 ? I1 : I0, T > 1 ? J1 : J0, vb);
    double rI[8], acc[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      rI[m] = r[I0 * TILE + 4 * m + grp];
      acc[m] = 0.0;
    }
    int t = 0;
    // uses the tile in v, then (refill) loads into v the tile two positions ahead
    auto step = [&](double2 *v, bool refill) {
      const double2 rj = *(const double2 *)(r + J0 * TILE + c2);
#pragma unroll
      for (int m = 0; m < 8; ++m) acc[m] += v[m].x * rj.x + v[m].y * rj.y;
      if (J0 != I0) {
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          cx += v[m].x * rI[m];
          cy += v[m].y * rI[m];
        }
        cx += __shfl_xor(cx, 16, 64);
        cy += __shfl_xor(cy, 16, 64);
        cx += __shfl_xor(cx, 32, 64);
        cy += __shfl_xor(cy, 32, 64);
        if (lane < 16) {
          y[J0 * TILE + c2] += cx;
          y[J0 * TILE + c2 + 1] += cy;
        }
      } else {
        // row I0 complete
#pragma unroll
        for (int m = 0; m < 8; ++m) {
          double a = acc[m];
          a += __shfl_xor(a, 1, 64);
          a += __shfl_xor(a, 2, 64);
          a += __shfl_xor(a, 4, 64);
          a += __shfl_xor(a, 8, 64);
          acc[m] = 0.0;
          if ((lane & 15) == 0) y[I0 * TILE + 4 * m + grp] += a;
        }
        if (I1 >= 0) {
#pragma unroll
          for (int m = 0; m < 8; ++m) rI[m] = r[I1 * TILE + 4 * m + grp];
        }
      }
      int k2, I2, J2;
      whole_next<NW>(nb, w, k1, I1, J1, k2, I2, J2);
      if (refill) load(I2, J2, v);
      k0 = k1;
      I0 = I1;
      J0 = J1;
      k1 = k2;
      I1 = I2;
      J1 = J2;
      ++t;
    };
    while (t + 3 < T) {
      step(va, true);
      step(vb, true);
    }
    // at most three tiles left: t in va, t + 1 in vb, t + 2 loaded into va
    if (t < T) step(va, t + 2 < T);
    if (t < T) step(vb, false);
    if (t < T) step(va, false);
  }
  whole_finish<NW>(S, ys, 1.0);
}

// The segment table of a launch covering several solves: whole-system
// workgroups first (begin offsets in systems), then items (begin in items).
__device__ __forceinline__ const Seg &seg_of(const Seg *__restrict__ segs, int nseg, int g) {
  return segs[nseg == 1 ? 0 : find_seg(segs, nseg, g)];
}


// FP64: a wavefront covers a 32x32 tile with 8 loads of 16 bytes per lane; lane l
// holds rows 4k + l/16 (k < 8), columns 2(l%16) and 2(l%16)+1. The next tile is
// loaded while the current one is used.
__device__ __forceinline__ void items_f64(const Seg *__restrict__ segs, int nseg, int total, int g0,
                                          int gstride) {
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 4, c2 = (lane & 15) * 2;
  for (int g = g0; g < total; g += gstride) {
    const Seg sg = segs[nseg == 1 ? 0 : find_seg(segs, nseg, g)];
    if (sg.done && *sg.done) continue;
    const GItem it = sg.items[g - sg.begin];
    const SysDev S = sg.sys[it.sys];
    const double *__restrict__ r = (const double *)S.rp;
    const int I = it.I;
    const int64_t rowbase = (int64_t)I * (I + 1) / 2;
    const double2 *__restrict__ t = (const double2 *)((const double *)S.tiles + (rowbase + it.j0) * (TILE * TILE));
    double2 v[8], w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = ldnt(t + k * 64 + lane);
    double rI[8], acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      rI[k] = r[I * TILE + 4 * k + grp];
      acc[k] = 0.0;
    }
    for (int J = it.j0; J < it.j1; ++J) {
      const bool more = J + 1 < it.j1;
      t += TILE * TILE / 2;
      if (more) {
#pragma unroll
        for (int k = 0; k < 8; ++k) w[k] = ldnt(t + k * 64 + lane);
      }
      const double2 rj = *(const double2 *)(r + J * TILE + c2);
#pragma unroll
      for (int k = 0; k < 8; ++k) acc[k] += v[k].x * rj.x + v[k].y * rj.y;
      if (J != I) {
        double cx = 0.0, cy = 0.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          cx += v[k].x * rI[k];
          cy += v[k].y * rI[k];
        }
        cx += __shfl_xor(cx, 16, 64);
        cy += __shfl_xor(cy, 16, 64);
        cx += __shfl_xor(cx, 32, 64);
        cy += __shfl_xor(cy, 32, 64);
        if (lane < 16) {
          double2 o;
          o.x = cx;
          o.y = cy;
          *(double2 *)((double *)S.colpart + (rowbase + J) * TILE + c2) = o;
        }
      }
      if (more) {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = w[k];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      double a = acc[k];
      a += __shfl_xor(a, 1, 64);
      a += __shfl_xor(a, 2, 64);
      a += __shfl_xor(a, 4, 64);
      a += __shfl_xor(a, 8, 64);
      acc[k] = a;
    }
    if ((lane & 15) == 0) {
      double *rowp = (double *)S.rowpart + (int64_t)it.slot * TILE;
#pragma unroll
      for (int k = 0; k < 8; ++k) rowp[4 * k + grp] = acc[k];
    }
  }
}

// Work items only, one per wavefront.
__global__ __launch_bounds__(256) void k_gemv_f64(const Seg *__restrict__ segs, int nseg, int total,
                                                  const int *__restrict__ done, PcgCheck ck) {
  __shared__ double red[256 / WAVE];
  if (done && *done) return;
  if (carried_check<256>(ck, red)) return;
  items_f64(segs, nseg, total, blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4);
}

// Workgroups [0, nwhole) solve whole systems (wsegs: begin offsets in systems),
// the others take the work items (segs), NW wavefronts per workgroup.
template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_gemv_whole_f64(const Seg *__restrict__ segs, int nseg, int total,
                                                              const Seg *__restrict__ wsegs, int nwhole,
                                                              const int *__restrict__ done,
                                                              const double *__restrict__ gin, PcgCheck ck) {
  extern __shared__ double ys_whole_d[];
  __shared__ double red[NW];
  if (done && *done) return;
  if (carried_check<NW * WAVE>(ck, red)) return;
  if ((int)blockIdx.x < nwhole) {
    const Seg &sg = seg_of(wsegs, nseg, blockIdx.x);
    if (sg.done && *sg.done) return;
    whole_f64<NW>(sg.sys[sg.whole[blockIdx.x - sg.begin]], ys_whole_d, gin);
    return;
  }
  items_f64(segs, nseg, total, (blockIdx.x - nwhole) * NW + (threadIdx.x >> 6), (gridDim.x - nwhole) * NW);
}

// FP32: 4 loads of 16 bytes per lane per tile; lane l holds rows 8m + l/8 (m < 4),
// columns 4(l%8) .. 4(l%8)+3. Two register buffers take turns, as for FP64 tiles.
template <int NW>
__device__ __forceinline__ void whole_f32(const SysDev &S, float *ys, const double *__restrict__ gin) {
  const float *r;
  float *y = whole_begin<NW>(S, ys, gin, r);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane >> 3, c4 = (lane & 7) * 4;
  const int nb = S.nb;
  const float4 *__restrict__ base = (const float4 *)S.tiles;
  const int T = wave_row_tiles<NW>(nb, w);
  if (T > 0) {
    auto load = [&](int ti, int tj, float4 *dst) {
      const float4 *t = base + ((int64_t)ti * (ti + 1) / 2 + tj) * (TILE * TILE / 4);
#pragma unroll
      for (int m = 0; m < 4; ++m) dst[m] = ldnt(t + m * 64 + lane);
    };
    int k0 = 0, I0 = snake_row<NW>(nb, w, 0), J0 = 0, k1, I1, J1;
    whole_next<NW>(nb, w, k0, I0, J0, k1, I1, J1);
    // both buffers are loaded whatever T, as for FP64 tiles
    float4 va[4], vb[4];
    load(I0, J0, va);
    load(T > 1 ? I1 : I0, T > 1 ? J1 : J0, vb);
    float rI[4], acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      rI[m] = r[I0 * TILE + 8 * m + grp];
      acc[m] = 0.0f;
    }
    int t = 0;
    auto step = [&](float4 *v, bool refill) {
      const float4 rj = *(const float4 *)(r + J0 * TILE + c4);
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m] += v[m].x * rj.x + v[m].y * rj.y + v[m].z * rj.z + v[m].w * rj.w;
      if (J0 != I0) {
        float c[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          c[0] += v[m].x * rI[m];
          c[1] += v[m].y * rI[m];
          c[2] += v[m].z * rI[m];
          c[3] += v[m].w * rI[m];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          c[j] += __shfl_xor(c[j], 8, 64);
          c[j] += __shfl_xor(c[j], 16, 64);
          c[j] += __shfl_xor(c[j], 32, 64);
        }
        if (lane < 8) {
#pragma unroll
          for (int j = 0; j < 4; ++j) y[J0 * TILE + c4 + j] += c[j];
        }
      } else {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          float a = acc[m];
          a += __shfl_xor(a, 1, 64);
          a += __shfl_xor(a, 2, 64);
          a += __shfl_xor(a, 4, 64);
          acc[m] = 0.0f;
          if ((lane & 7) == 0) y[I0 * TILE + 8 * m + grp] += a;
        }
        if (I1 >= 0) {
#pragma unroll
          for (int m = 0; m < 4; ++m) rI[m] = r[I1 * TILE + 8 * m + grp];
        }
      }
      int k2, I2, J2;
      whole_next<NW>(nb, w, k1, I1, J1, k2, I2, J2);
      if (refill) load(I2, J2, v);
      k0 = k1;
      I0 = I1;
      J0 = J1;
      k1 = k2;
      I1 = I2;
      J1 = J2;
      ++t;
    };
    while (t + 3 < T) {
      step(va, true);
      step(vb, true);
    }
    if (t < T) step(va, t + 2 < T);
    if (t < T) step(vb, false);
    if (t < T) step(va, false);
  }
  whole_finish<NW>(S, ys, 1.0);
}


// Work items of FP32 (and FP16) tiles. With CH > 1 the tiles of an item and
// their right-hand-side pieces are loaded in chunks of up to CH, all issued
// before the first is used, so an item costs one memory round trip per chunk
// rather than one per tile: that pays when a launch holds few items (a single
// small mesh), whose latency nothing else hides. With CH = 1 the item's tiles
// are streamed with the next one in flight, at twice the occupancy: that pays
// for the many items of a lock-step batch, and in the launches that also hold
// whole-system workgroups, whose occupancy the chunk's registers would lower.
// Both apply each tile with the same helper (explicit fused multiply-adds), so
// an item's result does not depend on the launch it is in.
constexpr int ITEM_CHUNK = 4;
// launches of at most this many work items take the chunked form (it holds
// three wavefronts per SIMD, 3072 on the 256 compute units)
constexpr int ITEM_CHUNK_MAX_ITEMS = 3072;

// One tile (I, J) of a work item, FP32: row contribution into acc, transposed
// contribution (J != I) to the tile's column partial.
__device__ __forceinline__ void item_tile_f32(const float4 (&v)[4], const float4 &rj, const float (&rI)[4],
                                              float (&acc)[4], bool offdiag, float *__restrict__ colp, int lane) {
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] += fmaf(v[m].w, rj.w, fmaf(v[m].z, rj.z, fmaf(v[m].y, rj.y, v[m].x * rj.x)));
  if (offdiag) {
    float c[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      c[0] = fmaf(v[m].x, rI[m], c[0]);
      c[1] = fmaf(v[m].y, rI[m], c[1]);
      c[2] = fmaf(v[m].z, rI[m], c[2]);
      c[3] = fmaf(v[m].w, rI[m], c[3]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[j] += __shfl_xor(c[j], 8, 64);
      c[j] += __shfl_xor(c[j], 16, 64);
      c[j] += __shfl_xor(c[j], 32, 64);
    }
    if (lane < 8) {
      float4 o;
      o.x = c[0];
      o.y = c[1];
      o.z = c[2];
      o.w = c[3];
      *(float4 *)colp = o;
    }
  }
}

template <int CH>
__device__ __forceinline__ void items_f32(const Seg *__restrict__ segs, int nseg, int total, int g0,
                                          int gstride) {
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 3, c4 = (lane & 7) * 4;
  for (int g = g0; g < total; g += gstride) {
    const Seg sg = segs[nseg == 1 ? 0 : find_seg(segs, nseg, g)];
    if (sg.done && *sg.done) continue;
    const GItem it = sg.items[g - sg.begin];
    const SysDev S = sg.sys[it.sys];
    const float *__restrict__ r = (const float *)S.rp;
    const int I = it.I;
    const int64_t rowbase = (int64_t)I * (I + 1) / 2;
    const float4 *__restrict__ t0 = (const float4 *)((const float *)S.tiles + (rowbase + it.j0) * (TILE * TILE));
    float rI[4], acc[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      rI[m] = r[I * TILE + 8 * m + grp];
      acc[m] = 0.0f;
    }
    auto colp = [&](int J) { return (float *)S.colpart + (rowbase + J) * TILE + c4; };
    if constexpr (CH == 1) {
      float4 v[4], w[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) v[m] = ldnt(t0 + m * 64 + lane);
      const float4 *t = t0;
      for (int J = it.j0; J < it.j1; ++J) {
        const bool more = J + 1 < it.j1;
        t += TILE * TILE / 4;
        if (more) {
#pragma unroll
          for (int m = 0; m < 4; ++m) w[m] = ldnt(t + m * 64 + lane);
        }
        const float4 rj = *(const float4 *)(r + J * TILE + c4);
        item_tile_f32(v, rj, rI, acc, J != I, colp(J), lane);
        if (more) {
#pragma unroll
          for (int m = 0; m < 4; ++m) v[m] = w[m];
        }
      }
    } else {
      for (int J0 = it.j0; J0 < it.j1; J0 += CH) {
        const int cn = it.j1 - J0 < CH ? it.j1 - J0 : CH;
        float4 v[CH][4], rjv[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (u < cn) {
            const float4 *t = t0 + (int64_t)(J0 - it.j0 + u) * (TILE * TILE / 4);
#pragma unroll
            for (int m = 0; m < 4; ++m) v[u][m] = ldnt(t + m * 64 + lane);
            rjv[u] = *(const float4 *)(r + (J0 + u) * TILE + c4);
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (u >= cn) break;
          item_tile_f32(v[u], rjv[u], rI, acc, J0 + u != I, colp(J0 + u), lane);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float a = acc[m];
      a += __shfl_xor(a, 1, 64);
      a += __shfl_xor(a, 2, 64);
      a += __shfl_xor(a, 4, 64);
      acc[m] = a;
    }
    if ((lane & 7) == 0) {
      float *rowp = (float *)S.rowpart + (int64_t)it.slot * TILE;
#pragma unroll
      for (int m = 0; m < 4; ++m) rowp[8 * m + grp] = acc[m];
    }
  }
}

// Work items only, one per wavefront (CH: tiles loaded together, see items_f32).
template <int CH>
__global__ __launch_bounds__(256) void k_gemv_f32(const Seg *__restrict__ segs, int nseg, int total,
                                                  const int *__restrict__ done, PcgCheck ck) {
  __shared__ double red[256 / WAVE];
  if (done && *done) return;
  if (carried_check<256>(ck, red)) return;
  items_f32<CH>(segs, nseg, total, blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4);
}

// Workgroups [0, nwhole) solve whole systems (wsegs: begin offsets in systems),
// the others take the work items (segs), NW wavefronts per workgroup.
template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_gemv_whole_f32(const Seg *__restrict__ segs, int nseg,
                                                                 int total, const Seg *__restrict__ wsegs,
                                                                 int nwhole, const int *__restrict__ done,
                                                                 const double *__restrict__ gin, PcgCheck ck) {
  extern __shared__ float ys_whole[];
  __shared__ double red[NW];
  if (done && *done) return;
  if (carried_check<NW * WAVE>(ck, red)) return;
  if ((int)blockIdx.x < nwhole) {
    const Seg &sg = seg_of(wsegs, nseg, blockIdx.x);
    if (sg.done && *sg.done) return;
    whole_f32<NW>(sg.sys[sg.whole[blockIdx.x - sg.begin]], ys_whole, gin);
    return;
  }
  items_f32<1>(segs, nseg, total, (blockIdx.x - nwhole) * NW + (threadIdx.x >> 6),
            (gridDim.x - nwhole) * NW);
}

// FP16 tiles (the inverse divided by a power-of-two scale per system, so every
// entry is at most 2^14), FP32 arithmetic: 2 loads of 16 bytes per lane per tile;
// lane l holds rows 16m + l/4 (m < 2), columns 8(l%4) .. 8(l%4)+7. The row and
// column sums are multiplied back by the scale when written.
typedef _Float16 nt_h8 __attribute__((ext_vector_type(8)));

// DPP lane moves inside rows of 16 lanes (no LDS permute); lanes with no source read 0.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
// every lane of each group of 4 receives the group's sum, (v0 + v1) + (v2 + v3)
__device__ __forceinline__ float quad_sum(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  return v;
}

// FP16 tiles, whole systems (lane layout of k_gemv_f16 below: 2 rows x 8 columns
// per lane). Here the triangle is walked by column strips instead of tile rows: a
// lane's 8 columns need a sum over 16 lane groups, its 2 rows over only 4 lanes,
// so the transposed contribution is kept per lane down the whole strip (summed
// across lanes once per strip) and the per-tile cross-lane work is the short row
// sum. The waves take the strips, longest first, in the snake order.
// A 2 KB tile is a small load per wavefront, so two tiles are kept in flight
// while a third is used: three register buffers in a fixed rotation (the loop
// body is unrolled three times, so no loaded register is ever copied, which
// would wait for its load). The main loop issues its loads unconditionally (the
// last tiles of the walk are handled after it), so that the compiler's count of
// loads in flight stays exact and a tile's use waits for that tile alone.
template <int NW>
__device__ __forceinline__ void whole_f16(const SysDev &S, float *ys, const double *__restrict__ gin) {
  const float *r;
  float *y = whole_begin<NW>(S, ys, gin, r);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane >> 2, c8 = (lane & 3) * 8;
  const int nb = S.nb;
  const nt_h8 *__restrict__ base = (const nt_h8 *)S.tiles;
  // the wavefront's column strips, longest first in a snake order over the waves:
  // strip J holds tiles (I, J), I = J .. nb-1
  auto strip = [&](int k) {
    const int p = k * NW + ((k & 1) ? NW - 1 - w : w);
    return p < nb ? p : -1;
  };
  int T = 0;
  for (int k = 0;; ++k) {
    const int J = strip(k);
    if (J < 0) break;
    T += nb - J;
  }
  if (T == 0) {
    whole_finish<NW>(S, ys, (double)S.scale);
    return;
  }
  // position after (k, I, J) in the wavefront's walk (J < 0: none)
  auto next = [&](int &k, int &I, int &J) {
    if (J < 0) return;
    if (++I >= nb) {
      J = strip(++k);
      I = J;
    }
  };
  auto load = [&](int ti, int tj, nt_h8 *dst) {
    const nt_h8 *t = base + ((int64_t)ti * (ti + 1) / 2 + tj) * (TILE * TILE / 8);
#pragma unroll
    for (int m = 0; m < 2; ++m) dst[m] = ldnt_global(t + m * 64 + lane);
  };
  // positions of the tiles t (in use), t + 1 and t + 2 (in flight)
  int k0 = 0, J0 = strip(0), I0 = J0;
  int k1 = k0, I1 = I0, J1 = J0;
  next(k1, I1, J1);
  int k2 = k1, I2 = I1, J2 = J1;
  next(k2, I2, J2);
  // all three buffers are loaded whatever T (a short walk loads its first tile
  // again), so that every path into the loop has issued the same loads
  nt_h8 va[2], vb[2], vc[2];
  load(I0, J0, va);
  load(T > 1 ? I1 : I0, T > 1 ? J1 : J0, vb);
  load(T > 2 ? I2 : I0, T > 2 ? J2 : J0, vc);
  float rj[8], c[8];
  auto load_rj = [&](int J) {
    const float4 ra = *(const float4 *)(r + J * TILE + c8);
    const float4 rb = *(const float4 *)(r + J * TILE + c8 + 4);
    const float t8[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) rj[e] = t8[e];
  };
  load_rj(J0);
#pragma unroll
  for (int e = 0; e < 8; ++e) c[e] = 0.0f;
  int t = 0;
  // uses the tile (I0, J0) held in v, then (refill) loads into v the tile three
  // positions ahead, and advances
  auto step = [&](nt_h8 *v, bool refill) {
    float rI[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) rI[m] = r[I0 * TILE + 16 * m + grp];
    // row contribution of tile (I0, J0): summed over the 4 lanes of a row group
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float a = 0.0f;
#pragma unroll
      for (int e = 0; e < 8; ++e) a += (float)v[m][e] * rj[e];
      a = quad_sum(a);
      if ((lane & 3) == 0) y[I0 * TILE + 16 * m + grp] += a;
    }
    // transposed contribution, kept per lane down the strip
    if (I0 != J0) {
#pragma unroll
      for (int e = 0; e < 8; ++e) c[e] += (float)v[0][e] * rI[0] + (float)v[1][e] * rI[1];
    }
    if (J1 != J0) {
      // strip J0 complete
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float a = c[e];
        a += __shfl_xor(a, 4, 64);
        a += __shfl_xor(a, 8, 64);
        a += __shfl_xor(a, 16, 64);
        a += __shfl_xor(a, 32, 64);
        c[e] = 0.0f;
        if (lane < 4) y[J0 * TILE + c8 + e] += a;
      }
      if (J1 >= 0) load_rj(J1);
    }
    int k3 = k2, I3 = I2, J3 = J2;
    next(k3, I3, J3);
    if (refill) load(I3, J3, v);
    k0 = k1, I0 = I1, J0 = J1;
    k1 = k2, I1 = I2, J1 = J2;
    k2 = k3, I2 = I3, J2 = J3;
    ++t;
  };
  while (t + 5 < T) {
    step(va, true);
    step(vb, true);
    step(vc, true);
  }
  // at most five tiles left: t, t + 1, t + 2 in va, vb, vc; t + 3 and t + 4
  // loaded into va and vb by the first two steps
  if (t < T) step(va, t + 3 < T);
  if (t < T) step(vb, t + 3 < T);
  if (t < T) step(vc, false);
  if (t < T) step(va, false);
  if (t < T) step(vb, false);
  // the tiles hold A_s^{-1} / scale
  whole_finish<NW>(S, ys, (double)S.scale);
}


// One tile (I, J) of a work item, FP16 storage: as item_tile_f32, the tile
// scaled by the system's power of two.
__device__ __forceinline__ void item_tile_f16(const nt_h8 (&v)[2], const float4 &ra, const float4 &rb,
                                              const float (&rI)[2], float (&acc)[2], bool offdiag, float scale,
                                              float *__restrict__ colp, int lane) {
  const float rj[8] = {ra.x, ra.y, ra.z, ra.w, rb.x, rb.y, rb.z, rb.w};
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[m] = fmaf((float)v[m][k], rj[k], acc[m]);
  if (offdiag) {
    float c[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = fmaf((float)v[1][k], rI[1], (float)v[0][k] * rI[0]);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      c[k] += __shfl_xor(c[k], 4, 64);
      c[k] += __shfl_xor(c[k], 8, 64);
      c[k] += __shfl_xor(c[k], 16, 64);
      c[k] += __shfl_xor(c[k], 32, 64);
    }
    if (lane < 4) {
      float4 o0, o1;
      o0.x = c[0] * scale;
      o0.y = c[1] * scale;
      o0.z = c[2] * scale;
      o0.w = c[3] * scale;
      o1.x = c[4] * scale;
      o1.y = c[5] * scale;
      o1.z = c[6] * scale;
      o1.w = c[7] * scale;
      *(float4 *)colp = o0;
      *(float4 *)(colp + 4) = o1;
    }
  }
}

// Work items of FP16 tiles, as for FP32 (CH = 1: streamed, else in chunks).
template <int CH>
__device__ __forceinline__ void items_f16(const Seg *__restrict__ segs, int nseg, int total, int g0,
                                          int gstride) {
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 2, c8 = (lane & 3) * 8;
  for (int g = g0; g < total; g += gstride) {
    const Seg sg = segs[nseg == 1 ? 0 : find_seg(segs, nseg, g)];
    if (sg.done && *sg.done) continue;
    const GItem it = sg.items[g - sg.begin];
    const SysDev S = sg.sys[it.sys];
    const float *__restrict__ r = (const float *)S.rp;
    const int I = it.I;
    const int64_t rowbase = (int64_t)I * (I + 1) / 2;
    const nt_h8 *__restrict__ t0 = (const nt_h8 *)((const _Float16 *)S.tiles + (rowbase + it.j0) * (TILE * TILE));
    float rI[2], acc[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      rI[m] = r[I * TILE + 16 * m + grp];
      acc[m] = 0.0f;
    }
    auto colp = [&](int J) { return (float *)S.colpart + (rowbase + J) * TILE + c8; };
    if constexpr (CH == 1) {
      nt_h8 v[2], w[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) v[m] = ldnt_global(t0 + m * 64 + lane);
      const nt_h8 *t = t0;
      for (int J = it.j0; J < it.j1; ++J) {
        const bool more = J + 1 < it.j1;
        t += TILE * TILE / 8;
        if (more) {
#pragma unroll
          for (int m = 0; m < 2; ++m) w[m] = ldnt_global(t + m * 64 + lane);
        }
        const float4 ra = *(const float4 *)(r + J * TILE + c8);
        const float4 rb = *(const float4 *)(r + J * TILE + c8 + 4);
        item_tile_f16(v, ra, rb, rI, acc, J != I, S.scale, colp(J), lane);
        if (more) {
#pragma unroll
          for (int m = 0; m < 2; ++m) v[m] = w[m];
        }
      }
    } else {
      for (int J0 = it.j0; J0 < it.j1; J0 += CH) {
        const int cn = it.j1 - J0 < CH ? it.j1 - J0 : CH;
        nt_h8 v[CH][2];
        float4 ra[CH], rb[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (u < cn) {
            const nt_h8 *t = t0 + (int64_t)(J0 - it.j0 + u) * (TILE * TILE / 8);
#pragma unroll
            for (int m = 0; m < 2; ++m) v[u][m] = ldnt_global(t + m * 64 + lane);
            ra[u] = *(const float4 *)(r + (J0 + u) * TILE + c8);
            rb[u] = *(const float4 *)(r + (J0 + u) * TILE + c8 + 4);
          }
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          if (u >= cn) break;
          item_tile_f16(v[u], ra[u], rb[u], rI, acc, J0 + u != I, S.scale, colp(J0 + u), lane);
        }
      }
    }
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      float a = acc[m];
      a += __shfl_xor(a, 1, 64);
      a += __shfl_xor(a, 2, 64);
      acc[m] = a * S.scale;
    }
    if ((lane & 3) == 0) {
      float *rowp = (float *)S.rowpart + (int64_t)it.slot * TILE;
#pragma unroll
      for (int m = 0; m < 2; ++m) rowp[16 * m + grp] = acc[m];
    }
  }
}

// Work items only, one per wavefront (CH: tiles loaded together, see items_f32).
template <int CH>
__global__ __launch_bounds__(256) void k_gemv_f16(const Seg *__restrict__ segs, int nseg, int total,
                                                  const int *__restrict__ done, PcgCheck ck) {
  __shared__ double red[256 / WAVE];
  if (done && *done) return;
  if (carried_check<256>(ck, red)) return;
  items_f16<CH>(segs, nseg, total, blockIdx.x * 4 + (threadIdx.x >> 6), gridDim.x * 4);
}

// Workgroups [0, nwhole) solve whole systems (wsegs: begin offsets in systems),
// the others take the work items (segs), NW wavefronts per workgroup.
template <int NW>
__global__ __launch_bounds__(NW * WAVE) void k_gemv_whole_f16(const Seg *__restrict__ segs, int nseg,
                                                                 int total, const Seg *__restrict__ wsegs,
                                                                 int nwhole, const int *__restrict__ done,
                                                                 const double *__restrict__ gin, PcgCheck ck) {
  extern __shared__ float ys_whole[];
  __shared__ double red[NW];
  if (done && *done) return;
  if (carried_check<NW * WAVE>(ck, red)) return;
  if ((int)blockIdx.x < nwhole) {
    const Seg &sg = seg_of(wsegs, nseg, blockIdx.x);
    if (sg.done && *sg.done) return;
    whole_f16<NW>(sg.sys[sg.whole[blockIdx.x - sg.begin]], ys_whole, gin);
    return;
  }
  items_f16<1>(segs, nseg, total, (blockIdx.x - nwhole) * NW + (threadIdx.x >> 6),
            (gridDim.x - nwhole) * NW);
}

// z_s[I*TILE + c] = sum of the row partials of tile row I + sum over I' > I of
// the transposed partials of tile (I', I).
template <typename T>
__global__ __launch_bounds__(256) void k_combine(const Seg *__restrict__ segs, int nseg, int total,
                                                 const int *__restrict__ done) {
  if (done && *done) return;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int g = (int)(gid / TILE), c = (int)(gid % TILE);
  if (g >= total) return;
  const Seg sg = segs[nseg == 1 ? 0 : find_seg(segs, nseg, g)];
  if (sg.done && *sg.done) return;
  const GRow rw = sg.rows[g - sg.begin];
  const SysDev S = sg.sys[rw.sys];
  const T *rowp = (const T *)S.rowpart;
  const T *colp = (const T *)S.colpart;
  double acc = 0.0;
  for (int k = 0; k < rw.nslot; ++k) acc += (double)rowp[(int64_t)(rw.slot0 + k) * TILE + c];
  // column partials of tiles (I2, I), I2 > I: loads issued four at a time, summed in order
  for (int I2 = rw.I + 1; I2 < S.nb; I2 += 4) {
    T v[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
      v[m] = (I2 + m < S.nb) ? colp[((int64_t)(I2 + m) * (I2 + m + 1) / 2 + rw.I) * TILE + c] : T(0);
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (I2 + m < S.nb) acc += (double)v[m];
  }
  S.zp[rw.I * TILE + c] = acc;
  // the reduced solution is also scattered onto the full box-vertex grid
  if (S.yfull) {
    const int K = rw.I * TILE + c;
    if (K < S.n) S.yfull[S.act_bv[K]] = acc;
  }
}

// ---------------------------------------------------------------------------
// Final step of one preconditioner application, per free vertex i:
//   out_i = add_i + sum_{(p,a) covering i} z_p[a]             (local part)
//               + sum_c f_ic sum_k Phi_k(xi_ic) y_r[corner]  (J y_r, Sec. 4)
// plus partial sums of r.out and r.out_old for the PCG beta.
// The loads of a vertex go out in three rounds, each issued together: its list
// bounds (cover and J pointers) with r_i (and out_i, add_i); the positions of
// its first eight local solutions with its first J entry; then those solutions
// and the entry's eight box-grid corners. Further entries (more than eight
// covering subdomains, more than one cell) are walked one by one. With LY the
// reduced solution on the box grid (n_bv doubles) is first staged in LDS and the
// corner gathers read LDS. The sums run in the same order either way: the local
// solutions in list order, then the J entries in list order.
// ---------------------------------------------------------------------------
template <bool LY>
__device__ __forceinline__ double y_at(const double *__restrict__ yfull, const double *ly, int64_t b) {
  if constexpr (LY)
    return ly[b];
  else
    return yfull[b];
}

template <typename T, bool LY>
__device__ __forceinline__ void final_body(int64_t nf, const int *__restrict__ done, const double *__restrict__ add,
                                           const int32_t *__restrict__ cover_ptr,
                                           const int32_t *__restrict__ cover_pos, const double *__restrict__ zp,
                                           const int32_t *__restrict__ jv_ptr, const int32_t *__restrict__ jv_base,
                                           const T *__restrict__ jv_w, const T *__restrict__ jv_xi, int64_t nent,
                                           int bx1, int bxy1, const double *__restrict__ yfull, int n_bv, double *ly,
                                           double *__restrict__ out, const double *__restrict__ rdot,
                                           double *__restrict__ part1, double *__restrict__ part2,
                                           Scalars *__restrict__ sc, int start, int blk, int nblk, double *red) {
  if (*done) return;
  if constexpr (LY) {
    // eight loads per thread in flight, then their LDS stores
    for (int t0 = threadIdx.x; t0 < n_bv; t0 += 8 * VW) {
      double v[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) v[m] = (t0 + m * VW < n_bv) ? yfull[t0 + m * VW] : 0.0;
#pragma unroll
      for (int m = 0; m < 8; ++m)
        if (t0 + m * VW < n_bv) ly[t0 + m * VW] = v[m];
    }
    __syncthreads();
  }
  double d1 = 0.0, d2 = 0.0;
  const int64_t G = (int64_t)nblk * VW;
  for (int64_t i = blk * (int64_t)VW + threadIdx.x; i < nf; i += G) {
    // round 1: list bounds and the per-vertex values
    int c0 = 0, c1 = 0, j0 = 0, j1 = 0;
    if (cover_ptr) {
      c0 = cover_ptr[i];
      c1 = cover_ptr[i + 1];
    }
    if (jv_ptr) {
      j0 = jv_ptr[i];
      j1 = jv_ptr[i + 1];
    }
    const double ad = add ? add[i] : 0.0;
    double ri = 0.0, zo = 0.0;
    if (rdot) {
      ri = rdot[i];
      if (part2) zo = out[i];
    }
    // round 2: positions of the first eight local solutions; the first J entry
    constexpr int NC = 8;
    int pos[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) pos[m] = (c0 + m < c1) ? cover_pos[c0 + m] : -1;
    const bool hj = j0 < j1;
    int b0 = 0;
    T w0 = T(0), x0 = T(0), y0 = T(0), z0 = T(0);
    if (hj) {
      b0 = jv_base[j0];
      w0 = jv_w[j0];
      x0 = jv_xi[j0];
      y0 = jv_xi[nent + j0];
      z0 = jv_xi[2 * nent + j0];
    }
    // round 3: the local solutions and the entry's box-grid corners
    double v[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) v[m] = (pos[m] >= 0) ? zp[pos[m]] : 0.0;
    double yc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      yc[q] = hj ? y_at<LY>(yfull, ly, b0 + (q & 1) + ((q >> 1) & 1) * bx1 + ((q >> 2) & 1) * bxy1) : 0.0;
    double acc = ad;
#pragma unroll
    for (int m = 0; m < NC; ++m)
      if (pos[m] >= 0) acc += v[m];
    // further covering subdomains (more than eight: two or more layers of overlap)
    for (int k = c0 + NC; k < c1; ++k) acc += zp[cover_pos[k]];
    if (jv_ptr) {
      // J y_r: the corners of the entry's cell are box vertices base + {0,1} +
      // bx1 {0,1} + bxy1 {0,1} of the full grid (inactive ones hold 0)
      T cs = T(0);
      if (hj) {
        T sv = T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) sv += trilin<T>(q, x0, y0, z0) * (T)yc[q];
        cs += w0 * sv;
      }
      for (int k = j0 + 1; k < j1; ++k) {
        const int bk = jv_base[k];
        const T x = jv_xi[k], y = jv_xi[nent + k], z = jv_xi[2 * nent + k];
        double yk[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) yk[q] = y_at<LY>(yfull, ly, bk + (q & 1) + ((q >> 1) & 1) * bx1 + ((q >> 2) & 1) * bxy1);
        T sv = T(0);
#pragma unroll
        for (int q = 0; q < 8; ++q) sv += trilin<T>(q, x, y, z) * (T)yk[q];
        cs += jv_w[k] * sv;
      }
      acc += (double)cs;
    }
    if (rdot) {
      if (part2) d2 += ri * zo;
      d1 += ri * acc;
    }
    out[i] = acc;
  }
  if (rdot) {
    const double s1 = block_sum<VW>(d1, red);
    if (threadIdx.x == 0) part1[blk] = s1;
    if (part2) {
      const double s2 = block_sum<VW>(d2, red);
      if (threadIdx.x == 0) part2[blk] = s2;
    }
    // one completed iteration (not for the first application)
    if (sc && !start && blk == 0 && threadIdx.x == 0) sc->iter = sc->iter + 1;
  }
}

// y_lds = 1: stage the reduced solution (n_bv doubles of dynamic LDS). Held to
// the register budget of eight wavefronts per SIMD, so that four workgroups fit
// a compute unit and the 1024-workgroup grid runs in one round (its many pointer
// arguments otherwise take more scalar registers than eight waves allow).
template <typename T>
__global__ __launch_bounds__(VW) __attribute__((amdgpu_waves_per_eu(8))) void k_final(int64_t nf, const int *__restrict__ done, const double *__restrict__ add,
                                              const int32_t *__restrict__ cover_ptr,
                                              const int32_t *__restrict__ cover_pos, const double *__restrict__ zp,
                                              const int32_t *__restrict__ jv_ptr, const int32_t *__restrict__ jv_base,
                                              const T *__restrict__ jv_w, const T *__restrict__ jv_xi, int64_t nent,
                                              int bx1, int bxy1, const double *__restrict__ yfull, int n_bv, int y_lds,
                                              double *__restrict__ out, const double *__restrict__ rdot,
                                              double *__restrict__ part1, double *__restrict__ part2,
                                              Scalars *__restrict__ sc, int start) {
  extern __shared__ double ly[];
  __shared__ double red[VW / WAVE];
  if (y_lds && jv_ptr)
    final_body<T, true>(nf, done, add, cover_ptr, cover_pos, zp, jv_ptr, jv_base, jv_w, jv_xi, nent, bx1, bxy1,
                        yfull, n_bv, ly, out, rdot, part1, part2, sc, start, blockIdx.x, gridDim.x, red);
  else
    final_body<T, false>(nf, done, add, cover_ptr, cover_pos, zp, jv_ptr, jv_base, jv_w, jv_xi, nent, bx1, bxy1,
                         yfull, n_bv, nullptr, out, rdot, part1, part2, sc, start, blockIdx.x, gridDim.x, red);
}

// ---------------------------------------------------------------------------
// One PCG iteration of every solve of a lock-step batch in one launch per step:
// workgroup g of a grouped launch belongs to the solve c with
// off[c] <= g < off[c + 1] and runs as workgroup g - off[c] of that solve's own
// launch (same grid per solve, same partial sums, so each result is bitwise the
// solo one). The dense solves of the batch are already one launch (k_gemv_*).
// ---------------------------------------------------------------------------
// The solver state of every solve of a batch in one array, for one
// device-to-host transfer per lock step.
__global__ __launch_bounds__(64) void k_gather_scalars(const IterDev *__restrict__ ctx, int n,
                                                       Scalars *__restrict__ out) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i < n) out[i] = *ctx[i].sc;
}

__device__ __forceinline__ int find_ctx(const int32_t *__restrict__ off, int n, int g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(OP_BLOCK) void k_op_fused_grp(const IterDev *__restrict__ ctx,
                                                           const int32_t *__restrict__ off, int n) {
  extern __shared__ double lds[];
  __shared__ double red[OP_BLOCK / WAVE];
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  op_fused_body(d.op, d.z, d.pa, d.pb, d.q, d.energy, d.sc, d.part1, d.part2, d.nvblk, blockIdx.x - off[c], lds, red);
}

__global__ __launch_bounds__(VW) void k_update_fused_grp(const IterDev *__restrict__ ctx,
                                                         const int32_t *__restrict__ off, int n) {
  __shared__ double red[VW / WAVE];
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  update_fused_body(d.nf, d.op, d.sc, d.x, d.r, d.pa, d.pb, d.q, d.energy, (int)d.op.n_blocks, d.prr,
                    blockIdx.x - off[c], off[c + 1] - off[c], red);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pre_grp(const IterDev *__restrict__ ctx, const int32_t *__restrict__ off,
                                                 int n) {
  __shared__ double red[256 / WAVE];
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  pre_body<T>(d.ng, d.n_pack, &d.sc->done, d.sub_idx, d.r, (T *)d.rp, d.ntask, d.jt_start, d.jc_vid,
              (const T *)d.jc_w, (const T *)d.jc_xi, d.nent, (T *)d.jt_part, d.sc, d.prr, d.nvblk, 0,
              blockIdx.x - off[c], off[c + 1] - off[c], red);
}

template <typename T>
__global__ __launch_bounds__(256) void k_jt_corners_grp(const IterDev *__restrict__ ctx,
                                                        const int32_t *__restrict__ off, int n) {
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  corners_body<T>(d.n_r, &d.sc->done, d.jr_ptr, d.jr_src, (const T *)d.jt_part, (T *)d.rp + d.n_pack,
                  blockIdx.x - off[c]);
}

template <typename T>
__global__ __launch_bounds__(VW) void k_final_grp(const IterDev *__restrict__ ctx, const int32_t *__restrict__ off,
                                                  int n) {
  extern __shared__ double ly[];
  __shared__ double red[VW / WAVE];
  const int c = find_ctx(off, n, blockIdx.x);
  const IterDev &d = ctx[c];
  if (d.y_lds)
    final_body<T, true>(d.nf, &d.sc->done, nullptr, d.cover_ptr, d.cover_pos, d.zp, d.jv_ptr, d.jv_base,
                        (const T *)d.jv_w, (const T *)d.jv_xi, d.nent, d.bx1, d.bxy1, d.yfull, d.n_bv, ly, d.z, d.r,
                        d.part1, d.flexible ? d.part2 : nullptr, d.sc, 0, blockIdx.x - off[c],
                        off[c + 1] - off[c], red);
  else
    final_body<T, false>(d.nf, &d.sc->done, nullptr, d.cover_ptr, d.cover_pos, d.zp, d.jv_ptr, d.jv_base,
                         (const T *)d.jv_w, (const T *)d.jv_xi, d.nent, d.bx1, d.bxy1, d.yfull, d.n_bv, nullptr,
                         d.z, d.r, d.part1, d.flexible ? d.part2 : nullptr, d.sc, 0, blockIdx.x - off[c],
                         off[c + 1] - off[c], red);
}

// ---------------------------------------------------------------------------
// Setup: dense assembly of the local systems A_p = R_p A R_p^T (Sec. 3) into
// lower-tile storage. Every element containing a vertex of R_p belongs to the
// overlapping subdomain, so row a of A_p is the sum over the elements incident
// to vertex R_p[a] of their element-matrix rows, restricted to columns in R_p.
// One workgroup per system, one thread per row (fixed order, no atomics).
// ---------------------------------------------------------------------------
struct AsmSys {
  int64_t tile_off;   // offset (tiles) in the scratch store
  int32_t vec_off;    // offset of R_p in sub_idx
  int32_t n, nb, pad;
};

__device__ __forceinline__ double *tile_elem(double *M, int64_t tile_off, int i, int j) {
  const int I = i / TILE, J = j / TILE;
  return M + (tile_off + (int64_t)I * (I + 1) / 2 + J) * (TILE * TILE) + (i % TILE) * TILE + (j % TILE);
}

// lds_n > 0: R_p (at most lds_n entries) is staged in dynamic LDS for the searches.
__global__ __launch_bounds__(256) void k_assemble_local(const AsmSys *__restrict__ sys, const int32_t *__restrict__ sub_idx,
                                                        const int32_t *__restrict__ vinc_ptr, const int32_t *__restrict__ vinc,
                                                        const int32_t *__restrict__ e2v, int64_t E, int64_t nf,
                                                        const double *__restrict__ Ae, double *__restrict__ M,
                                                        int lds_n) {
  extern __shared__ int32_t lrs[];
  const AsmSys S = sys[blockIdx.x];
  const int32_t *R = sub_idx + S.vec_off;
  if (lds_n > 0) {
    for (int a = threadIdx.x; a < S.n; a += blockDim.x) lrs[a] = R[a];
    __syncthreads();
    R = lrs;
  }
  for (int a = threadIdx.x; a < S.n; a += blockDim.x) {
    const int32_t v = R[a];
    for (int k = vinc_ptr[v]; k < vinc_ptr[v + 1]; ++k) {
      const int64_t e = vinc[k] >> 3;
      const int la = vinc[k] & 7;
#pragma unroll
      for (int lb = 0; lb < 8; ++lb) {
        const int32_t u = e2v[lb * E + e];
        if (u >= nf) continue;
        int lo = 0, hi = S.n - 1, pos = -1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int32_t x = R[mid];
          if (x == u) {
            pos = mid;
            break;
          }
          if (x < u)
            lo = mid + 1;
          else
            hi = mid - 1;
        }
        if (pos < 0 || pos / TILE > a / TILE) continue;   // lower tiles only (diagonal tiles full)
        *tile_elem(M, S.tile_off, a, pos) += Ae[ae_at(sym8(la, lb), e)];
      }
    }
  }
}

// Identity on the padding rows of each system (so padded systems stay SPD).
__global__ void k_pad_identity(const AsmSys *__restrict__ sys, int nsys, double *__restrict__ M) {
  const int s = blockIdx.x;
  if (s >= nsys) return;
  const AsmSys S = sys[s];
  for (int i = S.n + threadIdx.x; i < S.nb * TILE; i += blockDim.x) *tile_elem(M, S.tile_off, i, i) = 1.0;
}

// ---------------------------------------------------------------------------
// Setup: reduced operator by cell assembly, eq. (Aij): for each occupied cell,
// A_cell = sum over its elements of (J^e)^T A^e J^e, J^e[a][k] = Phi_k(xi_a) with
// xi_a the local coordinates of element vertex a in the cell (zero rows at
// Dirichlet vertices). One workgroup per cell of CM_SLOTS wavefronts: slot g
// (one wavefront, thread (a, l) of the 8 x 8 products) takes the cell's
// elements g, g + CM_SLOTS, ... in order, and the slots' sums are added in slot
// order at the end.
// ---------------------------------------------------------------------------
constexpr int CM_SLOTS = 8;
struct BoxDev {
  double lo[3], H[3];
  int32_t b[3], pad;
};

__global__ __launch_bounds__(64 * CM_SLOTS) void k_cell_mats(BoxDev box, const int32_t *__restrict__ occ_cells,
                                                             const int32_t *__restrict__ occ_ptr,
                                                             const int32_t *__restrict__ occ_elems,
                                                             const int32_t *__restrict__ e2v, int64_t E, int64_t NV,
                                                             int64_t nf, const double *__restrict__ xyz,
                                                             const double *__restrict__ Ae,
                                                             double *__restrict__ cellmat) {
  __shared__ double Je[CM_SLOTS][8][8], T1[CM_SLOTS][8][8], part[CM_SLOTS][64];
  const int o = blockIdx.x;
  const int c = occ_cells[o];
  const int c3[3] = {c % box.b[0], (c / box.b[0]) % box.b[1], c / (box.b[0] * box.b[1])};
  const int g = threadIdx.x / 64, t = threadIdx.x % 64, ta = t >> 3, tk = t & 7;
  const int k0 = occ_ptr[o], ne = occ_ptr[o + 1] - k0;
  double acc = 0.0;
  for (int r = 0; r * CM_SLOTS < ne; ++r) {
    const int kk = r * CM_SLOTS + g;
    const bool has = kk < ne;
    const int64_t e = has ? occ_elems[k0 + kk] : 0;
    double ae[8];
    if (has) {
#pragma unroll
      for (int b = 0; b < 8; ++b) ae[b] = Ae[ae_at(sym8(ta, b), e)];
      const int32_t u = e2v[ta * E + e];
      double w = 0.0;
      if (u < nf) {
        double xi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) xi[d] = ((xyz[d * NV + u] - box.lo[d]) - (double)c3[d] * box.H[d]) / box.H[d];
        w = trilin<double>(tk, xi[0], xi[1], xi[2]);
      }
      Je[g][ta][tk] = w;
    }
    __syncthreads();
    if (has) {  // T1 = A^e J^e : thread (a, l)
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 8; ++b) s += ae[b] * Je[g][b][tk];
      T1[g][ta][tk] = s;
    }
    __syncthreads();
    if (has) {  // (J^e)^T T1 : thread (k, l) = (ta, tk)
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < 8; ++a) s += Je[g][a][ta] * T1[g][a][tk];
      acc += s;
    }
    __syncthreads();
  }
  part[g][t] = acc;
  __syncthreads();
  if (g == 0) {
    double sum = 0.0;
#pragma unroll
    for (int h = 0; h < CM_SLOTS; ++h) sum += part[h][t];
    cellmat[(int64_t)o * 64 + t] = sum;
  }
}

// Dense A_r from the cell matrices: row K sums, over the occupied cells around
// box vertex K, that cell's row for K restricted to active corners.
__global__ __launch_bounds__(256) void k_assemble_reduced(int64_t nr, const int32_t *__restrict__ ar_ptr,
                                                          const int32_t *__restrict__ ar_src,
                                                          const int32_t *__restrict__ corner_act,
                                                          const double *__restrict__ cellmat, double *__restrict__ M) {
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  for (int k = ar_ptr[K]; k < ar_ptr[K + 1]; ++k) {
    const int o = ar_src[k] >> 3, q = ar_src[k] & 7;
#pragma unroll
    for (int l = 0; l < 8; ++l) {
      const int32_t L = corner_act[8 * o + l];
      if (L < 0 || L / TILE > K / TILE) continue;
      *tile_elem(M, 0, (int)K, L) += cellmat[(int64_t)o * 64 + q * 8 + l];
    }
  }
}

// ---------------------------------------------------------------------------
// Setup, standard interpolation (Sec. 4, eq. (Psi)): the Galerkin reduced
// operator A_r = J^T A J, one probe per class of box vertices congruent modulo
// (px, py, pz). A probe is v = J sum_{L in class} e_L; then A v and J^T A v come
// from the solve's own kernels, and entry K of the result is A_r[K, L] for the
// one L of the class within reach of K (the classes are spaced so that no two of
// them reach the same K).
// ---------------------------------------------------------------------------
struct ProbeDev {
  int32_t p[3], d[3], c[3], b[3];
  int32_t bx1, bxy1;
};

// v_i = phi_q(xi_i) for the corner q of vertex i's cell that lies in the class
// (at most one: a cell's corners differ by 1 per direction), else 0
__global__ __launch_bounds__(256) void k_probe_vec(int64_t nf, ProbeDev pr, const int32_t *__restrict__ jv_ptr,
                                                   const int32_t *__restrict__ jv_base, const double *__restrict__ jv_xi,
                                                   int64_t nent, double *__restrict__ v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nf) return;
  double out = 0.0;
  const int k = jv_ptr[i];
  if (k < jv_ptr[i + 1]) {
    const int32_t g = jv_base[k];
    const int32_t g3[3] = {g % pr.bx1, (g / pr.bx1) % (pr.bxy1 / pr.bx1), g / pr.bxy1};
    int q = 0;
    bool in = true;
    for (int d = 0; d < 3; ++d) {
      const int r = ((pr.c[d] - g3[d]) % pr.p[d] + pr.p[d]) % pr.p[d];
      if (r > 1) in = false;
      q |= (r & 1) << d;
    }
    if (in) out = trilin<double>(q, jv_xi[k], jv_xi[nent + k], jv_xi[2 * nent + k]);
  }
  v[i] = out;
}

// A_r[K, L] = rr[K] for the class member L within reach of K, stored when it
// falls in a lower tile of the dense reduced system
__global__ __launch_bounds__(256) void k_probe_scatter(int64_t nr, ProbeDev pr, const int32_t *__restrict__ act_bv,
                                                       const int32_t *__restrict__ bv_act, const double *__restrict__ rr,
                                                       double *__restrict__ M) {
  const int64_t K = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (K >= nr) return;
  const int32_t g = act_bv[K];
  const int32_t g3[3] = {g % pr.bx1, (g / pr.bx1) % (pr.bxy1 / pr.bx1), g / pr.bxy1};
  int32_t l3[3];
  for (int d = 0; d < 3; ++d) {
    // the class member nearest K in this direction: offset r or r - p, whichever
    // is within reach and on the grid (a period of b + 1 leaves one member)
    const int r = ((pr.c[d] - g3[d]) % pr.p[d] + pr.p[d]) % pr.p[d];
    const bool up = r <= pr.d[d] && g3[d] + r <= pr.b[d];
    const bool down = r - pr.p[d] >= -pr.d[d] && g3[d] + r - pr.p[d] >= 0;
    if (!up && !down) return;
    l3[d] = g3[d] + (up ? r : r - pr.p[d]);
  }
  const int32_t L = bv_act[l3[0] + pr.bx1 * l3[1] + pr.bxy1 * l3[2]];
  if (L < 0 || L / TILE > (int)K / TILE) return;
  *tile_elem(M, 0, (int)K, L) = rr[K];
}

// ---------------------------------------------------------------------------
// Setup: batched inverse of SPD systems by the symmetric block sweep (block
// Gauss-Jordan). Sweeping pivot block k of the current matrix M:
//   D = M_kk^{-1};  M_OO -= M_Ok D M_kO;  M_Ok <- M_Ok D;  M_kO <- D M_kO;
//   M_kk <- -D.
// After every block is swept, M = -A^{-1}. Only lower tiles are stored; the
// step is split into: pivot-block inverse, panel (P_I = M_Ik, G_I = P_I D), and
// the tile update. A non-positive pivot flags the system as not SPD.
// ---------------------------------------------------------------------------
struct SweepSys {
  int64_t tile_off;   // scratch tiles
  int64_t pan_off;    // panel slots (nb per system)
  int32_t nb, pad;
};

__device__ __forceinline__ double *tile_ptr(double *M, int64_t toff, int I, int J) {
  return M + (toff + (int64_t)I * (I + 1) / 2 + J) * (TILE * TILE);
}

// Save the diagonal of the assembled systems (the reference for the relative
// pivot test below).
__global__ __launch_bounds__(256) void k_save_diag(const SweepSys *__restrict__ sys, const double *__restrict__ M,
                                                   double *__restrict__ diag0) {
  const SweepSys S = sys[blockIdx.x];
  for (int i = threadIdx.x; i < S.nb * TILE; i += blockDim.x) {
    const int I = i / TILE;
    diag0[S.pan_off * TILE + i] = M[(S.tile_off + (int64_t)I * (I + 1) / 2 + I) * (TILE * TILE) + (i % TILE) * (TILE + 1)];
  }
}

// A pivot is the diagonal of a Schur complement of the SPD system; it must stay
// positive, and a pivot below PIVOT_RTOL times the original diagonal entry marks
// the system as numerically singular (e.g. the constant null space of an
// all-Neumann reduced operator).
constexpr double PIVOT_RTOL = 1e-13;

// The sweep runs SW tile columns per block step. Step kb sweeps the columns
// K = [k0, k0 + w), k0 = kb SW, w = min(SW, nb - k0), as one block:
//   D = M_KK^{-1};  G_I = M_IK D and P_I = M_IK for the tile rows I outside K;
//   M_IJ -= G_I P_J^T (I, J outside K);  M_IK <- G_I;  M_KK <- -D.
// Sweeping K at once equals sweeping its columns one by one, and every pass
// over the stored tiles does 32 x 32 x 32 w multiply-adds per tile instead of
// 32 x 32 x 32, so the passes over M fall from nb to about nb / SW. The
// pivot-block inverse costs (32 SW)^2 scalar updates per pivot, latency-bound:
// measured at SW = 1, 2 and 4, two tile columns per step gave the fastest
// setups (four halve the passes again but the 128 x 128 inverse costs more than
// that saves).
constexpr int SW = 2;                   // tile columns per block step
constexpr int BW = SW * TILE;           // pivot block edge
constexpr int BH = BW / 2;              // inner-dimension chunk of the update
constexpr int PIV_T = 256;              // threads of the pivot-block inverse
constexpr int PIV_TPR = PIV_T / BW;     // threads per row of the block
constexpr int PIV_EPT = BW / PIV_TPR;   // entries per thread (one row segment)
static_assert(PIV_EPT * PIV_TPR == BW && PIV_T % BW == 0, "pivot block layout");

// 32 x 32 x 32 tile products on the matrix cores: v_mfma_f64_16x16x4f64 takes a
// 16 x 4 block of A (lane l holds A[l%16][l/16]) and a 4 x 16 block of B (lane l
// holds B[l/16][l%16]) and accumulates into a 16 x 16 block of which lane l holds
// rows l/16, l/16 + 4, l/16 + 8 and l/16 + 12 of column l%16.
typedef double v4d __attribute__((ext_vector_type(4)));

// Workgroups are dealt to the 8 XCDs round robin (workgroup b to XCD b % 8):
// with a grid that is a multiple of 8, XCD x gets the contiguous work range
// [x per, (x + 1) per), so the tiles of one system share an L2.
__device__ __forceinline__ int xcd_grouped(int bid, int nblk) {
  const int per = nblk / 8;
  return (bid % 8) * per + bid / 8;
}

// Entry (i, c) of the pivot block M_KK (i, c < 32 w) from the lower tiles.
__device__ __forceinline__ double kblock_at(const double *M, int64_t toff, int k0, int i, int c) {
  const int I = i / TILE, J = c / TILE;
  if (I >= J) return tile_ptr((double *)M, toff, k0 + I, k0 + J)[(i % TILE) * TILE + c % TILE];
  return tile_ptr((double *)M, toff, k0 + J, k0 + I)[(c % TILE) * TILE + i % TILE];
}

// D = M_KK^{-1} by Gauss-Jordan on the 32 w x 32 w block, one workgroup per
// system: thread t holds row t / PIV_TPR, columns PIV_EPT (t % PIV_TPR) onwards,
// in registers; the PIV_TPR threads of a row are neighbouring lanes of one
// wavefront. Per pivot j every thread takes its row's entry in column j from the
// owning lane; row j is scaled by the reciprocal of the pivot and published
// through LDS (buffers alternating between pivots, one barrier per pivot), and
// every other row subtracts its multiple. Each pivot is a diagonal entry of a
// Schur complement of the SPD system and is tested as above.
__global__ __launch_bounds__(PIV_T) void k_bsweep_pivot(int kb, const SweepSys *__restrict__ sys,
                                                        const double *__restrict__ M, double *__restrict__ Dbuf,
                                                        const double *__restrict__ diag0, int *__restrict__ status) {
  static_assert(WAVE % PIV_TPR == 0, "a row's threads share a wavefront");
  __shared__ double rowb[2][BW];
  __shared__ int bad;
  const SweepSys S = sys[blockIdx.x];
  const int k0 = kb * SW;
  if (k0 >= S.nb) return;
  const int n = min(SW, S.nb - k0) * TILE;
  const int i = threadIdx.x / PIV_TPR, c0 = (threadIdx.x % PIV_TPR) * PIV_EPT;
  double a[PIV_EPT];
#pragma unroll
  for (int e = 0; e < PIV_EPT; ++e) {
    const int c = c0 + e;
    a[e] = (i < n && c < n) ? kblock_at(M, S.tile_off, k0, i, c) : (i == c ? 1.0 : 0.0);
  }
  if (threadIdx.x == 0) bad = 0;
  const double *d0 = diag0 + (S.pan_off + k0) * TILE;
  const int lane = threadIdx.x % WAVE, row_lane0 = lane - lane % PIV_TPR;
  __syncthreads();
  for (int j0 = 0; j0 < n; j0 += PIV_EPT) {
    const bool own = (c0 == j0);   // this thread holds columns j0 .. j0 + PIV_EPT - 1
    const int src = row_lane0 + j0 / PIV_EPT;
#pragma unroll
    for (int q = 0; q < PIV_EPT; ++q) {
      const int j = j0 + q, b = j & 1;
      const double f = __shfl(a[q], src, WAVE);   // entry (i, j) of this row
      if (i == j) {
        if (own && (!(f > PIVOT_RTOL * d0[j]) || !isfinite(f))) bad = 1;
        const double rp = 1.0 / f;
#pragma unroll
        for (int e = 0; e < PIV_EPT; ++e) {
          const double v = (own && e == q) ? rp : a[e] * rp;
          a[e] = v;
          rowb[b][c0 + e] = v;
        }
      }
      __syncthreads();
      if (i != j && i < n) {
#pragma unroll
        for (int e = 0; e < PIV_EPT; ++e) a[e] = ((own && e == q) ? 0.0 : a[e]) - f * rowb[b][c0 + e];
      }
    }
  }
  __syncthreads();
  double *out = Dbuf + (int64_t)blockIdx.x * BW * BW + (int64_t)i * BW + c0;
  if (i < n) {
#pragma unroll
    for (int e = 0; e < PIV_EPT; ++e)
      if (c0 + e < n) out[e] = a[e];
  }
  if (threadIdx.x == 0 && bad) status[blockIdx.x] = 1;
}

// grid: 8 ceil(ns maxnb / 8) workgroups over the (system, tile row I) pairs,
// system-major and XCD-grouped. For I outside K: P_I = M_IK (stored tiles
// (I, k0 + j) below K, transposes of (k0 + j, I) above it, each read in its
// stored order) as a 32 x BW row strip, kept, and G_I = P_I D on the matrix
// cores: wavefront v takes the 16-column blocks v and v + 4 for both row halves,
// with the block's D operands (from the L2) loaded into registers first.
__global__ __launch_bounds__(256) void k_bsweep_panel(int kb, int ns, int maxnb, const SweepSys *__restrict__ sys,
                                                      const double *__restrict__ M, const double *__restrict__ Dbuf,
                                                      double *__restrict__ Pbuf, double *__restrict__ Gbuf) {
  __shared__ double Pl[TILE][BW + 1];
  const int q = xcd_grouped((int)blockIdx.x, (int)gridDim.x);
  if (q >= ns * maxnb) return;
  const int s = q / maxnb, I = q % maxnb;
  const SweepSys S = sys[s];
  const int k0 = kb * SW;
  if (k0 >= S.nb || I >= S.nb) return;
  const int w = min(SW, S.nb - k0), n = w * TILE;
  if (I >= k0 && I < k0 + w) return;
  for (int t = threadIdx.x; t < TILE * BW; t += blockDim.x) {
    const int j = t / (TILE * TILE), e = t % (TILE * TILE);
    if (j < w) {
      if (I > k0)
        Pl[e / TILE][j * TILE + e % TILE] = tile_ptr((double *)M, S.tile_off, I, k0 + j)[e];
      else
        Pl[e % TILE][j * TILE + e / TILE] = tile_ptr((double *)M, S.tile_off, k0 + j, I)[e];
    } else {
      Pl[e / TILE][j * TILE + e % TILE] = 0.0;
    }
  }
  __syncthreads();
  double *po = Pbuf + (S.pan_off + I) * (TILE * BW);
  for (int t = threadIdx.x; t < TILE * BW; t += blockDim.x) po[t] = Pl[t / BW][t % BW];
  const double *D = Dbuf + (int64_t)s * BW * BW;
  double *go = Gbuf + (S.pan_off + I) * (TILE * BW);
  const int wv = threadIdx.x / WAVE, l = threadIdx.x % WAVE, cl = l % 16, kq = l / 16;
  const int nst = n / 4;
  for (int cb = wv; cb * 16 < n; cb += 4) {
    double dv[BW / 4];
#pragma unroll
    for (int st = 0; st < BW / 4; ++st) dv[st] = (st < nst) ? D[(4 * st + kq) * BW + cb * 16 + cl] : 0.0;
    v4d a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < BW / 4; ++st) {
      if (st < nst) {
        a0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Pl[cl][4 * st + kq], dv[st], a0, 0, 0, 0);
        a1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Pl[16 + cl][4 * st + kq], dv[st], a1, 0, 0, 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      go[(kq + 4 * r) * BW + cb * 16 + cl] = a0[r];
      go[(16 + kq + 4 * r) * BW + cb * 16 + cl] = a1[r];
    }
  }
}

// grid: 8 ceil(ntiles / 8) workgroups over the lower tiles of all systems
// (XCD-grouped). Tiles with both indices in K take -D, tiles with one take G
// (transposed above K); the others M_IJ -= G_I P_J^T on the matrix cores, each
// wavefront owning one 16 x 16 quadrant, the accumulator starting from M_IJ and
// the inner dimension staged through LDS (coalesced 16-byte loads) in chunks of
// BH. (Operands loaded by each lane straight from the strips, without LDS,
// touch one cache line per lane and load: measured twice as slow.)
__global__ __launch_bounds__(256) void k_bsweep_update(int kb, int ntiles, const SweepSys *__restrict__ sys,
                                                       const int32_t *__restrict__ tsys,
                                                       const int16_t *__restrict__ tI, const int16_t *__restrict__ tJ,
                                                       double *__restrict__ M, const double *__restrict__ Dbuf,
                                                       const double *__restrict__ Pbuf,
                                                       const double *__restrict__ Gbuf) {
  __shared__ double Gs[TILE][BH + 1];
  __shared__ double Ps[TILE][BH + 1];
  const int t0 = xcd_grouped((int)blockIdx.x, (int)gridDim.x);
  if (t0 >= ntiles) return;
  const int s = tsys[t0];
  const SweepSys S = sys[s];
  const int k0 = kb * SW;
  if (k0 >= S.nb) return;
  const int w = min(SW, S.nb - k0), n = w * TILE;
  const int I = tI[t0], J = tJ[t0];
  double *Mt = tile_ptr(M, S.tile_off, I, J);
  const bool iK = I >= k0 && I < k0 + w, jK = J >= k0 && J < k0 + w;
  if (iK && jK) {  // M_IJ <- -D, block (I - k0, J - k0)
    const double *dv = Dbuf + (int64_t)s * BW * BW + (I - k0) * TILE * BW + (J - k0) * TILE;
    for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) Mt[t] = -dv[(t / TILE) * BW + t % TILE];
    return;
  }
  if (jK) {  // I past K: M_IJ <- columns J - k0 of G_I
    const double *g = Gbuf + (S.pan_off + I) * (TILE * BW) + (J - k0) * TILE;
    for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) Mt[t] = g[(t / TILE) * BW + t % TILE];
    return;
  }
  if (iK) {  // J before K: M_IJ <- (columns I - k0 of G_J)^T
    const double *g = Gbuf + (S.pan_off + J) * (TILE * BW) + (I - k0) * TILE;
    for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) Mt[t] = g[(t % TILE) * BW + t / TILE];
    return;
  }
  const double *g = Gbuf + (S.pan_off + I) * (TILE * BW);
  const double *p = Pbuf + (S.pan_off + J) * (TILE * BW);
  const int wv = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
  const int r0 = (wv >> 1) * 16, c0 = (wv & 1) * 16, cl = l % 16, kq = l / 16;
  double *mo = Mt + (r0 + kq) * TILE + c0 + cl;
  v4d acc = {mo[0], mo[4 * TILE], mo[8 * TILE], mo[12 * TILE]};
  for (int h = 0; h * BH < n; ++h) {
    if (h > 0) __syncthreads();
    for (int t = threadIdx.x; t < TILE * BH / 2; t += blockDim.x) {
      const int i = t / (BH / 2), j = 2 * (t % (BH / 2));
      const double2 gv = *(const double2 *)(g + i * BW + h * BH + j);
      const double2 pv = *(const double2 *)(p + i * BW + h * BH + j);
      Gs[i][j] = -gv.x;
      Gs[i][j + 1] = -gv.y;
      Ps[i][j] = pv.x;
      Ps[i][j + 1] = pv.y;
    }
    __syncthreads();
    const int nst = min(BH, n - h * BH) / 4;
#pragma unroll 8
    for (int st = 0; st < nst; ++st)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Gs[r0 + cl][4 * st + kq], Ps[c0 + cl][4 * st + kq], acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) mo[4 * r * TILE] = acc[r];
}

// Per swept system: a power of two s with max |entry| / s <= 2^14 (1 when the
// system is zero), the scale of its FP16 tiles.
__global__ __launch_bounds__(256) void k_sys_scale(const SweepSys *__restrict__ sys, const double *__restrict__ M,
                                                   float *__restrict__ scale) {
  __shared__ double red[256 / WAVE];
  const SweepSys S = sys[blockIdx.x];
  const int64_t n = (int64_t)S.nb * (S.nb + 1) / 2 * (TILE * TILE);
  const double *base = M + S.tile_off * (TILE * TILE);
  double mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) mx = fmax(mx, fabs(base[i]));
  for (int o = WAVE / 2; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, WAVE));
  if ((threadIdx.x % WAVE) == 0) red[threadIdx.x / WAVE] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) m = fmax(m, red[w]);
    scale[blockIdx.x] = (m > 0.0) ? (float)ldexp(1.0, ilogb(m) - 13) : 1.0f;
  }
}

// -M -> output tiles (symmetrised diagonal tiles), divided by the system's scale
// (NULL: 1) and converted to T.
template <typename T>
__global__ __launch_bounds__(256) void k_sweep_pack(const SweepSys *__restrict__ sys, const int32_t *__restrict__ tsys,
                                                    const int16_t *__restrict__ tI, const int16_t *__restrict__ tJ,
                                                    const int64_t *__restrict__ out_off, const double *__restrict__ M,
                                                    const float *__restrict__ scale, T *__restrict__ out) {
  const int t0 = blockIdx.x;
  const int s = tsys[t0];
  const SweepSys S = sys[s];
  const int I = tI[t0], J = tJ[t0];
  const double *Mt = tile_ptr((double *)M, S.tile_off, I, J);
  T *o = out + (out_off[s] + (int64_t)I * (I + 1) / 2 + J) * (TILE * TILE);
  for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) {
    const int i = t / TILE, j = t % TILE;
    double v = -Mt[t];
    if (I == J) v = -0.5 * (Mt[t] + Mt[j * TILE + i]);
    if (scale) v /= (double)scale[s];
    o[t] = (T)v;
  }
}

// explicit instantiations used by the host code
template __global__ void k_gather<double>(int64_t, const int *, const int32_t *, const double *, double *);
template __global__ void k_gather<float>(int64_t, const int *, const int32_t *, const double *, float *);
template __global__ void k_jt_tasks<double>(int, const int *, const int32_t *, const int32_t *, const double *,
                                            const double *, int64_t, const double *, double *, PcgCheck);
template __global__ void k_jt_tasks<float>(int, const int *, const int32_t *, const int32_t *, const float *,
                                           const float *, int64_t, const double *, float *, PcgCheck);
template __global__ void k_jt_corners<double>(int64_t, const int *, const int32_t *, const int32_t *, const double *,
                                              double *);
template __global__ void k_jt_corners<float>(int64_t, const int *, const int32_t *, const int32_t *, const float *,
                                             float *);
template __global__ void k_combine<double>(const Seg *, int, int, const int *);
template __global__ void k_combine<float>(const Seg *, int, int, const int *);
template __global__ void k_sweep_pack<double>(const SweepSys *, const int32_t *, const int16_t *, const int16_t *,
                                              const int64_t *, const double *, const float *, double *);
template __global__ void k_sweep_pack<float>(const SweepSys *, const int32_t *, const int16_t *, const int16_t *,
                                             const int64_t *, const double *, const float *, float *);
template __global__ void k_sweep_pack<_Float16>(const SweepSys *, const int32_t *, const int16_t *, const int16_t *,
                                                const int64_t *, const double *, const float *, _Float16 *);

}  // namespace coarse
