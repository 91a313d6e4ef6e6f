// Kernel declarations and the small descriptor structs shared between the
// kernels (kernels.hip) and the host orchestration (api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "plan.h"

namespace coarse {

// Element matrices (36 unique FP64 entries of each symmetric 8x8 A^e) are stored
// per operator block of OP_BLOCK elements: [block][36][OP_BLOCK], so the block
// that applies them streams one contiguous 72 KB region.
__host__ __device__ inline int64_t ae_at(int k, int64_t e) {
  return ((e / OP_BLOCK) * 36 + k) * OP_BLOCK + (e % OP_BLOCK);
}

// The operator keeps only the 28 off-diagonal entries a < b of each A^e (its rows
// sum to zero), in the same blocked layout: [block][28][OP_BLOCK].
__host__ __device__ inline int64_t ae28_at(int k, int64_t e) {
  return ((e / OP_BLOCK) * 28 + k) * OP_BLOCK + (e % OP_BLOCK);
}

// Solver scalars living in device memory (one per context).
struct Scalars {
  double bb, rho[2], rr, pq, alpha, beta, tol2, res_true;
  double rr0;      // ||r_0||^2 of the first convergence test
  int32_t iter;    // completed iterations (parity of the double buffers)
  int32_t iters;   // iterations reported when the solve ended
  int32_t done, status, max_it, flexible, pad0, pad1;
};

// The convergence test of PCG carried by the first kernel of a preconditioner
// application (sc == nullptr: none): the workgroup partials of the residual
// norm, their count, and the start flag of pcg_check; lead != 0 lets workgroup 0
// record the outcome (one kernel per application records it).
struct PcgCheck {
  Scalars *sc;
  const double *part;
  int32_t n, start, lead, pad;
};

// One dense system of the batched local/reduced solve, with absolute pointers.
struct SysDev {
  const void *tiles;   // lower tiles of A_s^{-1}, TILE x TILE row-major each
  const void *rp;      // right-hand side (nb*TILE entries)
  void *colpart;       // per tile: transposed contribution (TILE entries)
  void *rowpart;       // per work item: row contribution (TILE entries)
  double *zp;          // solution (nb*TILE entries)
  double *yfull;       // reduced system only: solution scattered to all box vertices
  const int32_t *act_bv;   // reduced system only: active index -> box vertex
  const int32_t *gidx;     // local systems: internal vertex of each packed entry (-1: padding)
  int32_t nb, n;
  float scale;             // FP16 tiles hold A_s^{-1} / scale (1 otherwise)
  int32_t pad;
};

// GEMV work item: tiles (I, j0 .. j1-1) of system `sys`; `slot` indexes the
// system's row-partial area.
struct GItem {
  int32_t sys;
  int16_t I, j0, j1, pad;
  int32_t slot;
};

// Combine work: one tile row of one system.
struct GRow {
  int32_t sys, I, slot0, nslot;
};

// A contiguous range of items (or rows) of one context inside a batched launch.
struct Seg {
  const GItem *items;
  const GRow *rows;
  const int32_t *whole;   // systems solved by one workgroup each
  const SysDev *sys;
  const int *done;   // the owning solve's finished flag (batched launches), or null
  int32_t begin;     // first global index of this segment
  int32_t pad;
};

// Device pointers of one context used by the per-iteration kernels.
struct OpDev {
  int64_t E, n_blocks, n_shared;
  const double *Ae;           // [block][28][OP_BLOCK] off-diagonal element entries (ae28_at)
  const uint16_t *lconn;   // [E][8] block-local slots, one 16-byte load per element
  const int32_t *blk_slot_ptr, *slot_vid, *slot_dst, *slot_inc_ptr;
  const uint16_t *slot_inc;
  const uint16_t *slot_inc8;  // per slot: the first 8 incidences as one 16-byte record
  double *partials;
  const int32_t *sh_vid, *sh_ptr;
  const uint8_t *slot_pw;     // 1: this slot's block writes the vertex's search direction
  const uint8_t *blk_inc;     // per block, 1: sum through the incidence lists (see block_accumulate)
  const int2 *vq;             // free vertex -> (first partial, count); count 0: owned by one block
  int32_t lds_bytes;
  int32_t ae_nt;              // 1: the element matrices outgrow the last-level cache; stream them
                              // with non-temporal loads
};

// One local system of the inexact local solves, A_p in ELL form: entry (k, i) of
// the system at ell_off + k * npad + i (values; the column words, two uint16
// columns each, at ell_off / 2 + (k / 2) * npad + i).
struct LocSys {
  int64_t ell_off;
  int32_t vec_off;   // offset of R_p in the packed vectors (sub_idx, rp, zp, diag)
  int32_t n, npad, pad;
};

// The per-iteration state of one solve, for launches that cover every solve of
// a lock-step batch (T-typed arrays are float or double by the batch precision).
struct IterDev {
  OpDev op;
  int64_t nf;        // free vertices
  int64_t n_pack;    // packed local entries; the reduced system's entries follow
  int64_t nent, n_r;
  Scalars *sc;
  double *x, *r, *pa, *pb, *z, *q, *energy, *part1, *part2, *prr;
  const double *zp, *yfull;
  const int32_t *sub_idx, *jt_start, *jc_vid, *jr_ptr, *jr_src, *cover_ptr, *cover_pos, *jv_ptr, *jv_base;
  void *rp, *jt_part;
  const void *jc_w, *jc_xi, *jv_w, *jv_xi;
  int32_t nvblk;     // grid of the per-vertex kernels = number of their partials
  int32_t ng;        // gather workgroups of the restriction kernel
  int32_t ntask, bx1, bxy1, flexible;
  int32_t n_bv;      // box vertices of the full reduced grid
  int32_t y_lds;     // 1: the final kernel stages the reduced solution in LDS
  // inexact local solves (loc_iters > 0): n_loc systems, W entries per row
  const LocSys *loc_sys;
  const double *loc_diag;
  const uint32_t *loc_col;
  const void *loc_val;   // double (FP64 contexts) or float
  int32_t loc_w, loc_iters, n_loc, pad_loc;
};

}  // namespace coarse
