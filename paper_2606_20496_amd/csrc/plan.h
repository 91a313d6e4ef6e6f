// Host-side setup plan: every combinatorial structure the device kernels need,
// built once per mesh in plain C++ (no device calls). Device numerics (element
// matrices, local and reduced inverses) are computed later from these tables.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace coarse {

// Tile edge of the dense local / reduced inverse storage (both precisions).
constexpr int TILE = 32;
// Elements per workgroup of the operator kernel.
constexpr int OP_BLOCK = 256;
// Tiles per GEMV work item (one wavefront streams at most this many tiles).
constexpr int GEMV_SEG = 4;
// Systems of WHOLE_NB_MIN to WHOLE_NB_MAX tile rows are solved by one workgroup
// each (WHOLE_WAVES_F64 wavefronts for FP64 tiles, WHOLE_WAVES_NARROW for
// FP32/FP16); the others are cut into work items (a smaller system does too
// little work for a workgroup's fixed costs, a larger one too much for one unit).
constexpr int WHOLE_NB_MIN = 16;
constexpr int WHOLE_NB_MAX = 48;
constexpr int WHOLE_WAVES_F64 = 4;
constexpr int WHOLE_WAVES_NARROW = 8;
// Reduced-space entries per restriction task (one wavefront).
constexpr int JT_CHUNK = 256;

struct PlanInput {
  int64_t n_vert = 0, n_elem = 0;
  const double *xyz = nullptr;
  const int32_t *e2v = nullptr;
  const int32_t *part = nullptr;
  int32_t n_part = 0;
  const uint8_t *dirichlet = nullptr;
  int overlap = 1;
  int boxes[3] = {0, 0, 0};
  int interp = 0;
  // host threads: 0 = by mesh size (one below 2^20 elements, else up to 8); the
  // plan is the same for every thread count
  int threads = 0;
};

// One dense SPD system whose inverse is stored in lower-triangular tiles.
struct System {
  int64_t n = 0;        // true size
  int64_t nb = 0;       // tile rows (n_pad = nb*TILE)
  int64_t vec_off = 0;  // offset of its RHS / solution in the packed vectors
  int64_t tile_off = 0; // offset (in tiles) of tile (0,0) in the tile store
  int64_t row_off = 0;  // offset of its tile rows in the row table
};

// A GEMV work item: tiles (I, j0 .. j1-1) of one system.
struct GemvItem {
  int32_t sys, I, j0, j1;
};

struct Plan {
  std::string err;
  // sizes
  int64_t n_vert = 0, n_elem = 0, n_free = 0;
  int32_t n_part = 0;
  // internal numbering: vertices free-first; elements ordered by (part, Morton)
  std::vector<int32_t> vint_of_user;   // user vertex -> internal id
  std::vector<int32_t> user_of_vint;   // internal id -> user vertex
  std::vector<int32_t> elem_user;      // internal element -> user element
  std::vector<int32_t> e2v;            // SoA [8][E], internal vertex ids
  std::vector<double> xyz;             // SoA [3][n_vert], internal order
  std::vector<int32_t> mult;           // elements per vertex (internal)

  // operator blocks (OP_BLOCK consecutive internal elements)
  int64_t n_blocks = 0, max_slots = 0;
  std::vector<int32_t> blk_slot_ptr;   // [n_blocks+1]
  std::vector<int32_t> slot_vid;       // free internal vertex of each slot
  std::vector<int32_t> slot_dst;       // >=0: owned, write q[dst]; <0: partial -(k+1)
  std::vector<int32_t> slot_inc_ptr;   // [n_slots+1] into slot_inc
  std::vector<uint16_t> slot_inc;      // e_local*8 + a
  std::vector<uint16_t> slot_inc8;      // [slots][8]: the incidence list as one record (see plan.cpp)
  std::vector<uint8_t> blk_inc;        // [n_blocks] 1: two elements hold a vertex at the same local
                                       // corner, so the block sums through the incidence lists
  bool any_blk_inc = false;
  std::vector<uint16_t> lconn;         // [E][8]: slot of local vertex a (0xFFFF = Dirichlet), 16 B per element
  int64_t n_partials = 0;
  std::vector<int32_t> sh_vid;         // shared vertices
  std::vector<int32_t> sh_ptr;         // [n_shared+1] partial ids of shared vertex j: [sh_ptr[j], sh_ptr[j+1])
  std::vector<int32_t> sh_part;        // unused (partials are contiguous per vertex)
  std::vector<uint8_t> slot_pw;        // 1: the slot's block writes the vertex (first block touching it)
  std::vector<int32_t> vq;             // [n_free][2]: first partial and count (0 = owned)

  // free vertex -> incident (element, local vertex) pairs, element order
  std::vector<int32_t> vinc_ptr;       // [n_free+1]
  std::vector<int32_t> vinc;           // e*8 + a

  // local systems (Sec. 3)
  std::vector<std::vector<int32_t>> R;   // sorted internal ids per subdomain
  std::vector<int32_t> sub_of_sys;       // system -> subdomain (local systems only)
  std::vector<System> sys;               // local systems, then the reduced system
  int64_t n_local_sys = 0;
  int64_t vec_len = 0;                   // packed vector length (all systems)
  int64_t n_tiles = 0;
  std::vector<int32_t> sub_idx;          // [vec_len] internal vertex or -1 (padding / reduced)
  std::vector<int32_t> cover_ptr;        // [n_free+1]
  std::vector<int32_t> cover_pos;        // positions in the packed vectors
  int64_t n_rows = 0;                    // tile rows over all systems
  // local-system element lists for the dense assembly are implied by R (all
  // incident elements of a vertex in R_p lie in the overlapping subdomain)

  // reduced space (Sec. 4)
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, H[3] = {1, 1, 1};
  int32_t b[3] = {1, 1, 1};
  // standard interpolation: the Galerkin A_r = J^T A J is formed column by column
  // from probes; box vertices congruent modulo probe_p share a probe, and a probe
  // column couples box vertices at most probe_d apart per direction
  int32_t probe_p[3] = {1, 1, 1}, probe_d[3] = {0, 0, 0};
  int64_t n_bv = 0;                      // (b+1)^3 box vertices
  std::vector<int32_t> elem_cell;        // internal element -> cell id
  std::vector<int32_t> occ_cells;        // occupied cells (ids)
  std::vector<int32_t> cell_occ;         // cell id -> occupied index or -1
  std::vector<int32_t> occ_elem_ptr;     // [n_occ+1] elements per occupied cell
  std::vector<int32_t> occ_elems;
  std::vector<int32_t> occ_corner_act;   // [n_occ][8] active index of each corner or -1
  std::vector<int32_t> bv_act;           // box vertex -> active index or -1
  std::vector<int32_t> act_bv;           // active index -> box vertex
  int64_t n_r = 0;
  // vertex-major interpolation entries (prolongation J)
  std::vector<int32_t> jv_ptr;           // [n_free+1]
  std::vector<int32_t> jv_occ;           // occupied-cell index of the entry
  std::vector<int32_t> jv_base;          // box-vertex id of the entry's cell corner 0
  std::vector<double> jv_w;              // weight fraction n_ic/m_i
  std::vector<double> jv_xi;             // [3][n_entries] local coordinates
  // cell-major entries (restriction J^T)
  std::vector<int32_t> jc_vid;
  std::vector<double> jc_w;
  std::vector<double> jc_xi;             // [3][n_entries]
  std::vector<int32_t> jt_task_start;    // [n_tasks+1] entry ranges
  std::vector<int32_t> jt_task_occ;      // occupied cell of the task
  std::vector<int32_t> jr_ptr;           // [n_r+1] per active box vertex
  std::vector<int32_t> jr_src;           // task*8 + corner
  // dense reduced assembly: per active vertex, (occupied cell, corner) pairs
  std::vector<int32_t> ar_ptr;           // [n_r+1]
  std::vector<int32_t> ar_src;           // occ*8 + corner
};

// Build the plan; returns 0 or a negative coarse_status (message in plan.err).
int build_plan(const PlanInput &in, Plan &plan);

// The dense-solve work of the systems of a plan. Systems with WHOLE_NB_MIN <= nb
// <= WHOLE_NB_MAX go to `whole` (one workgroup each; the local systems largest first, then the
// reduced system), as many as fill whole rounds of n_cu compute units (none when
// there are fewer than n_cu): the smallest of the rest, and every larger system,
// have each tile row I cut into items of tiles_of_bucket[bucket(nb)] tiles
// (bucket b: nb <= bucket_max[b]; a value < 1 means GEMV_SEG), whose partial sums
// the row table combines.
struct GemvTable {
  std::vector<int32_t> whole;
  int32_t whole_local = 0;   // leading entries of `whole` that are local systems
  int32_t whole_nb_max = 0;
  std::vector<GemvItem> items;
  std::vector<int32_t> row_item0, row_nitem, row_sys, row_I;
};
// Systems before first_sys are left out (their solves are not dense).
void build_gemv_items(const Plan &P, const int *tiles_of_bucket, const int *bucket_max, int nbucket, int n_cu,
                      GemvTable &out, int64_t first_sys = 0);

}  // namespace coarse
