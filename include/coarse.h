/*
 * coarse.h — C-ABI of the MI355X (gfx950) two-level Schwarz coarse solver.
 *
 * The library solves the coarse (N = 1, element-vertex) Poisson system
 * A u = b of Ratnayaka, Fischer & Olson, "Coarse Solvers for Exascale Solution of
 * Poisson Problems", Sec. 3: A = Q^T A_L Q is the trilinear (Q1) finite-element
 * stiffness matrix on a globally unstructured hexahedral mesh with homogeneous
 * Dirichlet and Neumann boundaries. It is preconditioned by the two-level additive
 * Schwarz method of eq. (asm),
 *     z = sum_p R_p^T A_p^{-1} R_p r + J A_r^{-1} J^T r,
 * with exact local solves on overlapping subdomains (Sec. 3) and the non-nested
 * box-grid reduced space of Sec. 4 (element-centroid cells, J = W Q^T J_L S,
 * A_r assembled cell by cell as in eq. (Aij)), inside preconditioned conjugate
 * gradients. All arithmetic runs in the library's HIP kernels on the current
 * device; no CPU fallback exists.
 *
 * Conventions shared by every call
 *   - Return value: COARSE_OK (0) on success, a negative COARSE_E* code on error
 *     (the context, if any, is left unchanged and usable), COARSE_NOTCONV (+1) as
 *     a warning. coarse_last_error() returns a message for the last failing call.
 *   - Host arrays are read during the call only; the caller keeps ownership.
 *   - Vector arguments of apply/solve are DEVICE pointers to contiguous float64
 *     arrays of length n_vert in the caller's vertex numbering. Entries at
 *     Dirichlet vertices are ignored on input and written as 0 on output. Input
 *     and output must not alias.
 *   - All device work is ordered on the context's stream (coarse_opts.stream, or
 *     coarse_set_stream). A context must not be used from two streams or threads
 *     at once. No call after coarse_setup allocates device memory, except
 *     the first block solve of a context set up without opts.block_rhs (see
 *     coarse_solve_multi) and the lock-step batch calls, which hold their own
 *     tables (coarse_solve_batch_noalloc allocates nothing).
 */
#ifndef COARSE_H
#define COARSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum coarse_status {
  COARSE_OK = 0,
  COARSE_NOTCONV = 1,      /* max_it reached; u holds the last iterate            */
  COARSE_EINVAL = -1,      /* bad argument (null pointer, index out of range, ...) */
  COARSE_ENOMEM = -2,      /* device or host allocation failed                     */
  COARSE_EMESH = -3,       /* element with det(dx/dxi) <= 0 at a Gauss point, or a
                              vertex repeated within an element                    */
  COARSE_ESINGULAR = -4,   /* a local A_p or the reduced A_r is not SPD (e.g. an
                              all-Neumann problem, or an empty interior box, Sec. 4) */
  COARSE_EDEVICE = -5,     /* HIP runtime error                                    */
  COARSE_EBREAKDOWN = -6   /* PCG breakdown: p.Ap <= 0 or a non-finite value       */
};

enum coarse_precision {
  COARSE_FP64 = 0,   /* everything in float64                                      */
  COARSE_MIXED = 1,  /* local inverses, J/J^T and the reduced solve in float32;
                        A, the PCG vectors and dot products stay float64 (the
                        single-precision local/reduced solves of Sec. 6)          */
  COARSE_MIXED_F16 = 2 /* as COARSE_MIXED, with the local and reduced inverses
                        stored in float16 (each system's inverse divided by a
                        power-of-two scale so no entry exceeds 2^14) and applied
                        with float32 arithmetic: half the bytes of the dominant
                        kernel, a less exact preconditioner                       */
};

enum coarse_mode {
  COARSE_ADDITIVE = 0,     /* eq. (asm)                                            */
  COARSE_HYBRID_SYM = 1,   /* symmetrised hybrid of eqs. (asm1)-(asm2):
                              z0 = M_r r, z1 = z0 + M_loc (r - A z0),
                              z = z1 + M_r (r - A z1)                              */
  COARSE_LOCAL_ONLY = 2,   /* eq. (asm1) alone (ablation)                          */
  COARSE_REDUCED_ONLY = 3, /* J A_r^{-1} J^T alone (ablation)                      */
  COARSE_HYBRID = 4        /* eqs. (asm1)-(asm2) as written: z_loc = M_loc r,
                              z = z_loc + M_r (r - A z_loc). Not symmetric: the
                              default beta of a context in this mode is the
                              flexible one (opts.flexible is forced to 1)          */
};

enum coarse_interp {
  COARSE_J_CENTROID = 0,   /* element-centroid cells + W averaging, cell-assembled
                              A_r (Sec. 4, compact 3^d stencil)                    */
  COARSE_J_STANDARD = 1    /* J_ij = Phi_j(x_i) with the box bounding x_i and
                              A_r = J^T A J (Sec. 4, eq. (Psi); 5^d stencil)        */
};

typedef struct coarse_ctx coarse_ctx;   /* opaque; owns all device state */

/* Mesh (Sec. 3): n_elem hexahedra; e2v[8*e + v] is local vertex v = i + 2j + 4k,
 * (i,j,k) in {0,1}^3 lexicographic, of element e (ids in [0, n_vert)); xyz[3*u+d]
 * is coordinate d of vertex u. part[e] in [0, n_part) is the subdomain Omega_p of
 * element e (contiguous element clusters, Sec. 3); part == NULL asks the library
 * to cut the mesh by recursive coordinate bisection of the element centroids
 * into n_part pieces (n_part >= 1). */
typedef struct {
  int64_t n_vert;
  int64_t n_elem;
  const double *xyz;      /* host [n_vert][3]  */
  const int32_t *e2v;     /* host [n_elem][8]  */
  const int32_t *part;    /* host [n_elem] or NULL */
  int32_t n_part;
} coarse_mesh;

/* Boundary (Sec. 3): dirichlet[u] != 0 marks a homogeneous Dirichlet vertex;
 * every other boundary vertex is homogeneous Neumann. At least one Dirichlet
 * vertex is needed for A to be SPD. */
typedef struct {
  const uint8_t *dirichlet;   /* host [n_vert] */
} coarse_bc;

/* Largest basis of prior solutions a context may keep (opts.projection). */
#define COARSE_PROJECTION_MAX 64
/* right-hand sides of one block solve (coarse_solve_multi) */
#define COARSE_MULTI_MAX 16

/* Size buckets of the work-item table: bucket b holds the systems whose tile
 * count nb = ceil(n/32) is at most 2, 4, 8, 12, 16, 24, 48 for b = 0..6; bucket 7
 * holds all larger ones. */
#define COARSE_GEMV_BUCKETS 8

typedef struct {
  int overlap;      /* element layers added to each subdomain (Sec. 3), >= 1        */
  int boxes[3];     /* b_x, b_y, b_z boxes of the reduced grid (Sec. 4); a zero
                       entry means ceil(n_part^(1/3))                               */
  int precision;    /* enum coarse_precision                                       */
  int mode;         /* enum coarse_mode                                            */
  int interp;       /* enum coarse_interp                                          */
  int max_it;       /* PCG iteration cap                                           */
  int check_every;  /* PCG iterations queued between host convergence checks; the
                       result does not depend on it (finished iterations are
                       skipped on the device)                                      */
  int flexible;     /* 1: Polak-Ribiere beta (r, z_new - z_old)/(r,z)_old;
                       0: Fletcher-Reeves. Default 1 for the mixed forms, else 0  */
  void *stream;     /* hipStream_t; NULL = the null stream                         */
  int gemv_tiles[COARSE_GEMV_BUCKETS];
                    /* tiles per work item of the batched dense solve, per size
                       bucket of a system's tile count nb = ceil(n/32) (see
                       COARSE_GEMV_BUCKETS). 0 = 4. Used for the
                       systems cut into work items: those outside 16..48 tile
                       rows, all systems of a context with fewer systems than the
                       device has compute units, and the smallest ones past a
                       multiple of that count (the others are solved by one
                       workgroup each). Changes only the order of rounding inside
                       a row sum and the speed; a context keeps its choice for
                       life (results stay bitwise reproducible, alone or batched) */
  int projection;   /* l >= 0 prior solutions kept for coarse_solve_projected
                       (Sec. 5); 0 = none. The basis takes 2 l n_free doubles of
                       device memory, allocated by the setup; l <=
                       COARSE_PROJECTION_MAX                                       */
  int whole_waves;  /* wavefronts per workgroup of the systems solved by one
                       workgroup each (those of 16..48 tile rows, in contexts with
                       at least one system per compute unit): 2, 4 or 8 for FP64
                       tiles, 4, 8 or 16 for FP32/FP16 tiles; 0 = 4 (FP64) or 8.
                       Halved while the workgroup's LDS copies of the solution
                       would exceed 64 KiB. Changes the order of rounding only   */
  int block_rhs;    /* 1: the setup also allocates the vectors of the block solve
                       (coarse_solve_multi, about 9 * 16 doubles per free vertex),
                       so that no later call on the context allocates; 0 (default):
                       the first block-solve call allocates them                   */
  int local_iters;  /* 0 (default): exact local solves with the stored inverses
                       A_p^{-1} (Sec. 3, eq. (asm)). k > 0: inexact local solves
                       (the iterative local solver of Sec. 6.3): each r_p is solved
                       by k steps of conjugate gradients preconditioned by the
                       diagonal of A_p, from zero; A_p is stored sparse (ELL) and no
                       local inverse is formed. The preconditioner then depends
                       on r nonlinearly, so the flexible beta is used whatever
                       opts.flexible says. Needs every |R_p| <= 1024 and at most 26
                       off-diagonal entries per row of A_p (the 27-point coupling
                       of a vertex inside a structured hex block; else
                       COARSE_EINVAL at setup). Block solves (coarse_solve_multi,
                       coarse_multi_*) reject such a context (COARSE_EINVAL);
                       single solves and lock-step batches take it             */
  int reduced_refine; /* 1: after each reduced solve y = A_r^{-1} r_r, one step of
                       iterative refinement y += A_r^{-1} (r_r - A_r y), the
                       residual formed in FP64 by the 27-point stencil of A_r on
                       the box grid (Sec. 4, eq. (Aij)) and the correction by the
                       same stored inverse: brings the FP32 or FP16-stored reduced
                       solve of the mixed forms to about FP64 accuracy. Centroid
                       interpolation only (else COARSE_EINVAL at setup); block
                       solves and lock-step batches reject such a context.
                       0 (default): no refinement                              */
} coarse_opts;

typedef struct {
  int iters;            /* products with A inside the PCG loop                     */
  int status;           /* COARSE_OK, COARSE_NOTCONV or COARSE_EBREAKDOWN          */
  double relres;        /* ||r_k||_2 / ||b||_2 from the recurrence (free entries)   */
  double relres_true;   /* ||b - A u||_2 / ||b||_2 recomputed at the end            */
  double t_setup;       /* seconds spent in coarse_setup                            */
  double t_solve;       /* seconds spent in this solve (host clock, stream synced)  */
  double relres0;       /* ||b - A u_0||_2 / ||b||_2 of the initial guess u_0 (1 from
                           u_0 = 0)                                                */
  int n_basis;          /* prior solutions the initial guess was projected on      */
} coarse_stats;

typedef struct {
  int64_t n_free;        /* unknowns (non-Dirichlet vertices)                       */
  int64_t n_sub;         /* subdomains with a non-empty R_p                         */
  int64_t sum_np;        /* sum_p |R_p|                                             */
  int64_t max_np;        /* max_p |R_p|                                             */
  int64_t n_r;           /* reduced unknowns after compression (Sec. 4)             */
  int64_t n_cells;       /* boxes that own at least one element centroid            */
  int64_t local_bytes;   /* bytes of the stored local inverses                      */
  int64_t reduced_bytes; /* bytes of the stored reduced inverse                     */
  int64_t a_bytes;       /* bytes streamed by one application of A                  */
  int64_t inv_alg_bytes; /* sum over local and reduced systems of n(n+1)/2 stored
                            entries times the element size: the packed symmetric
                            inverses one preconditioner application must read     */
  int64_t n_jent;        /* entries of J: (free vertex, cell) pairs with a nonzero
                            weight fraction (Sec. 4, J = W Q^T J_L S)              */
  int64_t n_inc_blocks;  /* operator blocks (256 elements) in which two elements
                            hold one vertex at the same local corner; they sum
                            element outputs through per-vertex incidence lists,
                            all others corner by corner                         */
  int64_t device_bytes;  /* all device memory held by the context                   */
  int32_t boxes[3];
  int32_t precision;
  int32_t gemv_tiles[COARSE_GEMV_BUCKETS];   /* work-item table the context uses     */
  int32_t whole_waves;    /* wavefronts per whole-system workgroup in use          */
  int32_t reduced_stream; /* 1: the reduced system has more than 48 tile rows of
                             32, and the additive preconditioner solves it on a
                             second stream beside the local systems (profile
                             phase 7); 0: one dense-solve launch holds both     */
  int32_t local_iters;    /* opts.local_iters of the context (0: exact solves)    */
  int32_t ell_width;      /* inexact local solves: off-diagonal entries stored per
                             row of A_p (even; the largest row count rounded up);
                             local_bytes then counts the stored A_p (ELL entries
                             and diagonals), not inverses                         */
  int32_t reduced_refine; /* opts.reduced_refine of the context                   */
} coarse_info_t;

/* Fill *o with the defaults: overlap 1, boxes auto, FP64, additive, centroid J,
 * max_it 1000, check_every 4, flexible 0, null stream. */
void coarse_default_opts(coarse_opts *o);

/* Build everything a solve needs (Secs. 3-4): locality ordering, overlapping
 * subdomains and R_p, element matrices, the local inverses A_p^{-1} (batched
 * dense block-sweep on the device), the box grid, J and the reduced inverse
 * A_r^{-1}. Allocates all device memory of the context. On success *out owns it.
 * Errors: EINVAL, ENOMEM, EMESH, ESINGULAR, EDEVICE. */
int coarse_setup(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts,
                 coarse_ctx **out);

/* coarse_setup in two halves, for callers that prepare new meshes while the GPU
 * is busy with other work (a serving loop):
 *   coarse_plan_create: the host half. Validates opts, orders the elements and
 *     vertices, builds the overlapping subdomains and R_p (Sec. 3), the box grid,
 *     the element cells and the weights of J (Sec. 4) and every work table. It
 *     makes no HIP call and touches no device, so it may run on any host thread
 *     while other threads use the GPU. The plan holds copies of all it needs: the
 *     caller may free the mesh arrays on return. Errors: EINVAL, EMESH (mesh
 *     topology), ENOMEM (host memory).
 *   coarse_setup_from_plan: the device half, on `stream` (NULL = default stream;
 *     opts.stream of the plan is not used): uploads the plan, forms the element
 *     matrices, assembles and inverts every A_p and A_r. Errors as coarse_setup.
 *     The plan is not modified and may be used again or destroyed afterwards.
 *   coarse_plan_destroy: frees the plan (host memory only); NULL is accepted.
 * coarse_setup(mesh, bc, opts, out) is these three calls with opts.stream. */
typedef struct coarse_plan coarse_plan;
/* Replace the work-item table (opts.gemv_tiles) a plan hands to later device
 * setups; for tuning the batched dense solve without rebuilding the plan. */
int coarse_plan_set_gemv_tiles(coarse_plan *plan, const int *tiles);
int coarse_plan_create(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts,
                       coarse_plan **out);
int coarse_setup_from_plan(const coarse_plan *plan, void *stream, coarse_ctx **out);
int coarse_plan_destroy(coarse_plan *plan);

/* z = M^{-1} r: one application of the preconditioner selected by opts.mode
 * (eq. (asm) by default). r, z: device float64 [n_vert]. Errors: EINVAL. */
int coarse_apply_precond(coarse_ctx *ctx, const double *r, double *z);

/* q = A p, the Q1 operator of Sec. 3 (free rows/columns). Device float64 [n_vert]. */
int coarse_apply_A(coarse_ctx *ctx, const double *p, double *q);

/* Solve the coarse system A u = b of Sec. 3 (the element-vertex problem that the
 * paper's Sec. 1 embeds in a Krylov method) by preconditioned conjugate
 * gradients from u0 = 0 with the preconditioner of opts.mode, until
 * ||r||_2 <= tol ||b||_2 over the free entries (recurrence residual). Each
 * iteration: q = A p, alpha = (r,z)/(p,q), x += alpha p, r -= alpha q, the
 * convergence test, z = M^{-1} r, beta (Fletcher-Reeves, or Polak-Ribiere with
 * opts.flexible), p = z + beta p; iterations count the products with A. The
 * true residual ||b - A u|| is recomputed at the end (stats.relres_true).
 * b, u: device float64 [n_vert]. st may be NULL. Returns COARSE_OK, COARSE_NOTCONV
 * (warning) or COARSE_EBREAKDOWN / COARSE_EINVAL. b = 0 gives u = 0, iters = 0. */
int coarse_solve(coarse_ctx *ctx, const double *b, double *u, double tol, coarse_stats *st);

/* Solve A u = b for one of a sequence of right-hand sides with the same A, by
 * projection onto prior solutions (Sec. 5, the A-orthogonal best fit over the
 * span of the last solutions): with the stored basis x_1..x_n, A-orthonormal
 * (x_j^T A x_k = delta_jk, free entries), c_j = x_j^T b, u_bar = sum_j c_j x_j is
 * the best approximation of u in the A-norm over that span, and PCG starts from
 * u_0 = u_bar (r_0 = b - sum_j c_j A x_j), stopping at ||r||_2 <= tol ||b||_2 as
 * coarse_solve does. The solution then joins the basis by A-Gram-Schmidt
 * (classical, coefficients x_j^T A u) and normalisation; it is not added when its
 * A-orthogonal part has A-norm at most 1e-6 of its own (already in the span) or
 * is not finite. When the basis holds opts.projection vectors, the next append
 * empties it first. Needs opts.projection >= 1 at setup (else EINVAL); no device
 * allocation. b, u: device float64 [n_vert]; st as for coarse_solve, with
 * relres0 = ||r_0|| / ||b|| and n_basis = n. Returns as coarse_solve. */
int coarse_solve_projected(coarse_ctx *ctx, const double *b, double *u, double tol, coarse_stats *st);

/* Forget the stored prior solutions (the next coarse_solve_projected starts from
 * u_0 = 0). Errors: EINVAL. */
int coarse_projection_reset(coarse_ctx *ctx);

/* Block solve: k right-hand sides on the context's mesh (1 <= k <=
 * COARSE_MULTI_MAX), k independent PCG recurrences (Sec. 1, the same iteration
 * as coarse_solve for each column, to the same tolerance) advanced together so
 * that every read of the element matrices and of the stored dense inverses
 * serves all of them: the dense solves of the additive preconditioner (Sec. 3,
 * eq. (asm), and the reduced solve of Sec. 4) become products of each inverse
 * with a 16-column block, on the matrix cores (FP64 products for COARSE_FP64,
 * FP32 products of the FP32 or FP16-stored inverses for the mixed forms; the
 * operator, vectors and dot products are FP64 in every form). A column stops
 * changing once it has converged; the others go on. b, u: device float64
 * [k][n_vert] (column j at offset j * n_vert), b != u. st: NULL or k entries, one
 * per column (t_solve is the block's). Needs the additive mode (else EINVAL). The
 * first call allocates the block's vectors (about 9 * 16 doubles per free
 * vertex) for the context's life. Returns the worst column status, as
 * coarse_solve. Results per column are bitwise reproducible and independent of
 * the other columns, but not bitwise those of coarse_solve (another summation
 * order inside the dense solves). */
int coarse_solve_multi(coarse_ctx *ctx, int k, const double *b, double *u, double tol, coarse_stats *st);

/* z_j = M r_j for the k columns of r (the additive preconditioner of
 * coarse_solve_multi); r, z: device float64 [k][n_vert], r != z. Errors as
 * coarse_solve_multi. */
int coarse_apply_precond_multi(coarse_ctx *ctx, int k, const double *r, double *z);

/* The block solve in steps, for a loop that interleaves it with other work on the
 * context's stream (a serving loop's lock steps). Same iteration and results as
 * coarse_solve_multi. begin enqueues r = b and the first preconditioner
 * application (b: device float64 [k][n_vert], kept alive by the caller until end);
 * advance enqueues `iters` iterations of the live columns and a copy of the solver
 * state to pinned host memory; once the caller has synchronised the stream,
 * coarse_multi_done returns 1 when every column has finished (0 if not, as of the
 * last advance); end enqueues the true residuals and the solutions (u: [k][n_vert],
 * u != b), synchronises the stream, fills st (NULL or k entries) and returns the
 * worst column status. One block solve per context at a time: begin (and the other
 * block calls) fail with EINVAL while one is in progress, and so do advance, done
 * and end without one. */
int coarse_multi_begin(coarse_ctx *ctx, int k, const double *b, double tol);
int coarse_multi_advance(coarse_ctx *ctx, int iters);
int coarse_multi_done(const coarse_ctx *ctx);
int coarse_multi_end(coarse_ctx *ctx, double *u, coarse_stats *st);

/* Solve `count` independent systems (any mix of contexts, each with its own right-
 * hand side) in lock step: every PCG phase of all live systems is issued before
 * the next phase, and each phase of all of them is one launch.
 * Contexts must be distinct; the batch runs on the stream of ctxs[0]. Each result
 * equals what coarse_solve gives for that system alone (bitwise). */
int coarse_solve_batch(coarse_ctx *const *ctxs, const double *const *b, double *const *u,
                       int count, double tol, coarse_stats *st);

/* coarse_solve_batch without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same solves and the same results (bitwise), with
 * the batch's device tables in a fixed 1 MiB array of the library on each
 * device (held until the process ends) and its host staging in a fixed host
 * array, instead of memory allocated per call. No graph replay. It calls no
 * hipMalloc, hipFree or other allocating routine; the contexts' own memory is
 * allocated at their setup. count may not exceed COARSE_NOALLOC_MAX_SOLVES
 * (else COARSE_EINVAL, message in coarse_last_error(NULL)). Calls share those
 * arrays: two calls that overlap in time (on any device, from any thread) race
 * and must not be made. Returns as coarse_solve_batch. */
#define COARSE_NOALLOC_MAX_SOLVES 256
int coarse_solve_batch_noalloc(coarse_ctx *const *ctxs, const double *const *b, double *const *u, int count,
                               double tol, coarse_stats *st);

/* Continuous batching (lock-step solves). A batch advances every live solve by
 * whole PCG iterations, all on `stream`, with seven launches per iteration
 * whatever the number of live solves: the operator, the x/r update, the
 * restriction (R_p and the first stage of J^T), the J^T corner sums, the dense
 * local and reduced solves of all systems of all solves (one GEMV and one
 * partial-sum launch), and the overlap sum with the prolongation; an eighth
 * runs the inexact local solves of the solves set up with opts.local_iters > 0. Each workgroup
 * of such a launch works for one solve exactly as in that solve's own launch.
 * A submitted solve's first preconditioner application runs at submit. Solves join with
 * coarse_batch_submit and leave when coarse_batch_step reports them finished, so
 * requests that arrive while others are running are admitted between steps.
 * Results are bitwise identical to coarse_solve of the same context and RHS, or,
 * for a context set up with opts.projection > 0, to coarse_solve_projected (the
 * solve starts from the projection onto the context's prior solutions, and its
 * solution joins them when it is retired).
 * Contexts must use the additive preconditioner and share one precision; while
 * in a batch a context must not be used otherwise. `stream` orders the batch
 * against the caller (inputs must be ready on it before submit); use_graph = 1
 * captures one lock step as a HIP graph and replays it (needs a non-null stream;
 * the graph is rebuilt when the set of live solves changes). */
typedef struct coarse_batch coarse_batch;
int coarse_batch_create(void *stream, int use_graph, coarse_batch **out);
/* Start the solve of ctx for right-hand side b into u (device, as in
 * coarse_solve); tag is returned by coarse_batch_step when it finishes. */
int coarse_batch_submit(coarse_batch *bt, coarse_ctx *ctx, const double *b, double *u, double tol, int64_t tag);
/* Advance all live solves by `iters` lock steps, then retire up to cap of the
 * finished ones: their u is written (stream-ordered before later work on
 * `stream`) and they are reported in tags[] / stats[] (*n_done of them); other
 * finished solves stay live (their iterations are skipped) until a later step
 * retires them. */
int coarse_batch_step(coarse_batch *bt, int iters, int64_t *tags, coarse_stats *stats, int cap, int *n_done);
/* coarse_batch_step in two halves, so that the caller can do other work (for
 * instance the device half of another context's setup, on another stream) while
 * the lock steps run. coarse_batch_launch queues `iters` lock steps and the copy
 * of the solver states to the host, and returns without waiting;
 * coarse_batch_collect waits for them and retires finished solves exactly as
 * coarse_batch_step does (0 of them when nothing was launched). Between the two,
 * coarse_batch_submit and a second launch return COARSE_EINVAL, and the contexts
 * in the batch must not be used. launch followed by collect gives the same
 * results, bit for bit, as step. */
int coarse_batch_launch(coarse_batch *bt, int iters);
int coarse_batch_collect(coarse_batch *bt, int64_t *tags, coarse_stats *stats, int cap, int *n_done);
int coarse_batch_live(const coarse_batch *bt);
int coarse_batch_destroy(coarse_batch *bt);

/* Release all memory of the context. NULL is accepted. */
int coarse_destroy(coarse_ctx *ctx);

/* Device bytes held by the context (for admission by HBM budget). */
size_t coarse_device_bytes(const coarse_ctx *ctx);

/* Sizes of the built context. */
int coarse_get_info(const coarse_ctx *ctx, coarse_info_t *info);

/* w = A_r y with the 27-point stencil of the reduced operator on the structured
 * box grid (Sec. 4, eq. (Aij): the cell-assembled A_r of the centroid
 * interpolation couples a box vertex only with box vertices at most one box away
 * per direction). y and w are device arrays of (b_x+1)(b_y+1)(b_z+1) doubles,
 * box vertex (i, j, k) at i + (b_x+1)(j + (b_y+1)k) (coarse_info_t.boxes gives
 * b); w is written at every box vertex, 0 at the inactive ones (those that hold
 * no reduced unknown), and y is not read there. Ordered on the context's stream.
 * COARSE_EINVAL for a context with the standard interpolation (its Galerkin A_r
 * has a wider stencil) or without reduced unknowns. */
int coarse_apply_reduced_operator(coarse_ctx *ctx, const double *y, double *w);

/* Change the stream used by later calls on this context. */
int coarse_set_stream(coarse_ctx *ctx, void *stream);

/* Phase timers (HIP events on the context's stream around every launch of a
 * phase). enable != 0 is a bit mask of the phases to time (bit i = phase i;
 * 0xFF = all): it clears the accumulators and starts timing. enable = 0 waits for
 * the stream, stops, and writes the accumulated milliseconds and launch counts of
 * the first nphase phases into ms[] and counts[] (either may be NULL).
 * Phases: 0 operator A (with the search-direction update), 1 the convergence
 * test of PCG, with the first stage of J^T when the reduced system shares the
 * local systems' stream (additive mode) and the restriction gather R_p r for the
 * inexact local solves (with stored inverses the dense solves gather r_p
 * themselves), 2 reduced restriction J^T (corner sums), 3 batched dense solves
 * A_p^{-1} and A_r^{-1} (the tiled GEMV kernel alone), 4 partial-sum combine,
 * 5 overlap sum + J prolongation (with (r, z)), 6 PCG vector update, 7 the reduced
 * branch of the additive two-level preconditioner (both stages of J^T, the dense
 * solve of A_r and its partial sums) when it runs on the context's second stream
 * beside the local solves (coarse_info_t.reduced_stream; phases 3 and 4 then
 * cover the local systems alone, and phase 2 is not used). */
#define COARSE_NPHASE 8
int coarse_profile(coarse_ctx *ctx, int enable, double *ms, int64_t *counts, int nphase);

/* Host-only dry run of the combinatorial setup (no device is touched): fills
 * *info with n_free, n_sub, sum_np, max_np, n_r, n_cells and boxes; if sizes is
 * not NULL, sizes[p] receives |R_p| for p < n_part. Errors: EINVAL, EMESH. */
int coarse_plan_info(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts,
                     coarse_info_t *info, int64_t *sizes);

/* Message for a status code; last failure message of a context (or, when ctx
 * is NULL, of the last failed coarse_setup on the calling host thread). */
const char *coarse_strerror(int code);
const char *coarse_last_error(const coarse_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* COARSE_H */
