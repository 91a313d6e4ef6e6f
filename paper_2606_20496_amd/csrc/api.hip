// C-ABI of the coarse solver: context setup, preconditioner application and
// PCG, orchestrating the kernels of kernels.hip on one HIP stream.
#include "kernels.hip"
#include "multi.hip"
#include "local_pcg.hip"
#include "stencil.hip"
#include "capture_guard.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/coarse.h"

using namespace coarse;

namespace {

thread_local std::string g_setup_error;   // setups may run on several host threads

// graph captures of lock-step batches against setups, destructions and block-
// solve allocations made by any host thread
CaptureGuard g_guard;

struct Fail : std::runtime_error {
  int code;
  Fail(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess)                                                                              \
      throw Fail(e_ == hipErrorOutOfMemory ? COARSE_ENOMEM : COARSE_EDEVICE,                           \
                 std::string(#expr) + ": " + hipGetErrorString(e_));                                   \
  } while (0)

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The device's default stream-ordered memory pool keeps what it holds between
// setups (by default it would give memory back at every synchronisation).
std::mutex g_pool_mu;
bool g_pool_ready[64] = {};

void keep_pool_memory() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (g_pool_ready[dev]) return;
  hipMemPool_t pool = nullptr;
  HIPCHK(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t keep = UINT64_MAX;
  HIPCHK(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  g_pool_ready[dev] = true;
}

// Small pinned host blocks (solver states read back by the host) carved from
// 1 MiB slabs that the process keeps: setting up and destroying contexts then
// allocates and frees no pinned memory (freeing pinned memory synchronises the
// device).
class PinnedPool {
 public:
  static constexpr size_t kBlock = 4096, kSlab = size_t(1) << 20;
  void *get(size_t n) {
    if (n > kBlock) throw Fail(COARSE_EINVAL, "pinned block request too large");
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) {
      void *slab = nullptr;
      HIPCHK(hipHostMalloc(&slab, kSlab, hipHostMallocDefault));
      for (size_t k = 0; k < kSlab / kBlock; ++k) free_.push_back((char *)slab + k * kBlock);
    }
    void *p = free_.back();
    free_.pop_back();
    return p;
  }
  void put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<void *> free_;
};
PinnedPool g_pinned;

// Pinned host slabs for staging small uploads (a copy from pinned memory runs
// asynchronously; one from pageable memory is staged by the runtime, call by
// call). A setup takes slabs as it needs them and returns them once its stream
// has been synchronised. The slabs are kept for the life of the process.
class StagingPool {
 public:
  static constexpr size_t kSlab = size_t(1) << 20;
  void *get() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) {
      void *slab = nullptr;
      HIPCHK(hipHostMalloc(&slab, kSlab, hipHostMallocDefault));
      return slab;
    }
    void *p = free_.back();
    free_.pop_back();
    return p;
  }
  void put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<void *> free_;
};
StagingPool g_staging;

// Non-blocking streams for the contexts' second stream, kept for reuse:
// creating a stream costs far more than the rest of a small context's setup.
class StreamPool {
 public:
  hipStream_t get() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (!free_.empty()) {
        hipStream_t s = free_.back();
        free_.pop_back();
        return s;
      }
    }
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  // the caller has synchronised the stream
  void put(hipStream_t s) {
    if (!s) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(s);
  }

 private:
  std::mutex mu_;
  std::vector<hipStream_t> free_;
};
StreamPool g_streams;

// Device memory of a context (hipMalloc, freed at release), or with a stream
// the temporaries of a setup: stream-ordered allocations from the device's
// pool, freed in stream order, so that releasing them does not synchronise the
// device (a plain hipFree would wait for every stream, the solves of other
// contexts included).
//
// Small allocations (at most kSmall bytes) are carved from kChunk-byte blocks
// (256-byte aligned), so a context makes a handful of allocations instead of a
// hundred; `bytes` counts what the arena holds from the device.
struct Arena {
  static constexpr size_t kSmall = size_t(64) << 10, kChunk = size_t(512) << 10, kAlign = 256;
  std::vector<void *> ptrs;
  size_t bytes = 0;
  hipStream_t ordered = nullptr;
  bool stream_ordered = false;
  char *chunk = nullptr;
  size_t chunk_used = kChunk;
  Arena() = default;
  explicit Arena(hipStream_t s) : ordered(s), stream_ordered(true) { keep_pool_memory(); }
  void *raw(size_t nb) {
    void *p = nullptr;
    if (stream_ordered)
      HIPCHK(hipMallocAsync(&p, nb, ordered));
    else
      HIPCHK(hipMalloc(&p, nb));
    ptrs.push_back(p);
    bytes += nb;
    return p;
  }
  template <typename T>
  T *alloc(size_t n) {
    if (n == 0) n = 1;
    const size_t nb = n * sizeof(T);
    if (nb > kSmall) return (T *)raw(nb);
    const size_t nba = (nb + kAlign - 1) / kAlign * kAlign;
    if (chunk_used + nba > kChunk) {
      chunk = (char *)raw(kChunk);
      chunk_used = 0;
    }
    T *p = (T *)(chunk + chunk_used);
    chunk_used += nba;
    return p;
  }
  // Uploads are stream-ordered and not waited for. Small ones go through pinned
  // staging (the host data is copied at once, so the source may go away); the
  // staging slabs, like a temporary source of a large upload (an rvalue, kept in
  // `hold`), are released by drop_hold(), which the caller calls after its next
  // synchronisation of the stream. A large upload from an lvalue needs its
  // source to live until then.
  std::vector<std::shared_ptr<void>> hold;
  std::vector<void *> staging;
  size_t staging_used = StagingPool::kSlab;
  template <typename T>
  T *upload(const std::vector<T> &v, hipStream_t s) {
    T *p = alloc<T>(v.size());
    const size_t nb = v.size() * sizeof(T);
    if (nb == 0) return p;
    if (nb <= kSmall) {
      const size_t nba = (nb + kAlign - 1) / kAlign * kAlign;
      if (staging_used + nba > StagingPool::kSlab) {
        staging.push_back(g_staging.get());
        staging_used = 0;
      }
      char *h = (char *)staging.back() + staging_used;
      staging_used += nba;
      std::memcpy(h, v.data(), nb);
      HIPCHK(hipMemcpyAsync(p, h, nb, hipMemcpyHostToDevice, s));
    } else {
      HIPCHK(hipMemcpyAsync(p, v.data(), nb, hipMemcpyHostToDevice, s));
    }
    return p;
  }
  template <typename T>
  T *upload(std::vector<T> &&v, hipStream_t s) {
    if (v.size() * sizeof(T) <= kSmall) return upload(v, s);
    auto kept = std::make_shared<std::vector<T>>(std::move(v));
    hold.push_back(kept);
    return upload(*kept, s);
  }
  void drop_hold() {
    hold.clear();
    for (void *h : staging) g_staging.put(h);
    staging.clear();
    staging_used = StagingPool::kSlab;
  }
  void release() {
    for (void *p : ptrs) (void)(stream_ordered ? hipFreeAsync(p, ordered) : hipFree(p));
    ptrs.clear();
    bytes = 0;
    chunk = nullptr;
    chunk_used = kChunk;
  }
  ~Arena() {
    // staging still held: its copies may be in flight
    if (!staging.empty() && ordered) (void)hipStreamSynchronize(ordered);
    drop_hold();
    release();
  }
};

// Several small uploads as one copy: add() packs a host array into the arena's
// pinned staging and notes where its device address goes; commit() (also at the
// end of the batch's scope) carves one device block for all of them, issues one
// copy and writes the addresses. Arrays of more than Arena::kSmall bytes are
// uploaded on their own at add(). Commit before anything reads the addresses or
// the data.
class UploadBatch {
 public:
  UploadBatch(Arena &a, hipStream_t s) : a_(a), s_(s) {}
  UploadBatch(const UploadBatch &) = delete;
  UploadBatch &operator=(const UploadBatch &) = delete;
  ~UploadBatch() {
    try {
      commit();
    } catch (...) {
    }
  }
  template <typename P, typename T>
  void add(P *dst, const std::vector<T> &v) {
    const size_t nb = v.size() * sizeof(T);
    if (nb > Arena::kSmall) {
      *dst = (P)a_.upload(v, s_);
      return;
    }
    const size_t nba = (std::max<size_t>(nb, sizeof(T)) + Arena::kAlign - 1) / Arena::kAlign * Arena::kAlign;
    if (a_.staging_used + nba > StagingPool::kSlab) {
      commit();
      a_.staging.push_back(g_staging.get());
      a_.staging_used = 0;
    }
    if (fix_.empty()) start_ = a_.staging_used;
    const size_t off = a_.staging_used - start_;
    if (nb) std::memcpy((char *)a_.staging.back() + a_.staging_used, v.data(), nb);
    a_.staging_used += nba;
    fix_.push_back([dst, off](char *base) { *dst = (P)(base + off); });
  }
  template <typename P, typename T>
  void add(P *dst, std::vector<T> &&v) {
    if (v.size() * sizeof(T) > Arena::kSmall) {
      *dst = (P)a_.upload(std::move(v), s_);
      return;
    }
    add(dst, static_cast<const std::vector<T> &>(v));
  }
  void commit() {
    if (fix_.empty()) return;
    const size_t total = a_.staging_used - start_;
    char *d = a_.alloc<char>(total);
    HIPCHK(hipMemcpyAsync(d, (char *)a_.staging.back() + start_, total, hipMemcpyHostToDevice, s_));
    for (auto &f : fix_) f(d);
    fix_.clear();
  }

 private:
  Arena &a_;
  hipStream_t s_;
  size_t start_ = 0;
  std::vector<std::function<void(char *)>> fix_;
};

// largest box grid whose reduced solution the final kernel stages in LDS (with
// 512-thread workgroups, four per compute unit still fit its 160 KiB)
constexpr int64_t kYLdsMaxBytes = 40 * 1024;

// upper bounds on a system's tile count per work-item bucket (the last is open)
const int kGemvBucketMax[COARSE_GEMV_BUCKETS] = {2, 4, 8, 12, 16, 24, 48, 1 << 30};

inline unsigned nblk(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

// The dense solves of one application: the whole-system workgroups (nwhole
// systems, wsegs, nw wavefronts each) and the work items (segs), in one launch
// when there are whole systems; either may be empty.
// gin != nullptr: the whole-system workgroups of local systems gather their
// right-hand sides r_p = R_p gin themselves (through SysDev::gidx) instead of
// reading the packed vectors (work items always read the packed vectors)
template <int NW>
void launch_whole(hipStream_t s, int precision, const Seg *segs, int nseg, int nitems, const Seg *wsegs, int nwhole,
                  int whole_lds, const int *done, const double *gin, const PcgCheck &ck) {
  const unsigned g = (unsigned)nwhole + (nitems > 0 ? nblk(nitems, NW) : 0u);
  if (precision == COARSE_FP64)
    hipLaunchKernelGGL(k_gemv_whole_f64<NW>, dim3(g), dim3(NW * WAVE), whole_lds, s, segs, nseg, nitems, wsegs,
                       nwhole, done, gin, ck);
  else if (precision == COARSE_MIXED_F16)
    hipLaunchKernelGGL(k_gemv_whole_f16<NW>, dim3(g), dim3(NW * WAVE), whole_lds, s, segs, nseg, nitems, wsegs,
                       nwhole, done, gin, ck);
  else
    hipLaunchKernelGGL(k_gemv_whole_f32<NW>, dim3(g), dim3(NW * WAVE), whole_lds, s, segs, nseg, nitems, wsegs,
                       nwhole, done, gin, ck);
}

// ck.sc != nullptr: the launch carries the convergence test of PCG
void launch_gemv(hipStream_t s, int precision, int nw, const Seg *segs, int nseg, int nitems, const Seg *wsegs,
                 int nwhole, int whole_lds, const int *done, const double *gin, const PcgCheck &ck = PcgCheck{}) {
  if (nwhole > 0) {
    switch (nw) {
      case 2: launch_whole<2>(s, precision, segs, nseg, nitems, wsegs, nwhole, whole_lds, done, gin, ck); break;
      case 8: launch_whole<8>(s, precision, segs, nseg, nitems, wsegs, nwhole, whole_lds, done, gin, ck); break;
      case 16: launch_whole<16>(s, precision, segs, nseg, nitems, wsegs, nwhole, whole_lds, done, gin, ck); break;
      default: launch_whole<4>(s, precision, segs, nseg, nitems, wsegs, nwhole, whole_lds, done, gin, ck); break;
    }
  } else if (nitems > 0) {
    // one wavefront per work item (the kernel also loops over a smaller grid, but
    // one item per wavefront measured fastest on MI355X at every size tried)
    const unsigned g = nblk(nitems, 4);
    const bool chunk = nitems <= ITEM_CHUNK_MAX_ITEMS;   // few items: latency-bound
    if (precision == COARSE_FP64)
      hipLaunchKernelGGL(k_gemv_f64, dim3(g), dim3(256), 0, s, segs, nseg, nitems, done, ck);
    else if (precision == COARSE_MIXED_F16) {
      if (chunk)
        hipLaunchKernelGGL(k_gemv_f16<ITEM_CHUNK>, dim3(g), dim3(256), 0, s, segs, nseg, nitems, done, ck);
      else
        hipLaunchKernelGGL(k_gemv_f16<1>, dim3(g), dim3(256), 0, s, segs, nseg, nitems, done, ck);
    } else {
      if (chunk)
        hipLaunchKernelGGL(k_gemv_f32<ITEM_CHUNK>, dim3(g), dim3(256), 0, s, segs, nseg, nitems, done, ck);
      else
        hipLaunchKernelGGL(k_gemv_f32<1>, dim3(g), dim3(256), 0, s, segs, nseg, nitems, done, ck);
    }
  }
}

// Wavefronts per whole-system workgroup that a context may choose, per tile type
inline bool whole_waves_ok(int precision, int nw) {
  return precision == COARSE_FP64 ? (nw == 2 || nw == 4 || nw == 8) : (nw == 4 || nw == 8 || nw == 16);
}

}  // namespace

// Host half of a setup: everything the device half uploads, built without any
// HIP call (so it may be built on any host thread).
struct coarse_plan {
  Plan P;
  coarse_opts o;
  double t_plan = 0.0;
};

struct coarse_ctx {
  std::string err;
  hipStream_t stream = nullptr;
  // second stream of the additive preconditioner: the reduced-space branch (J^T
  // corner sums, the dense solve of A_r) runs beside the local dense solves
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int precision = 0, mode = 0, interp = 0, max_it = 1000, check_every = 4, flexible = 0;
  int64_t nv = 0, ne = 0, nf = 0, n_r = 0, nent = 0, ntask = 0;
  int64_t n_local_sys = 0, vec_len = 0, coarse_vec_off = 0;
  int32_t items_local = 0, items_total = 0, rows_local = 0, rows_total = 0;
  int32_t whole_local = 0, whole_total = 0;   // systems solved by one workgroup each
  int32_t whole_lds = 0;                      // LDS bytes of such a workgroup
  int whole_waves = 4;                        // wavefronts of such a workgroup
  int nvblk = 1;
  double t_setup = 0.0;
  coarse_info_t info{};
  Arena arena;

  OpDev op{};
  int32_t *user_of_vint = nullptr, *vint_of_user = nullptr;
  double *x = nullptr, *r = nullptr, *p = nullptr, *pb = nullptr, *z = nullptr, *q = nullptr, *bint = nullptr,
         *t1 = nullptr, *t2 = nullptr, *part1 = nullptr, *part2 = nullptr, *energy = nullptr;
  double *prr = nullptr;     // partial sums of ||r||^2 (and of ||b||^2 at the start)
  int last_iters = 0;        // iterations of the previous solve (first batch size)
  int gemv_tiles[COARSE_GEMV_BUCKETS] = {};   // work-item table this context was built with
  Scalars *sc = nullptr;
  Scalars *h_sc = nullptr;   // pinned host copy
  int *zero_flag = nullptr;  // a device int that is always 0
  int *done_flag = nullptr;  // &sc->done

  // initial guess by projection onto prior solutions: A-orthonormal basis X and
  // A X, proj_max rows of nf entries each, proj_n of them in use
  int proj_max = 0, proj_n = 0;
  double *proj_x = nullptr, *proj_ax = nullptr, *proj_part = nullptr, *proj_coef = nullptr;
  int *proj_count = nullptr;
  int *h_proj_count = nullptr;   // pinned host copy of the basis size after an append

  // batched dense solves
  int32_t *sub_idx = nullptr;
  void *rp = nullptr, *tiles = nullptr, *rowpart = nullptr, *colpart = nullptr;
  double *zp = nullptr;
  GItem *items = nullptr;
  int32_t *whole = nullptr;
  GRow *rows = nullptr;
  SysDev *sysdev = nullptr;
  Seg *seg_all = nullptr, *seg_local = nullptr, *seg_coarse = nullptr;
  Seg h_seg_all{}, h_seg_local{}, h_seg_coarse{};
  // the reduced system is too large for one workgroup: its dense solve (work
  // items and their partial sums) and the J^T corner sums run on the second
  // stream beside the local dense solves
  bool reduced_aside = false;
  int32_t *cover_ptr = nullptr, *cover_pos = nullptr;
  int y_lds = 0;   // the final kernel stages the reduced solution (n_bv doubles) in LDS

  // inexact local solves (local_iters > 0): A_p in ELL form, one workgroup of
  // loc_nt threads per subdomain
  // the reduced operator as a 27-point stencil on the box grid (centroid J), and
  // the refinement of the reduced solve (reduced_refine): its right-hand side,
  // solution and box-grid correction, and a copy of the system table that
  // points the reduced system at them
  double *ar_coef = nullptr;
  BoxGrid bgrid{};
  int reduced_refine = 0;
  void *r_res = nullptr;
  double *zcorr = nullptr, *ycorr = nullptr;
  SysDev *sysdev_corr = nullptr;
  Seg *seg_coarse_corr = nullptr;

  int local_iters = 0, loc_w = 0, loc_nt = 0;
  LocSys *locsys = nullptr;
  double *loc_diag = nullptr;
  uint32_t *loc_col = nullptr;
  void *loc_val = nullptr;

  // reduced space
  int32_t *jv_ptr = nullptr, *jv_occ = nullptr, *jc_vid = nullptr, *jt_start = nullptr, *jr_ptr = nullptr,
          *jr_src = nullptr, *corner_act = nullptr;
  void *jv_w = nullptr, *jv_xi = nullptr, *jc_w = nullptr, *jc_xi = nullptr, *jt_part = nullptr;
  int32_t *jv_base = nullptr, *act_bv = nullptr;
  double *yfull = nullptr;   // reduced solution on all (b+1)^3 box vertices (0 where inactive)
  int bx1 = 1, bxy1 = 1;

  // block solve of up to MC right-hand sides (FP64 contexts; buffers allocated
  // at its first use)
  std::vector<MSys> h_msys;   // per system: tiles, packed offset, size
  int64_t n_bv = 0, n_partials = 0, max_slots = 0;
  struct Multi {
    bool ready = false;
    double *X = nullptr, *R = nullptr, *Pa = nullptr, *Pb = nullptr, *Z = nullptr, *Q = nullptr, *B = nullptr;
    double *RP = nullptr, *ZP = nullptr, *tpart = nullptr, *yfull = nullptr, *partials = nullptr;
    double *part = nullptr, *part2 = nullptr, *energy = nullptr;
    MScal *ms = nullptr;
    MScal *h_ms = nullptr;   // pinned host copy
    int2 *rows = nullptr;
    MSys *sys = nullptr;
    int nrows = 0, nvb = 1, ng = 1, nt = 1, last_iters = 0;
    int32_t lds = 0;
    bool active = false;   // a block solve begun by coarse_multi_begin and not yet ended
    int k = 0;
    const double *b = nullptr;   // its right-hand sides
    double t0 = 0.0;
  } mb;

  // phase timers
  static constexpr int NPH = 8;
  int prof_mask = 0;
  double prof_ms[NPH] = {};
  int64_t prof_cnt[NPH] = {};
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  hipEvent_t ev_open[NPH] = {};

  ~coarse_ctx() {
    if (aux) {
      (void)hipStreamSynchronize(aux);
      g_streams.put(aux);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    g_pinned.put(h_sc);
    g_pinned.put(h_proj_count);
    g_pinned.put(mb.h_ms);
    for (auto &p : ev_pending) {
      ev_pool.push_back(p.second.first);
      ev_pool.push_back(p.second.second);
    }
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }

  hipEvent_t get_event() {
    if (ev_pool.empty()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      return e;
    }
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  void pbeg(int ph, hipStream_t s) {
    if (!((prof_mask >> ph) & 1)) return;
    ev_open[ph] = get_event();
    HIPCHK(hipEventRecord(ev_open[ph], s));
  }
  void pend(int ph, hipStream_t s) {
    if (!((prof_mask >> ph) & 1)) return;
    hipEvent_t e = get_event();
    HIPCHK(hipEventRecord(e, s));
    ev_pending.push_back({ph, {ev_open[ph], e}});
  }
  void pbeg(int ph) { pbeg(ph, stream); }
  void pend(int ph) { pend(ph, stream); }
  // after the stream has been synchronised: fold finished event pairs in
  void pcollect() {
    for (auto &p : ev_pending) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
      prof_ms[p.first] += ms;
      prof_cnt[p.first] += 1;
      ev_pool.push_back(p.second.first);
      ev_pool.push_back(p.second.second);
    }
    ev_pending.clear();
  }

  // ---- kernels on this context's stream ---------------------------------------
  void apply_op(const double *in, double *out, double *en, const int *done) {
    pbeg(0);
    hipLaunchKernelGGL(k_op_pass1, dim3((unsigned)op.n_blocks), dim3(OP_BLOCK), op.lds_bytes, stream, op, in, out, en,
                       done);
    if (op.n_shared > 0)
      hipLaunchKernelGGL(k_op_pass2, dim3(nblk(op.n_shared, 256)), dim3(256), 0, stream, op, out, done);
    pend(0);
  }

  template <typename T>
  void restrict_coarse(const double *in, const int *done) {
    pbeg(2);
    hipLaunchKernelGGL(k_jt_tasks<T>, dim3(nblk(ntask, 4)), dim3(256), 0, stream, (int)ntask, done, jt_start, jc_vid,
                       (const T *)jc_w, (const T *)jc_xi, nent, in, (T *)jt_part, PcgCheck{});
    corners<T>(done);
    pend(2);
  }

  // workgroups of k_pre: the gather part (one pass of UV entries per thread when
  // that takes at most 1024 workgroups, else several) and the J^T task part (one
  // task per wavefront, at most 2048 workgroups; both measured best on MI355X at
  // 64^3 and 128^3)
  int pre_gather_blocks() const { return (int)std::min<int64_t>(nblk(coarse_vec_off, 256 * UV), 1024); }
  int pre_task_blocks() const { return (int)std::min<int64_t>(nblk(ntask, 4), 2048); }

  template <typename T>
  void corners(const int *done, hipStream_t s) {
    hipLaunchKernelGGL(k_jt_corners<T>, dim3(nblk(n_r, 4)), dim3(256), 0, s, n_r, done, jr_ptr, jr_src,
                       (const T *)jt_part, (T *)rp + coarse_vec_off);
  }
  template <typename T>
  void corners(const int *done) {
    corners<T>(done, stream);
  }

  // the dense solves of a segment and the partial sums of its work items, on
  // stream s; ph_gemv / ph_comb < 0: not timed; gin != nullptr: the local
  // systems gather r_p = R_p gin themselves
  void gemv_combine(const Seg *segs, int nitems, int nrows, int nwhole, const int *done, hipStream_t s, int ph_gemv,
                    int ph_comb, const double *gin = nullptr, const PcgCheck &ck = PcgCheck{}) {
    if (nitems <= 0 && nwhole <= 0) return;
    if (ph_gemv >= 0) pbeg(ph_gemv, s);
    launch_gemv(s, precision, whole_waves, segs, 1, nitems, segs, nwhole, whole_lds, done, gin, ck);
    if (ph_gemv >= 0) pend(ph_gemv, s);
    if (nrows <= 0) return;
    if (ph_comb >= 0) pbeg(ph_comb, s);
    if (precision == COARSE_FP64)
      hipLaunchKernelGGL(k_combine<double>, dim3(nblk((int64_t)nrows * TILE, 256)), dim3(256), 0, s, segs, 1, nrows,
                         done);
    else
      hipLaunchKernelGGL(k_combine<float>, dim3(nblk((int64_t)nrows * TILE, 256)), dim3(256), 0, s, segs, 1, nrows,
                         done);
    if (ph_comb >= 0) pend(ph_comb, s);
  }
  void gemv_combine(const Seg *segs, int nitems, int nrows, int nwhole, const int *done,
                    const double *gin = nullptr, const PcgCheck &ck = PcgCheck{}) {
    gemv_combine(segs, nitems, nrows, nwhole, done, stream, 3, 4, gin, ck);
  }

  // one step of iterative refinement of the reduced solve just made on stream s:
  // the residual r_r - A_r y by the stencil sweep, its solve with the same
  // stored inverse, and y += the correction
  template <typename T>
  void refine_reduced(const int *done, hipStream_t s) {
    if (!reduced_refine || n_r <= 0) return;
    hipLaunchKernelGGL(k_ar_resid<T>, dim3(nblk(n_r, 256)), dim3(256), 0, s, n_r, done, (const int32_t *)act_bv,
                       (const double *)ar_coef, bgrid, (const double *)yfull, (const T *)rp + coarse_vec_off,
                       (T *)r_res);
    gemv_combine(seg_coarse_corr, items_total - items_local, rows_total - rows_local, whole_total - whole_local, done,
                 s, -1, -1);
    hipLaunchKernelGGL(k_ar_add, dim3(nblk(n_r, 256)), dim3(256), 0, s, n_r, done, (const int32_t *)act_bv,
                       (const double *)ycorr, yfull);
  }

  // the local solves of one application on the context's stream: the stored
  // inverses (gin != nullptr: they gather r_p = R_p gin themselves), or
  // local_iters steps of Jacobi-PCG per subdomain on the gathered packed vectors
  // (phase 3 either way)
  template <typename T>
  void local_part(const double *gin, const int *done, const PcgCheck &ck = PcgCheck{}) {
    if (local_iters <= 0) {
      gemv_combine(seg_local, items_local, rows_local, whole_local, done, gin, ck);
      return;
    }
    if (n_local_sys <= 0) return;
    pbeg(3);
    if (precision == COARSE_FP64)
      hipLaunchKernelGGL((k_local_pcg<double, T>), dim3((unsigned)n_local_sys), dim3(loc_nt), 0, stream, locsys, loc_w,
                         local_iters, done, (const T *)rp, (const double *)loc_diag, (const uint32_t *)loc_col,
                         (const double *)loc_val, zp);
    else
      hipLaunchKernelGGL((k_local_pcg<float, T>), dim3((unsigned)n_local_sys), dim3(loc_nt), 0, stream, locsys, loc_w,
                         local_iters, done, (const T *)rp, (const double *)loc_diag, (const uint32_t *)loc_col,
                         (const float *)loc_val, zp);
    pend(3);
  }

  // scal: count the iteration in the solver state (PCG); start: first application
  template <typename T>
  void final_step(const double *add, bool local, bool coarse, double *out, const double *rdot, double *p1, double *p2,
                  const int *done, bool scal, int start) {
    pbeg(5);
    const int yl = (coarse && y_lds) ? 1 : 0;
    hipLaunchKernelGGL(k_final<T>, dim3(nvblk), dim3(VW), yl ? n_bv * sizeof(double) : 0, stream, nf, done, add,
                       local ? cover_ptr : nullptr, (const int32_t *)cover_pos, (const double *)zp,
                       coarse ? jv_ptr : nullptr, jv_base,
                       (const T *)jv_w, (const T *)jv_xi, nent, bx1, bxy1, (const double *)yfull, (int)n_bv, yl, out,
                       rdot, p1, p2, scal ? sc : nullptr, start);
    pend(5);
  }

  // chk != nullptr: the convergence test of PCG runs first, from these partials.
  // When every local system is solved by a whole-system workgroup from its stored
  // inverse, the dense solves gather r_p = R_p in themselves (the packed vectors
  // are then not written); otherwise (work items, inexact local solves) a launch
  // of its own gathers them first.
  template <typename T>
  void precond_parts(const double *in, const double *add, bool local, bool coarse, double *out, const double *rdot,
                     double *p1, double *p2, const int *done, bool scal, int start, const double *chk) {
    const bool fuse = local && local_iters <= 0 && items_local == 0;
    const bool gather = local && !fuse;   // packed r_p written by a launch of its own
    const double *gin = fuse ? in : nullptr;
    if (local && coarse) {
      if (!reduced_aside && local_iters <= 0) {
        // a reduced system of at most WHOLE_NB_MAX tile rows joins the local
        // systems in one dense-solve launch: the convergence test and the first
        // stage of J^T in one launch, the corner sums, then the dense solves
        pbeg(1);
        const int ng = gather ? pre_gather_blocks() : 0;
        hipLaunchKernelGGL(k_pre<T>, dim3(std::max(ng + pre_task_blocks(), 1)), dim3(256), 0, stream, ng,
                           coarse_vec_off, done, sub_idx, in, (T *)rp, (int)ntask, jt_start, jc_vid, (const T *)jc_w,
                           (const T *)jc_xi, nent, (T *)jt_part, chk ? sc : nullptr, chk, nvblk, start);
        pend(1);
        pbeg(2);
        corners<T>(done);
        pend(2);
        gemv_combine(seg_all, items_total, rows_total, whole_total, done, gin);
        refine_reduced<T>(done, stream);
        final_step<T>(add, local, coarse, out, rdot, p1, p2, done, scal, start);
        return;
      }
      // The convergence test, the whole reduced-space branch on the second
      // stream (both stages of J^T, the dense solve of A_r and its partial sums)
      // beside the local solves; the two meet before the overlap sum. With
      // stored inverses in whole-system workgroups the local dense-solve launch
      // carries the test (its workgroup 0 records it) and so does the J^T launch
      // of the second stream (which records nothing); work items and the inexact
      // local solves need the gathered packed vectors, whose launch carries it
      // instead. Across hardware queues
      // each of the two waits costs some microseconds, which a large reduced
      // system (its long tile rows end the fused launch late, and its partial
      // sums need a combine pass) repays and a small one does not. Inexact local
      // solves have a launch of their own, so the reduced branch always runs
      // beside them.
      const PcgCheck ck_lead{chk ? sc : nullptr, chk, (int32_t)nvblk, start, 1, 0};
      const PcgCheck ck_aux{chk ? sc : nullptr, chk, (int32_t)nvblk, start, 0, 0};
      if (gather) {
        pbeg(1);
        hipLaunchKernelGGL(k_pre<T>, dim3(pre_gather_blocks()), dim3(256), 0, stream, pre_gather_blocks(),
                           coarse_vec_off, done, sub_idx, in, (T *)rp, 0, jt_start, jc_vid, (const T *)jc_w,
                           (const T *)jc_xi, nent, (T *)jt_part, chk ? sc : nullptr, chk, nvblk, start);
        pend(1);
      }
      HIPCHK(hipEventRecord(ev_fork, stream));
      HIPCHK(hipStreamWaitEvent(aux, ev_fork, 0));
      pbeg(7, aux);
      if (ntask > 0)
        hipLaunchKernelGGL(k_jt_tasks<T>, dim3(nblk(ntask, 4)), dim3(256), 0, aux, (int)ntask, done, jt_start,
                           jc_vid, (const T *)jc_w, (const T *)jc_xi, nent, in, (T *)jt_part,
                           gather ? PcgCheck{} : ck_aux);
      corners<T>(done, aux);
      gemv_combine(seg_coarse, items_total - items_local, rows_total - rows_local, whole_total - whole_local, done, aux,
                   -1, -1);
      refine_reduced<T>(done, aux);
      pend(7, aux);
      HIPCHK(hipEventRecord(ev_join, aux));
      local_part<T>(gin, done, gather ? PcgCheck{} : ck_lead);
      HIPCHK(hipStreamWaitEvent(stream, ev_join, 0));
    } else {
      if (chk) hipLaunchKernelGGL(k_check, dim3(1), dim3(256), 0, stream, sc, chk, nvblk, start);
      if (gather) {
        pbeg(1);
        hipLaunchKernelGGL(k_gather<T>, dim3(nblk(coarse_vec_off, VB)), dim3(VB), 0, stream, coarse_vec_off, done,
                           sub_idx, in, (T *)rp);
        pend(1);
      }
      if (coarse) restrict_coarse<T>(in, done);
    }
    if (local && !coarse)
      local_part<T>(gin, done);
    else if (coarse && !local) {
      gemv_combine(seg_coarse, items_total - items_local, rows_total - rows_local, whole_total - whole_local, done);
      refine_reduced<T>(done, stream);
    }
    final_step<T>(add, local, coarse, out, rdot, p1, p2, done, scal, start);
  }

  template <typename T>
  void precond_t(const double *in, double *out, const double *rdot, double *p1, double *p2, const int *done, bool scal,
                 int start, const double *chk) {
    switch (mode) {
      case COARSE_ADDITIVE:
        precond_parts<T>(in, nullptr, true, true, out, rdot, p1, p2, done, scal, start, chk);
        break;
      case COARSE_LOCAL_ONLY:
        precond_parts<T>(in, nullptr, true, false, out, rdot, p1, p2, done, scal, start, chk);
        break;
      case COARSE_REDUCED_ONLY:
        precond_parts<T>(in, nullptr, false, true, out, rdot, p1, p2, done, scal, start, chk);
        break;
      case COARSE_HYBRID_SYM:
        // z0 = M_r r; z1 = z0 + M_loc (r - A z0); z = z1 + M_r (r - A z1)
        precond_parts<T>(in, nullptr, false, true, t1, nullptr, nullptr, nullptr, done, false, start, chk);
        apply_op(t1, q, nullptr, done);
        hipLaunchKernelGGL(k_sub, dim3(nvblk), dim3(VB), 0, stream, nf, done, in, q, t2);
        precond_parts<T>(t2, t1, true, false, t1, nullptr, nullptr, nullptr, done, false, 0, nullptr);
        apply_op(t1, q, nullptr, done);
        hipLaunchKernelGGL(k_sub, dim3(nvblk), dim3(VB), 0, stream, nf, done, in, q, t2);
        precond_parts<T>(t2, t1, false, true, out, rdot, p1, p2, done, scal, start, nullptr);
        break;
      case COARSE_HYBRID:
        // eqs. (asm1)-(asm2): z_loc = M_loc r; z = z_loc + M_r (r - A z_loc)
        precond_parts<T>(in, nullptr, true, false, t1, nullptr, nullptr, nullptr, done, false, start, chk);
        apply_op(t1, q, nullptr, done);
        hipLaunchKernelGGL(k_sub, dim3(nvblk), dim3(VB), 0, stream, nf, done, in, q, t2);
        precond_parts<T>(t2, t1, false, true, out, rdot, p1, p2, done, scal, start, nullptr);
        break;
    }
  }

  void precond(const double *in, double *out, const double *rdot, double *p1, double *p2, const int *done,
               bool scal = false, int start = 0, const double *chk = nullptr) {
    if (precision == COARSE_FP64)
      precond_t<double>(in, out, rdot, p1, p2, done, scal, start, chk);
    else
      precond_t<float>(in, out, rdot, p1, p2, done, scal, start, chk);
  }

  // One PCG iteration k (skipped on the device once the solve has finished):
  //   beta, p_k = z_k + beta p_{k-1}, q = A p_k     (operator kernel)
  //   alpha, x += alpha p_k, r -= alpha q, ||r||^2  (update kernel)
  //   stop?, z = M r, (r, z)                        (preconditioner kernels)
  void iteration() {
    op_update();
    precond(r, z, r, part1, flexible ? part2 : nullptr, done_flag, true, 0, prr);
  }

  void op_update() {
    pbeg(0);
    if (op.ae_nt)
      hipLaunchKernelGGL((k_op_fused<true>), dim3((unsigned)op.n_blocks), dim3(OP_BLOCK), op.lds_bytes, stream, op,
                         (const double *)z, p, pb, q, energy, sc, (const double *)part1, (const double *)part2, nvblk);
    else
      hipLaunchKernelGGL((k_op_fused<false>), dim3((unsigned)op.n_blocks), dim3(OP_BLOCK), op.lds_bytes, stream, op,
                         (const double *)z, p, pb, q, energy, sc, (const double *)part1, (const double *)part2, nvblk);
    pend(0);
    pbeg(6);
    hipLaunchKernelGGL(k_update_fused, dim3(nvblk), dim3(VW), 0, stream, nf, op, sc, x, r, (const double *)p,
                       (const double *)pb, (const double *)q, (const double *)energy, (int)op.n_blocks, prr);
    pend(6);
  }

  // This context's per-iteration state for the grouped launches of a lock-step
  // batch (the same arguments its own launches of op_update, k_pre, the J^T
  // corners and k_final take in additive mode).
  void fill_iter(IterDev &d) const {
    d.op = op;
    d.nf = nf;
    d.n_pack = coarse_vec_off;
    d.nent = nent;
    d.n_r = n_r;
    d.sc = sc;
    d.x = x;
    d.r = r;
    d.pa = p;
    d.pb = pb;
    d.z = z;
    d.q = q;
    d.energy = energy;
    d.part1 = part1;
    d.part2 = part2;
    d.prr = prr;
    d.zp = zp;
    d.yfull = yfull;
    d.n_bv = (int32_t)n_bv;
    d.y_lds = y_lds;
    d.sub_idx = sub_idx;
    d.jt_start = jt_start;
    d.jc_vid = jc_vid;
    d.jr_ptr = jr_ptr;
    d.jr_src = jr_src;
    d.cover_ptr = cover_ptr;
    d.cover_pos = cover_pos;
    d.jv_ptr = jv_ptr;
    d.jv_base = jv_base;
    d.rp = rp;
    d.jt_part = jt_part;
    d.jc_w = jc_w;
    d.jc_xi = jc_xi;
    d.jv_w = jv_w;
    d.jv_xi = jv_xi;
    d.nvblk = nvblk;
    d.ng = pre_gather_blocks();
    d.ntask = (int32_t)ntask;
    d.bx1 = bx1;
    d.bxy1 = bxy1;
    d.flexible = flexible;
    d.loc_sys = locsys;
    d.loc_diag = loc_diag;
    d.loc_col = loc_col;
    d.loc_val = loc_val;
    d.loc_w = loc_w;
    d.loc_iters = local_iters;
    d.n_loc = local_iters > 0 ? (int32_t)n_local_sys : 0;
    d.pad_loc = 0;
  }

  // nproj > 0: start from the projection of the solution onto the first nproj
  // rows of the stored basis instead of u_0 = 0
  void start(const double *b, double tol, int nproj = 0) {
    hipLaunchKernelGGL(k_start, dim3(nvblk), dim3(VB), 0, stream, nf, user_of_vint, b, r, x, p, pb, z, bint, prr, sc,
                       tol * tol, max_it, flexible);
    if (nproj > 0) proj_guess(nproj);
    precond(r, z, r, part1, flexible ? part2 : nullptr, done_flag, true, nproj > 0 ? 2 : 1, prr);
  }

  // Sec. 5: c_j = X_j . b (and ||b||^2 as the last row), u_bar = sum c_j X_j in x,
  // r_0 = b - sum c_j A X_j in r with the partials of ||r_0||^2 in prr.
  void proj_guess(int n) {
    hipLaunchKernelGGL(k_proj_dots, dim3(nvblk, n + 1), dim3(VB), 0, stream, nf, n, (const double *)proj_x, nf,
                       (const double *)bint, (const double *)bint, proj_part);
    hipLaunchKernelGGL(k_proj_totals, dim3(n + 1), dim3(256), 0, stream, (const double *)proj_part, nvblk, proj_coef,
                       sc);
    hipLaunchKernelGGL(k_proj_guess, dim3(nvblk), dim3(VB), 0, stream, nf, n, (const double *)proj_coef,
                       (const double *)proj_x, (const double *)proj_ax, nf, x, r, prr);
  }

  // Append the solution in x (with q = A x, as finish() leaves them) as row n of
  // the basis: A-Gram-Schmidt against rows 0..n-1, then normalisation; the new
  // basis size goes to *h_proj_count once the stream is synchronised.
  void proj_append(int n) {
    hipLaunchKernelGGL(k_proj_dots, dim3(nvblk, n + 1), dim3(VB), 0, stream, nf, n, (const double *)proj_x, nf,
                       (const double *)q, (const double *)x, proj_part);
    hipLaunchKernelGGL(k_proj_totals, dim3(n + 1), dim3(256), 0, stream, (const double *)proj_part, nvblk, proj_coef,
                       nullptr);
    hipLaunchKernelGGL(k_proj_orth, dim3(nvblk), dim3(VB), 0, stream, nf, n, (const double *)proj_coef, proj_x,
                       proj_ax, nf, (const double *)x, (const double *)q, proj_part);
    hipLaunchKernelGGL(k_proj_scale, dim3(nvblk), dim3(VB), 0, stream, nf, n, (const double *)proj_part, nvblk,
                       (const double *)(proj_coef + n), proj_x, proj_ax, nf, proj_count);
    HIPCHK(hipMemcpyAsync(h_proj_count, proj_count, sizeof(int), hipMemcpyDeviceToHost, stream));
  }

  void finish(double *u) {
    apply_op(x, q, nullptr, zero_flag);
    hipLaunchKernelGGL(k_resnorm, dim3(nvblk), dim3(VB), 0, stream, nf, bint, q, part1);
    hipLaunchKernelGGL(k_res_total, dim3(1), dim3(VB), 0, stream, sc, (const double *)part1, nvblk);
    hipLaunchKernelGGL(k_permute_out, dim3(nblk(nv, VB)), dim3(VB), 0, stream, nv, nf, vint_of_user, x, u);
    HIPCHK(hipMemcpyAsync(h_sc, sc, sizeof(Scalars), hipMemcpyDeviceToHost, stream));
  }

  // ---- block solve (up to MC right-hand sides; FP64, additive) ---------------
  void m_init() {
    if (mb.ready) return;
    DeviceCallScope dc(g_guard);
    hipStream_t s = stream;
    arena.ordered = s;
    Arena &A = arena;
    const int64_t nfm = nf * MC;
    mb.X = A.alloc<double>(nfm);
    mb.R = A.alloc<double>(nfm);
    mb.Pa = A.alloc<double>(nfm);
    mb.Pb = A.alloc<double>(nfm);
    mb.Z = A.alloc<double>(nfm);
    mb.Q = A.alloc<double>(nfm);
    mb.B = A.alloc<double>(nfm);
    mb.RP = A.alloc<double>(vec_len * MC);
    mb.ZP = A.alloc<double>(vec_len * MC);
    mb.tpart = A.alloc<double>(std::max<int64_t>(1, ntask) * 8 * MC);
    mb.yfull = A.alloc<double>(std::max<int64_t>(1, n_bv) * MC);
    mb.partials = A.alloc<double>(std::max<int64_t>(1, n_partials) * MC);
    mb.nvb = (int)std::min<int64_t>(1024, nblk(nfm, 256));
    mb.ng = (int)std::min<int64_t>(1024, nblk(coarse_vec_off * MC, 256));
    mb.nt = (int)std::min<int64_t>(2048, nblk(ntask, 4));
    mb.part = A.alloc<double>((size_t)mb.nvb * MC);
    mb.part2 = A.alloc<double>((size_t)mb.nvb * MC);
    mb.energy = A.alloc<double>(std::max<int64_t>(1, op.n_blocks) * MC);
    mb.ms = A.alloc<MScal>(1);
    // packing pads and inactive box vertices are never written and stay 0
    HIPCHK(hipMemsetAsync(mb.RP, 0, vec_len * MC * sizeof(double), s));
    HIPCHK(hipMemsetAsync(mb.ZP, 0, vec_len * MC * sizeof(double), s));
    HIPCHK(hipMemsetAsync(mb.yfull, 0, std::max<int64_t>(1, n_bv) * MC * sizeof(double), s));
    HIPCHK(hipMemsetAsync(mb.ms, 0, sizeof(MScal), s));
    // one wavefront per tile row; rows of the largest systems first
    std::vector<int32_t> order(h_msys.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int32_t)k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return h_msys[a].nb > h_msys[b].nb; });
    std::vector<int2> rows;
    for (int32_t k : order)
      for (int32_t I = 0; I < h_msys[k].nb; ++I) rows.push_back(make_int2(k, I));
    mb.nrows = (int)rows.size();
    mb.rows = A.upload(rows, s);
    mb.sys = A.upload(h_msys, s);
    mb.h_ms = (MScal *)g_pinned.get(sizeof(MScal));
    mb.lds = (int32_t)((OP_BLOCK * 8 + max_slots * MCW) * sizeof(double));
    // the uploads above read host vectors of this function
    HIPCHK(hipStreamSynchronize(s));
    A.drop_hold();
    mb.ready = true;
  }

  void m_scal(const double *part, int n, int step) {
    // a flexible context takes the Polak-Ribiere beta: (r_{k+1}, z_k) from k_m_final
    const double *p2 = (step == MS_RZ && flexible) ? mb.part2 : nullptr;
    hipLaunchKernelGGL(k_m_scal, dim3(1), dim3(256), 0, stream, mb.ms, part, n, step, p2);
  }

  // Z = M R for every column (additive two-level preconditioner); T: the type
  // the context stores J in
  void m_precond() {
    if (precision == COARSE_FP64)
      m_precond_t<double>();
    else
      m_precond_t<float>();
  }

  template <typename T>
  void m_precond_t() {
    pbeg(1);
    hipLaunchKernelGGL(k_m_pre<T>, dim3(mb.ng + mb.nt), dim3(256), 0, stream, mb.ng, coarse_vec_off,
                       (const int32_t *)sub_idx, (const double *)mb.R, mb.RP, (int)ntask, (const int32_t *)jt_start,
                       (const int32_t *)jc_vid, (const T *)jc_w, (const T *)jc_xi, nent, mb.tpart,
                       (const MScal *)mb.ms);
    pend(1);
    pbeg(2);
    hipLaunchKernelGGL(k_m_corners, dim3(nblk(n_r * MC, 256)), dim3(256), 0, stream, n_r, (const int32_t *)jr_ptr,
                       (const int32_t *)jr_src, (const double *)mb.tpart, mb.RP + coarse_vec_off * MC,
                       (const MScal *)mb.ms);
    pend(2);
    pbeg(3);
    const dim3 gg((nblk(mb.nrows, 4) + 7) / 8 * 8);
    if (precision == COARSE_FP64)
      hipLaunchKernelGGL(k_m_gemv<double>, gg, dim3(256), 0, stream, (const int2 *)mb.rows, mb.nrows,
                         (const MSys *)mb.sys, (const double *)mb.RP, mb.ZP, mb.yfull, (const int32_t *)act_bv,
                         (const MScal *)mb.ms);
    else if (precision == COARSE_MIXED_F16)
      hipLaunchKernelGGL(k_m_gemv<_Float16>, gg, dim3(256), 0, stream, (const int2 *)mb.rows, mb.nrows,
                         (const MSys *)mb.sys, (const double *)mb.RP, mb.ZP, mb.yfull, (const int32_t *)act_bv,
                         (const MScal *)mb.ms);
    else
      hipLaunchKernelGGL(k_m_gemv<float>, gg, dim3(256), 0, stream, (const int2 *)mb.rows, mb.nrows,
                         (const MSys *)mb.sys, (const double *)mb.RP, mb.ZP, mb.yfull, (const int32_t *)act_bv,
                         (const MScal *)mb.ms);
    pend(3);
    pbeg(5);
    hipLaunchKernelGGL(k_m_final<T>, dim3(mb.nvb), dim3(256), 0, stream, nf, (const int32_t *)cover_ptr,
                       (const int32_t *)cover_pos, (const double *)mb.ZP, (const int32_t *)jv_ptr,
                       (const int32_t *)jv_base, (const T *)jv_w, (const T *)jv_xi, nent, bx1, bxy1,
                       (const double *)mb.yfull, mb.Z, (const double *)mb.R, mb.part, flexible ? mb.part2 : nullptr,
                       (const MScal *)mb.ms);
    pend(5);
  }

  // r = b for the k columns, x = 0, z_0 = M r_0, rho_0, beta_0 = 0
  void m_start(const double *b, int k, double tol) {
    hipLaunchKernelGGL(k_m_start, dim3(mb.nvb), dim3(256), 0, stream, nf, nv, (const int32_t *)user_of_vint, b, k,
                       mb.R, mb.X, mb.Pa, mb.Pb, mb.Z, mb.B, mb.part, mb.ms, tol * tol, max_it);
    m_scal(mb.part, mb.nvb, MS_BB);
    m_precond();
    m_scal(mb.part, mb.nvb, MS_RZ);
  }

  // one PCG iteration of every live column
  void m_iteration() {
    pbeg(0);
    hipLaunchKernelGGL(k_m_op, dim3((unsigned)op.n_blocks), dim3(OP_BLOCK), mb.lds, stream, op,
                       (const double *)mb.Z, mb.Pa, mb.Pb, mb.Q, mb.partials, mb.energy, (const MScal *)mb.ms, 1);
    pend(0);
    m_scal(mb.energy, (int)op.n_blocks, MS_PQ);
    pbeg(6);
    hipLaunchKernelGGL(k_m_update, dim3(mb.nvb), dim3(256), 0, stream, nf, op, (const double *)mb.partials,
                       (const MScal *)mb.ms, mb.X, mb.R, (const double *)mb.Pa, (const double *)mb.Pb,
                       (const double *)mb.Q, mb.part);
    pend(6);
    m_scal(mb.part, mb.nvb, MS_RR);
    m_precond();
    m_scal(mb.part, mb.nvb, MS_RZ);
  }

  // true residuals, the k solutions in caller order, the state to the host
  void m_finish(double *u, int k) {
    hipLaunchKernelGGL(k_m_op, dim3((unsigned)op.n_blocks), dim3(OP_BLOCK), mb.lds, stream, op, (const double *)mb.X,
                       nullptr, nullptr, mb.Q, mb.partials, nullptr, (const MScal *)mb.ms, 0);
    if (op.n_shared > 0)
      hipLaunchKernelGGL(k_m_op_pass2, dim3(nblk(op.n_shared * MC, 256)), dim3(256), 0, stream, op,
                         (const double *)mb.partials, mb.Q);
    hipLaunchKernelGGL(k_m_resnorm, dim3(mb.nvb), dim3(256), 0, stream, nf, (const double *)mb.B,
                       (const double *)mb.Q, mb.part);
    m_scal(mb.part, mb.nvb, MS_RES);
    hipLaunchKernelGGL(k_m_permute_out, dim3(nblk(nv * k, 256)), dim3(256), 0, stream, nv, nf,
                       (const int32_t *)vint_of_user, (const double *)mb.X, k, u);
    HIPCHK(hipMemcpyAsync(mb.h_ms, mb.ms, sizeof(MScal), hipMemcpyDeviceToHost, stream));
  }

  void fill_stats(coarse_stats *st, double t0) {
    if (!st) return;
    st->iters = h_sc->iters;
    st->status = h_sc->status;
    st->relres = h_sc->bb > 0 ? std::sqrt(h_sc->rr / h_sc->bb) : 0.0;
    st->relres_true = h_sc->bb > 0 ? std::sqrt(h_sc->res_true / h_sc->bb) : 0.0;
    st->relres0 = h_sc->bb > 0 ? std::sqrt(h_sc->rr0 / h_sc->bb) : 0.0;
    st->n_basis = 0;
    st->t_setup = t_setup;
    st->t_solve = now() - t0;
  }
};

namespace {

// ---------------------------------------------------------------------------
// Setup helpers
// ---------------------------------------------------------------------------
template <typename T>
std::vector<T> cast_vec(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

// Invert a list of dense SPD systems (assembled by `assemble`) into the tile
// store `out` (type T) with the batched block sweep, in chunks that bound the
// FP64 scratch. Returns the number of systems flagged not SPD.
template <typename T, typename Assemble>
int64_t invert_systems(coarse_ctx *c, const std::vector<System> &sys, const std::vector<int64_t> &which, T *out,
                       size_t scratch_tiles_max, std::vector<float> &scales, Assemble assemble) {
  hipStream_t s = c->stream;
  int64_t nbad = 0;
  size_t i0 = 0;
  while (i0 < which.size()) {
    // chunk [i0, i1)
    size_t i1 = i0;
    int64_t tiles = 0, pans = 0;
    while (i1 < which.size()) {
      const System &S = sys[which[i1]];
      const int64_t t = S.nb * (S.nb + 1) / 2;
      if (i1 > i0 && (size_t)(tiles + t) > scratch_tiles_max) break;
      tiles += t;
      pans += S.nb;
      ++i1;
    }
    const int64_t ns = (int64_t)(i1 - i0);
    std::vector<SweepSys> ss(ns);
    std::vector<AsmSys> as(ns);
    std::vector<int64_t> oo(ns);
    std::vector<int32_t> tsys;
    std::vector<int16_t> tI, tJ;
    int64_t toff = 0, poff = 0, maxnb = 0;
    for (int64_t k = 0; k < ns; ++k) {
      const System &S = sys[which[i0 + k]];
      ss[k].tile_off = toff;
      ss[k].pan_off = poff;
      ss[k].nb = (int32_t)S.nb;
      as[k].tile_off = toff;
      as[k].vec_off = (int32_t)S.vec_off;
      as[k].n = (int32_t)S.n;
      as[k].nb = (int32_t)S.nb;
      oo[k] = S.tile_off;
      for (int I = 0; I < S.nb; ++I)
        for (int J = 0; J <= I; ++J) {
          tsys.push_back((int32_t)k);
          tI.push_back((int16_t)I);
          tJ.push_back((int16_t)J);
        }
      toff += S.nb * (S.nb + 1) / 2;
      poff += S.nb;
      maxnb = std::max<int64_t>(maxnb, S.nb);
    }
    Arena tmp(s);
    double *M = tmp.alloc<double>((size_t)toff * TILE * TILE);
    // panel strips (32 x BW per tile row) and pivot-block inverses (BW x BW)
    double *Pb = tmp.alloc<double>((size_t)poff * TILE * BW);
    double *Gb = tmp.alloc<double>((size_t)poff * TILE * BW);
    double *Dv = tmp.alloc<double>((size_t)ns * BW * BW);
    int *st = tmp.alloc<int>(ns);
    double *diag0 = tmp.alloc<double>((size_t)poff * TILE);
    SweepSys *dss;
    AsmSys *das;
    int64_t *doo;
    int32_t *dts;
    int16_t *dti, *dtj;
    {
      UploadBatch ub(tmp, s);
      ub.add(&dss, ss);
      ub.add(&das, as);
      ub.add(&doo, oo);
      ub.add(&dts, tsys);
      ub.add(&dti, tI);
      ub.add(&dtj, tJ);
    }
    HIPCHK(hipMemsetAsync(M, 0, (size_t)toff * TILE * TILE * sizeof(double), s));
    HIPCHK(hipMemsetAsync(st, 0, ns * sizeof(int), s));
    hipLaunchKernelGGL(k_pad_identity, dim3((unsigned)ns), dim3(256), 0, s, das, (int)ns, M);
    assemble(das, (int)ns, M);
    const int64_t ntiles = (int64_t)tsys.size();
    hipLaunchKernelGGL(k_save_diag, dim3((unsigned)ns), dim3(256), 0, s, dss, (const double *)M, diag0);
    if (ns * maxnb > INT32_MAX / 2 || ntiles > INT32_MAX / 2) throw Fail(COARSE_EINVAL, "too many systems for one sweep");
    const unsigned pan_grid = (unsigned)(8 * ((ns * maxnb + 7) / 8)), upd_grid = (unsigned)(8 * ((ntiles + 7) / 8));
    for (int kb = 0; (int64_t)kb * SW < maxnb; ++kb) {
      hipLaunchKernelGGL(k_bsweep_pivot, dim3((unsigned)ns), dim3(PIV_T), 0, s, kb, dss, (const double *)M, Dv,
                         (const double *)diag0, st);
      hipLaunchKernelGGL(k_bsweep_panel, dim3(pan_grid), dim3(256), 0, s, kb, (int)ns, (int)maxnb, dss,
                         (const double *)M, (const double *)Dv, Pb, Gb);
      hipLaunchKernelGGL(k_bsweep_update, dim3(upd_grid), dim3(256), 0, s, kb, (int)ntiles, dss, dts, dti, dtj, M,
                         (const double *)Dv, (const double *)Pb, (const double *)Gb);
    }
    // FP16 storage: a power-of-two scale per system keeps every entry in range
    float *dscale = nullptr;
    if (std::is_same<T, _Float16>::value) {
      dscale = tmp.alloc<float>(ns);
      hipLaunchKernelGGL(k_sys_scale, dim3((unsigned)ns), dim3(256), 0, s, dss, (const double *)M, dscale);
    }
    hipLaunchKernelGGL(k_sweep_pack<T>, dim3((unsigned)ntiles), dim3(256), 0, s, dss, dts, dti, dtj, doo, M,
                       (const float *)dscale, out);
    HIPCHK(hipGetLastError());
    std::vector<int> hst(ns);
    std::vector<float> hsc(ns, 1.0f);
    HIPCHK(hipMemcpyAsync(hst.data(), st, ns * sizeof(int), hipMemcpyDeviceToHost, s));
    if (dscale) HIPCHK(hipMemcpyAsync(hsc.data(), dscale, ns * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int v : hst) nbad += (v != 0);
    for (int64_t k = 0; k < ns; ++k) scales[which[i0 + k]] = hsc[k];
    i0 = i1;
  }
  return nbad;
}

// T: vectors, interpolation and partial sums; TT: the stored inverse tiles.
template <typename T, typename TT>
void setup_precision(coarse_ctx *c, const Plan &P, const int *gemv_tiles, int whole_waves) {
  hipStream_t s = c->stream;
  Arena &A = c->arena;
  const int64_t NE = P.n_elem, NV = P.n_vert, nf = P.n_free;
  // geometry and element matrices
  Arena tmp(s);
  double *xyz = tmp.upload(P.xyz, s);
  int32_t *e2v = tmp.upload(P.e2v, s);
  // all 36 entries for the setup's assemblies; the 28 off-diagonal ones stay for the operator
  double *Ae = tmp.alloc<double>(36 * (int64_t)nblk(NE, OP_BLOCK) * OP_BLOCK);   // blocked, see ae_at
  double *Ae28 = A.alloc<double>(28 * (int64_t)nblk(NE, OP_BLOCK) * OP_BLOCK);   // see ae28_at
  int *bad = tmp.alloc<int>(1);
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_elem_matrices, dim3(nblk(NE, 256)), dim3(256), 0, s, NE, NV, xyz, e2v, Ae, Ae28, bad);
  int hbad = 0;
  HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hbad) throw Fail(COARSE_EMESH, std::to_string(hbad) + " element(s) with det(dx/dxi) <= 0 at a Gauss point");

  // operator
  OpDev &op = c->op;
  op.E = NE;
  op.n_blocks = P.n_blocks;
  op.n_shared = (int64_t)P.sh_vid.size();
  op.Ae = Ae28;
  {
    UploadBatch ub(A, s);
    ub.add(&op.lconn, P.lconn);
    ub.add(&op.blk_slot_ptr, P.blk_slot_ptr);
    ub.add(&op.slot_vid, P.slot_vid);
    ub.add(&op.slot_dst, P.slot_dst);
    // the incidence lists only serve blocks of differently oriented elements
    ub.add(&op.blk_inc, P.blk_inc);
    if (P.any_blk_inc) {
      ub.add(&op.slot_inc_ptr, P.slot_inc_ptr);
      ub.add(&op.slot_inc, P.slot_inc);
      ub.add(&op.slot_inc8, P.slot_inc8);
    } else {
      op.slot_inc_ptr = A.alloc<int32_t>(1);
      op.slot_inc = A.alloc<uint16_t>(1);
      op.slot_inc8 = A.alloc<uint16_t>(1);
    }
    ub.add(&op.sh_vid, P.sh_vid);
    ub.add(&op.sh_ptr, P.sh_ptr);
    ub.add(&op.slot_pw, P.slot_pw);
    ub.add(&op.vq, P.vq);
  }
  op.partials = A.alloc<double>(std::max<int64_t>(1, P.n_partials));
  op.lds_bytes = (int32_t)((OP_BLOCK * 8 + P.max_slots) * sizeof(double));
  // 256 MB: the MI355X last-level (Infinity) cache
  op.ae_nt = (P.n_elem * 28 * (int64_t)sizeof(double) > (int64_t)(256ull << 20)) ? 1 : 0;
  if (op.lds_bytes > 64 * 1024) throw Fail(COARSE_EINVAL, "operator block touches too many vertices");

  // vectors
  c->nf = nf;
  c->nv = NV;
  c->ne = NE;
  c->nvblk = (int)std::min<int64_t>(1024, nblk(nf, VB));
  std::vector<int32_t> uov(P.user_of_vint.begin(), P.user_of_vint.begin() + nf);
  {
    UploadBatch ub(A, s);
    ub.add(&c->user_of_vint, uov);
    ub.add(&c->vint_of_user, P.vint_of_user);
  }
  for (double **v : {&c->x, &c->r, &c->p, &c->pb, &c->z, &c->q, &c->bint, &c->t1, &c->t2}) {
    *v = A.alloc<double>(nf);
    HIPCHK(hipMemsetAsync(*v, 0, nf * sizeof(double), s));
  }
  const int64_t npart = std::max<int64_t>(c->nvblk, 1);
  c->part1 = A.alloc<double>(npart);
  c->part2 = A.alloc<double>(npart);
  c->energy = A.alloc<double>(std::max<int64_t>(1, P.n_blocks));
  c->sc = A.alloc<Scalars>(1);
  HIPCHK(hipMemsetAsync(c->sc, 0, sizeof(Scalars), s));
  c->done_flag = (int *)((char *)c->sc + offsetof(Scalars, done));
  c->prr = A.alloc<double>(npart);
  c->zero_flag = A.alloc<int>(1);
  HIPCHK(hipMemsetAsync(c->zero_flag, 0, sizeof(int), s));
  if (c->proj_max > 0) {
    c->proj_x = A.alloc<double>((size_t)c->proj_max * nf);
    c->proj_ax = A.alloc<double>((size_t)c->proj_max * nf);
    c->proj_part = A.alloc<double>((size_t)(c->proj_max + 1) * npart);
    c->proj_coef = A.alloc<double>(c->proj_max + 1);
    c->proj_count = A.alloc<int>(1);
    c->h_proj_count = (int *)g_pinned.get(sizeof(int));
  }

  // packed vectors, systems, tiles
  c->n_local_sys = P.n_local_sys;
  c->vec_len = P.vec_len;
  c->coarse_vec_off = P.sys.back().vec_off;
  c->n_r = P.n_r;
  c->sub_idx = A.upload(P.sub_idx, s);
  c->rp = A.alloc<T>(P.vec_len);
  HIPCHK(hipMemsetAsync(c->rp, 0, P.vec_len * sizeof(T), s));
  c->zp = A.alloc<double>(P.vec_len);
  HIPCHK(hipMemsetAsync(c->zp, 0, P.vec_len * sizeof(double), s));
  // with inexact local solves only the reduced system has an inverse: its tiles
  // start the store and the dense-solve tables leave the local systems out
  const bool inexact = c->local_iters > 0;
  std::vector<System> sysv = P.sys;
  int64_t n_tiles = P.n_tiles;
  if (inexact) {
    for (int64_t k = 0; k < P.n_local_sys; ++k) sysv[k].tile_off = 0;
    n_tiles -= P.sys[P.n_local_sys].tile_off;
    sysv[P.n_local_sys].tile_off = 0;
  }
  TT *tiles = A.alloc<TT>((size_t)n_tiles * TILE * TILE);
  std::vector<float> sys_scale(P.sys.size(), 1.0f);
  c->tiles = tiles;
  GemvTable G;
  int dev = 0, n_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  build_gemv_items(P, gemv_tiles, kGemvBucketMax, COARSE_GEMV_BUCKETS, n_cu, G, inexact ? P.n_local_sys : 0);
  // transposed partials only for the systems cut into work items
  std::vector<int64_t> colpart_off(P.sys.size(), -1);
  int64_t ncolpart = 0;
  {
    std::vector<char> is_whole(P.sys.size(), 0);
    for (int32_t k : G.whole) is_whole[k] = 1;
    for (size_t k = inexact ? (size_t)P.n_local_sys : 0; k < P.sys.size(); ++k)
      if (!is_whole[k]) {
        colpart_off[k] = ncolpart;
        ncolpart += P.sys[k].nb * (P.sys[k].nb + 1) / 2;
      }
  }
  c->colpart = A.alloc<T>((size_t)std::max<int64_t>(1, ncolpart) * TILE);
  for (int b = 0; b < COARSE_GEMV_BUCKETS; ++b) c->gemv_tiles[b] = gemv_tiles[b] >= 1 ? gemv_tiles[b] : GEMV_SEG;
  c->rowpart = A.alloc<T>((size_t)G.items.size() * TILE);
  {
    UploadBatch ub(A, s);
    ub.add(&c->cover_ptr, P.cover_ptr);
    ub.add(&c->cover_pos, P.cover_pos);
  }

  // inverses of the local systems (dense assembly of A_p), or A_p itself in
  // ELL form for the inexact local solves ...
  const size_t scratch_tiles = (size_t)(1536ull << 20) / (TILE * TILE * sizeof(double));
  int32_t *vinc_ptr, *vinc;
  {
    UploadBatch ub(tmp, s);
    ub.add(&vinc_ptr, P.vinc_ptr);
    ub.add(&vinc, P.vinc);
  }
  int64_t nbad = 0;
  int64_t ell_entries = 0;
  if (inexact) {
    using V = typename std::conditional<std::is_same<TT, double>::value, double, float>::type;
    std::vector<LocSys> ls((size_t)P.n_local_sys);
    int64_t maxn = 0;
    for (int64_t k = 0; k < P.n_local_sys; ++k) {
      ls[k].vec_off = (int32_t)P.sys[k].vec_off;
      ls[k].n = (int32_t)P.sys[k].n;
      ls[k].npad = (int32_t)((P.sys[k].n + 31) / 32 * 32);
      ls[k].pad = 0;
      maxn = std::max<int64_t>(maxn, P.sys[k].n);
    }
    if (maxn > LOC_NT_MAX)
      throw Fail(COARSE_EINVAL, "inexact local solves need subdomains of at most " + std::to_string(LOC_NT_MAX) +
                                    " free vertices (largest: " + std::to_string(maxn) + ")");
    LocSys *dls = tmp.upload(ls, s);
    int *wmax = tmp.alloc<int>(1);
    HIPCHK(hipMemsetAsync(wmax, 0, sizeof(int), s));
    if (P.n_local_sys > 0)
      hipLaunchKernelGGL(k_loc_count, dim3((unsigned)P.n_local_sys), dim3(512), 0, s, (const LocSys *)dls,
                         (const int32_t *)c->sub_idx, (const int32_t *)vinc_ptr, (const int32_t *)vinc,
                         (const int32_t *)e2v, NE, nf, wmax);
    int hw = 0;
    HIPCHK(hipMemcpyAsync(&hw, wmax, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hw > LOC_WMAX)
      throw Fail(COARSE_EINVAL, "inexact local solves need at most " + std::to_string(LOC_WMAX) +
                                    " off-diagonal entries per row of A_p");
    const int W = (hw + 1) / 2 * 2;
    for (int64_t k = 0; k < P.n_local_sys; ++k) {
      ls[k].ell_off = ell_entries;
      ell_entries += (int64_t)W * ls[k].npad;
    }
    c->locsys = A.upload(ls, s);
    c->loc_w = W;
    c->loc_nt = (int)std::max<int64_t>(WAVE, (maxn + WAVE - 1) / WAVE * WAVE);
    c->loc_diag = A.alloc<double>(std::max<int64_t>(1, c->coarse_vec_off));
    c->loc_col = A.alloc<uint32_t>(std::max<int64_t>(1, ell_entries / 2));
    V *val = A.alloc<V>(std::max<int64_t>(1, ell_entries));
    c->loc_val = val;
    HIPCHK(hipMemsetAsync(c->loc_diag, 0, std::max<int64_t>(1, c->coarse_vec_off) * sizeof(double), s));
    HIPCHK(hipMemsetAsync(c->loc_col, 0, std::max<int64_t>(1, ell_entries / 2) * sizeof(uint32_t), s));
    HIPCHK(hipMemsetAsync(val, 0, std::max<int64_t>(1, ell_entries) * sizeof(V), s));
    int *lbad = tmp.alloc<int>(1);
    HIPCHK(hipMemsetAsync(lbad, 0, sizeof(int), s));
    if (P.n_local_sys > 0)
      hipLaunchKernelGGL(k_loc_fill<V>, dim3((unsigned)P.n_local_sys), dim3(512), 0, s, (const LocSys *)c->locsys, W,
                         (const int32_t *)c->sub_idx, (const int32_t *)vinc_ptr, (const int32_t *)vinc,
                         (const int32_t *)e2v, NE, nf, (const double *)Ae, c->loc_diag, c->loc_col, val, lbad);
    int hb = 0;
    HIPCHK(hipMemcpyAsync(&hb, lbad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hb) throw Fail(COARSE_ESINGULAR, std::to_string(hb) + " row(s) of a local A_p with a non-positive diagonal");
  } else {
    std::vector<int64_t> loc(P.n_local_sys);
    for (int64_t k = 0; k < P.n_local_sys; ++k) loc[k] = k;
    // the searches of the assembly run in LDS when the largest R_p fits
    int64_t maxn = 0;
    for (int64_t k = 0; k < P.n_local_sys; ++k) maxn = std::max<int64_t>(maxn, P.sys[k].n);
    const int lds_n = maxn * (int64_t)sizeof(int32_t) <= 32768 ? (int)maxn : 0;
    nbad = invert_systems<TT>(c, P.sys, loc, tiles, scratch_tiles, sys_scale, [&](AsmSys *das, int ns, double *M) {
      hipLaunchKernelGGL(k_assemble_local, dim3((unsigned)ns), dim3(256), lds_n * sizeof(int32_t), s, das, c->sub_idx,
                         vinc_ptr, vinc, e2v, NE, nf, (const double *)Ae, M, lds_n);
    });
    if (nbad) throw Fail(COARSE_ESINGULAR, std::to_string(nbad) + " local system(s) A_p not positive definite");
  }

  // ... and of the reduced system (cell assembly, eq. (Aij))
  BoxDev box;
  for (int d = 0; d < 3; ++d) {
    box.lo[d] = P.lo[d];
    box.H[d] = P.H[d];
    box.b[d] = P.b[d];
  }
  const int64_t nocc = (int64_t)P.occ_cells.size();
  int32_t *occ_cells, *occ_ptr, *occ_elems, *ar_ptr, *ar_src;
  {
    UploadBatch ub(tmp, s);
    ub.add(&occ_cells, P.occ_cells);
    ub.add(&occ_ptr, P.occ_elem_ptr);
    ub.add(&occ_elems, P.occ_elems);
    ub.add(&ar_ptr, P.ar_ptr);
    ub.add(&ar_src, P.ar_src);
  }
  double *cellmat = tmp.alloc<double>(64 * std::max<int64_t>(1, nocc));
  {
    UploadBatch ub(A, s);
    ub.add(&c->corner_act, P.occ_corner_act);
    ub.add(&c->act_bv, P.act_bv);
  }
  c->bgrid = BoxGrid{P.b[0] + 1, P.b[1] + 1, P.b[2] + 1, 0};
  std::vector<int64_t> red = {P.n_local_sys};
  const int64_t nr = P.n_r;
  if (c->interp == COARSE_J_CENTROID) {
    hipLaunchKernelGGL(k_cell_mats, dim3((unsigned)nocc), dim3(64 * CM_SLOTS), 0, s, box, occ_cells, occ_ptr, occ_elems, e2v, NE,
                       NV, nf, xyz, (const double *)Ae, cellmat);
    // A_r also as its 27-point stencil on the box grid
    if (nr > 0) {
      c->ar_coef = A.alloc<double>(27 * nr);
      HIPCHK(hipMemsetAsync(c->ar_coef, 0, 27 * nr * sizeof(double), s));
      hipLaunchKernelGGL(k_ar_stencil_build, dim3(nblk(nr, 256)), dim3(256), 0, s, nr, (const int32_t *)ar_ptr,
                         (const int32_t *)ar_src, (const int32_t *)c->corner_act, (const int32_t *)occ_cells,
                         (const int32_t *)c->act_bv, c->bgrid, P.b[0], P.b[1], (const double *)cellmat, c->ar_coef);
    }
    nbad = invert_systems<TT>(c, sysv, red, tiles, scratch_tiles, sys_scale, [&](AsmSys *, int, double *M) {
      hipLaunchKernelGGL(k_assemble_reduced, dim3(nblk(nr, 256)), dim3(256), 0, s, nr, ar_ptr, ar_src,
                         (const int32_t *)c->corner_act, (const double *)cellmat, M);
    });
  } else {
    // Galerkin A_r = J^T A J by probes, in FP64 whatever the solve precision
    const int64_t ne = (int64_t)P.jv_w.size();
    int32_t *pjv_ptr = tmp.upload(P.jv_ptr, s);
    int32_t *pjv_base = tmp.upload(P.jv_base, s);
    double *pjv_xi = tmp.upload(P.jv_xi, s);
    int32_t *pjc_vid = tmp.upload(P.jc_vid, s);
    double *pjc_w = tmp.upload(P.jc_w, s);
    double *pjc_xi = tmp.upload(P.jc_xi, s);
    int32_t *pjt = tmp.upload(P.jt_task_start, s);
    int32_t *pjr_ptr = tmp.upload(P.jr_ptr, s);
    int32_t *pjr_src = tmp.upload(P.jr_src, s);
    int32_t *pbv_act = tmp.upload(P.bv_act, s);
    int32_t *pact_bv = tmp.upload(P.act_bv, s);
    const int64_t ntask = (int64_t)P.jt_task_occ.size();
    double *pv = tmp.alloc<double>(nf), *pq = tmp.alloc<double>(nf), *prr = tmp.alloc<double>(nr);
    double *ptp = tmp.alloc<double>(8 * std::max<int64_t>(1, ntask));
    ProbeDev pr{};
    for (int d = 0; d < 3; ++d) {
      pr.p[d] = P.probe_p[d];
      pr.d[d] = P.probe_d[d];
      pr.b[d] = P.b[d];
    }
    pr.bx1 = P.b[0] + 1;
    pr.bxy1 = (P.b[0] + 1) * (P.b[1] + 1);
    nbad = invert_systems<TT>(c, sysv, red, tiles, scratch_tiles, sys_scale, [&](AsmSys *, int, double *M) {
      for (pr.c[2] = 0; pr.c[2] < pr.p[2]; ++pr.c[2])
        for (pr.c[1] = 0; pr.c[1] < pr.p[1]; ++pr.c[1])
          for (pr.c[0] = 0; pr.c[0] < pr.p[0]; ++pr.c[0]) {
            hipLaunchKernelGGL(k_probe_vec, dim3(nblk(nf, 256)), dim3(256), 0, s, nf, pr, (const int32_t *)pjv_ptr,
                               (const int32_t *)pjv_base, (const double *)pjv_xi, ne, pv);
            c->apply_op(pv, pq, nullptr, c->zero_flag);
            hipLaunchKernelGGL(k_jt_tasks<double>, dim3(nblk(ntask, 4)), dim3(256), 0, s, (int)ntask,
                               (const int *)c->zero_flag, (const int32_t *)pjt, (const int32_t *)pjc_vid,
                               (const double *)pjc_w, (const double *)pjc_xi, ne, (const double *)pq, ptp,
                               PcgCheck{});
            hipLaunchKernelGGL(k_jt_corners<double>, dim3(nblk(nr, 4)), dim3(256), 0, s, nr,
                               (const int *)c->zero_flag, (const int32_t *)pjr_ptr, (const int32_t *)pjr_src,
                               (const double *)ptp, prr);
            hipLaunchKernelGGL(k_probe_scatter, dim3(nblk(nr, 256)), dim3(256), 0, s, nr, pr,
                               (const int32_t *)pact_bv, (const int32_t *)pbv_act, (const double *)prr, M);
          }
    });
  }
  if (nbad) throw Fail(COARSE_ESINGULAR, "reduced system A_r not positive definite (empty interior box?)");

  // reduced solution on the full box-vertex grid (inactive vertices stay 0)
  c->yfull = A.alloc<double>(P.n_bv);
  c->y_lds = (P.n_bv * (int64_t)sizeof(double) <= kYLdsMaxBytes) ? 1 : 0;
  HIPCHK(hipMemsetAsync(c->yfull, 0, P.n_bv * sizeof(double), s));
  c->bx1 = P.b[0] + 1;
  c->bxy1 = (P.b[0] + 1) * (P.b[1] + 1);

  // GEMV items, combine rows, system table, segments
  std::vector<SysDev> sd(P.sys.size());
  for (size_t k = 0; k < P.sys.size(); ++k) {
    const System &S = sysv[k];
    const bool no_inverse = inexact && (int64_t)k < P.n_local_sys;
    sd[k].tiles = no_inverse ? nullptr : tiles + (size_t)S.tile_off * TILE * TILE;
    sd[k].rp = (T *)c->rp + S.vec_off;
    sd[k].colpart = colpart_off[k] >= 0 ? (T *)c->colpart + (size_t)colpart_off[k] * TILE : nullptr;
    sd[k].zp = c->zp + S.vec_off;
    sd[k].nb = (int32_t)S.nb;
    sd[k].n = (int32_t)S.n;
    sd[k].scale = sys_scale[k];
    sd[k].pad = 0;
    const bool red_sys = (int64_t)k == P.n_local_sys;
    sd[k].yfull = red_sys ? c->yfull : nullptr;
    sd[k].act_bv = red_sys ? c->act_bv : nullptr;
    sd[k].gidx = red_sys ? nullptr : (const int32_t *)c->sub_idx + S.vec_off;
  }
  c->h_msys.resize(P.sys.size());
  for (size_t k = 0; k < P.sys.size(); ++k) {
    const System &S = P.sys[k];
    MSys &m = c->h_msys[k];
    m.tiles = sd[k].tiles;
    m.voff = S.vec_off;
    m.nb = (int32_t)S.nb;
    m.n = (int32_t)S.n;
    m.red = (int64_t)k == P.n_local_sys ? 1 : 0;
    m.scale = sys_scale[k];
  }
  c->n_bv = P.n_bv;
  c->n_partials = P.n_partials;
  c->max_slots = P.max_slots;
  // item slots: index within the system's item list
  std::vector<int64_t> sys_item0(P.sys.size(), -1);
  for (size_t i = 0; i < G.items.size(); ++i)
    if (sys_item0[G.items[i].sys] < 0) sys_item0[G.items[i].sys] = (int64_t)i;
  for (size_t k = 0; k < P.sys.size(); ++k)
    sd[k].rowpart = sys_item0[k] >= 0 ? (T *)c->rowpart + (size_t)sys_item0[k] * TILE : nullptr;
  std::vector<GItem> gi(G.items.size());
  int32_t il = 0;
  for (size_t i = 0; i < G.items.size(); ++i) {
    const GemvItem &it = G.items[i];
    gi[i].sys = it.sys;
    gi[i].I = (int16_t)it.I;
    gi[i].j0 = (int16_t)it.j0;
    gi[i].j1 = (int16_t)it.j1;
    gi[i].pad = 0;
    gi[i].slot = (int32_t)(i - sys_item0[it.sys]);
    if (it.sys < P.n_local_sys) il = (int32_t)i + 1;
  }
  if (P.sys.back().nb > 32767 / 2) throw Fail(COARSE_EINVAL, "reduced system too large");
  std::vector<GRow> gr(G.row_sys.size());
  int32_t rl = 0;
  for (int64_t k = 0; k < (int64_t)gr.size(); ++k) {
    gr[k].sys = G.row_sys[k];
    gr[k].I = G.row_I[k];
    gr[k].slot0 = (int32_t)(G.row_item0[k] - sys_item0[G.row_sys[k]]);
    gr[k].nslot = G.row_nitem[k];
    if (G.row_sys[k] < P.n_local_sys) rl = (int32_t)k + 1;
  }
  {
    UploadBatch ub(A, s);
    ub.add(&c->items, gi);
    ub.add(&c->rows, gr);
    ub.add(&c->whole, G.whole);
    ub.add(&c->sysdev, sd);
  }
  c->items_local = il;
  c->items_total = (int32_t)gi.size();
  c->rows_local = rl;
  c->rows_total = (int32_t)gr.size();
  c->whole_local = G.whole_local;
  c->whole_total = (int32_t)G.whole.size();
  // wavefronts per whole-system workgroup: the caller's choice or the default for
  // the tile type, halved while one solution copy per wave of the largest such
  // system, plus its staged right-hand side, would not fit the 64 KiB of LDS a
  // workgroup may use
  int nw = whole_waves_ok(c->precision, whole_waves) ? whole_waves
                                                     : (sizeof(TT) == 8 ? WHOLE_WAVES_F64 : WHOLE_WAVES_NARROW);
  while (nw > 2 && (int64_t)(nw + 1) * G.whole_nb_max * TILE * (int64_t)sizeof(T) > 65536) nw /= 2;
  c->whole_waves = nw;
  c->whole_lds = (nw + 1) * G.whole_nb_max * TILE * (int32_t)sizeof(T);
  c->h_seg_all = Seg{c->items, c->rows, c->whole, c->sysdev, nullptr, 0, 0};
  c->h_seg_local = c->h_seg_all;
  c->h_seg_coarse = Seg{c->items + il, c->rows + rl, c->whole + c->whole_local, c->sysdev, nullptr, 0, 0};
  {
    UploadBatch ub(A, s);
    ub.add(&c->seg_all, std::vector<Seg>{c->h_seg_all});
    ub.add(&c->seg_local, std::vector<Seg>{c->h_seg_local});
    ub.add(&c->seg_coarse, std::vector<Seg>{c->h_seg_coarse});
  }
  c->reduced_aside = P.n_r > 0 && P.sys[P.n_local_sys].nb > WHOLE_NB_MAX;
  if (c->reduced_refine && P.n_r > 0) {
    const System &R = P.sys[P.n_local_sys];
    c->r_res = A.alloc<T>(R.nb * TILE);
    HIPCHK(hipMemsetAsync(c->r_res, 0, R.nb * TILE * sizeof(T), s));
    c->zcorr = A.alloc<double>(R.nb * TILE);
    c->ycorr = A.alloc<double>(P.n_bv);
    HIPCHK(hipMemsetAsync(c->ycorr, 0, P.n_bv * sizeof(double), s));
    std::vector<SysDev> sc = sd;
    sc[P.n_local_sys].rp = c->r_res;
    sc[P.n_local_sys].zp = c->zcorr;
    sc[P.n_local_sys].yfull = c->ycorr;
    c->sysdev_corr = A.upload(sc, s);
    Seg h = c->h_seg_coarse;
    h.sys = c->sysdev_corr;
    c->seg_coarse_corr = A.upload(std::vector<Seg>{h}, s);
  }

  // reduced-space interpolation entries
  c->nent = (int64_t)P.jv_w.size();
  c->ntask = (int64_t)P.jt_task_occ.size();
  {
    UploadBatch ub(A, s);
    ub.add(&c->jv_ptr, P.jv_ptr);
    ub.add(&c->jv_base, P.jv_base);
    ub.add(&c->jv_w, cast_vec<T>(P.jv_w));
    ub.add(&c->jv_xi, cast_vec<T>(P.jv_xi));
    ub.add(&c->jc_vid, P.jc_vid);
    ub.add(&c->jc_w, cast_vec<T>(P.jc_w));
    ub.add(&c->jc_xi, cast_vec<T>(P.jc_xi));
    ub.add(&c->jt_start, P.jt_task_start);
    ub.add(&c->jr_ptr, P.jr_ptr);
    ub.add(&c->jr_src, P.jr_src);
  }
  c->jt_part = A.alloc<T>(8 * std::max<int64_t>(1, c->ntask));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  A.drop_hold();

  // sizes
  coarse_info_t &in = c->info;
  in.n_free = nf;
  in.n_sub = P.n_local_sys;
  in.sum_np = 0;
  in.max_np = 0;
  for (int64_t k = 0; k < P.n_local_sys; ++k) {
    in.sum_np += P.sys[k].n;
    in.max_np = std::max<int64_t>(in.max_np, P.sys[k].n);
  }
  in.n_r = P.n_r;
  in.n_cells = nocc;
  const int64_t tl = P.sys.back().tile_off;
  in.local_bytes = tl * TILE * TILE * (int64_t)sizeof(TT);
  in.reduced_bytes = (P.n_tiles - tl) * TILE * TILE * (int64_t)sizeof(TT);
  in.inv_alg_bytes = 0;
  for (size_t k = inexact ? (size_t)P.n_local_sys : 0; k < P.sys.size(); ++k)
    in.inv_alg_bytes += P.sys[k].n * (P.sys[k].n + 1) / 2 * (int64_t)sizeof(TT);
  in.local_iters = c->local_iters;
  in.ell_width = c->loc_w;
  in.reduced_refine = c->reduced_refine;
  if (inexact) {
    // ELL values and column words, and the diagonals
    const int64_t vb = std::is_same<TT, double>::value ? 8 : 4;
    in.local_bytes = ell_entries * (vb + 2) + c->coarse_vec_off * 8;
  }
  in.n_jent = (int64_t)P.jv_w.size();
  in.n_inc_blocks = 0;
  int64_t inc_slots = 0;
  for (int64_t blk = 0; blk < P.n_blocks; ++blk)
    if (P.blk_inc[blk]) {
      ++in.n_inc_blocks;
      inc_slots += P.blk_slot_ptr[blk + 1] - P.blk_slot_ptr[blk];
    }
  // element matrices and connectivity; slot vertex, destination and writer flag;
  // the 16-byte incidence record of slots in incidence-list blocks; p read, q written
  in.a_bytes = NE * (28 * 8 + 8 * 2) + (int64_t)P.slot_vid.size() * 9 + inc_slots * 16 + nf * 16;
  for (int d = 0; d < 3; ++d) in.boxes[d] = P.b[d];
  in.precision = c->precision;
  for (int b = 0; b < COARSE_GEMV_BUCKETS; ++b) in.gemv_tiles[b] = c->gemv_tiles[b];
  in.reduced_stream = (c->reduced_aside || inexact) ? 1 : 0;
  in.whole_waves = c->whole_waves;
}

coarse_ctx *as_ctx(const coarse_ctx *c) { return const_cast<coarse_ctx *>(c); }

int fail_ctx(coarse_ctx *c, const Fail &f) {
  if (c) c->err = f.what();
  return f.code;
}

PlanInput make_input(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *o) {
  PlanInput in;
  in.n_vert = mesh->n_vert;
  in.n_elem = mesh->n_elem;
  in.xyz = mesh->xyz;
  in.e2v = mesh->e2v;
  in.part = mesh->part;
  in.n_part = mesh->n_part;
  in.dirichlet = bc->dirichlet;
  in.overlap = o->overlap;
  for (int d = 0; d < 3; ++d) in.boxes[d] = o->boxes[d];
  in.interp = o->interp;
  return in;
}

}  // namespace

// ---------------------------------------------------------------------------
// Lock-step batch of independent solves (continuous batching). Every live solve
// advances one PCG iteration per lock step: its own kernels (operator, update,
// convergence test, R_p, J^T, then the overlap sum and prolongation) run on one of
// a few side streams, and the dense local and reduced solves of all live solves
// go into ONE GEMV launch and ONE combine launch on the main stream. Solves join
// and leave only between steps. A solve's arithmetic never depends on the others,
// so its result is bitwise the same alone or in any mix.
// ---------------------------------------------------------------------------
struct coarse_batch {
  // grouped launches of one lock step: operator, update, restriction, J^T
  // corners, overlap sum (the dense solves use the segment tables)
  enum { G_OP, G_UPD, G_PRE, G_COR, G_FIN, G_LOC, NG };
  std::string err;
  hipStream_t main = nullptr;
  struct Entry {
    coarse_ctx *c;
    const double *b;
    double *u;
    int64_t tag;
    double t0;
    hipStream_t saved_stream;
    int nproj;   // prior solutions its initial guess was projected on
  };
  std::vector<Entry> live;
  int precision = -1, whole_waves = 4;
  bool dirty = true, use_graph = false;
  bool pending = false;      // lock steps launched, their solver states not yet collected
  Seg *d_seg = nullptr;      // [3][cap]: item, row and whole-system segments
  Seg *h_seg = nullptr;      // pinned staging
  IterDev *d_iter = nullptr, *h_iter = nullptr;   // [cap] per-solve state
  int32_t *d_off = nullptr, *h_off = nullptr;     // [NG][cap + 1] workgroup offsets
  Scalars *d_sc = nullptr, *h_sc = nullptr;       // [cap] solver states, gathered each step
  int cap = 0, n_items = 0, n_rows = 0, n_whole = 0, whole_lds = 0;
  int grid[NG] = {};
  int op_lds = 0, fin_lds = 0;
  int loc_nt = 0;   // workgroup size of the grouped inexact local solves
  hipGraphExec_t gexec = nullptr;
  // tables in memory the batch does not own (the allocation-free entry point):
  // fixed capacity, never reallocated or freed, no graph
  bool ext = false;

  void init(hipStream_t s, bool graph) {
    main = s;
    use_graph = graph && s != nullptr;   // the null stream cannot be captured
  }

  // Device tables carved from `dev` and host staging from `host` (each at least
  // table_bytes(cap_) bytes, 256-byte aligned), for at most cap_ solves.
  static constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
  static constexpr size_t table_bytes(int cap_) {
    return align256(3 * (size_t)cap_ * sizeof(Seg)) + align256((size_t)cap_ * sizeof(IterDev)) +
           align256((size_t)NG * (cap_ + 1) * sizeof(int32_t)) + align256((size_t)cap_ * sizeof(Scalars));
  }
  void use_external(void *dev, void *host, int cap_) {
    char *d = (char *)dev, *h = (char *)host;
    size_t o = 0;
    d_seg = (Seg *)(d + o);
    h_seg = (Seg *)(h + o);
    o += align256(3 * (size_t)cap_ * sizeof(Seg));
    d_iter = (IterDev *)(d + o);
    h_iter = (IterDev *)(h + o);
    o += align256((size_t)cap_ * sizeof(IterDev));
    d_off = (int32_t *)(d + o);
    h_off = (int32_t *)(h + o);
    o += align256((size_t)NG * (cap_ + 1) * sizeof(int32_t));
    d_sc = (Scalars *)(d + o);
    h_sc = (Scalars *)(h + o);
    cap = cap_;
    ext = true;
    use_graph = false;
  }

  ~coarse_batch() {
    if (main) (void)hipStreamSynchronize(main);
    for (auto &e : live) e.c->stream = e.saved_stream;
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (!ext) free_tables();
  }

  void free_tables() {
    if (d_seg) (void)hipFree(d_seg);
    if (h_seg) (void)hipHostFree(h_seg);
    if (d_iter) (void)hipFree(d_iter);
    if (h_iter) (void)hipHostFree(h_iter);
    if (d_off) (void)hipFree(d_off);
    if (h_off) (void)hipHostFree(h_off);
    if (d_sc) (void)hipFree(d_sc);
    if (h_sc) (void)hipHostFree(h_sc);
    d_sc = nullptr;
    h_sc = nullptr;
    d_seg = nullptr;
    h_seg = nullptr;
    d_iter = nullptr;
    h_iter = nullptr;
    d_off = nullptr;
    h_off = nullptr;
  }

  int submit(coarse_ctx *c, const double *b, double *u, double tol, int64_t tag) {
    if (pending) {
      err = "lock steps launched and not yet collected";
      return COARSE_EINVAL;
    }
    if (c->mode != COARSE_ADDITIVE) {
      err = "batched solves use the additive preconditioner";
      return COARSE_EINVAL;
    }
    if (c->reduced_refine) {
      err = "batched solves do not refine the reduced solve (opts.reduced_refine = 0)";
      return COARSE_EINVAL;
    }
    if (precision >= 0 && c->precision != precision) {
      err = "all solves of a batch share one precision";
      return COARSE_EINVAL;
    }
    if (!live.empty() && c->whole_waves != whole_waves) {
      err = "all solves of a batch share one whole-system wavefront count";
      return COARSE_EINVAL;
    }
    for (auto &e : live)
      if (e.c == c) {
        err = "context already in the batch";
        return COARSE_EINVAL;
      }
    precision = c->precision;
    whole_waves = c->whole_waves;
    c->prof_mask = 0;   // no per-phase events inside lock steps (they may be captured)
    Entry e{c, b, u, tag, now(), c->stream, c->proj_max > 0 ? c->proj_n : 0};
    // every launch of a batched solve goes to the batch's stream, so the start
    // is ordered before the lock steps (also when they are a replayed graph)
    c->stream = main;
    // a context set up with a projection basis starts from the projection onto
    // its prior solutions (Sec. 5), as coarse_solve_projected does
    const int nproj = c->proj_max > 0 ? c->proj_n : 0;
    c->start(b, 1.0 * tol, nproj);
    live.push_back(e);
    dirty = true;
    return COARSE_OK;
  }

  void rebuild_tables() {
    const int n = (int)live.size();
    if (n > cap && ext) throw Fail(COARSE_EINVAL, "more solves than the batch's fixed tables hold");
    if (n > cap) {
      DeviceCallScope dc(g_guard);
      HIPCHK(hipStreamSynchronize(main));
      free_tables();
      cap = std::max(2 * n, 16);
      HIPCHK(hipMalloc(&d_seg, 3 * cap * sizeof(Seg)));
      HIPCHK(hipHostMalloc((void **)&h_seg, 3 * cap * sizeof(Seg), hipHostMallocDefault));
      HIPCHK(hipMalloc(&d_iter, cap * sizeof(IterDev)));
      HIPCHK(hipHostMalloc((void **)&h_iter, cap * sizeof(IterDev), hipHostMallocDefault));
      HIPCHK(hipMalloc(&d_off, NG * (cap + 1) * sizeof(int32_t)));
      HIPCHK(hipHostMalloc((void **)&h_off, NG * (cap + 1) * sizeof(int32_t), hipHostMallocDefault));
      HIPCHK(hipMalloc(&d_sc, cap * sizeof(Scalars)));
      HIPCHK(hipHostMalloc((void **)&h_sc, cap * sizeof(Scalars), hipHostMallocDefault));
    }
    n_items = n_rows = n_whole = 0;
    op_lds = whole_lds = fin_lds = loc_nt = 0;
    for (int g = 0; g < NG; ++g) h_off[g * (cap + 1)] = 0;
    for (int k = 0; k < n; ++k) {
      coarse_ctx *c = live[k].c;
      h_seg[k] = Seg{c->items, c->rows, c->whole, c->sysdev, c->done_flag, n_items, 0};
      h_seg[cap + k] = Seg{c->items, c->rows, c->whole, c->sysdev, c->done_flag, n_rows, 0};
      h_seg[2 * cap + k] = Seg{c->items, c->rows, c->whole, c->sysdev, c->done_flag, n_whole, 0};
      n_items += c->items_total;
      n_rows += c->rows_total;
      n_whole += c->whole_total;
      whole_lds = std::max(whole_lds, (int)c->whole_lds);
      c->fill_iter(h_iter[k]);
      const int64_t blocks[NG] = {c->op.n_blocks, c->nvblk, c->pre_gather_blocks() + c->pre_task_blocks(),
                                  nblk(c->n_r, 4), c->nvblk, c->local_iters > 0 ? c->n_local_sys : 0};
      if (c->local_iters > 0) loc_nt = std::max(loc_nt, c->loc_nt);
      for (int g = 0; g < NG; ++g) {
        const int64_t next = h_off[g * (cap + 1) + k] + blocks[g];
        if (next > INT32_MAX / 2) throw Fail(COARSE_EINVAL, "lock-step batch too large for one launch");
        h_off[g * (cap + 1) + k + 1] = (int32_t)next;
      }
      op_lds = std::max(op_lds, (int)c->op.lds_bytes);
      if (c->y_lds) fin_lds = std::max(fin_lds, (int)(c->n_bv * sizeof(double)));
    }
    for (int g = 0; g < NG; ++g) grid[g] = h_off[g * (cap + 1) + n];
    HIPCHK(hipMemcpyAsync(d_seg, h_seg, 3 * cap * sizeof(Seg), hipMemcpyHostToDevice, main));
    HIPCHK(hipMemcpyAsync(d_iter, h_iter, n * sizeof(IterDev), hipMemcpyHostToDevice, main));
    HIPCHK(hipMemcpyAsync(d_off, h_off, NG * (cap + 1) * sizeof(int32_t), hipMemcpyHostToDevice, main));
    if (gexec) {
      HIPCHK(hipGraphExecDestroy(gexec));
      gexec = nullptr;
    }
    dirty = false;
  }

  // one lock step of every live solve: seven launches whatever the batch size
  // (eight when some of the solves use inexact local solves)
  template <typename T>
  void lock_step_t() {
    const int n = (int)live.size();
    const int32_t *off = d_off;
    const int L = cap + 1;
    hipLaunchKernelGGL(k_op_fused_grp, dim3(grid[G_OP]), dim3(OP_BLOCK), op_lds, main, (const IterDev *)d_iter, off, n);
    hipLaunchKernelGGL(k_update_fused_grp, dim3(grid[G_UPD]), dim3(VW), 0, main, (const IterDev *)d_iter, off + L, n);
    hipLaunchKernelGGL(k_pre_grp<T>, dim3(grid[G_PRE]), dim3(256), 0, main, (const IterDev *)d_iter, off + 2 * L, n);
    hipLaunchKernelGGL(k_jt_corners_grp<T>, dim3(grid[G_COR]), dim3(256), 0, main, (const IterDev *)d_iter,
                       off + 3 * L, n);
    launch_gemv(main, precision, whole_waves, d_seg, n, n_items, d_seg + 2 * cap, n_whole, whole_lds, nullptr, nullptr);
    if (n_rows > 0)
      hipLaunchKernelGGL(k_combine<T>, dim3(nblk((int64_t)n_rows * TILE, 256)), dim3(256), 0, main,
                         (const Seg *)(d_seg + cap), n, n_rows, (const int *)nullptr);
    // inexact local solves of the solves that use them
    if (grid[G_LOC] > 0) {
      if (precision == COARSE_FP64)
        hipLaunchKernelGGL((k_local_pcg_grp<double, T>), dim3(grid[G_LOC]), dim3(loc_nt), 0, main,
                           (const IterDev *)d_iter, off + 5 * L, n);
      else
        hipLaunchKernelGGL((k_local_pcg_grp<float, T>), dim3(grid[G_LOC]), dim3(loc_nt), 0, main,
                           (const IterDev *)d_iter, off + 5 * L, n);
    }
    hipLaunchKernelGGL(k_final_grp<T>, dim3(grid[G_FIN]), dim3(VW), fin_lds, main, (const IterDev *)d_iter,
                       off + 4 * L, n);
  }
  void lock_step() {
    if (precision == COARSE_FP64)
      lock_step_t<double>();
    else
      lock_step_t<float>();
  }

  int step(int iters, int64_t *tags, coarse_stats *stats, int capn, int *n_done) {
    const int rc = launch(iters);
    if (rc != COARSE_OK) return rc;
    return collect(tags, stats, capn, n_done);
  }

  // Queue `iters` lock steps and the copy of the solver states to the host,
  // without waiting for them.
  int launch(int iters) {
    if (pending) {
      err = "lock steps launched and not yet collected";
      return COARSE_EINVAL;
    }
    if (live.empty()) return COARSE_OK;
    if (dirty) rebuild_tables();
    // a graph is captured only while no setup, destruction or allocation runs
    // on another thread; otherwise this step's launches go out directly (the
    // same kernels and arguments, so the same results)
    if (use_graph && !gexec && g_guard.try_begin_capture()) {
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(main, hipStreamCaptureModeRelaxed);
      if (e == hipSuccess) {
        try {
          lock_step();
        } catch (...) {
          (void)hipStreamEndCapture(main, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          g_guard.end_capture();
          throw;
        }
        e = hipStreamEndCapture(main, &graph);
      }
      g_guard.end_capture();
      HIPCHK(e);
      e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(e);
    }
    if (use_graph && gexec) {
      for (int i = 0; i < iters; ++i) HIPCHK(hipGraphLaunch(gexec, main));
    } else {
      for (int i = 0; i < iters; ++i) lock_step();
    }
    const int n = (int)live.size();
    hipLaunchKernelGGL(k_gather_scalars, dim3(nblk(n, 64)), dim3(64), 0, main, (const IterDev *)d_iter, n, d_sc);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h_sc, d_sc, n * sizeof(Scalars), hipMemcpyDeviceToHost, main));
    pending = true;
    return COARSE_OK;
  }

  // Wait for the launched lock steps, then retire up to capn finished solves.
  int collect(int64_t *tags, coarse_stats *stats, int capn, int *n_done) {
    *n_done = 0;
    if (!pending) return COARSE_OK;
    pending = false;
    const int n = (int)live.size();
    HIPCHK(hipStreamSynchronize(main));
    for (int k = 0; k < n; ++k) *live[k].c->h_sc = h_sc[k];
    // retire at most capn finished solves; any others stay (their iterations are
    // skipped on the device) and are retired by a later step
    std::vector<Entry> keep;
    std::vector<Entry> fin;
    for (auto &e : live) ((e.c->h_sc->done && (int)fin.size() < capn) ? fin : keep).push_back(e);
    if (fin.empty()) return COARSE_OK;
    for (auto &e : fin) {
      e.c->finish(e.u);
      // the solution joins the basis of a context that keeps one (a full basis
      // starts again from it)
      if (e.c->proj_max > 0) e.c->proj_append(e.c->proj_n >= e.c->proj_max ? 0 : e.c->proj_n);
    }
    HIPCHK(hipStreamSynchronize(main));
    for (auto &e : fin) {
      e.c->last_iters = e.c->h_sc->iters;
      if (e.c->proj_max > 0) e.c->proj_n = *e.c->h_proj_count;
      if (tags) tags[*n_done] = e.tag;
      if (stats) {
        e.c->fill_stats(&stats[*n_done], e.t0);
        stats[*n_done].n_basis = e.nproj;
      }
      ++*n_done;
      e.c->stream = e.saved_stream;
    }
    live.swap(keep);
    dirty = true;
    return COARSE_OK;
  }
};

namespace {

// ---------------------------------------------------------------------------
// Memory of the allocation-free lock-step batch (coarse_solve_batch_noalloc):
// its device tables (solve segments, per-solve iteration state, workgroup
// offsets, gathered solver states) live in a file-scope device array instead
// of memory the batch allocates, and its host staging in a file-scope host
// array. In host code the name `scratch` stands for the symbol only; the
// array's device address on each device comes from hipGetSymbolAddress (taken
// once per device, with that device current) and only that address reaches
// kernels and copies. Every call on one device shares that device's array.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(1) << 20;
static_assert(coarse_batch::table_bytes(COARSE_NOALLOC_MAX_SOLVES) <= kScratchBytes,
              "allocation-free batch tables exceed the scratch array");
__device__ __align__(256) unsigned char scratch[kScratchBytes];
alignas(256) unsigned char g_noalloc_host[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device.
void *scratch_address() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Fail(COARSE_EDEVICE, "device id beyond the scratch address table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Fail(COARSE_EDEVICE, "no device address for the scratch array");
    g_scratch_dev[dev] = p;
  }
  return g_scratch_dev[dev];
}

// PCG from u_0 = 0 (or, with `projected`, from the projection onto the stored
// basis, which then takes in the new solution), with host convergence checks
// every check_every queued iterations.
int run_solve(coarse_ctx *c, const double *b, double *u, double tol, coarse_stats *st, bool projected) {
  const double t0 = now();
  const int nproj = projected ? c->proj_n : 0;
  try {
    c->start(b, tol, nproj);
    int batch = std::max(c->check_every, c->last_iters);
    for (;;) {
      for (int j = 0; j < batch; ++j) c->iteration();
      batch = c->check_every;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(c->h_sc, c->sc, sizeof(Scalars), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      c->pcollect();
      if (c->h_sc->done) break;
    }
    c->finish(u);
    // a full basis starts again from the new solution alone
    if (projected) c->proj_append(c->proj_n >= c->proj_max ? 0 : c->proj_n);
    HIPCHK(hipStreamSynchronize(c->stream));
    if (projected) c->proj_n = *c->h_proj_count;
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  c->fill_stats(st, t0);
  if (st) st->n_basis = nproj;
  c->last_iters = c->h_sc->iters;
  const int status = c->h_sc->status;
  if (status == -6) c->err = "PCG breakdown (p.Ap <= 0 or non-finite value)";
  if (status == 1) c->err = "iteration limit reached";
  return status;
}

int check_multi(coarse_ctx *c, int k) {
  if (k < 1 || k > COARSE_MULTI_MAX) {
    c->err = "the block solve takes 1 to COARSE_MULTI_MAX right-hand sides";
    return COARSE_EINVAL;
  }
  if (c->mode != COARSE_ADDITIVE || c->h_msys.empty()) {
    c->err = "the block solve needs a context with the additive preconditioner";
    return COARSE_EINVAL;
  }
  if (c->local_iters > 0 || c->reduced_refine) {
    c->err = "the block solve needs exact local solves and no reduced refinement";
    return COARSE_EINVAL;
  }
  if ((OP_BLOCK * 8 + c->max_slots * MCW) * (int64_t)sizeof(double) > 65536) {
    c->err = "operator blocks with too many distinct vertices for the block solve";
    return COARSE_EINVAL;
  }
  return COARSE_OK;
}

}  // namespace

extern "C" {

void coarse_default_opts(coarse_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->overlap = 1;
  o->precision = COARSE_FP64;
  o->mode = COARSE_ADDITIVE;
  o->interp = COARSE_J_CENTROID;
  o->max_it = 1000;
  o->check_every = 4;
  o->flexible = 0;
  o->stream = nullptr;
  o->projection = 0;
}

int coarse_plan_info(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts, coarse_info_t *info,
                     int64_t *sizes) {
  if (!mesh || !bc || !info) return COARSE_EINVAL;
  coarse_opts o;
  coarse_default_opts(&o);
  if (opts) o = *opts;
  Plan P;
  int rc = build_plan(make_input(mesh, bc, &o), P);
  if (rc) {
    g_setup_error = P.err;
    return rc;
  }
  std::memset(info, 0, sizeof(*info));
  info->n_free = P.n_free;
  info->n_sub = P.n_local_sys;
  for (int64_t k = 0; k < P.n_local_sys; ++k) {
    info->sum_np += P.sys[k].n;
    info->max_np = std::max<int64_t>(info->max_np, P.sys[k].n);
  }
  info->n_r = P.n_r;
  info->n_cells = (int64_t)P.occ_cells.size();
  info->n_jent = (int64_t)P.jv_w.size();
  for (int64_t blk = 0; blk < P.n_blocks; ++blk) info->n_inc_blocks += P.blk_inc[blk];
  for (int d = 0; d < 3; ++d) info->boxes[d] = P.b[d];
  info->precision = o.precision;
  if (sizes)
    for (int32_t p = 0; p < P.n_part; ++p) sizes[p] = (int64_t)P.R[p].size();
  return 0;
}

int coarse_plan_create(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts, coarse_plan **out) {
  if (!mesh || !bc || !out) {
    g_setup_error = "null argument";
    return COARSE_EINVAL;
  }
  *out = nullptr;
  coarse_opts o;
  coarse_default_opts(&o);
  if (opts) o = *opts;
  if (o.precision != COARSE_FP64 && o.precision != COARSE_MIXED && o.precision != COARSE_MIXED_F16) {
    g_setup_error = "unknown precision";
    return COARSE_EINVAL;
  }
  if (o.mode < 0 || o.mode > COARSE_HYBRID || o.max_it < 1 || o.check_every < 1) {
    g_setup_error = "bad mode, max_it or check_every";
    return COARSE_EINVAL;
  }
  if (o.whole_waves != 0 && !whole_waves_ok(o.precision, o.whole_waves)) {
    g_setup_error = "whole_waves must be 0, or 2, 4 or 8 for FP64 tiles and 4, 8 or 16 for FP32/FP16 tiles";
    return COARSE_EINVAL;
  }
  if (o.projection < 0 || o.projection > COARSE_PROJECTION_MAX) {
    g_setup_error = "projection must be in [0, COARSE_PROJECTION_MAX]";
    return COARSE_EINVAL;
  }
  if (o.local_iters < 0 || o.local_iters > 10000) {
    g_setup_error = "local_iters must be in [0, 10000]";
    return COARSE_EINVAL;
  }
  if (o.reduced_refine && o.interp != COARSE_J_CENTROID) {
    g_setup_error = "reduced_refine needs the centroid interpolation (27-point A_r)";
    return COARSE_EINVAL;
  }
  try {
    const double t0 = now();
    std::unique_ptr<coarse_plan> pl(new coarse_plan());
    pl->o = o;
    int rc = build_plan(make_input(mesh, bc, &o), pl->P);
    if (rc) {
      g_setup_error = pl->P.err;
      return rc;
    }
    pl->t_plan = now() - t0;
    *out = pl.release();
  } catch (const std::bad_alloc &) {
    g_setup_error = "host allocation failed";
    return COARSE_ENOMEM;
  }
  return COARSE_OK;
}

int coarse_plan_set_gemv_tiles(coarse_plan *plan, const int *tiles) {
  if (!plan || !tiles) return COARSE_EINVAL;
  for (int b = 0; b < COARSE_GEMV_BUCKETS; ++b) plan->o.gemv_tiles[b] = tiles[b];
  return COARSE_OK;
}

int coarse_plan_destroy(coarse_plan *plan) {
  delete plan;
  return COARSE_OK;
}

int coarse_setup(const coarse_mesh *mesh, const coarse_bc *bc, const coarse_opts *opts, coarse_ctx **out) {
  if (out) *out = nullptr;
  coarse_plan *pl = nullptr;
  int rc = coarse_plan_create(mesh, bc, opts, &pl);
  if (rc) return rc;
  rc = coarse_setup_from_plan(pl, pl->o.stream, out);
  coarse_plan_destroy(pl);
  return rc;
}

int coarse_setup_from_plan(const coarse_plan *plan, void *stream, coarse_ctx **out) {
  if (!plan || !out) {
    g_setup_error = "null argument";
    return COARSE_EINVAL;
  }
  *out = nullptr;
  const coarse_opts &o = plan->o;
  const Plan &P = plan->P;
  const double t0 = now() - plan->t_plan;
  DeviceCallScope dc(g_guard);
  std::unique_ptr<coarse_ctx> c(new coarse_ctx());
  c->stream = (hipStream_t)stream;
  try {
    // the context's memory is stream-ordered too: destroying it (evictions in a
    // serving loop) then never synchronises the device
    keep_pool_memory();
  } catch (const Fail &f) {
    g_setup_error = f.what();
    return f.code;
  }
  c->arena.ordered = c->stream;
  c->arena.stream_ordered = true;
  c->precision = o.precision;
  c->mode = o.mode;
  c->interp = o.interp;
  c->max_it = o.max_it;
  c->check_every = o.check_every;
  // the hybrid of eqs. (asm1)-(asm2) is not symmetric, and inexact local solves
  // are not linear in r (their CG coefficients depend on it): the flexible beta
  c->flexible = (o.flexible || o.mode == COARSE_HYBRID || o.local_iters > 0) ? 1 : 0;
  c->local_iters = o.local_iters;
  c->reduced_refine = o.reduced_refine ? 1 : 0;
  c->proj_max = o.projection;
  try {
    c->aux = g_streams.get();
    HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
    c->h_sc = (Scalars *)g_pinned.get(sizeof(Scalars));
    if (o.precision == COARSE_FP64)
      setup_precision<double, double>(c.get(), P, o.gemv_tiles, o.whole_waves);
    else if (o.precision == COARSE_MIXED)
      setup_precision<float, float>(c.get(), P, o.gemv_tiles, o.whole_waves);
    else
      setup_precision<float, _Float16>(c.get(), P, o.gemv_tiles, o.whole_waves);
  } catch (const Fail &f) {
    g_setup_error = f.what();
    (void)hipStreamSynchronize(c->stream);
    return f.code;
  } catch (const std::bad_alloc &) {
    g_setup_error = "host allocation failed";
    return COARSE_ENOMEM;
  }
  // the block solve's vectors, when asked for and the context can run it
  if (o.block_rhs && check_multi(c.get(), 1) == COARSE_OK) {
    try {
      c->m_init();
      HIPCHK(hipStreamSynchronize(c->stream));
    } catch (const Fail &f) {
      g_setup_error = f.what();
      return f.code;
    }
  }
  c->t_setup = now() - t0;
  c->info.device_bytes = (int64_t)c->arena.bytes;
  *out = c.release();
  return COARSE_OK;
}

int coarse_apply_precond(coarse_ctx *c, const double *r, double *z) {
  if (!c || !r || !z || r == z) return COARSE_EINVAL;
  try {
    hipLaunchKernelGGL(k_gather_user, dim3(c->nvblk), dim3(VB), 0, c->stream, c->nf, c->user_of_vint, r, c->r);
    c->precond(c->r, c->z, nullptr, nullptr, nullptr, c->zero_flag);
    hipLaunchKernelGGL(k_permute_out, dim3(nblk(c->nv, VB)), dim3(VB), 0, c->stream, c->nv, c->nf, c->vint_of_user,
                       c->z, z);
    HIPCHK(hipGetLastError());
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_apply_A(coarse_ctx *c, const double *p, double *q) {
  if (!c || !p || !q || p == q) return COARSE_EINVAL;
  try {
    hipLaunchKernelGGL(k_gather_user, dim3(c->nvblk), dim3(VB), 0, c->stream, c->nf, c->user_of_vint, p, c->p);
    c->apply_op(c->p, c->q, nullptr, c->zero_flag);
    hipLaunchKernelGGL(k_permute_out, dim3(nblk(c->nv, VB)), dim3(VB), 0, c->stream, c->nv, c->nf, c->vint_of_user,
                       c->q, q);
    HIPCHK(hipGetLastError());
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_apply_reduced_operator(coarse_ctx *c, const double *y, double *w) {
  if (!c || !y || !w || y == w) return COARSE_EINVAL;
  if (!c->ar_coef) {
    c->err = "no stencil of A_r (standard interpolation, or no reduced unknowns)";
    return COARSE_EINVAL;
  }
  try {
    HIPCHK(hipMemsetAsync(w, 0, c->n_bv * sizeof(double), c->stream));
    hipLaunchKernelGGL(k_ar_apply, dim3(nblk(c->n_r, 256)), dim3(256), 0, c->stream, c->n_r,
                       (const int32_t *)c->act_bv, (const double *)c->ar_coef, c->bgrid, y, w);
    HIPCHK(hipGetLastError());
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_solve(coarse_ctx *c, const double *b, double *u, double tol, coarse_stats *st) {
  if (!c || !b || !u || b == u || !(tol > 0)) return COARSE_EINVAL;
  return run_solve(c, b, u, tol, st, false);
}

namespace {

// the per-column statistics of a finished block solve; returns the worst status
int multi_stats(coarse_ctx *c, int k, coarse_stats *st, double t0) {
  const MScal &m = *c->mb.h_ms;
  int worst = COARSE_OK, most = 0;
  for (int j = 0; j < k; ++j) {
    most = std::max(most, m.iters[j]);
    const int s = m.status[j];
    if (s < 0 || (s > 0 && worst == COARSE_OK)) worst = s;
    if (!st) continue;
    coarse_stats &o = st[j];
    o.iters = m.iters[j];
    o.status = s;
    o.relres = m.bb[j] > 0 ? std::sqrt(m.rr[j] / m.bb[j]) : 0.0;
    o.relres_true = m.bb[j] > 0 ? std::sqrt(m.res_true[j] / m.bb[j]) : 0.0;
    o.relres0 = m.bb[j] > 0 ? std::sqrt(m.rr0[j] / m.bb[j]) : 0.0;
    o.n_basis = 0;
    o.t_setup = c->t_setup;
    o.t_solve = now() - t0;
  }
  c->mb.last_iters = most;
  if (worst == -6) c->err = "PCG breakdown (p.Ap <= 0 or non-finite value)";
  if (worst == 1) c->err = "iteration limit reached";
  return worst;
}

}  // namespace

int coarse_multi_begin(coarse_ctx *c, int k, const double *b, double tol) {
  if (!c || !b || !(tol > 0)) return COARSE_EINVAL;
  int rc = check_multi(c, k);
  if (rc) return rc;
  if (c->mb.active) {
    c->err = "a block solve is in progress on this context";
    return COARSE_EINVAL;
  }
  try {
    c->m_init();
    c->mb.t0 = now();
    c->m_start(b, k, tol);
    HIPCHK(hipMemcpyAsync(c->mb.h_ms, c->mb.ms, sizeof(MScal), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipGetLastError());
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  c->mb.active = true;
  c->mb.k = k;
  c->mb.b = b;
  return COARSE_OK;
}

int coarse_multi_advance(coarse_ctx *c, int iters) {
  if (!c || iters < 0) return COARSE_EINVAL;
  if (!c->mb.active) {
    c->err = "no block solve in progress on this context";
    return COARSE_EINVAL;
  }
  try {
    for (int j = 0; j < iters; ++j) c->m_iteration();
    HIPCHK(hipMemcpyAsync(c->mb.h_ms, c->mb.ms, sizeof(MScal), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipGetLastError());
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_multi_done(const coarse_ctx *c) {
  if (!c || !c->mb.active) return COARSE_EINVAL;
  return c->mb.h_ms->all_done ? 1 : 0;
}

int coarse_multi_end(coarse_ctx *c, double *u, coarse_stats *st) {
  if (!c || !u) return COARSE_EINVAL;
  if (!c->mb.active) {
    c->err = "no block solve in progress on this context";
    return COARSE_EINVAL;
  }
  if (u == c->mb.b) {
    c->err = "the solutions may not overwrite the right-hand sides";
    return COARSE_EINVAL;
  }
  c->mb.active = false;
  try {
    c->m_finish(u, c->mb.k);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->pcollect();
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return multi_stats(c, c->mb.k, st, c->mb.t0);
}

int coarse_solve_multi(coarse_ctx *c, int k, const double *b, double *u, double tol, coarse_stats *st) {
  if (!c || !b || !u || b == u || !(tol > 0)) return COARSE_EINVAL;
  int rc = check_multi(c, k);
  if (rc) return rc;
  if (c->mb.active) {
    c->err = "a block solve is in progress on this context";
    return COARSE_EINVAL;
  }
  const double t0 = now();
  try {
    c->m_init();
    c->m_start(b, k, tol);
    int batch = std::max(c->check_every, c->mb.last_iters);
    for (;;) {
      for (int j = 0; j < batch; ++j) c->m_iteration();
      batch = c->check_every;
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(c->mb.h_ms, c->mb.ms, sizeof(MScal), hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipStreamSynchronize(c->stream));
      c->pcollect();
      if (c->mb.h_ms->all_done) break;
    }
    c->m_finish(u, k);
    HIPCHK(hipStreamSynchronize(c->stream));
    c->pcollect();
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return multi_stats(c, k, st, t0);
}

int coarse_apply_precond_multi(coarse_ctx *c, int k, const double *r, double *z) {
  if (!c || !r || !z || r == z) return COARSE_EINVAL;
  int rc = check_multi(c, k);
  if (rc) return rc;
  if (c->mb.active) {
    c->err = "a block solve is in progress on this context";
    return COARSE_EINVAL;
  }
  try {
    c->m_init();
    c->m_start(r, k, 1.0);
    hipLaunchKernelGGL(k_m_permute_out, dim3(nblk(c->nv * k, 256)), dim3(256), 0, c->stream, c->nv, c->nf,
                       (const int32_t *)c->vint_of_user, (const double *)c->mb.Z, k, z);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->pcollect();
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_solve_projected(coarse_ctx *c, const double *b, double *u, double tol, coarse_stats *st) {
  if (!c || !b || !u || b == u || !(tol > 0)) return COARSE_EINVAL;
  if (c->proj_max <= 0) {
    c->err = "the context was set up without a projection basis (opts.projection = 0)";
    return COARSE_EINVAL;
  }
  return run_solve(c, b, u, tol, st, true);
}

int coarse_projection_reset(coarse_ctx *c) {
  if (!c) return COARSE_EINVAL;
  c->proj_n = 0;
  return COARSE_OK;
}

int coarse_solve_batch(coarse_ctx *const *ctxs, const double *const *b, double *const *u, int count, double tol,
                       coarse_stats *st) {
  if (!ctxs || !b || !u || count < 0) return COARSE_EINVAL;
  if (count == 0) return COARSE_OK;
  for (int i = 0; i < count; ++i)
    for (int j = 0; j < i; ++j)
      if (ctxs[i] == ctxs[j] || !ctxs[i]) return COARSE_EINVAL;
  coarse_batch *bt = nullptr;
  int rc = coarse_batch_create(ctxs[0]->stream, 0, &bt);
  if (rc) return rc;
  int worst = COARSE_OK;
  for (int i = 0; i < count && worst >= 0; ++i) {
    rc = coarse_batch_submit(bt, ctxs[i], b[i], u[i], tol, i);
    if (rc < 0) worst = rc;
  }
  std::vector<int64_t> tags(count);
  std::vector<coarse_stats> sts(count);
  while (worst >= 0 && coarse_batch_live(bt) > 0) {
    int nd = 0;
    rc = coarse_batch_step(bt, ctxs[0]->check_every, tags.data(), sts.data(), count, &nd);
    if (rc < 0) {
      worst = rc;
      break;
    }
    for (int k = 0; k < nd; ++k) {
      if (st) st[tags[k]] = sts[k];
      const int s = sts[k].status;
      if (s < 0 || (s > 0 && worst == COARSE_OK)) worst = s;
    }
  }
  coarse_batch_destroy(bt);
  return worst;
}

int coarse_solve_batch_noalloc(coarse_ctx *const *ctxs, const double *const *b, double *const *u, int count,
                               double tol, coarse_stats *st) {
  if (!ctxs || !b || !u || count < 0) return COARSE_EINVAL;
  if (count > COARSE_NOALLOC_MAX_SOLVES) {
    g_setup_error = "coarse_solve_batch_noalloc takes at most COARSE_NOALLOC_MAX_SOLVES systems";
    return COARSE_EINVAL;
  }
  if (count == 0) return COARSE_OK;
  for (int i = 0; i < count; ++i) {
    if (!ctxs[i] || !b[i] || !u[i] || b[i] == u[i]) return COARSE_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[i] == ctxs[j]) return COARSE_EINVAL;
  }
  if (!(tol > 0)) return COARSE_EINVAL;
  int64_t tags[COARSE_NOALLOC_MAX_SOLVES];
  coarse_stats sts[COARSE_NOALLOC_MAX_SOLVES];
  coarse_batch bt;
  int worst = COARSE_OK;
  try {
    bt.init(ctxs[0]->stream, false);
    // every table entry a step reads is written first: nothing to clear
    bt.use_external(scratch_address(), g_noalloc_host, COARSE_NOALLOC_MAX_SOLVES);
    for (int i = 0; i < count && worst >= 0; ++i) {
      const int rc = bt.submit(ctxs[i], b[i], u[i], tol, i);
      if (rc < 0) worst = rc;
    }
    while (worst >= 0 && !bt.live.empty()) {
      int nd = 0;
      bt.step(ctxs[0]->check_every, tags, sts, count, &nd);
      for (int k = 0; k < nd; ++k) {
        if (st) st[tags[k]] = sts[k];
        const int s = sts[k].status;
        if (s < 0 || (s > 0 && worst == COARSE_OK)) worst = s;
      }
    }
  } catch (const Fail &f) {
    g_setup_error = f.what();
    return f.code;
  }
  if (worst < 0 && !bt.err.empty()) g_setup_error = bt.err;
  return worst;
}

int coarse_batch_create(void *stream, int use_graph, coarse_batch **out) {
  if (!out) return COARSE_EINVAL;
  *out = nullptr;
  std::unique_ptr<coarse_batch> bt(new coarse_batch());
  try {
    bt->init((hipStream_t)stream, use_graph != 0);
  } catch (const Fail &f) {
    g_setup_error = f.what();
    return f.code;
  }
  *out = bt.release();
  return COARSE_OK;
}

int coarse_batch_submit(coarse_batch *bt, coarse_ctx *c, const double *b, double *u, double tol, int64_t tag) {
  if (!bt || !c || !b || !u || b == u || !(tol > 0)) return COARSE_EINVAL;
  try {
    return bt->submit(c, b, u, tol, tag);
  } catch (const Fail &f) {
    bt->err = f.what();
    return f.code;
  }
}

int coarse_batch_step(coarse_batch *bt, int iters, int64_t *tags, coarse_stats *stats, int cap, int *n_done) {
  if (!bt || iters < 1 || !n_done || cap < 0) return COARSE_EINVAL;
  try {
    return bt->step(iters, tags, stats, cap, n_done);
  } catch (const Fail &f) {
    bt->err = f.what();
    return f.code;
  }
}

int coarse_batch_launch(coarse_batch *bt, int iters) {
  if (!bt || iters < 1) return COARSE_EINVAL;
  try {
    return bt->launch(iters);
  } catch (const Fail &f) {
    bt->err = f.what();
    return f.code;
  }
}

int coarse_batch_collect(coarse_batch *bt, int64_t *tags, coarse_stats *stats, int cap, int *n_done) {
  if (!bt || !n_done || cap < 0) return COARSE_EINVAL;
  try {
    return bt->collect(tags, stats, cap, n_done);
  } catch (const Fail &f) {
    bt->err = f.what();
    return f.code;
  }
}

int coarse_batch_live(const coarse_batch *bt) { return bt ? (int)bt->live.size() : 0; }

int coarse_batch_destroy(coarse_batch *bt) {
  if (!bt) return COARSE_OK;
  DeviceCallScope dc(g_guard);
  delete bt;
  return COARSE_OK;
}

int coarse_destroy(coarse_ctx *c) {
  if (!c) return COARSE_OK;
  DeviceCallScope dc(g_guard);
  (void)hipStreamSynchronize(c->stream);
  // the memory goes back to the pool in the order of the context's stream (its
  // second stream is drained by the destructor first)
  c->arena.ordered = c->stream;
  delete c;
  return COARSE_OK;
}

size_t coarse_device_bytes(const coarse_ctx *c) { return c ? c->arena.bytes : 0; }

int coarse_get_info(const coarse_ctx *c, coarse_info_t *info) {
  if (!c || !info) return COARSE_EINVAL;
  *info = c->info;
  info->device_bytes = (int64_t)c->arena.bytes;
  return COARSE_OK;
}

int coarse_profile(coarse_ctx *c, int enable, double *ms, int64_t *counts, int nphase) {
  if (!c || nphase < 0) return COARSE_EINVAL;
  try {
    HIPCHK(hipStreamSynchronize(c->stream));
    c->pcollect();
    if (enable) {
      for (int i = 0; i < coarse_ctx::NPH; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_cnt[i] = 0;
      }
      c->prof_mask = enable & ((1 << coarse_ctx::NPH) - 1);
    } else {
      c->prof_mask = 0;
      for (int i = 0; i < std::min(nphase, (int)coarse_ctx::NPH); ++i) {
        if (ms) ms[i] = c->prof_ms[i];
        if (counts) counts[i] = c->prof_cnt[i];
      }
    }
  } catch (const Fail &f) {
    return fail_ctx(c, f);
  }
  return COARSE_OK;
}

int coarse_set_stream(coarse_ctx *c, void *stream) {
  if (!c) return COARSE_EINVAL;
  c->stream = (hipStream_t)stream;
  return COARSE_OK;
}

const char *coarse_strerror(int code) {
  switch (code) {
    case COARSE_OK: return "success";
    case COARSE_NOTCONV: return "iteration limit reached before the tolerance";
    case COARSE_EINVAL: return "invalid argument";
    case COARSE_ENOMEM: return "out of memory";
    case COARSE_EMESH: return "invalid mesh (inverted element or repeated vertex)";
    case COARSE_ESINGULAR: return "singular local or reduced system";
    case COARSE_EDEVICE: return "HIP runtime error";
    case COARSE_EBREAKDOWN: return "PCG breakdown";
    default: return "unknown status";
  }
}

const char *coarse_last_error(const coarse_ctx *c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

}  // extern "C"
