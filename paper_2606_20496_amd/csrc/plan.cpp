// Host-side combinatorial setup of the coarse solver (see plan.h).
//
// Follows the paper's problem statement and method:
//   Sec. 3  element-vertex connectivity, homogeneous Dirichlet vertices removed,
//           overlapping subdomains (layers of vertex-sharing elements) and R_p
//           on the vertices interior to each overlapping subdomain;
//   Sec. 4  bounding box cut into boxes, elements assigned to the cell of their
//           centroid, the averaged interpolation J = W Q^T J_L S, compression of
//           box vertices whose column of J is zero.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace coarse {

namespace {

uint64_t spread3(uint64_t x) {
  x &= 0x1fffff;
  x = (x | (x << 32)) & 0x1f00000000ffffULL;
  x = (x | (x << 16)) & 0x1f0000ff0000ffULL;
  x = (x | (x << 8)) & 0x100f00f00f00f00fULL;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ULL;
  x = (x | (x << 2)) & 0x1249249249249249ULL;
  return x;
}

// Element centroid: the plain mean of the 8 vertices, summed in local order.
inline void centroid(const double *xyz, const int32_t *ev, double c[3]) {
  for (int d = 0; d < 3; ++d) {
    double s = xyz[3 * (int64_t)ev[0] + d];
    for (int v = 1; v < 8; ++v) s = s + xyz[3 * (int64_t)ev[v] + d];
    c[d] = s / 8.0;
  }
}

// Recursive coordinate bisection of element centroids into n pieces.
void rcb(std::vector<int32_t> &idx, int64_t lo, int64_t hi, int32_t label0, int32_t n,
         const std::vector<double> &cen, std::vector<int32_t> &part) {
  if (n <= 1 || hi - lo <= 1) {
    for (int64_t i = lo; i < hi; ++i) part[idx[i]] = label0;
    return;
  }
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = lo; i < hi; ++i)
    for (int d = 0; d < 3; ++d) {
      mn[d] = std::min(mn[d], cen[3 * (int64_t)idx[i] + d]);
      mx[d] = std::max(mx[d], cen[3 * (int64_t)idx[i] + d]);
    }
  int ax = 0;
  for (int d = 1; d < 3; ++d)
    if (mx[d] - mn[d] > mx[ax] - mn[ax]) ax = d;
  int32_t nl = n / 2;
  int64_t mid = lo + (hi - lo) * nl / n;
  std::nth_element(idx.begin() + lo, idx.begin() + mid, idx.begin() + hi, [&](int32_t a, int32_t b) {
    double ca = cen[3 * (int64_t)a + ax], cb = cen[3 * (int64_t)b + ax];
    return ca < cb || (ca == cb && a < b);
  });
  rcb(idx, lo, mid, label0, nl, cen, part);
  rcb(idx, mid, hi, label0 + nl, n - nl, cen, part);
}

// Trilinear weight of corner k = kx + 2ky + 4kz at local coordinates xi.
inline double phi(int k, const double xi[3]) {
  double fx = (k & 1) ? xi[0] : 1.0 - xi[0];
  double fy = (k & 2) ? xi[1] : 1.0 - xi[1];
  double fz = (k & 4) ? xi[2] : 1.0 - xi[2];
  return fx * fy * fz;
}

// Run f(begin, end, t) over [0, n) cut into nt contiguous ranges, one thread
// each (t = 0..nt-1); the ranges, and so every result, do not depend on timing.
template <typename F>
void parallel_for(int64_t n, int nt, F f) {
  if (nt <= 1 || n < 2 * nt) {
    f((int64_t)0, n, 0);
    return;
  }
  std::vector<std::thread> ts;
  for (int t = 1; t < nt; ++t) ts.emplace_back([&f, n, nt, t] { f(n * t / nt, n * (t + 1) / nt, t); });
  f((int64_t)0, n / nt, 0);
  for (auto &th : ts) th.join();
}

// Host threads for a plan: large meshes only (the plans of small meshes run
// side by side on a server's own worker threads).
int plan_threads(int64_t n_elem) {
  if (n_elem < (int64_t(1) << 20)) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max<unsigned>(1, std::min<unsigned>(8, hw));
}

// Phase timings of the host setup on stderr when COARSE_TRACE is set.
struct Trace {
  bool on = std::getenv("COARSE_TRACE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char *what) {
    if (!on) return;
    const auto n = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[coarse plan] %-28s %8.3f ms\n", what, std::chrono::duration<double, std::milli>(n - t).count());
    t = n;
  }
};

}  // namespace

int build_plan(const PlanInput &in, Plan &P) {
  Trace tr;
  const int64_t NV = in.n_vert, NE = in.n_elem;
  const int NT = in.threads > 0 ? std::min(in.threads, 64) : plan_threads(NE);
  if (NV <= 0 || NE <= 0 || !in.xyz || !in.e2v || !in.dirichlet) {
    P.err = "empty mesh or null array";
    return -1;
  }
  if (NV >= (int64_t(1) << 31) || NE >= (int64_t(1) << 31) / 8) {
    P.err = "mesh too large for 32-bit indices";
    return -1;
  }
  if (in.overlap < 1 || in.n_part < 1) {
    P.err = "overlap and n_part must be >= 1";
    return -1;
  }
  if (in.interp != 0 && in.interp != 1) {
    P.err = "unknown interpolation scheme";
    return -1;
  }
  P.n_vert = NV;
  P.n_elem = NE;
  for (int64_t e = 0; e < NE; ++e) {
    const int32_t *ev = in.e2v + 8 * e;
    for (int v = 0; v < 8; ++v) {
      if (ev[v] < 0 || ev[v] >= NV) {
        P.err = "e2v entry out of range at element " + std::to_string(e);
        return -1;
      }
      for (int w = 0; w < v; ++w)
        if (ev[w] == ev[v]) {
          P.err = "vertex repeated within element " + std::to_string(e);
          return -3;
        }
    }
  }
  for (int64_t u = 0; u < 3 * NV; ++u)
    if (!std::isfinite(in.xyz[u])) {
      P.err = "non-finite vertex coordinate";
      return -1;
    }

  tr.mark("validate");
  // ---- partition labels -------------------------------------------------------
  std::vector<double> cen(3 * NE);
  parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int) {
    for (int64_t e = e0; e < e1; ++e) centroid(in.xyz, in.e2v + 8 * e, &cen[3 * e]);
  });
  std::vector<int32_t> part(NE);
  P.n_part = in.n_part;
  if (in.part) {
    for (int64_t e = 0; e < NE; ++e) {
      if (in.part[e] < 0 || in.part[e] >= in.n_part) {
        P.err = "part label out of range at element " + std::to_string(e);
        return -1;
      }
      part[e] = in.part[e];
    }
  } else {
    std::vector<int32_t> idx(NE);
    std::iota(idx.begin(), idx.end(), 0);
    rcb(idx, 0, NE, 0, in.n_part, cen, part);
  }

  tr.mark("partition");
  // ---- bounding box of all vertices (Sec. 4) ----------------------------------
  for (int d = 0; d < 3; ++d) {
    P.lo[d] = 1e300;
    P.hi[d] = -1e300;
  }
  for (int64_t u = 0; u < NV; ++u)
    for (int d = 0; d < 3; ++d) {
      P.lo[d] = std::min(P.lo[d], in.xyz[3 * u + d]);
      P.hi[d] = std::max(P.hi[d], in.xyz[3 * u + d]);
    }

  tr.mark("bounding box");
  // ---- element order: (subdomain, Morton code of centroid) --------------------
  {
    std::vector<uint64_t> key(NE);
    parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int) {
      for (int64_t e = e0; e < e1; ++e) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) {
          double ext = P.hi[d] - P.lo[d];
          double t = ext > 0 ? (cen[3 * e + d] - P.lo[d]) / ext : 0.0;
          t = std::min(std::max(t, 0.0), 1.0);
          q[d] = (uint64_t)(t * 2097151.0);
        }
        key[e] = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
      }
    });
    // order by (subdomain, key, element): elements bucketed by subdomain (in
    // element order), then each subdomain's run sorted by (key, element)
    std::vector<int64_t> pst(in.n_part + 1, 0);
    for (int64_t e = 0; e < NE; ++e) pst[part[e] + 1]++;
    for (int32_t q = 0; q < in.n_part; ++q) pst[q + 1] += pst[q];
    P.elem_user.resize(NE);
    {
      std::vector<int64_t> fill(pst.begin(), pst.end() - 1);
      for (int64_t e = 0; e < NE; ++e) P.elem_user[fill[part[e]]++] = (int32_t)e;
    }
    parallel_for(in.n_part, NT, [&](int64_t q0, int64_t q1, int) {
      for (int64_t q = q0; q < q1; ++q)
        std::sort(P.elem_user.begin() + pst[q], P.elem_user.begin() + pst[q + 1], [&](int32_t a, int32_t b) {
          if (key[a] != key[b]) return key[a] < key[b];
          return a < b;
        });
    });
  }

  tr.mark("element order");
  // ---- vertex numbering: free vertices first, by first touch -------------------
  // The first touch of a vertex is the least slot 8 ei + v (element ei in the
  // order above, corner v) naming it. Free vertices are numbered in first-touch
  // order, then the Dirichlet vertices that elements use, in the same order:
  // first touches found by an atomic minimum, counted per range of elements,
  // then numbered per range from the ranges' prefix sums.
  P.vint_of_user.assign(NV, -1);
  int64_t nf = 0, nd = 0;
  if (NT == 1) {
    // one thread: the same numbering in two plain passes
    for (int64_t ei = 0; ei < NE; ++ei) {
      const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
      for (int v = 0; v < 8; ++v)
        if (!in.dirichlet[ev[v]] && P.vint_of_user[ev[v]] < 0) P.vint_of_user[ev[v]] = (int32_t)nf++;
    }
    nd = nf;
    for (int64_t ei = 0; ei < NE; ++ei) {
      const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
      for (int v = 0; v < 8; ++v)
        if (P.vint_of_user[ev[v]] < 0) P.vint_of_user[ev[v]] = (int32_t)nd++;
    }
  } else {
    const int64_t NONE = INT64_MAX;
    std::unique_ptr<std::atomic<int64_t>[]> first(new std::atomic<int64_t>[NV]);
    parallel_for(NV, NT, [&](int64_t u0, int64_t u1, int) {
      for (int64_t u = u0; u < u1; ++u) first[u].store(NONE, std::memory_order_relaxed);
    });
    parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int) {
      for (int64_t ei = e0; ei < e1; ++ei) {
        const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
        for (int v = 0; v < 8; ++v) {
          const int64_t key = 8 * ei + v;
          std::atomic<int64_t> &f = first[ev[v]];
          int64_t cur = f.load(std::memory_order_relaxed);
          while (key < cur && !f.compare_exchange_weak(cur, key, std::memory_order_relaxed)) {
          }
        }
      }
    });
    std::vector<int64_t> cnt_f(NT + 1, 0), cnt_d(NT + 1, 0);
    parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int t) {
      int64_t cf = 0, cd = 0;
      for (int64_t ei = e0; ei < e1; ++ei) {
        const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
        for (int v = 0; v < 8; ++v)
          if (first[ev[v]].load(std::memory_order_relaxed) == 8 * ei + v) (in.dirichlet[ev[v]] ? cd : cf)++;
      }
      cnt_f[t + 1] = cf;
      cnt_d[t + 1] = cd;
    });
    for (int t = 0; t < NT; ++t) {
      cnt_f[t + 1] += cnt_f[t];
      cnt_d[t + 1] += cnt_d[t];
    }
    nf = cnt_f[NT];
    parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int t) {
      int64_t idf = cnt_f[t], idd = nf + cnt_d[t];
      for (int64_t ei = e0; ei < e1; ++ei) {
        const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
        for (int v = 0; v < 8; ++v)
          if (first[ev[v]].load(std::memory_order_relaxed) == 8 * ei + v)
            P.vint_of_user[ev[v]] = (int32_t)(in.dirichlet[ev[v]] ? idd++ : idf++);
      }
    });
    nd = nf + cnt_d[NT];
  }
  for (int64_t u = 0; u < NV; ++u)
    if (!in.dirichlet[u] && P.vint_of_user[u] < 0) {
      P.err = "free vertex " + std::to_string(u) + " belongs to no element";
      return -1;
    }
  P.n_free = nf;
  // unused Dirichlet vertices get the remaining ids
  for (int64_t u = 0; u < NV; ++u)
    if (P.vint_of_user[u] < 0) P.vint_of_user[u] = (int32_t)nd++;
  if (nf == 0) {
    P.err = "no free vertices";
    return -1;
  }
  P.user_of_vint.assign(NV, 0);
  P.xyz.resize(3 * NV);
  parallel_for(NV, NT, [&](int64_t u0, int64_t u1, int) {
    for (int64_t u = u0; u < u1; ++u) {
      P.user_of_vint[P.vint_of_user[u]] = (int32_t)u;
      for (int d = 0; d < 3; ++d) P.xyz[d * NV + P.vint_of_user[u]] = in.xyz[3 * u + d];
    }
  });
  P.e2v.resize(8 * NE);
  std::vector<int32_t> part_int(NE);
  parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int) {
    for (int64_t ei = e0; ei < e1; ++ei) {
      const int32_t *ev = in.e2v + 8 * (int64_t)P.elem_user[ei];
      for (int v = 0; v < 8; ++v) P.e2v[v * NE + ei] = P.vint_of_user[ev[v]];
      part_int[ei] = part[P.elem_user[ei]];
    }
  });
  auto E2V = [&](int64_t e, int v) { return P.e2v[v * NE + e]; };

  tr.mark("vertex numbering");
  // ---- multiplicity and vertex -> element incidence (all vertices) ------------
  P.mult.assign(NV, 0);
  for (int64_t e = 0; e < NE; ++e)
    for (int v = 0; v < 8; ++v) P.mult[E2V(e, v)]++;
  std::vector<int32_t> inc_ptr(NV + 1, 0), inc(8 * NE);
  for (int64_t u = 0; u < NV; ++u) inc_ptr[u + 1] = inc_ptr[u] + P.mult[u];
  {
    std::vector<int32_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int64_t e = 0; e < NE; ++e)
      for (int v = 0; v < 8; ++v) inc[fill[E2V(e, v)]++] = (int32_t)(e * 8 + v);
  }
  P.vinc_ptr.assign(inc_ptr.begin(), inc_ptr.begin() + nf + 1);
  P.vinc.assign(inc.begin(), inc.begin() + inc_ptr[nf]);

  tr.mark("incidence");
  // ---- operator blocks ---------------------------------------------------------
  {
    const int64_t nb = (NE + OP_BLOCK - 1) / OP_BLOCK;
    P.n_blocks = nb;
    P.blk_slot_ptr.assign(1, 0);
    P.blk_inc.assign(nb, 0);
    P.lconn.assign(8 * NE, 0xFFFF);
    // each block on its own (in parallel): its vertices (sorted), each vertex's
    // incidence list in (element, local vertex) order, its local connectivity,
    // whether the block holds all of a vertex's incidences; then the blocks are
    // concatenated in order
    struct BlockOut {
      std::vector<int32_t> verts, list_ptr;
      std::vector<uint16_t> lists;
      std::vector<uint8_t> owned;
      uint8_t inc = 0;
    };
    std::vector<BlockOut> bo(nb);
    const int nt_blk = (nb >= 2 * NT) ? NT : 1;
    // per range of blocks: the slot of each vertex of the current block (-1
    // elsewhere, reset after the block), so a block's vertices are found without
    // sorting its incidences; only the distinct vertices are sorted
    std::vector<std::vector<int32_t>> slot_of_t(nt_blk);
    parallel_for(nb, nt_blk, [&](int64_t b0, int64_t b1, int t) {
      std::vector<int32_t> &slot_of = slot_of_t[t];
      slot_of.assign(nf, -1);
      std::vector<int32_t> uniq, fill;
      std::vector<uint8_t> seen;
      for (int64_t blk = b0; blk < b1; ++blk) {
        const int64_t e0 = blk * OP_BLOCK, e1 = std::min<int64_t>(NE, e0 + OP_BLOCK);
        uniq.clear();
        int64_t nent = 0;
        for (int64_t e = e0; e < e1; ++e)
          for (int v = 0; v < 8; ++v) {
            const int32_t u = E2V(e, v);
            if (u >= nf) continue;
            ++nent;
            if (slot_of[u] < 0) {
              slot_of[u] = 0;
              uniq.push_back(u);
            }
          }
        std::sort(uniq.begin(), uniq.end());
        const int32_t ns = (int32_t)uniq.size();
        BlockOut &o = bo[blk];
        o.verts = uniq;
        o.list_ptr.assign(ns + 1, 0);
        for (int32_t sl = 0; sl < ns; ++sl) slot_of[uniq[sl]] = sl;
        for (int64_t e = e0; e < e1; ++e)
          for (int v = 0; v < 8; ++v) {
            const int32_t u = E2V(e, v);
            if (u < nf) o.list_ptr[slot_of[u] + 1]++;
          }
        for (int32_t sl = 0; sl < ns; ++sl) o.list_ptr[sl + 1] += o.list_ptr[sl];
        // each vertex's incidences in (element, local vertex) order
        fill.assign(o.list_ptr.begin(), o.list_ptr.end() - 1);
        seen.assign(ns, 0);
        o.lists.resize(nent);
        for (int64_t e = e0; e < e1; ++e)
          for (int v = 0; v < 8; ++v) {
            const int32_t u = E2V(e, v);
            if (u >= nf) continue;
            const int32_t sl = slot_of[u];
            o.lists[fill[sl]++] = (uint16_t)((e - e0) * 8 + v);
            P.lconn[e * 8 + v] = (uint16_t)sl;
            if ((seen[sl] >> v) & 1) o.inc = 1;
            seen[sl] |= (uint8_t)(1u << v);
          }
        o.owned.resize(ns);
        for (int32_t sl = 0; sl < ns; ++sl) {
          o.owned[sl] = (int64_t)(o.list_ptr[sl + 1] - o.list_ptr[sl]) == (int64_t)P.mult[uniq[sl]] ? 1 : 0;
          slot_of[uniq[sl]] = -1;
        }
      }
    });
    slot_of_t.clear();
    // the blocks' slots and lists concatenated in block order: offsets first,
    // then each block copies its part (in parallel)
    std::vector<int64_t> soff(nb + 1, 0), loff(nb + 1, 0);
    for (int64_t blk = 0; blk < nb; ++blk) {
      soff[blk + 1] = soff[blk] + (int64_t)bo[blk].verts.size();
      loff[blk + 1] = loff[blk] + (int64_t)bo[blk].lists.size();
      P.blk_inc[blk] = bo[blk].inc;
      if (bo[blk].inc) P.any_blk_inc = true;
      P.max_slots = std::max<int64_t>(P.max_slots, (int64_t)bo[blk].verts.size());
    }
    const int64_t nslot = soff[nb];
    P.blk_slot_ptr.resize(nb + 1);
    for (int64_t blk = 0; blk <= nb; ++blk) P.blk_slot_ptr[blk] = (int32_t)soff[blk];
    P.slot_vid.resize(nslot);
    P.slot_dst.resize(nslot);
    P.slot_inc.resize(loff[nb]);
    P.slot_inc_ptr.resize(nslot + 1);
    P.slot_inc_ptr[0] = 0;
    P.slot_inc8.resize(8 * nslot);
    parallel_for(nb, nt_blk, [&](int64_t b0, int64_t b1, int) {
      for (int64_t blk = b0; blk < b1; ++blk) {
        BlockOut &o = bo[blk];
        const int64_t s0 = soff[blk], l0b = loff[blk];
        std::copy(o.lists.begin(), o.lists.end(), P.slot_inc.begin() + l0b);
        for (size_t sl = 0; sl < o.verts.size(); ++sl) {
          const int64_t gs = s0 + (int64_t)sl;
          const int32_t u = o.verts[sl];
          P.slot_vid[gs] = u;
          const int32_t l0 = o.list_ptr[sl], l1 = o.list_ptr[sl + 1];
          P.slot_inc_ptr[gs + 1] = (int32_t)(l0b + l1);
          // the same list as one 16-byte record (0xFFFF ends it; 0xFFFE first: the
          // list is longer than 8 and only the CSR form holds it)
          const int len = l1 - l0;
          for (int k = 0; k < 8; ++k)
            P.slot_inc8[8 * gs + k] =
                len > 8 ? (k == 0 ? 0xFFFE : 0xFFFF) : (k < len ? o.lists[l0 + k] : (uint16_t)0xFFFF);
          P.slot_dst[gs] = o.owned[sl] ? u : -1;   // shared slots patched below
        }
        o = BlockOut();   // release the block's lists once they are copied
      }
    });
    std::vector<int64_t> shared_blocks;  // (slot global index) of shared slots
    for (int64_t gs = 0; gs < nslot; ++gs)
      if (P.slot_dst[gs] < 0) shared_blocks.push_back(gs);
    // partial ids grouped by vertex (vertices in order of first appearance, each
    // vertex's partials contiguous and in block order), so the sum over a shared
    // vertex reads one contiguous range
    P.n_partials = (int64_t)shared_blocks.size();
    std::vector<int32_t> sh_index(NV, -1);
    std::vector<int32_t> count;
    for (int64_t k = 0; k < P.n_partials; ++k) {
      const int32_t u = P.slot_vid[shared_blocks[k]];
      if (sh_index[u] < 0) {
        sh_index[u] = (int32_t)count.size();
        count.push_back(0);
        P.sh_vid.push_back(u);
      }
      count[sh_index[u]]++;
    }
    P.sh_ptr.assign(count.size() + 1, 0);
    for (size_t j = 0; j < count.size(); ++j) P.sh_ptr[j + 1] = P.sh_ptr[j] + count[j];
    {
      std::vector<int32_t> fill(P.sh_ptr.begin(), P.sh_ptr.end() - 1);
      for (int64_t k = 0; k < P.n_partials; ++k) {
        const int64_t gs = shared_blocks[k];
        const int32_t pid = fill[sh_index[P.slot_vid[gs]]]++;
        P.slot_dst[gs] = -(pid + 1);
      }
    }
    P.sh_part.clear();
    // one writer per vertex: the owning block, or the first block sharing it
    P.slot_pw.assign(P.slot_vid.size(), 0);
    std::vector<char> seen(nf, 0);
    for (size_t gs = 0; gs < P.slot_vid.size(); ++gs) {
      const int32_t u = P.slot_vid[gs];
      if (!seen[u]) {
        seen[u] = 1;
        P.slot_pw[gs] = 1;
      }
    }
    // per free vertex: (first partial, count), count 0 = owned by one block
    P.vq.assign(2 * nf, 0);
    for (size_t j = 0; j < P.sh_vid.size(); ++j) {
      P.vq[2 * P.sh_vid[j]] = P.sh_ptr[j];
      P.vq[2 * P.sh_vid[j] + 1] = P.sh_ptr[j + 1] - P.sh_ptr[j];
    }
  }

  tr.mark("operator blocks");
  // ---- overlapping subdomains and R_p (Sec. 3) --------------------------------
  {
    std::vector<int64_t> pstart(in.n_part + 1, 0);
    for (int64_t e = 0; e < NE; ++e) pstart[part_int[e] + 1]++;
    for (int p = 0; p < in.n_part; ++p) pstart[p + 1] += pstart[p];
    P.R.assign(in.n_part, {});
    // overlap 1: the elements that join subdomain p are those of other parts that
    // share a vertex with it; one pass over the vertices whose elements span
    // several parts lists them as (part, element) pairs, bucketed by part
    // (a vertex touching more than 64 subdomains sends every subdomain through the
    // general layer loop below instead)
    std::vector<int64_t> lay_ptr;
    std::vector<int32_t> lay;
    bool by_vertex = in.overlap == 1;
    if (by_vertex) {
      lay_ptr.assign(in.n_part + 1, 0);
      auto visit = [&](auto &&emit) -> bool {
        int32_t parts[64];
        for (int64_t u = 0; u < NV; ++u) {
          int np = 0;
          for (int32_t k = inc_ptr[u]; k < inc_ptr[u + 1]; ++k) {
            const int32_t q = part_int[inc[k] >> 3];
            bool have = false;
            for (int j = 0; j < np; ++j) have |= (parts[j] == q);
            if (have) continue;
            if (np == 64) return false;
            parts[np++] = q;
          }
          if (np < 2) continue;
          for (int32_t k = inc_ptr[u]; k < inc_ptr[u + 1]; ++k) {
            const int32_t f = inc[k] >> 3, q = part_int[f];
            for (int j = 0; j < np; ++j)
              if (parts[j] != q) emit(parts[j], f);
          }
        }
        return true;
      };
      by_vertex = visit([&](int32_t q, int32_t) { lay_ptr[q + 1]++; });
      if (by_vertex) {
        for (int32_t q = 0; q < in.n_part; ++q) lay_ptr[q + 1] += lay_ptr[q];
        lay.resize(lay_ptr[in.n_part]);
        std::vector<int64_t> fill(lay_ptr.begin(), lay_ptr.end() - 1);
        visit([&](int32_t q, int32_t f) { lay[fill[q]++] = f; });
      }
    }
    // subdomains in parallel, each thread with its own marks
    parallel_for(in.n_part, NT, [&](int64_t p0, int64_t p1, int) {
    std::vector<int32_t> emark(NE, -1), vmark(NV, -1), vcnt(NV, 0);
    std::vector<int32_t> cur, nxt, touched;
    for (int32_t p = (int32_t)p0; p < (int32_t)p1; ++p) {
      cur.clear();
      for (int64_t e = pstart[p]; e < pstart[p + 1]; ++e) {
        cur.push_back((int32_t)e);
        emark[e] = p;
      }
      std::vector<int32_t> all = cur;
      if (by_vertex) {
        for (int64_t k = lay_ptr[p]; k < lay_ptr[p + 1]; ++k)
          if (emark[lay[k]] != p) {
            emark[lay[k]] = p;
            all.push_back(lay[k]);
          }
      }
      for (int layer = 0; !by_vertex && layer < in.overlap; ++layer) {
        nxt.clear();
        for (int32_t e : all)
          for (int v = 0; v < 8; ++v) {
            int32_t u = E2V(e, v);
            for (int32_t k = inc_ptr[u]; k < inc_ptr[u + 1]; ++k) {
              int32_t f = inc[k] >> 3;
              if (emark[f] != p) {
                emark[f] = p;
                nxt.push_back(f);
              }
            }
          }
        all.insert(all.end(), nxt.begin(), nxt.end());
      }
      // a free vertex is in R_p when all its incidences lie in the extended
      // subdomain: the incidences counted there equal its multiplicity
      std::vector<int32_t> &R = P.R[p];
      touched.clear();
      for (int32_t e : all)
        for (int v = 0; v < 8; ++v) {
          int32_t u = E2V(e, v);
          if (u >= nf) continue;
          if (vmark[u] != p) {
            vmark[u] = p;
            vcnt[u] = 0;
            touched.push_back(u);
          }
          vcnt[u]++;
        }
      for (int32_t u : touched)
        if (vcnt[u] == P.mult[u]) R.push_back(u);
      std::sort(R.begin(), R.end());
    }
    });
  }

  tr.mark("overlap and R_p");
  // ---- box grid and element cells (Sec. 4) ------------------------------------
  int32_t bauto = (int32_t)std::ceil(std::cbrt((double)in.n_part) - 1e-9);
  for (int d = 0; d < 3; ++d) {
    P.b[d] = in.boxes[d] > 0 ? in.boxes[d] : std::max(1, bauto);
    P.H[d] = (P.hi[d] - P.lo[d]) / (double)P.b[d];
    if (!(P.H[d] > 0)) {
      P.err = "degenerate bounding box";
      return -1;
    }
  }
  const int64_t bx1 = P.b[0] + 1, by1 = P.b[1] + 1, bz1 = P.b[2] + 1;
  P.n_bv = bx1 * by1 * bz1;
  const int64_t ncell = (int64_t)P.b[0] * P.b[1] * P.b[2];
  auto cell_of = [&](const double x[3], int32_t c3[3]) {
    for (int d = 0; d < 3; ++d) {
      double t = std::floor((x[d] - P.lo[d]) / P.H[d]);
      int64_t c = (int64_t)t;
      if (t < 0) c = 0;
      if (t > P.b[d] - 1) c = P.b[d] - 1;
      c3[d] = (int32_t)c;
    }
  };
  auto corner_bv = [&](const int32_t c3[3], int k) -> int64_t {
    return (c3[0] + (k & 1)) + bx1 * ((c3[1] + ((k >> 1) & 1)) + by1 * (c3[2] + ((k >> 2) & 1)));
  };
  auto cell_id = [&](const int32_t c3[3]) -> int64_t { return c3[0] + (int64_t)P.b[0] * (c3[1] + (int64_t)P.b[1] * c3[2]); };
  auto cell_xyz = [&](int64_t c, int32_t c3[3]) {
    c3[0] = (int32_t)(c % P.b[0]);
    c3[1] = (int32_t)((c / P.b[0]) % P.b[1]);
    c3[2] = (int32_t)(c / ((int64_t)P.b[0] * P.b[1]));
  };
  auto local_xi = [&](const double x[3], const int32_t c3[3], double xi[3]) {
    for (int d = 0; d < 3; ++d) xi[d] = ((x[d] - P.lo[d]) - (double)c3[d] * P.H[d]) / P.H[d];
  };

  P.elem_cell.resize(NE);
  parallel_for(NE, NT, [&](int64_t e0, int64_t e1, int) {
    for (int64_t e = e0; e < e1; ++e) {
      // the centroid from the internal-order coordinates (better locality than
      // the user order; the same sum, corner by corner)
      double c[3];
      for (int d = 0; d < 3; ++d) {
        const double *xd = P.xyz.data() + d * NV;
        double sum = xd[E2V(e, 0)];
        for (int v = 1; v < 8; ++v) sum = sum + xd[E2V(e, v)];
        c[d] = sum / 8.0;
      }
      int32_t c3[3];
      cell_of(c, c3);
      P.elem_cell[e] = (int32_t)cell_id(c3);
    }
  });

  // vertex-major entries: (free vertex, cell) with weight fraction n_ic / m_i;
  // ranges of vertices in parallel, concatenated in vertex order
  std::vector<int32_t> ent_cell;  // cell id of each entry
  P.jv_ptr.assign(1, 0);
  {
    struct EntOut {
      std::vector<int32_t> cell, count;
      std::vector<double> w, xi;
    };
    const int nt = (nf >= 2 * NT) ? NT : 1;
    std::vector<EntOut> eo(nt);
    parallel_for(nf, nt, [&](int64_t i0, int64_t i1, int t) {
      EntOut &o = eo[t];
      std::vector<int32_t> cells;
      for (int64_t i = i0; i < i1; ++i) {
        const double x[3] = {P.xyz[i], P.xyz[NV + i], P.xyz[2 * NV + i]};
        const size_t before = o.cell.size();
        if (in.interp == 0) {
          cells.clear();
          for (int32_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) cells.push_back(P.elem_cell[inc[k] >> 3]);
          std::sort(cells.begin(), cells.end());
          for (size_t a = 0; a < cells.size();) {
            size_t b2 = a;
            while (b2 < cells.size() && cells[b2] == cells[a]) ++b2;
            int32_t c3[3];
            cell_xyz(cells[a], c3);
            double xi[3];
            local_xi(x, c3, xi);
            o.cell.push_back(cells[a]);
            o.w.push_back((double)(b2 - a) / (double)P.mult[i]);
            for (int d = 0; d < 3; ++d) o.xi.push_back(xi[d]);
            a = b2;
          }
        } else {
          int32_t c3[3];
          cell_of(x, c3);
          double xi[3];
          local_xi(x, c3, xi);
          o.cell.push_back((int32_t)cell_id(c3));
          o.w.push_back(1.0);
          for (int d = 0; d < 3; ++d) o.xi.push_back(xi[d]);
        }
        o.count.push_back((int32_t)(o.cell.size() - before));
      }
    });
    std::vector<int64_t> base(nt + 1, 0);
    for (int t = 0; t < nt; ++t) base[t + 1] = base[t] + (int64_t)eo[t].cell.size();
    P.jv_ptr.resize(nf + 1);
    ent_cell.resize(base[nt]);
    P.jv_w.resize(base[nt]);
    P.jv_xi.resize(3 * base[nt]);
    parallel_for(nf, nt, [&](int64_t i0, int64_t, int t) {
      EntOut &o = eo[t];
      int64_t k = base[t];
      for (size_t a = 0; a < o.count.size(); ++a) {
        k += o.count[a];
        P.jv_ptr[i0 + 1 + (int64_t)a] = (int32_t)k;
      }
      std::copy(o.cell.begin(), o.cell.end(), ent_cell.begin() + base[t]);
      std::copy(o.w.begin(), o.w.end(), P.jv_w.begin() + base[t]);
      std::copy(o.xi.begin(), o.xi.end(), P.jv_xi.begin() + 3 * base[t]);
      o = EntOut();
    });
  }
  const int64_t nent = (int64_t)ent_cell.size();

  // occupied cells: cells owning an element (centroid scheme) or an entry
  P.cell_occ.assign(ncell, -1);
  {
    std::vector<char> occ(ncell, 0);
    for (int64_t e = 0; e < NE; ++e) occ[P.elem_cell[e]] = 1;
    for (int64_t k = 0; k < nent; ++k) occ[ent_cell[k]] = 1;
    for (int64_t c = 0; c < ncell; ++c)
      if (occ[c]) {
        P.cell_occ[c] = (int32_t)P.occ_cells.size();
        P.occ_cells.push_back((int32_t)c);
      }
  }
  const int64_t nocc = (int64_t)P.occ_cells.size();
  P.occ_elem_ptr.assign(nocc + 1, 0);
  for (int64_t e = 0; e < NE; ++e) P.occ_elem_ptr[P.cell_occ[P.elem_cell[e]] + 1]++;
  for (int64_t o = 0; o < nocc; ++o) P.occ_elem_ptr[o + 1] += P.occ_elem_ptr[o];
  P.occ_elems.resize(NE);
  {
    std::vector<int32_t> fill(P.occ_elem_ptr.begin(), P.occ_elem_ptr.end() - 1);
    for (int64_t e = 0; e < NE; ++e) P.occ_elems[fill[P.cell_occ[P.elem_cell[e]]]++] = (int32_t)e;
  }

  // compression: a box vertex is kept when some entry gives it a nonzero weight
  P.bv_act.assign(P.n_bv, -1);
  {
    std::vector<char> act(P.n_bv, 0);
    for (int64_t k = 0; k < nent; ++k) {
      int32_t c3[3];
      cell_xyz(ent_cell[k], c3);
      const double xi[3] = {P.jv_xi[3 * k], P.jv_xi[3 * k + 1], P.jv_xi[3 * k + 2]};
      for (int q = 0; q < 8; ++q)
        if (phi(q, xi) != 0.0) act[corner_bv(c3, q)] = 1;
    }
    for (int64_t g = 0; g < P.n_bv; ++g)
      if (act[g]) {
        P.bv_act[g] = (int32_t)P.act_bv.size();
        P.act_bv.push_back((int32_t)g);
      }
  }
  P.n_r = (int64_t)P.act_bv.size();
  if (P.n_r == 0) {
    P.err = "reduced space is empty";
    return -4;
  }
  P.occ_corner_act.resize(8 * nocc);
  for (int64_t o = 0; o < nocc; ++o) {
    int32_t c3[3];
    cell_xyz(P.occ_cells[o], c3);
    for (int q = 0; q < 8; ++q) P.occ_corner_act[8 * o + q] = P.bv_act[corner_bv(c3, q)];
  }
  P.jv_occ.resize(nent);
  for (int64_t k = 0; k < nent; ++k) P.jv_occ[k] = P.cell_occ[ent_cell[k]];
  P.jv_base.resize(nent);
  for (int64_t k = 0; k < nent; ++k) {
    int32_t c3[3];
    cell_xyz(ent_cell[k], c3);
    P.jv_base[k] = (int32_t)corner_bv(c3, 0);
  }

  // cell-major copy of the entries, cut into restriction tasks
  {
    std::vector<int32_t> ent_vid(nent);
    parallel_for(nf, NT, [&](int64_t i0, int64_t i1, int) {
      for (int64_t i = i0; i < i1; ++i)
        for (int32_t k = P.jv_ptr[i]; k < P.jv_ptr[i + 1]; ++k) ent_vid[k] = (int32_t)i;
    });
    // entries by occupied cell, in entry order within a cell (a counting sort)
    std::vector<int32_t> order(nent);
    {
      std::vector<int64_t> ost(nocc + 1, 0);
      for (int64_t k = 0; k < nent; ++k) ost[P.jv_occ[k] + 1]++;
      for (int64_t o = 0; o < nocc; ++o) ost[o + 1] += ost[o];
      for (int64_t k = 0; k < nent; ++k) order[ost[P.jv_occ[k]]++] = (int32_t)k;
    }
    P.jc_vid.resize(nent);
    P.jc_w.resize(nent);
    P.jc_xi.resize(3 * nent);
    parallel_for(nent, NT, [&](int64_t j0, int64_t j1, int) {
      for (int64_t j = j0; j < j1; ++j) {
        int32_t k = order[j];
        P.jc_vid[j] = ent_vid[k];
        P.jc_w[j] = P.jv_w[k];
        for (int d = 0; d < 3; ++d) P.jc_xi[d * nent + j] = P.jv_xi[3 * (int64_t)k + d];
      }
    });
    // vertex-major xi to SoA as well
    std::vector<double> soa(3 * nent);
    parallel_for(nent, NT, [&](int64_t k0, int64_t k1, int) {
      for (int64_t k = k0; k < k1; ++k)
        for (int d = 0; d < 3; ++d) soa[d * nent + k] = P.jv_xi[3 * k + d];
    });
    P.jv_xi.swap(soa);
    P.jt_task_start.assign(1, 0);
    std::vector<std::vector<int32_t>> occ_tasks(nocc);
    int64_t j = 0;
    while (j < nent) {
      int32_t o = P.jv_occ[order[j]];
      int64_t j1 = j;
      while (j1 < nent && P.jv_occ[order[j1]] == o) ++j1;
      for (int64_t s = j; s < j1; s += JT_CHUNK) {
        occ_tasks[o].push_back((int32_t)P.jt_task_occ.size());
        P.jt_task_occ.push_back(o);
        P.jt_task_start.push_back((int32_t)std::min<int64_t>(j1, s + JT_CHUNK));
      }
      j = j1;
    }
    // per active box vertex: (task, corner) sources in fixed cell order
    P.jr_ptr.assign(1, 0);
    P.ar_ptr.assign(1, 0);
    for (int64_t K = 0; K < P.n_r; ++K) {
      int64_t g = P.act_bv[K];
      int32_t gx = (int32_t)(g % bx1), gy = (int32_t)((g / bx1) % by1), gz = (int32_t)(g / (bx1 * by1));
      for (int dz = 1; dz >= 0; --dz)
        for (int dy = 1; dy >= 0; --dy)
          for (int dx = 1; dx >= 0; --dx) {
            int32_t c3[3] = {gx - dx, gy - dy, gz - dz};
            if (c3[0] < 0 || c3[1] < 0 || c3[2] < 0 || c3[0] >= P.b[0] || c3[1] >= P.b[1] || c3[2] >= P.b[2]) continue;
            int32_t o = P.cell_occ[cell_id(c3)];
            if (o < 0) continue;
            int q = dx + 2 * dy + 4 * dz;
            for (int32_t t : occ_tasks[o]) P.jr_src.push_back(t * 8 + q);
            P.ar_src.push_back(o * 8 + q);
          }
      P.jr_ptr.push_back((int32_t)P.jr_src.size());
      P.ar_ptr.push_back((int32_t)P.ar_src.size());
    }
  }

  if (in.interp != 0) {
    // J e_L lives on the vertices of the cells around box vertex L; A reaches one
    // element further. With elements spanning at most ext_d in direction d, the
    // column couples box vertices within 1 + ceil(ext_d / H_d) of L.
    double ext[3] = {0, 0, 0};
    for (int64_t e = 0; e < NE; ++e)
      for (int d = 0; d < 3; ++d) {
        double mn = 1e300, mx = -1e300;
        for (int v = 0; v < 8; ++v) {
          const double x = P.xyz[d * NV + E2V(e, v)];
          mn = std::min(mn, x);
          mx = std::max(mx, x);
        }
        ext[d] = std::max(ext[d], mx - mn);
      }
    for (int d = 0; d < 3; ++d) {
      P.probe_d[d] = 1 + (int32_t)std::ceil(ext[d] / P.H[d]);
      P.probe_p[d] = std::min<int32_t>(2 * P.probe_d[d] + 1, P.b[d] + 1);
    }
  }
  tr.mark("reduced space");
  // ---- dense systems, packed vectors, tiles and GEMV items --------------------
  {
    int64_t voff = 0, toff = 0, roff = 0;
    auto add_sys = [&](int64_t n) {
      System s;
      s.n = n;
      s.nb = (n + TILE - 1) / TILE;
      s.vec_off = voff;
      s.tile_off = toff;
      s.row_off = roff;
      voff += s.nb * TILE;
      toff += s.nb * (s.nb + 1) / 2;
      roff += s.nb;
      P.sys.push_back(s);
    };
    for (int32_t p = 0; p < in.n_part; ++p)
      if (!P.R[p].empty()) {
        add_sys((int64_t)P.R[p].size());
        P.sub_of_sys.push_back(p);
      }
    P.n_local_sys = (int64_t)P.sys.size();
    add_sys(P.n_r);
    P.vec_len = voff;
    P.n_tiles = toff;
    P.n_rows = roff;
    P.sub_idx.assign(voff, -1);
    std::vector<int32_t> ccount(nf + 1, 0);
    for (int64_t s = 0; s < P.n_local_sys; ++s) {
      const auto &R = P.R[P.sub_of_sys[s]];
      for (size_t a = 0; a < R.size(); ++a) {
        P.sub_idx[P.sys[s].vec_off + a] = R[a];
        ccount[R[a] + 1]++;
      }
    }
    for (int64_t i = 0; i < nf; ++i) {
      if (ccount[i + 1] == 0) {
        P.err = "free vertex not covered by any subdomain";
        return -1;
      }
      ccount[i + 1] += ccount[i];
    }
    P.cover_ptr = ccount;
    P.cover_pos.resize(ccount[nf]);
    std::vector<int32_t> fill(ccount.begin(), ccount.end() - 1);
    for (int64_t s = 0; s < P.n_local_sys; ++s) {
      const auto &R = P.R[P.sub_of_sys[s]];
      for (size_t a = 0; a < R.size(); ++a) P.cover_pos[fill[R[a]]++] = (int32_t)(P.sys[s].vec_off + a);
    }
  }
  tr.mark("systems and items");
  return 0;
}

void build_gemv_items(const Plan &P, const int *tiles_of_bucket, const int *bucket_max, int nbucket, int n_cu,
                      GemvTable &out, int64_t first_sys) {
  out = GemvTable();
  // whole-system candidates, largest first; the smallest beyond a multiple of
  // n_cu would form a last round that few compute units work on
  std::vector<int32_t> cand;
  for (int64_t s = first_sys; s < (int64_t)P.sys.size(); ++s)
    if (P.sys[s].nb >= WHOLE_NB_MIN && P.sys[s].nb <= WHOLE_NB_MAX) cand.push_back((int32_t)s);
  std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) { return P.sys[a].nb > P.sys[b].nb; });
  // fewer systems than compute units: one workgroup per system would leave most
  // of the chip idle and make one unit stream a whole system, so every system
  // goes to work items
  size_t keep = cand.size();
  if (n_cu > 0) keep -= keep % (size_t)n_cu;
  std::vector<char> whole(P.sys.size(), 0);
  for (size_t i = 0; i < keep; ++i) whole[cand[i]] = 1;
  for (int64_t s = first_sys; s < (int64_t)P.sys.size(); ++s) {
    const System &S = P.sys[s];
    if (whole[s]) {
      out.whole.push_back((int32_t)s);
      out.whole_nb_max = std::max<int32_t>(out.whole_nb_max, (int32_t)S.nb);
      continue;
    }
    int b = 0;
    while (b + 1 < nbucket && S.nb > bucket_max[b]) ++b;
    const int64_t seg = (tiles_of_bucket && tiles_of_bucket[b] >= 1) ? tiles_of_bucket[b] : GEMV_SEG;
    for (int64_t I = 0; I < S.nb; ++I) {
      out.row_item0.push_back((int32_t)out.items.size());
      for (int64_t j0 = 0; j0 <= I; j0 += seg) {
        GemvItem it;
        it.sys = (int32_t)s;
        it.I = (int32_t)I;
        it.j0 = (int32_t)j0;
        it.j1 = (int32_t)std::min<int64_t>(I + 1, j0 + seg);
        out.items.push_back(it);
      }
      out.row_nitem.push_back((int32_t)(out.items.size() - out.row_item0.back()));
      out.row_sys.push_back((int32_t)s);
      out.row_I.push_back((int32_t)I);
    }
  }
  // local systems largest first (the longest workgroups start first), then the
  // reduced system
  auto mid = std::stable_partition(out.whole.begin(), out.whole.end(), [&](int32_t s) { return s < P.n_local_sys; });
  out.whole_local = (int32_t)(mid - out.whole.begin());
  std::stable_sort(out.whole.begin(), mid, [&](int32_t a, int32_t b) { return P.sys[a].nb > P.sys[b].nb; });
}

}  // namespace coarse
