// Builds the host plan of one mesh with several thread counts and checks that
// every field equals the one-thread plan. Mesh files in the directory given as
// the first argument: xyz.bin (double [n_vert][3]), e2v.bin (int32 [n_elem][8]),
// dir.bin (uint8 [n_vert]), meta.bin (int32: n_part, boxes[3], overlap, interp)
// and, when the mesh brings subdomain labels, part.bin (int32 [n_elem]).
// Prints "same <threads>" per count, or the fields that differ; exit status 0
// when all plans are the same.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "plan.h"

using namespace coarse;

template <typename T>
static std::vector<T> read_all(const std::string &f, bool *found = nullptr) {
  std::ifstream s(f, std::ios::binary | std::ios::ate);
  if (found) *found = (bool)s;
  if (!s) return {};
  const size_t n = (size_t)s.tellg();
  s.seekg(0);
  std::vector<T> v(n / sizeof(T));
  s.read((char *)v.data(), (std::streamsize)(v.size() * sizeof(T)));
  return v;
}

static int compare(const Plan &a, const Plan &b) {
  int bad = 0;
#define SAME(f)                                   \
  if (!(a.f == b.f)) {                            \
    std::printf("field %s differs\n", #f);        \
    bad = 1;                                      \
  }
#define SAME_ARR(f)                                \
  if (std::memcmp(a.f, b.f, sizeof(a.f)) != 0) {   \
    std::printf("field %s differs\n", #f);         \
    bad = 1;                                       \
  }
  SAME(n_vert) SAME(n_elem) SAME(n_free) SAME(n_part)
  SAME(vint_of_user) SAME(user_of_vint) SAME(elem_user) SAME(e2v) SAME(xyz) SAME(mult)
  SAME(n_blocks) SAME(max_slots) SAME(blk_slot_ptr) SAME(slot_vid) SAME(slot_dst) SAME(slot_inc_ptr)
  SAME(slot_inc) SAME(slot_inc8) SAME(blk_inc) SAME(any_blk_inc) SAME(lconn) SAME(n_partials) SAME(sh_vid)
  SAME(sh_ptr) SAME(sh_part) SAME(slot_pw) SAME(vq)
  SAME(vinc_ptr) SAME(vinc)
  SAME(R) SAME(sub_of_sys) SAME(n_local_sys) SAME(vec_len) SAME(n_tiles) SAME(sub_idx) SAME(cover_ptr)
  SAME(cover_pos) SAME(n_rows)
  SAME_ARR(lo) SAME_ARR(hi) SAME_ARR(H) SAME_ARR(b) SAME_ARR(probe_p) SAME_ARR(probe_d)
  SAME(n_bv) SAME(elem_cell) SAME(occ_cells) SAME(cell_occ) SAME(occ_elem_ptr) SAME(occ_elems)
  SAME(occ_corner_act) SAME(bv_act) SAME(act_bv) SAME(n_r)
  SAME(jv_ptr) SAME(jv_occ) SAME(jv_base) SAME(jv_w) SAME(jv_xi)
  SAME(jc_vid) SAME(jc_w) SAME(jc_xi) SAME(jt_task_start) SAME(jt_task_occ) SAME(jr_ptr) SAME(jr_src)
  SAME(ar_ptr) SAME(ar_src)
#undef SAME
#undef SAME_ARR
  bool sys_same = a.sys.size() == b.sys.size();
  for (size_t s = 0; sys_same && s < a.sys.size(); ++s) {
    const System &x = a.sys[s], &y = b.sys[s];
    sys_same = x.n == y.n && x.nb == y.nb && x.vec_off == y.vec_off && x.tile_off == y.tile_off &&
               x.row_off == y.row_off;
  }
  if (!sys_same) {
    std::printf("field sys differs\n");
    bad = 1;
  }
  return bad;
}

int main(int argc, char **argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: %s mesh_dir threads...\n", argv[0]);
    return 2;
  }
  const std::string d = argv[1];
  bool has_part = false;
  const auto xyz = read_all<double>(d + "/xyz.bin");
  const auto e2v = read_all<int32_t>(d + "/e2v.bin");
  const auto dir = read_all<uint8_t>(d + "/dir.bin");
  const auto meta = read_all<int32_t>(d + "/meta.bin");
  const auto part = read_all<int32_t>(d + "/part.bin", &has_part);
  if (meta.size() != 6) return 2;
  PlanInput in;
  in.n_vert = (int64_t)dir.size();
  in.n_elem = (int64_t)e2v.size() / 8;
  in.xyz = xyz.data();
  in.e2v = e2v.data();
  in.part = has_part ? part.data() : nullptr;
  in.n_part = meta[0];
  in.dirichlet = dir.data();
  for (int k = 0; k < 3; ++k) in.boxes[k] = meta[1 + k];
  in.overlap = meta[4];
  in.interp = meta[5];
  in.threads = 1;
  Plan ref;
  int rc = build_plan(in, ref);
  if (rc != 0) {
    std::printf("plan failed: %d %s\n", rc, ref.err.c_str());
    return 1;
  }
  int bad = 0;
  for (int a = 2; a < argc; ++a) {
    in.threads = std::atoi(argv[a]);
    Plan p;
    rc = build_plan(in, p);
    if (rc != 0) {
      std::printf("plan failed with %d threads: %d %s\n", in.threads, rc, p.err.c_str());
      return 1;
    }
    if (compare(ref, p)) {
      std::printf("differs %d\n", in.threads);
      bad = 1;
    } else {
      std::printf("same %d\n", in.threads);
    }
  }
  return bad;
}
