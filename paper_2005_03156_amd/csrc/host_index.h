// Host-side copy of an index, shared by the index builder (index.cpp) and the
// cell-cover builder (cover.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "common.h"

namespace bm {

struct HostIndex {
  int32_t n_levels = 0, g0 = 0, leaf_base = 0, n_leaves = 0;
  int4 root_child = {0, 0, -1, 0};
  int4 root_box = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
  int64_t n_verts = 0;
  std::vector<GroupRec> grp;
  std::vector<LeafRec> leaf;
  std::vector<int4> ent;
  std::vector<uint64_t> slot_mask;
  std::vector<int32_t> parent;
};

// Does segment a-b meet the closed rectangle [qx0, qx1] x [qy0, qy1]? Exact:
// the boxes must overlap and the four corners must not lie strictly on one
// side of the line.
inline bool seg_meets_square(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t qx0, int64_t qy0, int64_t qx1,
                             int64_t qy1) {
  if (std::max(ax, bx) < qx0 || std::min(ax, bx) > qx1 || std::max(ay, by) < qy0 || std::min(ay, by) > qy1)
    return false;
  const __int128 dx = bx - ax, dy = by - ay;
  auto side = [&](int64_t px, int64_t py) {
    const __int128 c = dx * (__int128)(py - ay) - dy * (__int128)(px - ax);
    return (c > 0) - (c < 0);
  };
  const int s0 = side(qx0, qy0), s1 = side(qx1, qy0), s2 = side(qx0, qy1), s3 = side(qx1, qy1);
  if (s0 > 0 && s1 > 0 && s2 > 0 && s3 > 0) return false;
  if (s0 < 0 && s1 < 0 && s2 < 0 && s3 < 0) return false;
  return true;
}

// The crossing rule for one edge and a point (the predicate the kernels
// evaluate): the edge takes part when exactly one end is strictly above p,
// and counts when it meets the line y = p.y strictly right of p. The cross
// product is formed only when p lies in the edge's box, so it fits in int64.
inline unsigned crosses_host(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
  const bool a_up = ay > py, b_up = by > py;
  if (a_up == b_up) return 0;
  const int64_t xlo = std::min(ax, bx), xhi = std::max(ax, bx);
  if (px < xlo) return 1;
  if (px >= xhi) return 0;
  const int64_t c = (ax - px) * (by - py) - (bx - px) * (ay - py);
  return b_up ? (c > 0) : (c < 0);
}

// Validate a descriptor and build the host index (index.cpp).
int build_host(const bm_index_desc* d, HostIndex& h);
// Copy a device index back to the host (index.cpp).
int index_to_host(const bm_index* ix, HostIndex& h);

template <class T>
bool write_vec(FILE* f, const std::vector<T>& v) {
  const int64_t n = (int64_t)v.size();
  return fwrite(&n, sizeof n, 1, f) == 1 && (n == 0 || fwrite(v.data(), sizeof(T), n, f) == (size_t)n);
}

template <class T>
bool read_vec(FILE* f, std::vector<T>& v, int64_t max_n) {
  int64_t n = 0;
  if (fread(&n, sizeof n, 1, f) != 1 || n < 0 || n > max_n) return false;
  v.resize(n);
  return n == 0 || fread(v.data(), sizeof(T), n, f) == (size_t)n;
}

template <class T>
int download(const T* src, int64_t n, std::vector<T>& v) {
  v.resize(n);
  if (n == 0) return BM_OK;
  hipError_t e = hipMemcpy(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost);
  return e == hipSuccess ? BM_OK : fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
}

}  // namespace bm
