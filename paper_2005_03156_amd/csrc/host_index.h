// Host-side copy of an index, shared by the index builder (index.cpp) and the
// cell-cover builder (cover.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <climits>
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
