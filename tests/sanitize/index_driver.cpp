// The host index and cell-cover builders (index.cpp, cover.cpp) in a program
// of their own, so that they can be built with AddressSanitizer and
// UndefinedBehaviorSanitizer. Reads a block partition from a binary file and
// writes the index file and the cover file exactly as bm_index_build_file
// and bm_cover_build_file do.
//
// Input (little-endian): int64 B, int64 V, int64 L, int32 keep_all_levels,
// int32 cell_log2; int64 vert_off[B + 1]; int32 verts_xy[2 V];
// int64 n_groups[L]; then per level: int64 count, int32 parent[count].
// Usage: index_driver <input> <index out> <cover out>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "blockmap.h"

namespace bm {
int index_build_file(const bm_index_desc* d, const char* path);
int cover_build_file(const bm_index_desc* d, const bm_cover_cfg* cfg, const char* path);
int fail(int code, const std::string& msg) {
  std::fprintf(stderr, "builder: %s\n", msg.c_str());
  return code;
}
}  // namespace bm

template <class T>
static bool get(FILE* f, T* p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t B = 0, V = 0, L = 0;
  int32_t keep = 0, cell_log2 = 0;
  bool ok = get(f, &B, 1) && get(f, &V, 1) && get(f, &L, 1) && get(f, &keep, 1) && get(f, &cell_log2, 1) &&
            B >= 0 && V >= 0 && L >= 0 && L <= 64;
  std::vector<int64_t> vert_off(ok ? B + 1 : 0), n_groups(ok ? L : 0);
  std::vector<int32_t> verts(ok ? 2 * V : 0);
  ok = ok && get(f, vert_off.data(), vert_off.size()) && get(f, verts.data(), verts.size()) &&
       get(f, n_groups.data(), n_groups.size());
  std::vector<std::vector<int32_t>> parents(ok ? L : 0);
  for (int64_t l = 0; ok && l < L; ++l) {
    int64_t c = 0;
    ok = get(f, &c, 1) && c >= 0;
    if (ok) {
      parents[l].resize(c);
      ok = get(f, parents[l].data(), c);
    }
  }
  std::fclose(f);
  if (!ok) return 2;
  std::vector<const int32_t*> par(L);
  for (int64_t l = 0; l < L; ++l) par[l] = parents[l].data();
  bm_index_desc d{};
  d.n_blocks = B;
  d.vert_off = vert_off.data();
  d.verts_xy = verts.data();
  d.n_levels = (int32_t)L;
  d.n_groups = L ? n_groups.data() : nullptr;
  d.parent = L ? par.data() : nullptr;
  d.keep_all_levels = keep;
  int rc = bm::index_build_file(&d, argv[2]);
  if (rc != BM_OK) return 10 + rc;
  bm_cover_cfg cfg{};
  cfg.cell_log2 = cell_log2;
  cfg.threads = 4;
  rc = bm::cover_build_file(&d, &cfg, argv[3]);
  return rc == BM_OK ? 0 : 30 + rc;
}
