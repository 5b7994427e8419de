/* The CPU oracle (oracle/oracle.c) in a program of its own, so that it can be
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (the latter
 * guards its integer reasoning). Reads blocks, a hierarchy and points from a
 * binary file and writes three int32 results per point: brute force over
 * every block, brute force with box rejection, and the hierarchy route.
 *
 * Input (little-endian): int64 B, int64 V, int64 L, int64 N;
 * int64 vert_off[B + 1]; int32 verts_xy[2 V]; int64 n_groups[L]; per level
 * int64 count, int32 parent[count]; int32 xy[2 N].
 * Usage: oracle_driver <input> <output> */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct orc_hier orc_hier;
typedef struct {
  int64_t bbox_tests, leaf_cands, edge_tests, straddles, x_ambiguous, hits;
} orc_counts;
void orc_ring_boxes(int64_t nb, const int64_t* vert_off, const int32_t* verts, int32_t* box);
void orc_brute(int64_t nb, const int64_t* vert_off, const int32_t* verts, const int32_t* box, int64_t n,
               const int32_t* xy, int32_t* out, int32_t* hits);
orc_hier* orc_hier_create(int64_t nb, const int64_t* vert_off, const int32_t* verts, int32_t L,
                          const int64_t* n_groups, const int32_t* const* parent);
void orc_hier_destroy(orc_hier* h);
void orc_hier_map(const orc_hier* h, int64_t n, const int32_t* xy, int32_t* out, orc_counts* counts);

static int get(FILE* f, void* p, size_t size, size_t n) { return fread(p, size, n, f) == n; }

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hdr[4];
  if (!get(f, hdr, 8, 4)) return 2;
  const int64_t B = hdr[0], V = hdr[1], L = hdr[2], N = hdr[3];
  if (B < 0 || V < 0 || L < 0 || L > 64 || N < 0) return 2;
  int64_t* vert_off = malloc(8 * (B + 1));
  int32_t* verts = malloc(8 * (V + 1));
  int64_t* n_groups = malloc(8 * (L + 1));
  int32_t** parent = calloc(L + 1, sizeof(int32_t*));
  int ok = get(f, vert_off, 8, B + 1) && get(f, verts, 4, 2 * V) && get(f, n_groups, 8, L);
  for (int64_t l = 0; ok && l < L; ++l) {
    int64_t c = 0;
    ok = get(f, &c, 8, 1) && c >= 0;
    if (ok) {
      parent[l] = malloc(4 * (c + 1));
      ok = get(f, parent[l], 4, c);
    }
  }
  int32_t* xy = malloc(8 * (N + 1));
  ok = ok && get(f, xy, 4, 2 * N);
  fclose(f);
  if (!ok) return 2;
  int32_t* box = malloc(16 * (B + 1));
  int32_t* out = malloc(12 * (N + 1));
  orc_ring_boxes(B, vert_off, verts, box);
  orc_brute(B, vert_off, verts, NULL, N, xy, out, NULL);
  orc_brute(B, vert_off, verts, box, N, xy, out + N, NULL);
  orc_hier* h = orc_hier_create(B, vert_off, verts, (int32_t)L, L ? n_groups : NULL,
                                (const int32_t* const*)parent);
  orc_counts cnt;
  orc_hier_map(h, N, xy, out + 2 * N, &cnt);
  orc_hier_destroy(h);
  FILE* g = fopen(argv[2], "wb");
  ok = g && fwrite(out, 4, 3 * N, g) == (size_t)(3 * N);
  if (g) fclose(g);
  for (int64_t l = 0; l < L; ++l) free(parent[l]);
  free(parent); free(n_groups); free(verts); free(vert_off); free(xy); free(box); free(out);
  return ok ? 0 : 3;
}
