/*
 * CPU oracle for point -> block mapping. TEST INFRASTRUCTURE ONLY: the unit
 * tests, the smoke check and the benchmark's CPU-baseline leg call it; the
 * GPU library never links, loads or calls anything here, and nothing here is
 * shared with the GPU library.
 *
 * What is computed (paper Sec. III and III-A): the block containing each
 * point, found with the crossing-number test of Shimrat: cast a ray from the
 * point towards +x and count how often it crosses the block boundary; an odd
 * count means inside. Points on a boundary are resolved with the half-open
 * rule (an upward edge owns its lower end, a downward edge its lower end, a
 * horizontal edge never counts, and the crossing must lie strictly to the
 * right of the point), so that in a gap-free partition every point belongs to
 * exactly one block. The result for a point is the smallest block index whose
 * ring gives an odd count, or -1 when there is none.
 *
 * Two routes, both plain:
 *   orc_brute  - every block for every point (the definition; Sec. III-A's
 *                O(N_pt N_poly) simple implementation).
 *   orc_hier_* - the hierarchy of Sec. III: test the point against every
 *                top-level group box, then against the boxes of the children
 *                of each surviving group, level by level, and run the
 *                crossing-number test on every surviving block.
 * Arithmetic is exact: coordinates are integers and the crossing decision is
 * an integer comparison evaluated in 128 bits.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_API __attribute__((visibility("default")))

typedef __int128 i128;

/* Does the ray from (px,py) towards +x cross the edge (ax,ay)->(bx,by)?
 * Straddle: exactly one end lies strictly above the ray's line. Crossing: the
 * edge meets the line at x_int = ax + (py-ay)(bx-ax)/(by-ay), and px < x_int.
 * Multiplying by (by-ay) turns this into (px-ax)(by-ay) < (py-ay)(bx-ax),
 * with the inequality reversed when by-ay < 0. */
static inline int ray_crosses(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px,
                              int64_t py) {
  int a_above = ay > py, b_above = by > py;
  if (a_above == b_above) return 0;
  i128 lhs = (i128)(px - ax) * (i128)(by - ay);
  i128 rhs = (i128)(py - ay) * (i128)(bx - ax);
  return (by > ay) ? (lhs < rhs) : (lhs > rhs);
}

/* Even-odd crossing count over ring verts[0..m), closed from the last vertex
 * back to the first (a stored closing duplicate is a zero-length edge, which
 * never straddles). */
static inline int inside_ring(const int32_t* v, int64_t m, int64_t px, int64_t py) {
  int odd = 0;
  for (int64_t k = 0; k < m; ++k) {
    int64_t k1 = (k + 1 == m) ? 0 : k + 1;
    odd ^= ray_crosses(v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1], px, py);
  }
  return odd;
}

ORC_API int orc_inside(const int32_t* ring, int64_t m, int32_t px, int32_t py) {
  return inside_ring(ring, m, px, py);
}

/* Half-open box of each ring: [min x, max x) x [min y, max y). */
ORC_API void orc_ring_boxes(int64_t nb, const int64_t* vert_off, const int32_t* verts,
                            int32_t* box /* [nb][4]: xmin xmax ymin ymax */) {
  for (int64_t b = 0; b < nb; ++b) {
    int32_t x0 = INT32_MAX, x1 = INT32_MIN, y0 = INT32_MAX, y1 = INT32_MIN;
    for (int64_t k = vert_off[b]; k < vert_off[b + 1]; ++k) {
      int32_t x = verts[2 * k], y = verts[2 * k + 1];
      if (x < x0) x0 = x;
      if (x > x1) x1 = x;
      if (y < y0) y0 = y;
      if (y > y1) y1 = y;
    }
    box[4 * b] = x0; box[4 * b + 1] = x1; box[4 * b + 2] = y0; box[4 * b + 3] = y1;
  }
}

static inline int in_box(const int32_t* bx, int32_t px, int32_t py) {
  return bx[0] <= px && px < bx[1] && bx[2] <= py && py < bx[3];
}

/* Definition route: out[i] = smallest b whose ring contains point i, or -1.
 * box == NULL scans every block; otherwise blocks whose half-open box misses
 * the point are skipped (exact: a point outside that box has an even count).
 * hits (nullable) receives the number of containing blocks per point. */
ORC_API void orc_brute(int64_t nb, const int64_t* vert_off, const int32_t* verts,
                       const int32_t* box, int64_t n, const int32_t* xy, int32_t* out,
                       int32_t* hits) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n; ++i) {
    int32_t px = xy[2 * i], py = xy[2 * i + 1];
    int32_t best = -1, cnt = 0;
    for (int64_t b = 0; b < nb; ++b) {
      if (box && !in_box(box + 4 * b, px, py)) continue;
      if (inside_ring(verts + 2 * vert_off[b], vert_off[b + 1] - vert_off[b], px, py)) {
        if (best < 0) best = (int32_t)b;
        ++cnt;
        if (!hits) break;
      }
    }
    out[i] = best;
    if (hits) hits[i] = cnt;
  }
}

/* ------------------------------------------------------ hierarchy route ---- */

typedef struct {
  int64_t bbox_tests;   /* point-vs-box comparisons, all levels */
  int64_t leaf_cands;   /* (point, block) pairs that reach the crossing test */
  int64_t edge_tests;   /* ring edges examined */
  int64_t straddles;    /* edges whose y-span holds the point */
  int64_t x_ambiguous;  /* straddles with min(ax,bx) <= px < max(ax,bx) */
  int64_t hits;         /* containing blocks found */
} orc_counts;

typedef struct {
  int32_t L;             /* group levels; level L is the blocks */
  int64_t* size;         /* [L+1] entity count per level */
  int32_t** box;         /* [L+1] boxes per level (entity order) */
  int64_t** child_off;   /* [L] CSR per group level */
  int64_t** child;       /* [L] children of each group, ascending index */
  int64_t nb;
  const int64_t* vert_off;
  const int32_t* verts;
} orc_hier;

ORC_API void orc_hier_destroy(orc_hier* h) {
  if (!h) return;
  for (int32_t l = 0; l <= h->L; ++l) free(h->box[l]);
  for (int32_t l = 0; l < h->L; ++l) { free(h->child_off[l]); free(h->child[l]); }
  free(h->size); free(h->box); free(h->child_off); free(h->child);
  free(h);
}

/* The arrays passed in must outlive the handle (vertices are not copied). */
ORC_API orc_hier* orc_hier_create(int64_t nb, const int64_t* vert_off, const int32_t* verts,
                                  int32_t L, const int64_t* n_groups,
                                  const int32_t* const* parent) {
  orc_hier* h = (orc_hier*)calloc(1, sizeof(orc_hier));
  h->L = L; h->nb = nb; h->vert_off = vert_off; h->verts = verts;
  h->size = (int64_t*)malloc(sizeof(int64_t) * (L + 1));
  h->box = (int32_t**)calloc(L + 1, sizeof(int32_t*));
  h->child_off = (int64_t**)calloc(L > 0 ? L : 1, sizeof(int64_t*));
  h->child = (int64_t**)calloc(L > 0 ? L : 1, sizeof(int64_t*));
  for (int32_t l = 0; l < L; ++l) h->size[l] = n_groups[l];
  h->size[L] = nb;
  h->box[L] = (int32_t*)malloc(sizeof(int32_t) * 4 * (nb > 0 ? nb : 1));
  orc_ring_boxes(nb, vert_off, verts, h->box[L]);
  /* group box = smallest box holding the boxes of all its children */
  for (int32_t l = L - 1; l >= 0; --l) {
    int64_t G = h->size[l], E = h->size[l + 1];
    int32_t* gb = (int32_t*)malloc(sizeof(int32_t) * 4 * (G > 0 ? G : 1));
    for (int64_t g = 0; g < G; ++g) {
      gb[4 * g] = INT32_MAX; gb[4 * g + 1] = INT32_MIN;
      gb[4 * g + 2] = INT32_MAX; gb[4 * g + 3] = INT32_MIN;
    }
    const int32_t* cb = h->box[l + 1];
    for (int64_t e = 0; e < E; ++e) {
      int32_t* t = gb + 4 * (int64_t)parent[l][e];
      const int32_t* s = cb + 4 * e;
      if (s[0] < t[0]) t[0] = s[0];
      if (s[1] > t[1]) t[1] = s[1];
      if (s[2] < t[2]) t[2] = s[2];
      if (s[3] > t[3]) t[3] = s[3];
    }
    h->box[l] = gb;
    /* children lists by counting sort on the parent index */
    int64_t* off = (int64_t*)calloc(G + 1, sizeof(int64_t));
    int64_t* ch = (int64_t*)malloc(sizeof(int64_t) * (E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) off[parent[l][e] + 1]++;
    for (int64_t g = 0; g < G; ++g) off[g + 1] += off[g];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (G > 0 ? G : 1));
    memcpy(fill, off, sizeof(int64_t) * G);
    for (int64_t e = 0; e < E; ++e) ch[fill[parent[l][e]]++] = e;
    free(fill);
    h->child_off[l] = off;
    h->child[l] = ch;
  }
  return h;
}

typedef struct { int64_t* v; int64_t n, cap; } vec;
static inline void vpush(vec* a, int64_t x) {
  if (a->n == a->cap) {
    a->cap = a->cap ? 2 * a->cap : 64;
    a->v = (int64_t*)realloc(a->v, sizeof(int64_t) * a->cap);
  }
  a->v[a->n++] = x;
}

ORC_API void orc_hier_map(const orc_hier* h, int64_t n, const int32_t* xy, int32_t* out,
                          orc_counts* counts /* nullable */) {
  orc_counts tot = {0, 0, 0, 0, 0, 0};
#pragma omp parallel
  {
    vec cur = {0, 0, 0}, nxt = {0, 0, 0};
    orc_counts c = {0, 0, 0, 0, 0, 0};
#pragma omp for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
      int32_t px = xy[2 * i], py = xy[2 * i + 1];
      /* top level: every group (or every block when there is no hierarchy) */
      cur.n = 0;
      for (int64_t g = 0; g < h->size[0]; ++g) {
        c.bbox_tests++;
        if (in_box(h->box[0] + 4 * g, px, py)) vpush(&cur, g);
      }
      /* lower levels: children of the surviving groups only */
      for (int32_t l = 0; l < h->L; ++l) {
        nxt.n = 0;
        for (int64_t t = 0; t < cur.n; ++t) {
          int64_t g = cur.v[t];
          for (int64_t q = h->child_off[l][g]; q < h->child_off[l][g + 1]; ++q) {
            int64_t e = h->child[l][q];
            c.bbox_tests++;
            if (in_box(h->box[l + 1] + 4 * e, px, py)) vpush(&nxt, e);
          }
        }
        vec tmp = cur; cur = nxt; nxt = tmp;
      }
      /* leaf: crossing-number test on every candidate block */
      int32_t best = -1;
      for (int64_t t = 0; t < cur.n; ++t) {
        int64_t b = cur.v[t];
        const int32_t* r = h->verts + 2 * h->vert_off[b];
        int64_t m = h->vert_off[b + 1] - h->vert_off[b];
        c.leaf_cands++;
        c.edge_tests += m;
        for (int64_t k = 0; k < m; ++k) {
          int64_t k1 = (k + 1 == m) ? 0 : k + 1;
          int32_t ay = r[2 * k + 1], by = r[2 * k1 + 1], ax = r[2 * k], bx = r[2 * k1];
          if ((ay > py) != (by > py)) {
            c.straddles++;
            int32_t lo = ax < bx ? ax : bx, hi = ax < bx ? bx : ax;
            if (lo <= px && px < hi) c.x_ambiguous++;
          }
        }
        if (inside_ring(r, m, px, py)) {
          c.hits++;
          if (best < 0 || b < best) best = (int32_t)b;
        }
      }
      out[i] = best;
    }
#pragma omp critical
    {
      tot.bbox_tests += c.bbox_tests; tot.leaf_cands += c.leaf_cands;
      tot.edge_tests += c.edge_tests; tot.straddles += c.straddles;
      tot.x_ambiguous += c.x_ambiguous; tot.hits += c.hits;
    }
    free(cur.v); free(nxt.v);
  }
  if (counts) *counts = tot;
}

/* ------------------------------------------------ per-block aggregation ---- */

/* Points per block, the count that the paper's purpose (Sec. I-II: merging
 * demographic data by block) starts from: counts[b] += number of i with
 * ids[i] == b, for b in [0, nb); counts[nb] += number of the other ids (-1,
 * no block). counts holds nb + 1 entries and is accumulated into. */
ORC_API void orc_count_per_block(int64_t n, const int32_t* ids, int64_t nb, uint64_t* counts) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t b = ids[i];
    if (b >= 0 && b < nb) counts[b]++;
    else counts[nb]++;
  }
}

/* Per-point join of a per-block attribute (App. A gathers each point's block
 * FIPS code from the block's record): out[i] = table[ids[i]] when ids[i] is in
 * [0, nb), else fill. */
ORC_API void orc_join_per_block(int64_t n, const int32_t* ids, int64_t nb, const int64_t* table,
                                int64_t fill, int64_t* out) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t b = ids[i];
    out[i] = (b >= 0 && b < nb) ? table[b] : fill;
  }
}

/* Number of worker threads OpenMP will use (for reporting). */
#ifdef _OPENMP
#include <omp.h>
ORC_API int orc_threads(void) { return omp_get_max_threads(); }
ORC_API void orc_set_threads(int t) { omp_set_num_threads(t); }
#else
ORC_API int orc_threads(void) { return 1; }
ORC_API void orc_set_threads(int t) { (void)t; }
#endif
