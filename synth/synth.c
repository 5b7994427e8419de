/*
 * Seeded synthetic workloads for the point -> block mapping problem.
 *
 * This module generates INPUTS only: block polygons (watertight partitions of
 * a square), the group hierarchy above them, and query points. It holds none
 * of the mapping arithmetic (no bounding boxes, no crossing tests): both the
 * GPU library and the CPU oracle consume its arrays, and neither shares any
 * other code with the other.
 *
 * The paper's inputs are US census shapefiles (56 states, 3,233 counties,
 * 219,831 block groups) and mobile-device locations (Sec. II, Sec. V); neither
 * is available, so these generators stand in for them with the same structure:
 * irregular, non-convex polygons that tile a region without gaps or overlaps,
 * grouped into a nested hierarchy, and clustered query points.
 *
 * Randomness is counter based so that any chunk of any stream can be
 * regenerated independently and in parallel: value i of stream `key` is
 * splitmix64(key + splitmix64(i)), with splitmix64 the finaliser published by
 * Steele, Lea and Flood ("Fast splittable pseudorandom number generators",
 * OOPSLA 2014).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SYN_API __attribute__((visibility("default")))

/* ---------------------------------------------------------------- RNG ---- */

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t rnd(uint64_t key, uint64_t i) { return mix64(key + mix64(i)); }

/* uniform double in [0, 1) with 53 random bits */
static inline double u01(uint64_t key, uint64_t i) {
  return (double)(rnd(key, i) >> 11) * (1.0 / 9007199254740992.0);
}

/* key of (seed, config, stream, index): streams 0 = geometry, 1 = points,
 * 2 = batches / requests; index = chunk, batch or request number */
SYN_API uint64_t syn_key(uint64_t seed, uint64_t cfg, uint64_t stream, uint64_t k) {
  return mix64(mix64(mix64(mix64(seed) ^ cfg) ^ (stream * 0x100000001B3ull)) ^ k);
}

SYN_API uint64_t syn_rand_u64(uint64_t key, uint64_t i) { return rnd(key, i); }
SYN_API double syn_rand_u01(uint64_t key, uint64_t i) { return u01(key, i); }

static inline double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

static inline int32_t to_i32(double v) {
  v = rint(v);
  if (v < -2147483648.0) v = -2147483648.0;
  if (v > 2147483647.0) v = 2147483647.0;
  return (int32_t)v;
}

/* --------------------------------------- jittered shared-edge grid ---- */

typedef struct {
  int32_t n;     /* cells per side; blocks are the n*n cells, id = row*n + col */
  int64_t c;     /* cell size in integer units; the hull is [0, n*c]^2 */
  int32_t klaw;  /* interior points per edge: 0 = uniform {kmin..kmax},
                    1 = min(kmax, kmin + G) with G ~ Geometric(kp) on {0,1,..} */
  int32_t kmin, kmax;
  double kp;
  double vjit;   /* grid-vertex jitter, uniform +-vjit*c per axis */
  double pjit;   /* perpendicular offset of edge points, uniform +-pjit*c */
  double taper;  /* |offset| <= taper * distance to the nearer edge endpoint */
  uint64_t key;
} syn_grid;

static inline int32_t edge_k(const syn_grid* g, int64_t e) {
  uint64_t kk = mix64(g->key ^ 0x6B5Aull);
  if (g->klaw == 0) {
    int32_t span = g->kmax - g->kmin + 1;
    return g->kmin + (int32_t)(rnd(kk, (uint64_t)e) % (uint64_t)span);
  }
  double u = u01(kk, (uint64_t)e);
  double G = floor(log1p(-u) / log1p(-g->kp));
  double k = g->kmin + G;
  return (int32_t)(k > g->kmax ? g->kmax : k);
}

static inline void grid_vertex(const syn_grid* g, int32_t i, int32_t j, double* x, double* y) {
  uint64_t kv = mix64(g->key ^ 0x7E47ull);
  uint64_t id = (uint64_t)j * (uint64_t)(g->n + 1) + (uint64_t)i;
  double c = (double)g->c;
  double px = (double)i * c, py = (double)j * c;
  /* hull vertices move only along the hull; the four corners stay fixed */
  if (i != 0 && i != g->n) px += (2.0 * u01(kv, 2 * id) - 1.0) * g->vjit * c;
  if (j != 0 && j != g->n) py += (2.0 * u01(kv, 2 * id + 1) - 1.0) * g->vjit * c;
  *x = rint(px);
  *y = rint(py);
}

/* horizontal edge (i,j)->(i+1,j): id j*n+i ; vertical edge (i,j)->(i,j+1):
 * id (n+1)*n + j*(n+1)+i */
static inline int64_t hedge_id(const syn_grid* g, int32_t i, int32_t j) { return (int64_t)j * g->n + i; }
static inline int64_t vedge_id(const syn_grid* g, int32_t i, int32_t j) {
  return (int64_t)(g->n + 1) * g->n + (int64_t)j * (g->n + 1) + i;
}

/* interior points of edge e from (ax,ay) to (bx,by), in that direction */
static void edge_points(const syn_grid* g, int64_t e, int boundary, double ax, double ay, double bx,
                        double by, int32_t k, int32_t* out /* 2k */) {
  uint64_t ko = mix64(mix64(g->key ^ 0x0FF5ull) + (uint64_t)e);
  double dx = bx - ax, dy = by - ay;
  double L = sqrt(dx * dx + dy * dy);
  for (int32_t m = 1; m <= k; ++m) {
    double t = (double)m / (double)(k + 1);
    double off = 0.0;
    if (!boundary) {
      off = (2.0 * u01(ko, (uint64_t)m) - 1.0) * g->pjit * (double)g->c;
      double lim = g->taper * (t < 1.0 - t ? t : 1.0 - t) * L;
      off = clampd(off, -lim, lim);
    }
    double x = ax + t * dx - off * dy / L;
    double y = ay + t * dy + off * dx / L;
    out[2 * (m - 1)] = to_i32(x);
    out[2 * (m - 1) + 1] = to_i32(y);
  }
}

/* Ring sizes (no closing duplicate). vert_off has n*n+1 entries. Returns the
 * total vertex count. */
SYN_API int64_t syn_grid_offsets(const syn_grid* g, int64_t* vert_off) {
  int32_t n = g->n;
  vert_off[0] = 0;
  for (int32_t j = 0; j < n; ++j)
    for (int32_t i = 0; i < n; ++i) {
      int64_t b = (int64_t)j * n + i;
      int64_t cnt = 4 + edge_k(g, hedge_id(g, i, j)) + edge_k(g, vedge_id(g, i + 1, j)) +
                    edge_k(g, hedge_id(g, i, j + 1)) + edge_k(g, vedge_id(g, i, j));
      vert_off[b + 1] = vert_off[b] + cnt;
    }
  return vert_off[(int64_t)n * n];
}

static void put_reversed(int32_t* dst, const int32_t* src, int32_t k) {
  for (int32_t m = 0; m < k; ++m) {
    dst[2 * m] = src[2 * (k - 1 - m)];
    dst[2 * m + 1] = src[2 * (k - 1 - m) + 1];
  }
}

/* Fill every ring counter-clockwise: bottom edge, right edge, top edge
 * reversed, left edge reversed. Shared edges are generated once from their
 * own key, so both neighbours hold the identical point list. */
SYN_API void syn_grid_fill(const syn_grid* g, const int64_t* vert_off, int32_t* verts) {
  int32_t n = g->n;
#pragma omp parallel
  {
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(g->kmax + 1));
#pragma omp for schedule(static)
    for (int64_t b = 0; b < (int64_t)n * n; ++b) {
      int32_t j = (int32_t)(b / n), i = (int32_t)(b % n);
      double x00, y00, x10, y10, x11, y11, x01, y01;
      grid_vertex(g, i, j, &x00, &y00);
      grid_vertex(g, i + 1, j, &x10, &y10);
      grid_vertex(g, i + 1, j + 1, &x11, &y11);
      grid_vertex(g, i, j + 1, &x01, &y01);
      int32_t* o = verts + 2 * vert_off[b];
      int32_t k;
      /* bottom: (i,j) -> (i+1,j) */
      *o++ = (int32_t)x00; *o++ = (int32_t)y00;
      k = edge_k(g, hedge_id(g, i, j));
      edge_points(g, hedge_id(g, i, j), j == 0, x00, y00, x10, y10, k, o);
      o += 2 * k;
      /* right: (i+1,j) -> (i+1,j+1) */
      *o++ = (int32_t)x10; *o++ = (int32_t)y10;
      k = edge_k(g, vedge_id(g, i + 1, j));
      edge_points(g, vedge_id(g, i + 1, j), i + 1 == n, x10, y10, x11, y11, k, o);
      o += 2 * k;
      /* top, stored (i,j+1) -> (i+1,j+1), walked backwards */
      *o++ = (int32_t)x11; *o++ = (int32_t)y11;
      k = edge_k(g, hedge_id(g, i, j + 1));
      edge_points(g, hedge_id(g, i, j + 1), j + 1 == n, x01, y01, x11, y11, k, tmp);
      put_reversed(o, tmp, k);
      o += 2 * k;
      /* left, stored (i,j) -> (i,j+1), walked backwards */
      *o++ = (int32_t)x01; *o++ = (int32_t)y01;
      k = edge_k(g, vedge_id(g, i, j));
      edge_points(g, vedge_id(g, i, j), i == 0, x00, y00, x01, y01, k, tmp);
      put_reversed(o, tmp, k);
    }
    free(tmp);
  }
}

/* Nested rectangular bands over the n*n block grid: level l has rows[l] x
 * cols[l] groups (coarse to fine). Composed fine -> coarse so that every group
 * lies inside exactly one group of the level above. parent[l] receives, for
 * every entity of level l+1 (the blocks for the last level), the index of its
 * group at level l. */
SYN_API void syn_band_hierarchy(int32_t n, int32_t levels, const int32_t* rows, const int32_t* cols,
                                int32_t** parent) {
  /* entity (r, c) at the finer level of size R x C maps to (r*R'/R, c*C'/C) */
  for (int32_t l = levels - 1; l >= 0; --l) {
    int32_t R = (l == levels - 1) ? n : rows[l + 1];
    int32_t C = (l == levels - 1) ? n : cols[l + 1];
    for (int32_t r = 0; r < R; ++r)
      for (int32_t c = 0; c < C; ++c) {
        int64_t pr = (int64_t)r * rows[l] / R, pc = (int64_t)c * cols[l] / C;
        parent[l][(int64_t)r * C + c] = (int32_t)(pr * cols[l] + pc);
      }
  }
}

/* ---------------------------------------------------------- points ---- */

/* Mixture setup: K components, weights exp(wsig * N(0,1)) (equal if wsig==0),
 * centres uniform on [0,W]^2, sigma log-uniform on [sig_lo, sig_hi] * W.
 * cumw receives the normalised cumulative weights. */
SYN_API void syn_mixture_setup(uint64_t key, int32_t K, double W, double wsig, double sig_lo,
                               double sig_hi, double* cumw, double* cx, double* cy, double* sig) {
  double s = 0.0;
  for (int32_t k = 0; k < K; ++k) {
    double w = 1.0;
    if (wsig > 0.0) {
      double a = u01(key, 8 * (uint64_t)k), b = u01(key, 8 * (uint64_t)k + 1);
      double z = sqrt(-2.0 * log1p(-a)) * cos(2.0 * M_PI * b);
      w = exp(wsig * z);
    }
    s += w;
    cumw[k] = s;
    cx[k] = u01(key, 8 * (uint64_t)k + 2) * W;
    cy[k] = u01(key, 8 * (uint64_t)k + 3) * W;
    double lo = log(sig_lo), hi = log(sig_hi);
    sig[k] = exp(lo + u01(key, 8 * (uint64_t)k + 4) * (hi - lo)) * W;
  }
  for (int32_t k = 0; k < K; ++k) cumw[k] /= s;
  cumw[K - 1] = 1.0;
}

/* Points i0 .. i0+n-1 of a stream: with probability p_unif uniform on
 * [lo, hi)^2, else Gaussian around a mixture component drawn by weight.
 * Rounded to the nearest integer and clamped to int32. */
SYN_API void syn_mixture_points(uint64_t key, int64_t i0, int64_t n, int32_t K, const double* cumw,
                                const double* cx, const double* cy, const double* sig,
                                double p_unif, double lo, double hi, int32_t* xy) {
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    uint64_t g = (uint64_t)(i0 + j);
    double x, y;
    if (u01(key, 4 * g) < p_unif) {
      x = lo + u01(key, 4 * g + 1) * (hi - lo);
      y = lo + u01(key, 4 * g + 2) * (hi - lo);
    } else {
      double u = u01(key, 4 * g + 1);
      int32_t a = 0, b = K - 1; /* first k with cumw[k] > u */
      while (a < b) {
        int32_t m = (a + b) / 2;
        if (cumw[m] > u) b = m; else a = m + 1;
      }
      double r = sqrt(-2.0 * log1p(-u01(key, 4 * g + 2)));
      double t = 2.0 * M_PI * u01(key, 4 * g + 3);
      x = cx[a] + sig[a] * r * cos(t);
      y = cy[a] + sig[a] * r * sin(t);
    }
    xy[2 * j] = to_i32(x);
    xy[2 * j + 1] = to_i32(y);
  }
}

/* Batch or request sizes: round(exp(U[0, ln hi])) for law 0 (log-uniform on
 * [1, hi]); round(exp(ln(median) + s * N(0,1))) for law 1 (lognormal);
 * clamped to [1, hi]. */
SYN_API void syn_sizes(uint64_t key, int64_t nb, int32_t law, double median, double s, double hi,
                       int64_t* out) {
  for (int64_t b = 0; b < nb; ++b) {
    double v;
    if (law == 0) {
      v = exp(u01(key, 2 * (uint64_t)b) * log(hi));
    } else {
      double a = u01(key, 2 * (uint64_t)b), c = u01(key, 2 * (uint64_t)b + 1);
      double z = sqrt(-2.0 * log1p(-a)) * cos(2.0 * M_PI * c);
      v = exp(log(median) + s * z);
    }
    v = rint(v);
    if (v < 1.0) v = 1.0;
    if (v > hi) v = hi;
    out[b] = (int64_t)v;
  }
}
