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

/* key of (seed, workload seed stream, stream, index): streams 0 = geometry, 1 = points,
 * 2 = batches / requests; index = chunk, batch or request number */
SYN_API uint64_t syn_key(uint64_t seed, uint64_t wid, uint64_t stream, uint64_t k) {
  return mix64(mix64(mix64(mix64(seed) ^ wid) ^ (stream * 0x100000001B3ull)) ^ k);
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

/* ------------------------------------------- graded quadtree mesh ---- */
/*
 * A square of R x R root cells, each of side 2^lg_cell units. Root cell c is
 * cut into a 2^d x 2^d grid of equal leaves, d = depth[c] in [0, maxd];
 * neighbouring root cells (8-neighbourhood) differ in depth by at most one,
 * so a leaf side meets at most two leaves of the other side. All leaf corners
 * lie on a lattice of step 2^(lg_cell - maxd) ("lattice units"). A leaf side
 * whose neighbour is one level finer carries the neighbour's corner at its
 * midpoint (a T-junction) so the rings stay watertight.
 *
 * Shared features are derived from lattice coordinates alone, so both sides of
 * a boundary generate them identically and independently:
 *   - lattice vertex (X, Y): jittered by +-vjit of the smallest adjacent leaf
 *     (hull vertices only along the hull, hull corners fixed);
 *   - segment between two consecutive boundary vertices: k interior points,
 *     k from a Lomax (Pareto II) law, perpendicular offset +-pjit of the
 *     segment length tapered to taper * distance to the nearer end (no offset
 *     on the hull). Blocks over vmax vertices have their segments' k scaled
 *     down (a shared segment takes the smaller of its two blocks' factors).
 * Leaves are numbered by root cell (row-major), then row-major inside it.
 */
typedef struct {
  int32_t R, lg_cell, maxd;
  const int8_t* depth;      /* [R*R] */
  const int64_t* leaf_off;  /* [R*R+1] leaves before each root cell */
  double vjit, pjit, taper;
  double k_lambda, k_alpha; /* Lomax scale and shape */
  int32_t vmax;             /* vertex cap per block */
  uint64_t key;
  float* factor;            /* [n_leaves] k scale per block (filled by syn_qt_offsets) */
} syn_qt;

static inline int qt_depth_at(const syn_qt* q, int64_t cx, int64_t cy) {
  if (cx < 0 || cy < 0 || cx >= q->R || cy >= q->R) return -1;
  return q->depth[cy * q->R + cx];
}

/* depth of the leaf containing lattice cell (X, Y) (lower-left corner lattice
 * coordinate of a finest cell), -1 outside */
static inline int qt_depth_cell(const syn_qt* q, int64_t X, int64_t Y) {
  const int64_t per = (int64_t)1 << q->maxd;
  if (X < 0 || Y < 0) return -1;
  return qt_depth_at(q, X / per, Y / per);
}

/* leaf id of the leaf containing finest lattice cell (X, Y) */
static inline int64_t qt_leaf_at(const syn_qt* q, int64_t X, int64_t Y) {
  const int64_t per = (int64_t)1 << q->maxd;
  if (X < 0 || Y < 0 || X >= per * q->R || Y >= per * q->R) return -1;
  const int64_t cx = X / per, cy = Y / per, c = cy * q->R + cx;
  const int d = q->depth[c];
  const int64_t L = per >> d;
  const int64_t i = (X - cx * per) / L, j = (Y - cy * per) / L;
  return q->leaf_off[c] + j * ((int64_t)1 << d) + i;
}

static void qt_vertex(const syn_qt* q, int64_t X, int64_t Y, double* x, double* y) {
  const int64_t per = (int64_t)1 << q->maxd, N = per * q->R;
  const double unit = (double)((int64_t)1 << (q->lg_cell - q->maxd));
  int dmax = -1;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      int d = qt_depth_cell(q, X - a, Y - b);
      if (d > dmax) dmax = d;
    }
  const double s = unit * (double)(per >> (dmax < 0 ? 0 : dmax));
  const uint64_t kv = mix64(q->key ^ 0x7E47ull);
  const uint64_t id = (uint64_t)Y * (uint64_t)(N + 1) + (uint64_t)X;
  double px = (double)X * unit, py = (double)Y * unit;
  if (X != 0 && X != N) px += (2.0 * u01(kv, 2 * id) - 1.0) * q->vjit * s;
  if (Y != 0 && Y != N) py += (2.0 * u01(kv, 2 * id + 1) - 1.0) * q->vjit * s;
  *x = rint(px);
  *y = rint(py);
}

/* raw interior point count of the segment between lattice vertices A < B */
static inline int32_t qt_seg_k_raw(const syn_qt* q, uint64_t sid) {
  const double u = u01(mix64(q->key ^ 0x6B5Aull), sid);
  double k = floor(q->k_lambda * (pow(1.0 - u, -1.0 / q->k_alpha) - 1.0));
  if (k > (double)q->vmax) k = (double)q->vmax;
  return (int32_t)k;
}

/* segment id from its two lattice endpoints (order independent) */
static inline uint64_t qt_seg_id(const syn_qt* q, int64_t X0, int64_t Y0, int64_t X1, int64_t Y1) {
  const int64_t N = ((int64_t)1 << q->maxd) * q->R + 1;
  uint64_t a = (uint64_t)(Y0 * N + X0), b = (uint64_t)(Y1 * N + X1);
  if (a > b) { uint64_t t = a; a = b; b = t; }
  return mix64(a) ^ (b * 0x9E3779B97F4A7C15ull);
}

/* The boundary of leaf (corner (X0,Y0), side L lattice units) as up to 8
 * lattice vertices, counter-clockwise from the lower-left corner. */
static int qt_ring_corners(const syn_qt* q, int64_t X0, int64_t Y0, int64_t L, int d,
                           int64_t* vx, int64_t* vy) {
  int n = 0;
  const int64_t cx[4] = {X0, X0 + L, X0 + L, X0};
  const int64_t cy[4] = {Y0, Y0, Y0 + L, Y0 + L};
  /* finest cell just across the middle of each side: below, right, above, left */
  const int64_t h = L / 2;
  const int64_t ox[4] = {X0 + h, X0 + L, X0 + h, X0 - 1};
  const int64_t oy[4] = {Y0 - 1, Y0 + h, Y0 + L, Y0 + h};
  for (int s = 0; s < 4; ++s) {
    vx[n] = cx[s]; vy[n] = cy[s]; ++n;
    if (L >= 2 && qt_depth_cell(q, ox[s], oy[s]) > d) {
      vx[n] = (cx[s] + cx[(s + 1) & 3]) / 2;
      vy[n] = (cy[s] + cy[(s + 1) & 3]) / 2;
      ++n;
    }
  }
  return n;
}

static void qt_leaf_geom(const syn_qt* q, int64_t leaf, int64_t* X0, int64_t* Y0, int64_t* L, int* d) {
  /* root cell by binary search on leaf_off */
  int64_t lo = 0, hi = (int64_t)q->R * q->R - 1;
  while (lo < hi) {
    int64_t m = (lo + hi + 1) / 2;
    if (q->leaf_off[m] <= leaf) lo = m; else hi = m - 1;
  }
  const int64_t c = lo, per = (int64_t)1 << q->maxd;
  *d = q->depth[c];
  *L = per >> *d;
  const int64_t r = leaf - q->leaf_off[c], side = (int64_t)1 << *d;
  *X0 = (c % q->R) * per + (r % side) * *L;
  *Y0 = (c / q->R) * per + (r / side) * *L;
}

/* The leaf across the segment A -> B, which its own leaf walks counter-
 * clockwise (interior on the left): take the finest lattice cell just to the
 * right of the segment; -1 beyond the hull. */
static int64_t qt_other_leaf(const syn_qt* q, int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  int64_t X, Y;
  if (ay == by) {
    X = ax < bx ? ax : bx;
    Y = bx > ax ? ay - 1 : ay;
  } else {
    Y = ay < by ? ay : by;
    X = by > ay ? ax : ax - 1;
  }
  return qt_leaf_at(q, X, Y);
}

static int32_t qt_seg_k(const syn_qt* q, int64_t self, int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  const int32_t raw = qt_seg_k_raw(q, qt_seg_id(q, ax, ay, bx, by));
  float f = q->factor ? q->factor[self] : 1.0f;
  if (q->factor) {
    int64_t o = qt_other_leaf(q, ax, ay, bx, by);
    if (o >= 0 && q->factor[o] < f) f = q->factor[o];
  }
  if (f >= 1.0f) return raw;
  return (int32_t)floor((double)raw * (double)f);
}

/* Offsets of every ring (no closing duplicate); also fills q->factor. */
SYN_API int64_t syn_qt_offsets(syn_qt* q, int64_t n_leaves, int64_t* vert_off) {
  float* fac = q->factor;
  q->factor = NULL;
  /* pass 1: raw totals -> scale factors */
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t leaf = 0; leaf < n_leaves; ++leaf) {
    int64_t X0, Y0, L, vx[8], vy[8];
    int d;
    qt_leaf_geom(q, leaf, &X0, &Y0, &L, &d);
    const int nc = qt_ring_corners(q, X0, Y0, L, d, vx, vy);
    int64_t tot = nc, ks = 0;
    for (int s = 0; s < nc; ++s) ks += qt_seg_k_raw(q, qt_seg_id(q, vx[s], vy[s], vx[(s + 1) % nc], vy[(s + 1) % nc]));
    tot += ks;
    fac[leaf] = (tot > q->vmax && ks > 0) ? (float)((double)(q->vmax - nc) / (double)ks) : 1.0f;
  }
  q->factor = fac;
  /* pass 2: final counts */
  vert_off[0] = 0;
#pragma omp parallel for schedule(dynamic, 4096)
  for (int64_t leaf = 0; leaf < n_leaves; ++leaf) {
    int64_t X0, Y0, L, vx[8], vy[8];
    int d;
    qt_leaf_geom(q, leaf, &X0, &Y0, &L, &d);
    const int nc = qt_ring_corners(q, X0, Y0, L, d, vx, vy);
    int64_t tot = nc;
    for (int s = 0; s < nc; ++s) tot += qt_seg_k(q, leaf, vx[s], vy[s], vx[(s + 1) % nc], vy[(s + 1) % nc]);
    vert_off[leaf + 1] = tot;
  }
  for (int64_t leaf = 0; leaf < n_leaves; ++leaf) vert_off[leaf + 1] += vert_off[leaf];
  return vert_off[n_leaves];
}

SYN_API void syn_qt_fill(const syn_qt* q, int64_t n_leaves, const int64_t* vert_off, int32_t* verts) {
#pragma omp parallel
  {
    int32_t* tmp = (int32_t*)malloc(sizeof(int32_t) * 2 * (size_t)(q->vmax + 8));
#pragma omp for schedule(dynamic, 4096)
    for (int64_t leaf = 0; leaf < n_leaves; ++leaf) {
      int64_t X0, Y0, L, vx[8], vy[8];
      int d;
      qt_leaf_geom(q, leaf, &X0, &Y0, &L, &d);
      const int nc = qt_ring_corners(q, X0, Y0, L, d, vx, vy);
      const int64_t per = (int64_t)1 << q->maxd, N = per * q->R;
      int32_t* o = verts + 2 * vert_off[leaf];
      for (int s = 0; s < nc; ++s) {
        const int64_t ax = vx[s], ay = vy[s], bx = vx[(s + 1) % nc], by = vy[(s + 1) % nc];
        double fx, fy, gx, gy;
        qt_vertex(q, ax, ay, &fx, &fy);
        *o++ = (int32_t)fx;
        *o++ = (int32_t)fy;
        const int32_t k = qt_seg_k(q, leaf, ax, ay, bx, by);
        if (k == 0) continue;
        /* generate in canonical direction (smaller lattice id first) */
        const int rev = (ay * (N + 1) + ax) > (by * (N + 1) + bx);
        const int64_t cax = rev ? bx : ax, cay = rev ? by : ay, cbx = rev ? ax : bx, cby = rev ? ay : by;
        double px0, py0, px1, py1;
        qt_vertex(q, cax, cay, &px0, &py0);
        qt_vertex(q, cbx, cby, &px1, &py1);
        const int hull = (cax == cbx && (cax == 0 || cax == N)) || (cay == cby && (cay == 0 || cay == N));
        const uint64_t ko = mix64(mix64(q->key ^ 0x0FF5ull) + qt_seg_id(q, cax, cay, cbx, cby));
        const double dx = px1 - px0, dy = py1 - py0, Ls = sqrt(dx * dx + dy * dy);
        for (int32_t m = 1; m <= k; ++m) {
          const double t = (double)m / (double)(k + 1);
          double off = 0.0;
          if (!hull) {
            off = (2.0 * u01(ko, (uint64_t)m) - 1.0) * q->pjit * Ls;
            const double lim = q->taper * (t < 1.0 - t ? t : 1.0 - t) * Ls;
            off = clampd(off, -lim, lim);
          }
          tmp[2 * (m - 1)] = to_i32(px0 + t * dx - off * dy / Ls);
          tmp[2 * (m - 1) + 1] = to_i32(py0 + t * dy + off * dx / Ls);
        }
        if (rev) put_reversed(o, tmp, k);
        else memcpy(o, tmp, sizeof(int32_t) * 2 * (size_t)k);
        o += 2 * k;
      }
    }
    free(tmp);
  }
}

/* leaf -> (root cell, quadtree node at depth min(d, 2) inside it) for the
 * hierarchy; writes per leaf the index of its depth-2 group and per group its
 * root cell. Returns the number of groups. */
SYN_API int64_t syn_qt_groups(const syn_qt* q, int64_t n_leaves, int32_t* leaf_group, int32_t* group_cell) {
  int64_t ng = 0;
  const int64_t C = (int64_t)q->R * q->R;
  for (int64_t c = 0; c < C; ++c) {
    const int d = q->depth[c];
    const int dg = d < 2 ? d : 2;
    const int64_t side = (int64_t)1 << d, gside = (int64_t)1 << dg, sh = d - dg;
    for (int64_t r = 0; r < side * side; ++r) {
      const int64_t i = r % side, j = r / side;
      leaf_group[q->leaf_off[c] + r] = (int32_t)(ng + (j >> sh) * gside + (i >> sh));
    }
    for (int64_t g = 0; g < gside * gside; ++g) group_cell[ng + g] = (int32_t)c;
    ng += gside * gside;
  }
  (void)n_leaves;
  return ng;
}
