// Cell cover of an index: the "fast approach" of the paper (Sec. IV, true-hit
// filtering). The plane is cut into a quadtree of non-overlapping square
// cells; a cell that no block edge enters lies wholly inside one block (or
// outside all of them) and stores that answer, so a point falling there needs
// no crossing test at all. Cells that an edge enters are split further, down
// to a finest side of 2^cell_log2; those left at the finest level are
// boundary cells and list every block that can contain one of their points.
// The cells are indexed by a radix trie that consumes four quadtree levels
// (4 bits of each coordinate) per trie level, as the paper's F4 variant does;
// the last trie level takes the remaining 1-4 quadtree levels.
//
// Exactness. A block's answer at an integer point p is decided by the
// crossing rule for p nudged by an infinitesimal (+e1, +e2), 0 < e2 << e1:
// the nudged points of a cell [x0, x0+s) x [y0, y0+s) all lie in the open
// square (x0, x0+s) x (y0, y0+s). Inside and outside change only across the
// ring itself, so if no edge of a block meets the closed square, the block's
// answer is the same at all of them and one crossing test at any point of the
// cell gives it for the whole cell. Every edge counts here, horizontal ones
// too: they never cross a ray, but the answer flips across them (the ray
// passes above or below the ends of the neighbouring edges). The index keeps
// only the edges that can cross a ray (in its y-slab lists), so the builder
// takes the horizontal edges from the rings themselves. The segment/square
// test below is exact integer arithmetic; a touch counted on the square's
// border only makes the cover finer, never wrong.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "host_index.h"

struct bm_cover {
  bm::KCover k;
  const bm_index* index;
  int device;
  bm_cover_info info;
  void* allocs[8];
  int n_allocs;
};

namespace bm {
namespace {

constexpr char kCoverMagic[8] = {'B', 'M', 'C', 'O', 'V', '0', '0', '1'};

struct HostCover {
  CoverShape shape{};
  std::vector<uint32_t> ent;        // trie nodes, root first
  std::vector<uint32_t> cell_off;   // [cells + 1] into cell_leaf
  std::vector<uint32_t> cell_leaf;  // leaf positions (index order) per boundary cell
  std::vector<int32_t> cell_rep;    // answer at each boundary cell's centre (approximate mode)
  int64_t counts[4] = {0, 0, 0, 0};  // interior, node, boundary, empty entries
};

inline int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

inline int tag_of(uint32_t v) { return v == kCoverEmpty ? 3 : (int)(v >> 30); }

struct TooBig {};  // thrown when a cover outgrows the 30-bit entry and cell numbers

struct Child {
  int e;
  int64_t x, y;
  std::vector<int32_t> cand;
};

// Horizontal edges of every leaf (index order), as (x_lo, y, x_hi, y).
struct HorizEdges {
  std::vector<int64_t> off;  // [leaves + 1]
  std::vector<int4> e;
};

class Builder {
 public:
  Builder(const HostIndex& h, const HorizEdges& hz, const CoverShape& sh) : h_(h), hz_(hz), sh_(sh) {}

  int entry_log2(int lev) const {
    int l2 = sh_.log_side;
    for (int t = 0; t <= lev; ++t) l2 -= t == sh_.n_levels - 1 ? sh_.last_bits : 4;
    return l2;
  }

  // Leaf l contains point p (exact, through the leaf's y-slab edge lists).
  bool contains(int l, int64_t px, int64_t py) const {
    const LeafRec& r = h_.leaf[l];
    if (!(r.box.x <= px && px < r.box.y && r.box.z <= py && py < r.box.w)) return false;
    int64_t first, len;
    slab(l, (py - r.box.z) >> (r.packed & 0xff), first, len);
    unsigned acc = 0;
    for (int64_t j = 0; j < len; ++j) {
      const int4& e = h_.ent[first + j];
      acc ^= crosses_host(e.x, e.y, e.z, e.w, px, py);
    }
    return acc != 0;
  }

  // Smallest block index among `cand` containing p, or -1.
  int32_t answer(const int32_t* cand, int n, int64_t px, int64_t py) const {
    int32_t best = -1;
    for (int k = 0; k < n; ++k) {
      const int l = cand[k];
      const int32_t id = h_.leaf[l].leaf_id;
      if ((best < 0 || id < best) && contains(l, px, py)) best = id;
    }
    return best;
  }

  // The node over the square with low corner (x0, y0) at trie level `lev`,
  // for the leaves `cand` whose boxes meet it, with its whole subtree.
  // Returns the node's first entry in o.ent.
  uint32_t node(HostCover& o, int64_t x0, int64_t y0, int lev, const int32_t* cand, int nc) {
    std::vector<Child> kids;
    const uint32_t base = classify(o, x0, y0, lev, cand, nc, kids);
    for (Child& k : kids) {
      const uint32_t c = node(o, k.x, k.y, lev + 1, k.cand.data(), (int)k.cand.size());
      o.ent[base + k.e] = kCoverNode | c;
      o.counts[1]++;
    }
    return base;
  }

  // Fill the entries of one node; entries an edge enters above the finest
  // level are returned in `kids` (their candidates copied) for the caller to
  // build and link.
  uint32_t classify(HostCover& o, int64_t x0, int64_t y0, int lev, const int32_t* cand, int nc,
                    std::vector<Child>& kids) {
    const int bits = lev == sh_.n_levels - 1 ? sh_.last_bits : 4;
    const int F = 1 << bits, ne = F * F;
    const int64_t s = (int64_t)1 << entry_log2(lev);
    const bool finest = lev == sh_.n_levels - 1;
    if (o.ent.size() + ne > kCoverPayload || o.cell_rep.size() >= kCoverPayload) throw TooBig();
    const uint32_t base = (uint32_t)o.ent.size();
    o.ent.resize(base + ne, kCoverEmpty);
    if ((int)sc_.size() <= lev) sc_.resize(lev + 1);
    Scratch& S = sc_[lev];
    // candidates per entry (box overlap), as CSR
    S.cnt.assign(ne + 1, 0);
    S.rng.resize(4 * (size_t)nc);
    for (int k = 0; k < nc; ++k) {
      const int4& b = h_.leaf[cand[k]].box;
      int* R = &S.rng[4 * (size_t)k];
      R[0] = (int)std::clamp<int64_t>(floor_div((int64_t)b.x - x0, s), 0, F - 1);
      R[1] = (int)std::clamp<int64_t>(floor_div((int64_t)b.y - 1 - x0, s), -1, F - 1);
      R[2] = (int)std::clamp<int64_t>(floor_div((int64_t)b.z - y0, s), 0, F - 1);
      R[3] = (int)std::clamp<int64_t>(floor_div((int64_t)b.w - 1 - y0, s), -1, F - 1);
      if (b.x >= b.y || b.z >= b.w || (int64_t)b.x >= x0 + (int64_t)F * s || (int64_t)b.z >= y0 + (int64_t)F * s ||
          (int64_t)b.y <= x0 || (int64_t)b.w <= y0)
        R[1] = -1;  // an empty box holds no point; a box off the node holds none of its points
      for (int j = R[2]; j <= R[3]; ++j)
        for (int i = R[0]; i <= R[1]; ++i) S.cnt[j * F + i + 1]++;
    }
    for (int e = 0; e < ne; ++e) S.cnt[e + 1] += S.cnt[e];
    S.list.resize(S.cnt[ne]);
    S.fill.assign(S.cnt.begin(), S.cnt.end() - 1);
    for (int k = 0; k < nc; ++k) {
      const int* R = &S.rng[4 * (size_t)k];
      for (int j = R[2]; j <= R[3]; ++j)
        for (int i = R[0]; i <= R[1]; ++i) S.list[S.fill[j * F + i]++] = cand[k];
    }
    // entries met by an edge (and, at the finest level, by which leaves)
    S.touched.assign(ne, 0);
    S.tl.clear();
    const int64_t ytop = y0 + (int64_t)F * s;
    for (int k = 0; k < nc; ++k) {
      const int l = cand[k];
      const LeafRec& r = h_.leaf[l];
      if (r.box.x >= r.box.y || r.box.z >= r.box.w) continue;
      const int sh = r.packed & 0xff, logK = (r.packed >> 8) & 0xff;
      const int64_t K = (int64_t)1 << logK;
      const int64_t ylo = std::max<int64_t>(y0, r.box.z), yhi = std::min<int64_t>(ytop, (int64_t)r.box.w - 1);
      if (ylo > yhi) continue;
      const int64_t b0 = std::min<int64_t>(K - 1, (ylo - r.box.z) >> sh);
      const int64_t b1 = std::min<int64_t>(K - 1, (yhi - r.box.z) >> sh);
      for (int64_t b = b0; b <= b1; ++b) {
        int64_t first, len;
        slab(l, b, first, len);
        for (int64_t q = 0; q < len; ++q) {
          const int4& e = h_.ent[first + q];
          // an edge is listed in every slab it spans: take it once
          const int64_t eb = ((int64_t)std::min(e.y, e.w) - r.box.z) >> sh;
          if (std::max(eb, b0) != b) continue;
          mark(S, F, s, x0, y0, finest, l, e);
        }
      }
      for (int64_t q = hz_.off[l]; q < hz_.off[l + 1]; ++q) {
        const int4& e = hz_.e[q];
        if (e.y >= y0 && e.y <= ytop) mark(S, F, s, x0, y0, finest, l, e);
      }
    }
    if (finest) {
      std::sort(S.tl.begin(), S.tl.end());
      S.tl.erase(std::unique(S.tl.begin(), S.tl.end()), S.tl.end());
    }
    // classify the entries
    size_t tpos = 0;
    for (int e = 0; e < ne; ++e) {
      const int i = e % F, j = e / F;
      const int64_t ex = x0 + i * s, ey = y0 + j * s;
      const int32_t* ec = S.list.data() + S.cnt[e];
      const int en = S.cnt[e + 1] - S.cnt[e];
      uint32_t v = kCoverEmpty;
      if (ex > INT32_MAX || ey > INT32_MAX || en == 0) {
        v = kCoverEmpty;  // no block box meets it (or no int32 point lies in it)
      } else if (!S.touched[e]) {
        const int32_t a = answer(ec, en, ex, ey);
        v = a < 0 ? kCoverEmpty : (kCoverInterior | (uint32_t)a);
      } else if (finest) {
        const uint32_t cell = (uint32_t)o.cell_rep.size();
        const size_t c0 = o.cell_leaf.size();
        while (tpos < S.tl.size() && (int)(S.tl[tpos] >> 32) < e) ++tpos;
        for (; tpos < S.tl.size() && (int)(S.tl[tpos] >> 32) == e; ++tpos)
          o.cell_leaf.push_back((uint32_t)S.tl[tpos]);
        // a leaf no edge enters holds either all points of the cell or none:
        // it is listed when it holds the cell's corner
        for (int k = 0; k < en; ++k)
          if (std::find(o.cell_leaf.begin() + c0, o.cell_leaf.end(), (uint32_t)ec[k]) == o.cell_leaf.end() &&
              contains(ec[k], ex, ey))
            o.cell_leaf.push_back((uint32_t)ec[k]);
        o.cell_off.push_back((uint32_t)o.cell_leaf.size());
        const int64_t cx = std::min<int64_t>(ex + s / 2, INT32_MAX), cy = std::min<int64_t>(ey + s / 2, INT32_MAX);
        o.cell_rep.push_back(answer(ec, en, cx, cy));
        v = kCoverBoundary | cell;
      } else {
        kids.push_back({e, ex, ey, std::vector<int32_t>(ec, ec + en)});
        continue;  // linked by the caller
      }
      o.ent[base + e] = v;
      o.counts[tag_of(v)]++;
    }
    return base;
  }

 private:
  struct Scratch {
    std::vector<int> cnt, fill, rng;
    std::vector<int32_t> list;
    std::vector<uint8_t> touched;
    std::vector<int64_t> tl;  // (entry << 32 | leaf) pairs of edge touches
  };

  // Mark the entries (side s, F per axis, from (x0, y0)) whose closed square
  // edge e of leaf l meets.
  static void mark(Scratch& S, int F, int64_t s, int64_t x0, int64_t y0, bool finest, int l, const int4& e) {
    const int64_t xmin = std::min(e.x, e.z), xmax = std::max(e.x, e.z);
    const int64_t ymin = std::min(e.y, e.w), ymax = std::max(e.y, e.w);
    const int i0 = (int)std::max<int64_t>(0, floor_div(xmin - x0 - 1, s));
    const int i1 = (int)std::min<int64_t>(F - 1, floor_div(xmax - x0, s));
    const int j0 = (int)std::max<int64_t>(0, floor_div(ymin - y0 - 1, s));
    const int j1 = (int)std::min<int64_t>(F - 1, floor_div(ymax - y0, s));
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) {
        const int64_t qx = x0 + i * s, qy = y0 + j * s;
        if (!seg_meets_square(e.x, e.y, e.z, e.w, qx, qy, qx + s, qy + s)) continue;
        S.touched[j * F + i] = 1;
        if (finest) S.tl.push_back(((int64_t)(j * F + i) << 32) | (uint32_t)l);
      }
  }

  void slab(int l, int64_t b, int64_t& first, int64_t& len) const {
    const LeafRec& r = h_.leaf[l];
    const int logK = (r.packed >> 8) & 0xff;
    uint32_t o0, o1;
    if (r.packed & kLeafExtOff) {
      const int64_t nq = (((int64_t)1 << logK) + 1 + 3) >> 2;
      const uint32_t* o = reinterpret_cast<const uint32_t*>(h_.ent.data() + (r.ent - nq));
      o0 = o[b];
      o1 = o[b + 1];
    } else {
      o0 = r.off[b];
      o1 = r.off[b + 1];
    }
    first = r.ent + o0;
    len = (int64_t)o1 - o0;
  }

  const HostIndex& h_;
  const HorizEdges& hz_;
  CoverShape sh_;
  std::vector<Scratch> sc_;
};

CoverShape choose_shape(const HostIndex& h, const bm_index_desc* d, int cell_log2) {
  CoverShape sh{};
  const int4 rb = h.root_box;
  const bool empty = rb.x >= rb.y || rb.z >= rb.w;
  sh.ox = empty ? 0 : rb.x;
  sh.oy = empty ? 0 : rb.z;
  const int64_t ext = empty ? 1 : std::max<int64_t>((int64_t)rb.y - rb.x, (int64_t)rb.w - rb.z);
  int L = 0;
  while (((int64_t)1 << L) < ext) ++L;
  if (cell_log2 <= 0) {
    // About 1/64 of the median block's larger box side (most points of a
    // block then fall in interior cells), but no finer than the total ring
    // length over 2^26, which keeps the boundary cells to some tens of
    // millions; rounded to the nearest power of two. (220,900-block grid,
    // 100M points: 2^15 maps in 2.73 ms exact and 1.99 ms approximate, 2^16
    // in 3.21 and 2.03 ms, 2^17 in 4.15 and 2.08 ms; the cover takes 1.66 GB,
    // 0.60 GB and 0.26 GB.)
    std::vector<int64_t> side;
    side.reserve(h.leaf.size());
    for (const LeafRec& r : h.leaf)
      if (r.box.x < r.box.y && r.box.z < r.box.w)
        side.push_back(std::max<int64_t>((int64_t)r.box.y - r.box.x, (int64_t)r.box.w - r.box.z));
    double med = 1;
    if (!side.empty()) {
      std::nth_element(side.begin(), side.begin() + side.size() / 2, side.end());
      med = (double)side[side.size() / 2];
    }
    double len = 0;
    const int2* v = reinterpret_cast<const int2*>(d->verts_xy);
    for (int64_t b = 0; b < d->n_blocks; ++b)
      for (int64_t k = d->vert_off[b]; k < d->vert_off[b + 1]; ++k) {
        const int2 p = v[k], q = v[k + 1 < d->vert_off[b + 1] ? k + 1 : d->vert_off[b]];
        len += std::hypot((double)q.x - p.x, (double)q.y - p.y);
      }
    const double want = std::max({1.0, med / 64, len / (double)(1 << 26)});
    cell_log2 = std::max(1, std::min(30, (int)std::lround(std::log2(want))));
  }
  if (L < cell_log2 + 1) L = cell_log2 + 1;
  const int D = L - cell_log2;
  sh.log_side = L;
  sh.cell_log2 = cell_log2;
  sh.n_levels = (D + 3) / 4;
  sh.last_bits = D - 4 * (sh.n_levels - 1);
  return sh;
}

// Append `p` (built with local offsets) to `out`, relocating its node and
// cell references; returns the relocated first entry of p.
uint32_t append_part(HostCover& out, const HostCover& p) {
  const uint32_t eb = (uint32_t)out.ent.size(), cb = (uint32_t)out.cell_rep.size(),
                 lb = (uint32_t)out.cell_leaf.size();
  out.ent.reserve(out.ent.size() + p.ent.size());
  for (uint32_t v : p.ent) {
    const int t = tag_of(v);
    out.ent.push_back(t == 1 ? (kCoverNode | ((v & kCoverPayload) + eb))
                             : t == 2 ? (kCoverBoundary | ((v & kCoverPayload) + cb)) : v);
  }
  out.cell_leaf.insert(out.cell_leaf.end(), p.cell_leaf.begin(), p.cell_leaf.end());
  for (size_t c = 1; c < p.cell_off.size(); ++c) out.cell_off.push_back(p.cell_off[c] + lb);
  out.cell_rep.insert(out.cell_rep.end(), p.cell_rep.begin(), p.cell_rep.end());
  for (int t = 0; t < 4; ++t) out.counts[t] += p.counts[t];
  return eb;
}

// The root node is classified here; the subtrees below its entries are
// independent tasks built on `threads` threads, each into its own output,
// and appended in entry order, so the result does not depend on scheduling.
// Order-independent fingerprint term of one directed edge.
inline uint64_t edge_mix(int32_t ax, int32_t ay, int32_t bx, int32_t by) {
  uint64_t z = ((uint64_t)(uint32_t)ax << 32 | (uint32_t)ay) * 0x9E3779B97F4A7C15ull ^
               ((uint64_t)(uint32_t)bx << 32 | (uint32_t)by);
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// The horizontal edges of every leaf, taken from the rings of `d`, which must
// be the descriptor the index was built from: each leaf's box, and the count
// and fingerprint of its non-horizontal edges, are checked against the index.
int horizontal_edges(const HostIndex& h, const bm_index_desc* d, HorizEdges& hz) {
  if (!d || d->n_blocks != h.n_leaves || (d->n_blocks > 0 && (!d->vert_off || !d->verts_xy)))
    return fail(BM_EINVAL, "bm_cover: the descriptor does not describe this index's blocks");
  hz.off.assign((size_t)h.n_leaves + 1, 0);
  hz.e.clear();
  const int2* v = reinterpret_cast<const int2*>(d->verts_xy);
  for (int32_t l = 0; l < h.n_leaves; ++l) {
    const LeafRec& r = h.leaf[l];
    const int64_t b = r.leaf_id, a0 = d->vert_off[b], a1 = d->vert_off[b + 1];
    if (b < 0 || b >= d->n_blocks || a1 - a0 < 3) return fail(BM_EINVAL, "bm_cover: descriptor/index mismatch");
    int4 box = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    uint64_t fp = 0, cnt = 0;
    for (int64_t k = a0; k < a1; ++k) {
      const int2 p = v[k], q = v[k + 1 < a1 ? k + 1 : a0];
      box.x = std::min(box.x, p.x);
      box.y = std::max(box.y, p.x);
      box.z = std::min(box.z, p.y);
      box.w = std::max(box.w, p.y);
      if (p.y == q.y && p.x != q.x) hz.e.push_back(make_int4(std::min(p.x, q.x), p.y, std::max(p.x, q.x), p.y));
      if (p.y != q.y) {
        fp += edge_mix(p.x, p.y, q.x, q.y);
        ++cnt;
      }
    }
    // the same over the index's slab lists, each edge once (in its first slab)
    uint64_t fi = 0, ci = 0;
    if (r.box.z < r.box.w) {
      const int sh = r.packed & 0xff, logK = (r.packed >> 8) & 0xff;
      const int64_t K = (int64_t)1 << logK;
      const uint32_t* xo = (r.packed & kLeafExtOff)
                               ? reinterpret_cast<const uint32_t*>(h.ent.data() + (r.ent - ((K + 1 + 3) >> 2)))
                               : nullptr;
      for (int64_t sb = 0; sb < K; ++sb) {
        const int64_t o0 = xo ? xo[sb] : r.off[sb], o1 = xo ? xo[sb + 1] : r.off[sb + 1];
        for (int64_t q = r.ent + o0; q < r.ent + o1; ++q) {
          const int4& e = h.ent[q];
          if ((((int64_t)std::min(e.y, e.w) - r.box.z) >> sh) != sb) continue;
          fi += edge_mix(e.x, e.y, e.z, e.w);
          ++ci;
        }
      }
    }
    if (box.x != r.box.x || box.y != r.box.y || box.z != r.box.z || box.w != r.box.w || fp != fi || cnt != ci)
      return fail(BM_EINVAL, "bm_cover: block " + std::to_string(b) + "'s ring differs from the index's");
    hz.off[l + 1] = (int64_t)hz.e.size();
  }
  return BM_OK;
}

int build_cover(const HostIndex& h, const bm_index_desc* d, const bm_cover_cfg* cfg, HostCover& out) {
  const int cl = cfg ? cfg->cell_log2 : 0;
  if (cl < 0 || cl > 30) return fail(BM_EINVAL, "bm_cover: cell_log2 must be in [0, 30] (0 = automatic)");
  HorizEdges hz;
  int rc = horizontal_edges(h, d, hz);
  if (rc != BM_OK) return rc;
  out = HostCover();
  out.shape = choose_shape(h, d, cl);
  const CoverShape& sh = out.shape;
  int threads = cfg && cfg->threads > 0 ? cfg->threads : (int)std::thread::hardware_concurrency();
  threads = std::max(1, std::min(threads, 256));
  std::vector<int32_t> all(h.leaf.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int32_t)i;
  out.cell_off.assign(1, 0);
  try {
    Builder root(h, hz, sh);
    std::vector<Child> kids;
    root.classify(out, sh.ox, sh.oy, 0, all.data(), (int)all.size(), kids);
    std::vector<HostCover> part(kids.size());
    std::atomic<size_t> next{0};
    std::atomic<int> status{BM_OK};
    auto work = [&]() {
      try {
        Builder b(h, hz, sh);
        for (;;) {
          const size_t t = next.fetch_add(1);
          if (t >= kids.size()) break;
          part[t].cell_off.assign(1, 0);
          b.node(part[t], kids[t].x, kids[t].y, 1, kids[t].cand.data(), (int)kids[t].cand.size());
          std::vector<int32_t>().swap(kids[t].cand);
        }
      } catch (const std::bad_alloc&) {
        status = BM_ENOMEM;
        next = kids.size();
      } catch (const TooBig&) {
        status = BM_ERANGE;
        next = kids.size();
      }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
    if (status == BM_ERANGE) throw TooBig();
    if (status != BM_OK) return fail(BM_ENOMEM, "bm_cover: host allocation failed");
    for (size_t t = 0; t < kids.size(); ++t) {
      const uint32_t c = append_part(out, part[t]);
      part[t] = HostCover();
      out.ent[kids[t].e] = kCoverNode | c;
      out.counts[1]++;
    }
  } catch (const std::bad_alloc&) {
    return fail(BM_ENOMEM, "bm_cover: host allocation failed");
  } catch (const TooBig&) {
    out = HostCover();
    return fail(BM_ERANGE, "bm_cover: the cover exceeds 2^30 trie entries or cells; raise cell_log2");
  }
  if (out.ent.size() > kCoverPayload || out.cell_leaf.size() > UINT32_MAX || out.cell_rep.size() > kCoverPayload)
    return fail(BM_ERANGE, "bm_cover: the cover exceeds 2^30 trie entries or cells; raise cell_log2");
  return BM_OK;
}

bool write_cover(const HostCover& c, const char* path) {
  FILE* f = fopen(path, "wb");
  if (!f) return false;
  const int32_t sc[6] = {c.shape.ox, c.shape.oy, c.shape.log_side, c.shape.n_levels, c.shape.last_bits,
                         c.shape.cell_log2};
  bool ok = fwrite(kCoverMagic, 1, 8, f) == 8 && fwrite(sc, sizeof sc, 1, f) == 1 &&
            fwrite(c.counts, sizeof c.counts, 1, f) == 1 && write_vec(f, c.ent) && write_vec(f, c.cell_off) &&
            write_vec(f, c.cell_leaf) && write_vec(f, c.cell_rep);
  ok = (fclose(f) == 0) && ok;
  return ok;
}

template <class T>
int upload_to(bm_cover* cv, const std::vector<T>& v, const T** dst) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(v.size() * sizeof(T), sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  cv->allocs[cv->n_allocs++] = p;
  cv->info.device_bytes += (int64_t)bytes;
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  *dst = static_cast<const T*>(p);
  return BM_OK;
}

void free_cover(bm_cover* cv) {
  if (!cv) return;
  for (int i = 0; i < cv->n_allocs; ++i) (void)hipFree(cv->allocs[i]);
  delete cv;
}

}  // namespace

int cover_create(const bm_index* index, const bm_index_desc* desc, const bm_cover_cfg* cfg, bm_cover** out) {
  if (!index || !desc || !out) return fail(BM_EINVAL, "bm_cover_create: null argument");
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  HostIndex h;
  int rc = index_to_host(index, h);
  if (rc != BM_OK) return rc;
  HostCover c;
  rc = build_cover(h, desc, cfg, c);
  if (rc != BM_OK) return rc;
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  bm_cover* cv = new (std::nothrow) bm_cover();
  if (!cv) return fail(BM_ENOMEM, "bm_cover_create: host allocation failed");
  cv->index = index;
  cv->device = index->device;
  KCover& k = cv->k;
  if (rc == BM_OK) rc = upload_to(cv, c.ent, &k.ent);
  if (rc == BM_OK) rc = upload_to(cv, c.cell_off, &k.cell_off);
  if (rc == BM_OK) rc = upload_to(cv, c.cell_leaf, &k.cell_leaf);
  if (rc == BM_OK) rc = upload_to(cv, c.cell_rep, &k.cell_rep);
  if (rc != BM_OK) {
    free_cover(cv);
    return rc;
  }
  k.ox = c.shape.ox;
  k.oy = c.shape.oy;
  k.log_side = c.shape.log_side;
  k.n_levels = c.shape.n_levels;
  k.last_bits = c.shape.last_bits;
  bm_cover_info& in = cv->info;
  in.origin_x = c.shape.ox;
  in.origin_y = c.shape.oy;
  in.log2_side = c.shape.log_side;
  in.trie_levels = c.shape.n_levels;
  in.last_level_bits = c.shape.last_bits;
  in.cell_log2 = c.shape.cell_log2;
  in.interior_entries = c.counts[0];
  in.node_entries = c.counts[1];
  in.boundary_cells = c.counts[2];
  in.empty_entries = c.counts[3];
  in.trie_entries = (int64_t)c.ent.size();
  in.cell_leaves = (int64_t)c.cell_leaf.size();
  in.build_seconds = secs;
  *out = cv;
  return BM_OK;
}

int cover_build_file(const bm_index_desc* desc, const bm_cover_cfg* cfg, const char* path) {
  if (!desc || !path) return fail(BM_EINVAL, "bm_cover_build_file: null argument");
  HostIndex h;
  int rc = build_host(desc, h);
  if (rc != BM_OK) return rc;
  HostCover c;
  rc = build_cover(h, desc, cfg, c);
  if (rc != BM_OK) return rc;
  return write_cover(c, path) ? BM_OK : fail(BM_EIO, std::string("bm_cover_build_file: write failed on ") + path);
}

void cover_destroy(bm_cover* cv) { free_cover(cv); }

const KCover& cover_view(const bm_cover* cv) { return cv->k; }
const bm_index* cover_index(const bm_cover* cv) { return cv->index; }
int cover_device(const bm_cover* cv) { return cv->device; }
const bm_cover_info& cover_info(const bm_cover* cv) { return cv->info; }

}  // namespace bm
