// Index construction: validation, node ordering, half-open boxes, slot
// tables, y-slab edge lists, upload, save/load.
//
// The hierarchy of the paper (Sec. III-B: states holding counties holding
// blocks, each with a bounding box and, for blocks, a polygon) becomes one
// node array on the device. Nodes are renumbered level by level so that the
// children of every group are contiguous (a stable counting sort on the
// parent's new position); leaves keep their caller-given block index in
// leaf_id. Leaf boxes are the half-open extent of their ring; a group's box is
// the smallest box holding its children's boxes, so the filter never loses a
// containing block whatever the grouping.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "host_index.h"

namespace bm {
namespace {

constexpr int kTableMinChildren = 2;    // below this a group's children are simply all tested
constexpr int kTableMaxChildren = 256;  // above this too
constexpr int kThinFanout = 4;          // group levels with fewer children per group are left out
constexpr int64_t kMaxRingVerts = (int64_t)1 << 24;       // vertices per ring
constexpr int64_t kMaxSlabEdges = 4 * kMaxRingVerts + 64;  // the longest slab list such a ring gives
constexpr int kTableLogSlots = 7;       // slots per axis: 128 (16 for up to 16 children, 8 for up to 8)

const int4 kEmptyBox = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};

// Device layout of the boxes that filter steps test: the group records, then
// from a 64-byte boundary a copy of every leaf's box (16 bytes, so that the
// boxes of sibling leaves share cache lines), in one allocation. At most
// 2^26 nodes keep it below 2^31 bytes.
size_t leaf_boxes_offset(const HostIndex& h) { return (h.grp.size() * sizeof(GroupRec) + 63) & ~(size_t)63; }
size_t box_block_bytes(const HostIndex& h) { return leaf_boxes_offset(h) + h.leaf.size() * sizeof(int4); }

inline void grow(int4& a, const int4& b) {
  a.x = std::min(a.x, b.x);
  a.y = std::max(a.y, b.y);
  a.z = std::min(a.z, b.z);
  a.w = std::max(a.w, b.w);
}

// Slot table of a group with 2..256 children: the group box is cut into S = 128
// equal power-of-two slots per axis (S = 16 for up to 16 children, S = 8 for up
// to 8, where the table then fills one 128-byte line), and the row of slot s of
// an axis (W = ceil(children / 64) words) holds a bit for every child whose box
// overlaps it on that axis; x-rows first, then y-rows, starting on a 128-byte
// boundary. For a point in the group box, (x-slot mask & y-slot mask) is a superset
// of the children whose boxes contain it; the exact half-open box test is then
// run on those children only, so the filter's result is unchanged.
template <class BoxOf>
int4 make_table(BoxOf box_of, int c0, int c1, const int4& g, std::vector<uint64_t>& masks) {
  int4 r = make_int4(c0, c1, -1, 0);
  const int m = c1 - c0;
  if (m < kTableMinChildren || m > kTableMaxChildren || g.x >= g.y || g.z >= g.w) return r;
  const int logS = m <= 8 ? 3 : m <= 16 ? 4 : kTableLogSlots, S = 1 << logS, W = (m + 63) / 64;
  const int64_t wx = (int64_t)g.y - g.x, wy = (int64_t)g.w - g.z;
  int shx = 0, shy = 0;
  while (((int64_t)S << shx) < wx) ++shx;
  while (((int64_t)S << shy) < wy) ++shy;
  const size_t off = (masks.size() + 15) & ~(size_t)15;
  if (off + 2 * (size_t)S * W > (size_t)kMaxSlotWords) return r;
  masks.resize(off + 2 * (size_t)S * W, 0);
  for (int c = c0; c < c1; ++c) {
    const int4 b = box_of(c);
    if (b.x >= b.y || b.z >= b.w) continue;  // an empty box holds no point
    const int w = (c - c0) >> 6;
    const uint64_t bit = 1ull << ((c - c0) & 63);
    const int64_t sx0 = ((int64_t)b.x - g.x) >> shx, sx1 = ((int64_t)b.y - 1 - g.x) >> shx;
    const int64_t sy0 = ((int64_t)b.z - g.z) >> shy, sy1 = ((int64_t)b.w - 1 - g.z) >> shy;
    for (int64_t t = sx0; t <= sx1; ++t) masks[off + t * W + w] |= bit;
    for (int64_t t = sy0; t <= sy1; ++t) masks[off + (S + t) * W + w] |= bit;
  }
  r.z = (int)off;
  r.w = logS | (shx << 8) | (shy << 16) | (W << 24);
  return r;
}

// y-slabs of one ring (closed: v[0..m], v[m] = v[0]) with box bx. Only edges
// whose half-open y-span [min y, max y) overlaps a slab can meet a horizontal
// line through it, so the crossing test of a point needs only the edges listed
// for its slab. An edge with equal end heights never takes part and is left
// out. About per_slab edges per slab; fewer slabs when long edges would
// repeat too often. Appends to `ent` (offsets out of line when they do not
// fit in the record) and fills the record's slab fields, with rec.ent
// relative to the start of `ent`.
void build_slabs(const int2* v, int64_t m, const int4& bx, std::vector<int4>& ent, LeafRec& rec,
                 const int per_slab) {
  const int64_t ymin = bx.z, height = (int64_t)bx.w - bx.z;
  int logK = 0;
  while (logK < 12 && ((int64_t)per_slab << logK) < m) ++logK;
  if (height <= 0) logK = 0;
  std::vector<int64_t> cnt;
  int sh = 0;
  int64_t total = 0;
  for (;; --logK) {
    const int64_t K = (int64_t)1 << logK;
    sh = 0;
    while (height > 0 && (K << sh) < height) ++sh;
    cnt.assign(K + 1, 0);
    total = 0;
    for (int64_t k = 0; k < m; ++k) {
      const int64_t lo = std::min(v[k].y, v[k + 1].y), hi = std::max(v[k].y, v[k + 1].y);
      if (lo == hi) continue;
      const int64_t b0 = (lo - ymin) >> sh, b1 = (hi - 1 - ymin) >> sh;
      for (int64_t b = b0; b <= b1; ++b) cnt[b + 1]++;
      total += b1 - b0 + 1;
    }
    if (total > 4 * m + 64 && logK > 0) continue;
    break;
  }
  const int64_t K = (int64_t)1 << logK;
  for (int64_t b = 0; b < K; ++b) cnt[b + 1] += cnt[b];
  rec.packed = sh | (logK << 8);
  memset(rec.off, 0, sizeof rec.off);
  if (K + 1 <= (int64_t)sizeof rec.off && total <= 255) {
    for (int64_t b = 0; b <= K; ++b) rec.off[b] = (unsigned char)cnt[b];
  } else {
    rec.packed |= kLeafExtOff;
    const int64_t nq = (K + 1 + 3) / 4;
    const size_t q0 = ent.size();
    ent.resize(q0 + nq, make_int4(0, 0, 0, 0));
    uint32_t* o = reinterpret_cast<uint32_t*>(ent.data() + q0);
    for (int64_t b = 0; b <= K; ++b) o[b] = (uint32_t)cnt[b];
  }
  const size_t e0 = ent.size();
  rec.ent = (long long)e0;
  ent.resize(e0 + (size_t)total);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t k = 0; k < m; ++k) {
    const int64_t lo = std::min(v[k].y, v[k + 1].y), hi = std::max(v[k].y, v[k + 1].y);
    if (lo == hi) continue;
    const int64_t b0 = (lo - ymin) >> sh, b1 = (hi - 1 - ymin) >> sh;
    for (int64_t b = b0; b <= b1; ++b) ent[e0 + fill[b]++] = make_int4(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y);
  }
}

// The cell map of one ring (closed: v[0..m], v[m] = v[0]) with box bx: the
// box cut into kLeafCells x kLeafCells cells of 2^sx x 2^sy units. A cell
// whose closed rectangle meets an edge of the ring (horizontal and zero-length
// edges included, tested exactly) is kCellTest. Every other cell holds one
// answer: the integer points of a cell [x, x + 2^sx) x [y, y + 2^sy) are
// decided as if nudged by (+e1, +e2) with 0 < e2 << e1 << 1, so they all lie
// in the open rectangle, which no edge meets. Edge-free cells that share a
// side share that answer too, so it is taken once per 4-connected group of
// them, by the crossing rule at the lower-left point of one cell.
void build_cells(const int2* v, int64_t m, const int4& bx, uint32_t (&cell)[kLeafCells]) {
  for (uint32_t& c : cell) c = 0xAAAAAAAAu;  // every cell kCellTest
  const int64_t x0 = bx.x, y0 = bx.z, w = (int64_t)bx.y - bx.x, h = (int64_t)bx.w - bx.z;
  if (w <= 0 || h <= 0) return;  // an empty box holds no point
  const int sx = cell_shift((unsigned)w), sy = cell_shift((unsigned)h);
  constexpr int C = kLeafCells;
  bool hit[C][C] = {};  // [row][column]: an edge meets the closed cell
  for (int64_t k = 0; k < m; ++k) {
    const int64_t ax = v[k].x, ay = v[k].y, bx2 = v[k + 1].x, by2 = v[k + 1].y;
    // columns c whose closed x-range [x0 + c 2^sx, x0 + (c+1) 2^sx] can meet
    // the edge's, and likewise rows
    const int64_t c0 = std::max<int64_t>(0, ((std::min(ax, bx2) - x0) >> sx) - 1);
    const int64_t c1 = std::min<int64_t>(C - 1, (std::max(ax, bx2) - x0) >> sx);
    const int64_t r0 = std::max<int64_t>(0, ((std::min(ay, by2) - y0) >> sy) - 1);
    const int64_t r1 = std::min<int64_t>(C - 1, (std::max(ay, by2) - y0) >> sy);
    for (int64_t r = r0; r <= r1; ++r)
      for (int64_t c = c0; c <= c1; ++c)
        if (!hit[r][c] && seg_meets_square(ax, ay, bx2, by2, x0 + (c << sx), y0 + (r << sy), x0 + ((c + 1) << sx),
                                            y0 + ((r + 1) << sy)))
          hit[r][c] = true;
  }
  int comp[C][C];
  for (auto& row : comp)
    for (int& x : row) x = -1;
  int todo[C * C];
  for (int r = 0; r < C; ++r)
    for (int c = 0; c < C; ++c) {
      if (hit[r][c] || comp[r][c] >= 0) continue;
      // the answer of this group: the crossing rule at the cell's lower-left point
      const int64_t px = x0 + ((int64_t)c << sx), py = y0 + ((int64_t)r << sy);
      unsigned par = 0;
      for (int64_t k = 0; k < m; ++k) par ^= crosses_host(v[k].x, v[k].y, v[k + 1].x, v[k + 1].y, px, py);
      const uint32_t cls = par ? kCellIn : kCellOut;
      int n = 0;
      todo[n++] = r * C + c;
      comp[r][c] = 1;
      while (n) {
        const int q = todo[--n], qr = q / C, qc = q % C;
        cell[qr] = (cell[qr] & ~(3u << (2 * qc))) | (cls << (2 * qc));
        const int nr[4] = {qr - 1, qr + 1, qr, qr}, nc[4] = {qc, qc, qc - 1, qc + 1};
        for (int t = 0; t < 4; ++t)
          if (nr[t] >= 0 && nr[t] < C && nc[t] >= 0 && nc[t] < C && !hit[nr[t]][nc[t]] && comp[nr[t]][nc[t]] < 0) {
            comp[nr[t]][nc[t]] = 1;
            todo[n++] = nr[t] * C + nc[t];
          }
      }
    }
}

}  // namespace

int build_host(const bm_index_desc* d, HostIndex& h) {
  if (!d) return fail(BM_EINVAL, "bm_index_create: null descriptor");
  const int64_t B = d->n_blocks;
  if (B < 0 || B > INT32_MAX) return fail(BM_EINVAL, "bm_index_create: n_blocks out of range");
  if (d->n_levels < 0 || d->n_levels > 64) return fail(BM_EINVAL, "bm_index_create: n_levels out of range");
  if (B > 0 && (!d->vert_off || !d->verts_xy)) return fail(BM_EINVAL, "bm_index_create: null ring arrays");
  int L = d->n_levels;
  if (L > 0 && (!d->n_groups || !d->parent)) return fail(BM_EINVAL, "bm_index_create: null hierarchy arrays");

  // level sizes, coarse to fine; the last level is the blocks
  std::vector<int64_t> size(L + 1);
  int64_t total_nodes = 0;
  for (int l = 0; l < L; ++l) {
    if (d->n_groups[l] < 1 || d->n_groups[l] > INT32_MAX)
      return fail(BM_EINVAL, "bm_index_create: n_groups[" + std::to_string(l) + "] out of range");
    if (!d->parent[l]) return fail(BM_EINVAL, "bm_index_create: null parent[" + std::to_string(l) + "]");
    size[l] = d->n_groups[l];
    total_nodes += size[l];
  }
  size[L] = B;
  total_nodes += B;
  if (total_nodes > kMaxNodes)
    return fail(BM_ERANGE, "bm_index_create: more than 2^" + std::to_string(32 - kSlotBits) +
                               " nodes (groups of all levels plus blocks)");

  // rings
  if (B > 0) {
    if (d->vert_off[0] != 0) return fail(BM_EINVAL, "bm_index_create: vert_off[0] must be 0");
    for (int64_t b = 0; b < B; ++b) {
      const int64_t m = d->vert_off[b + 1] - d->vert_off[b];
      if (m < 3)
        return fail(BM_EINVAL, "bm_index_create: ring " + std::to_string(b) + " has fewer than 3 vertices");
      // A slab lists at most 4m + 64 edges, so the edge chunks that one
      // crossing-test round of 64 pairs deals out stay below 2^31.
      if (m > kMaxRingVerts)
        return fail(BM_EINVAL, "bm_index_create: ring " + std::to_string(b) + " has more than 2^24 vertices");
    }
    const int64_t V = d->vert_off[B];
    for (int64_t k = 0; k < 2 * V; ++k)
      if (d->verts_xy[k] < 0)
        return fail(BM_ERANGE, "bm_index_create: vertex coordinate outside [0, 2^31-1] at vertex " +
                                   std::to_string(k / 2));
    h.n_verts = V;
  }
  // parents
  for (int l = 0; l < L; ++l) {
    const int32_t* par = d->parent[l];
    for (int64_t e = 0; e < size[l + 1]; ++e)
      if (par[e] < 0 || par[e] >= size[l])
        return fail(BM_EINVAL, "bm_index_create: parent[" + std::to_string(l) + "][" + std::to_string(e) +
                                   "] out of range");
  }

  // Thin group levels are left out: a level whose groups hold fewer than
  // kThinFanout children on average costs each point one more round of group
  // items for little filtering, so the level above adopts its children (the
  // root, for level 0). Group boxes are unions of their children's boxes, so
  // the candidates stay a superset of the true hits and no result changes. A
  // level stays if leaving it out would give a group more children than a
  // slot table holds. (220,900-block grid with tracts of ~3 blocks: mapping
  // kernel 5.03 -> 4.70 ms per 100M points.) A caller may ask to keep every
  // level.
  std::vector<const int32_t*> par(d->parent, d->parent + L);
  std::vector<std::vector<int32_t>> composed;
  composed.reserve(L);
  for (int l = d->keep_all_levels ? -1 : L - 1; l >= 0; --l) {
    const int64_t G = size[l], E = size[l + 1];
    if (E >= kThinFanout * G) continue;
    if (l == 0) {
      if (E > kTableMaxChildren) continue;
    } else {
      std::vector<int32_t> cnt(size[l - 1], 0);
      bool fits = true;
      for (int64_t e = 0; e < E && fits; ++e) fits = ++cnt[par[l - 1][par[l][e]]] <= kTableMaxChildren;
      if (!fits) continue;
      composed.emplace_back(E);
      for (int64_t e = 0; e < E; ++e) composed.back()[e] = par[l - 1][par[l][e]];
      par[l - 1] = composed.back().data();
    }
    par.erase(par.begin() + l);
    size.erase(size.begin() + l);
    total_nodes -= G;
    --L;
  }

  // new positions: level 0 keeps its order; a finer level is sorted stably by
  // the new position of its parent
  std::vector<int64_t> base(L + 2, 0);
  for (int l = 0; l <= L; ++l) base[l + 1] = base[l] + size[l];
  std::vector<std::vector<int32_t>> pos(L + 1);
  std::vector<int32_t> leaf_order;  // new leaf position -> caller's block index
  pos[0].resize(size[0]);
  for (int64_t e = 0; e < size[0]; ++e) pos[0][e] = (int32_t)e;
  if (L == 0) {
    leaf_order.resize(B);
    for (int64_t e = 0; e < B; ++e) leaf_order[e] = (int32_t)e;
  }
  h.grp.assign(base[L], GroupRec{kEmptyBox, make_int4(0, 0, -1, 0)});
  h.parent.assign(total_nodes, -1);
  for (int l = 0; l < L; ++l) {
    const int32_t* pl = par[l];
    const int64_t G = size[l], E = size[l + 1];
    std::vector<int64_t> cnt(G + 1, 0);
    for (int64_t e = 0; e < E; ++e) cnt[pos[l][pl[e]] + 1]++;
    for (int64_t g = 0; g < G; ++g) cnt[g + 1] += cnt[g];
    for (int64_t g = 0; g < G; ++g)  // children of the group at new position g
      h.grp[base[l] + g].child =
          make_int4((int)(base[l + 1] + cnt[g]), (int)(base[l + 1] + cnt[g + 1]), -1, 0);
    pos[l + 1].resize(E);
    if (l + 1 == L) leaf_order.resize(E);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t e = 0; e < E; ++e) {
      const int64_t np = fill[pos[l][pl[e]]]++;
      pos[l + 1][e] = (int32_t)np;
      if (l + 1 == L) leaf_order[np] = (int32_t)e;
      h.parent[base[l + 1] + np] = (int32_t)(base[l] + pos[l][pl[e]]);
    }
  }

  // leaves, in parallel over ranges: box, id, y-slab lists. About three edges
  // per slab keep a crossing test's slab short; an index too large for the
  // last-level cache (estimated as its leaf records plus two 16-byte entries
  // per vertex) lists about six, so that long edges repeat in fewer slabs
  // (8M-block quadtree: 8.68 -> 6.93 GB on the device, mapping time unchanged;
  // six would cost the 220,900-block grid 1.5 %).
  const int per_slab =
      (int64_t)B * (int64_t)sizeof(LeafRec) + 32 * (int64_t)d->vert_off[d->n_blocks] > kPresortBigIndex ? 6 : 3;
  h.leaf.assign(B, LeafRec{});
  const int T = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)std::thread::hardware_concurrency(), 16,
                                                              B / 4096 + 1}));
  std::vector<std::vector<int4>> part(T);
  auto work = [&](int t) {
    const int64_t lo = B * t / T, hi = B * (t + 1) / T;
    std::vector<int2> ring;
    for (int64_t nb = lo; nb < hi; ++nb) {
      const int32_t b = leaf_order[nb];
      const int32_t* src = d->verts_xy + 2 * d->vert_off[b];
      const int64_t m = d->vert_off[b + 1] - d->vert_off[b];
      ring.resize(m + 1);
      int4 bx = kEmptyBox;
      for (int64_t k = 0; k < m; ++k) {
        ring[k] = make_int2(src[2 * k], src[2 * k + 1]);
        grow(bx, make_int4(ring[k].x, ring[k].x, ring[k].y, ring[k].y));
      }
      ring[m] = ring[0];
      LeafRec& rec = h.leaf[nb];
      rec.box = bx;
      rec.leaf_id = b;
      build_slabs(ring.data(), m, bx, part[t], rec, per_slab);
      build_cells(ring.data(), m, bx, rec.cell);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(work, t);
    work(0);
    for (auto& x : th) x.join();
  }
  size_t tot = 0;
  for (int t = 0; t < T; ++t) tot += part[t].size();
  h.ent.resize(std::max<size_t>(tot, 1));
  size_t at = 0;
  for (int t = 0; t < T; ++t) {
    const int64_t lo = B * t / T, hi = B * (t + 1) / T;
    for (int64_t nb = lo; nb < hi; ++nb) h.leaf[nb].ent += (long long)at;
    if (!part[t].empty()) memcpy(h.ent.data() + at, part[t].data(), part[t].size() * sizeof(int4));
    at += part[t].size();
    std::vector<int4>().swap(part[t]);
  }
  auto box_of = [&](int64_t c) { return c >= base[L] ? h.leaf[c - base[L]].box : h.grp[c].box; };
  // group boxes, finest group level first
  for (int l = L - 1; l >= 0; --l)
    for (int64_t g = 0; g < size[l]; ++g) {
      const int4 cr = h.grp[base[l] + g].child;
      int4 bx = kEmptyBox;
      for (int c = cr.x; c < cr.y; ++c) grow(bx, box_of(c));
      h.grp[base[l] + g].box = bx;
    }
  // slot tables: every group, then the virtual root over level 0
  for (int64_t g = 0; g < base[L]; ++g)
    h.grp[g].child = make_table(box_of, h.grp[g].child.x, h.grp[g].child.y, h.grp[g].box, h.slot_mask);
  int4 rb = kEmptyBox;
  for (int64_t e = 0; e < size[0]; ++e) grow(rb, box_of(e));
  if ((int64_t)h.ent.size() > kMaxEnt)
    return fail(BM_ERANGE, "bm_index_create: the slab edge lists exceed 2^31 entries");
  h.root_box = rb;
  h.root_child = make_table(box_of, 0, (int)size[0], rb, h.slot_mask);
  h.n_levels = L;
  h.g0 = (int32_t)size[0];
  h.leaf_base = (int32_t)base[L];
  h.n_leaves = (int32_t)B;
  return BM_OK;
}

namespace {

// Device copy of v followed by `pad` zeroed elements.
template <class T>
int upload(bm_index* ix, const std::vector<T>& v, const T** dst, size_t pad = 0) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>((v.size() + pad) * sizeof(T), sizeof(T));
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ix->allocs[ix->n_allocs++] = p;
  ix->bytes += (int64_t)bytes;
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  if (pad) {
    e = hipMemset(static_cast<T*>(p) + v.size(), 0, pad * sizeof(T));
    if (e != hipSuccess) return fail(BM_EHIP, std::string("hipMemset: ") + hipGetErrorString(e));
  }
  *dst = static_cast<const T*>(p);
  return BM_OK;
}

int upload_boxes(bm_index* ix, const HostIndex& h, const GroupRec** grp) {
  void* p = nullptr;
  const size_t lo = leaf_boxes_offset(h), bytes = std::max<size_t>(box_block_bytes(h), 64);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  ix->allocs[ix->n_allocs++] = p;
  ix->bytes += (int64_t)bytes;
  char* c = static_cast<char*>(p);
  std::vector<int4> boxes(h.leaf.size());
  for (size_t b = 0; b < h.leaf.size(); ++b) boxes[b] = h.leaf[b].box;
  if (!h.grp.empty()) e = hipMemcpy(c, h.grp.data(), h.grp.size() * sizeof(GroupRec), hipMemcpyHostToDevice);
  if (e == hipSuccess && !boxes.empty())
    e = hipMemcpy(c + lo, boxes.data(), boxes.size() * sizeof(int4), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(BM_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  *grp = reinterpret_cast<const GroupRec*>(c);
  return BM_OK;
}

void free_index(bm_index* ix) {
  if (!ix) return;
  for (int i = 0; i < ix->n_allocs; ++i) (void)hipFree(ix->allocs[i]);
  delete ix;
}

// The adaptive sort bins of SortMap: each coarse cell's depth raised, one
// level at a time, where the most blocks (by box centre) share a bin, while
// the bins stay within kSortMapBins; false when the extent is too small for
// bins of at least 64 units, or there are no leaves.
bool build_sort_map(const HostIndex& h, int& log_side, int& n_bins, std::vector<uint32_t>& cell,
                    std::vector<int4>& sq) {
  const int4 rb = h.root_box;
  if (rb.x >= rb.y || rb.z >= rb.w || h.leaf.empty()) return false;
  const int64_t ext = std::max<int64_t>((int64_t)rb.y - rb.x, (int64_t)rb.w - rb.z);
  int L = 0;
  while (((int64_t)1 << L) < ext) ++L;
  if (L < kSortCoarseBits + kSortMaxDepth + 6 || L > 31) return false;
  const int cs = L - kSortCoarseBits;
  constexpr int kSide = 1 << kSortCoarseBits;
  std::vector<int64_t> blocks(kSortCells, 0);
  for (const LeafRec& r : h.leaf)
    if (r.box.x < r.box.y && r.box.z < r.box.w) {
      const int64_t x = ((((int64_t)r.box.x + r.box.y - 1) >> 1) - rb.x) >> cs;
      const int64_t y = ((((int64_t)r.box.z + r.box.w - 1) >> 1) - rb.z) >> cs;
      blocks[(size_t)(y * kSide + x)]++;
    }
  std::vector<int> d(kSortCells, 0);
  int64_t bins = kSortCells;
  // max-heap on blocks per bin (blocks / 4^d), ties to the lower cell
  auto per_bin = [&](int c) { return (double)blocks[c] / (double)((int64_t)1 << (2 * d[c])); };
  std::vector<std::pair<double, int>> heap;
  for (int c = 0; c < kSortCells; ++c) heap.push_back({per_bin(c), -c});
  std::make_heap(heap.begin(), heap.end());
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end());
    const auto [load, negc] = heap.back();
    heap.pop_back();
    const int c = -negc;
    if (load <= 1.0) break;
    const int64_t add = 3 * ((int64_t)1 << (2 * d[c]));
    if (d[c] >= kSortMaxDepth || bins + add > kSortMapBins) continue;
    d[c]++;
    bins += add;
    heap.push_back({per_bin(c), -c});
    std::push_heap(heap.begin(), heap.end());
  }
  // bins in Z-order: coarse cells by Morton index, each cell's bins by theirs
  auto spread = [](uint32_t v) {
    uint32_t r = 0;
    for (int b = 0; b < 16; ++b) r |= ((v >> b) & 1u) << (2 * b);
    return r;
  };
  std::vector<int> zorder(kSortCells);
  for (int c = 0; c < kSortCells; ++c) zorder[spread((uint32_t)(c % kSide)) | (spread((uint32_t)(c / kSide)) << 1)] = c;
  cell.assign(kSortCells, 0);
  sq.assign(kSortMapBins, make_int4(0, 0, 0, 0));
  uint32_t first = 0;
  for (int z = 0; z < kSortCells; ++z) {
    const int c = zorder[z], dc = d[c];
    cell[c] = first | ((uint32_t)dc << 16);
    const int fs = cs - dc;  // log side of the cell's bins
    const uint32_t n = 1u << dc;
    for (uint32_t fy = 0; fy < n; ++fy)
      for (uint32_t fx = 0; fx < n; ++fx) {
        const uint32_t x0 = ((uint32_t)(c % kSide) << cs) + (fx << fs);
        const uint32_t y0 = ((uint32_t)(c / kSide) << cs) + (fy << fs);
        sq[first + (spread(fx) | (spread(fy) << 1))] = make_int4((int)x0, (int)y0, fs, 0);
      }
    first += n * n;
  }
  log_side = L;
  n_bins = (int)first;
  return true;
}

int make_device(HostIndex& h, bm_index** out) {
  bm_index* ix = new (std::nothrow) bm_index();
  if (!ix) return fail(BM_ENOMEM, "bm_index_create: host allocation failed");
  hipError_t e = hipGetDevice(&ix->device);
  if (e != hipSuccess) {
    delete ix;
    return fail(BM_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  e = hipDeviceGetAttribute(&ix->num_cu, hipDeviceAttributeMultiprocessorCount, ix->device);
  if (e != hipSuccess || ix->num_cu < 1) ix->num_cu = 256;
  KIndex& k = ix->k;
  int rc = BM_OK;
  if (rc == BM_OK) rc = upload_boxes(ix, h, &k.grp);
  if (rc == BM_OK) rc = upload(ix, h.leaf, &k.leaf);
  k.lbox_off = (uint32_t)leaf_boxes_offset(h);
  if (rc == BM_OK) rc = upload(ix, h.ent, &k.ent, kEntPad);
  if (rc == BM_OK) rc = upload(ix, h.slot_mask, reinterpret_cast<const uint64_t**>(&k.slot_mask));
  if (rc == BM_OK) rc = upload(ix, h.parent, &k.parent);
  if (rc != BM_OK) {
    free_index(ix);
    return rc;
  }
  k.n_levels = h.n_levels;
  k.root_child = h.root_child;
  k.root_box = h.root_box;
  k.g0 = h.g0;
  k.leaf_base = h.leaf_base;
  k.n_leaves = h.n_leaves;
  k.presort_chunk = ix->bytes > kPresortBigIndex ? kPresortChunkBigIndex : kPresortChunk;
  k.presort_bin_bits = ix->bytes > kPresortBigIndex ? 6 : 5;
  k.sort_map = SortMap{nullptr, nullptr, make_int2(0, 0), 0, 0};
  if (k.presort_bin_bits == 6) {
    int L = 0, nb = 0;
    std::vector<uint32_t> cell;
    std::vector<int4> sq;
    if (build_sort_map(h, L, nb, cell, sq)) {
      rc = upload(ix, cell, &k.sort_map.cell);
      if (rc == BM_OK) rc = upload(ix, sq, &k.sort_map.sq);
      if (rc != BM_OK) {
        free_index(ix);
        return rc;
      }
      k.sort_map.org = make_int2(h.root_box.x, h.root_box.z);
      k.sort_map.log_side = L;
      k.sort_map.n_bins = nb;
    }
  }
  ix->n_blocks = h.n_leaves;
  ix->n_nodes = (int64_t)h.parent.size();
  ix->n_verts = h.n_verts;
  ix->n_masks = (int64_t)h.slot_mask.size();
  ix->n_ent = (int64_t)h.ent.size();
  *out = ix;
  return BM_OK;
}

// ---- flat file: magic, scalars, then the arrays
constexpr char kMagic[8] = {'B', 'M', 'I', 'D', 'X', '0', '0', '3'};

int write_host(const HostIndex& h, const char* path) {
  FILE* f = fopen(path, "wb");
  if (!f) return fail(BM_EIO, std::string("cannot open ") + path);
  const int32_t sc[12] = {h.n_levels, h.g0, h.leaf_base, h.n_leaves,
                          h.root_child.x, h.root_child.y, h.root_child.z, h.root_child.w,
                          h.root_box.x, h.root_box.y, h.root_box.z, h.root_box.w};
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(sc, sizeof sc, 1, f) == 1 &&
            fwrite(&h.n_verts, sizeof h.n_verts, 1, f) == 1 && write_vec(f, h.grp) && write_vec(f, h.leaf) &&
            write_vec(f, h.ent) && write_vec(f, h.slot_mask) && write_vec(f, h.parent);
  ok = (fclose(f) == 0) && ok;
  return ok ? BM_OK : fail(BM_EIO, std::string("write failed on ") + path);
}

// Structural checks of a loaded index, so that a damaged file cannot send
// the kernels out of bounds.
bool consistent(const HostIndex& h) {
  const int64_t N = (int64_t)h.parent.size(), lb = h.leaf_base, B = h.n_leaves;
  if (h.n_levels < 0 || h.g0 < 0 || lb < 0 || B < 0 || lb + B != N || (int64_t)h.grp.size() != lb ||
      (int64_t)h.leaf.size() != B || h.g0 > N || (h.n_levels == 0 ? h.g0 != B : h.g0 > lb))
    return false;
  const int64_t NE = (int64_t)h.ent.size();
  if (N > kMaxNodes || NE > kMaxEnt || (int64_t)h.slot_mask.size() > kMaxSlotWords) return false;
  auto table_ok = [&](const int4& c) {
    if (c.z < 0) return true;
    const int logS = c.w & 0xff, shx = (c.w >> 8) & 0xff, shy = (c.w >> 16) & 0xff, m = c.y - c.x;
    const int W = (int)((unsigned)c.w >> 24);
    if (logS < 3 || logS > 7 || shx > 31 || shy > 31 || m < 1 || m > kTableMaxChildren || W != (m + 63) / 64)
      return false;
    const int64_t S = 1 << logS;
    if ((int64_t)c.z + 2 * S * W > (int64_t)h.slot_mask.size()) return false;
    for (int64_t t = 0; t < 2 * S; ++t)
      for (int w = 0; w < W; ++w) {
        const int left = m - 64 * w;  // children in word w
        const uint64_t keep = left >= 64 ? ~0ull : ((1ull << left) - 1);
        if (h.slot_mask[c.z + t * W + w] & ~keep) return false;
      }
    return true;
  };
  for (int64_t g = 0; g < lb; ++g) {
    const int4 c = h.grp[g].child;
    if (c.x < 0 || c.x > c.y || c.y > N || c.x <= g || !table_ok(c)) return false;
  }
  if (h.root_child.x != 0 || h.root_child.y != h.g0 || !table_ok(h.root_child)) return false;
  for (int64_t e = 0; e < N; ++e)
    if (h.parent[e] < -1 || h.parent[e] >= e) return false;
  for (int64_t b = 0; b < B; ++b) {
    const LeafRec& r = h.leaf[b];
    const int sh = r.packed & 0xff, logK = (r.packed >> 8) & 0xff;
    if (sh > 31 || logK > 12 || (r.packed & ~(0xffff | kLeafExtOff)) != 0) return false;
    const int64_t K = (int64_t)1 << logK;
    if (r.box.w > r.box.z && (int64_t)r.box.w - r.box.z > (K << sh)) return false;
    if (r.ent < 0 || r.ent > NE) return false;
    std::vector<int64_t> off(K + 1);
    if (r.packed & kLeafExtOff) {
      const int64_t nq = (K + 1 + 3) / 4;
      if (r.ent < nq) return false;
      const uint32_t* o = reinterpret_cast<const uint32_t*>(h.ent.data() + r.ent - nq);
      for (int64_t j = 0; j <= K; ++j) off[j] = o[j];
    } else {
      if (K + 1 > (int64_t)sizeof r.off) return false;
      for (int64_t j = 0; j <= K; ++j) off[j] = r.off[j];
    }
    if (off[0] != 0) return false;
    for (int64_t j = 0; j < K; ++j)
      if (off[j] > off[j + 1] || off[j + 1] - off[j] > kMaxSlabEdges) return false;
    if (r.ent + off[K] > NE) return false;
  }
  return true;
}

}  // namespace

int index_create(const bm_index_desc* d, bm_index** out) {
  if (!out) return fail(BM_EINVAL, "bm_index_create: null output pointer");
  *out = nullptr;
  HostIndex h;
  int rc = build_host(d, h);
  if (rc != BM_OK) return rc;
  return make_device(h, out);
}

void index_destroy(bm_index* ix) { free_index(ix); }

int index_to_host(const bm_index* ix, HostIndex& h) {
  const KIndex& k = ix->k;
  int rc = BM_OK;
  if (rc == BM_OK) rc = download(k.grp, (int64_t)k.leaf_base, h.grp);
  if (rc == BM_OK) rc = download(k.leaf, (int64_t)k.n_leaves, h.leaf);
  if (rc == BM_OK) rc = download(k.ent, ix->n_ent, h.ent);
  if (rc == BM_OK) rc = download(reinterpret_cast<const uint64_t*>(k.slot_mask), ix->n_masks, h.slot_mask);
  if (rc == BM_OK) rc = download(k.parent, ix->n_nodes, h.parent);
  if (rc != BM_OK) return rc;
  h.n_levels = k.n_levels;
  h.g0 = k.g0;
  h.leaf_base = k.leaf_base;
  h.n_leaves = k.n_leaves;
  h.root_child = k.root_child;
  h.root_box = k.root_box;
  h.n_verts = ix->n_verts;
  return BM_OK;
}

int index_save(const bm_index* ix, const char* path) {
  if (!ix || !path) return fail(BM_EINVAL, "bm_index_save: null argument");
  HostIndex h;
  const int rc = index_to_host(ix, h);
  return rc == BM_OK ? write_host(h, path) : rc;
}

int index_build_file(const bm_index_desc* d, const char* path) {
  if (!path) return fail(BM_EINVAL, "bm_index_build_file: null path");
  HostIndex h;
  int rc = build_host(d, h);
  if (rc != BM_OK) return rc;
  return write_host(h, path);
}

int index_load(const char* path, bm_index** out) {
  if (!path || !out) return fail(BM_EINVAL, "bm_index_load: null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(BM_EIO, std::string("bm_index_load: cannot open ") + path);
  HostIndex h;
  char magic[8];
  int32_t sc[12];
  const int64_t lim = (int64_t)1 << 36;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(sc, sizeof sc, 1, f) == 1 &&
            fread(&h.n_verts, sizeof h.n_verts, 1, f) == 1 && read_vec(f, h.grp, INT32_MAX) &&
            read_vec(f, h.leaf, INT32_MAX) && read_vec(f, h.ent, lim) && read_vec(f, h.slot_mask, INT32_MAX) &&
            read_vec(f, h.parent, INT32_MAX);
  fclose(f);
  if (!ok) return fail(BM_EIO, std::string("bm_index_load: malformed file ") + path);
  h.n_levels = sc[0];
  h.g0 = sc[1];
  h.leaf_base = sc[2];
  h.n_leaves = sc[3];
  h.root_child = make_int4(sc[4], sc[5], sc[6], sc[7]);
  h.root_box = make_int4(sc[8], sc[9], sc[10], sc[11]);
  if (!consistent(h)) return fail(BM_EIO, std::string("bm_index_load: inconsistent index in ") + path);
  return make_device(h, out);
}

}  // namespace bm
