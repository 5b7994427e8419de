// Point -> block mapping kernels for gfx950 (wave64).
//
// One kernel does the whole path for a tile of 64 points per wavefront:
//   1. hierarchical box filter (paper Sec. III): the root's slot table gives
//      each point its candidate level-0 groups, whose boxes are tested
//      exactly (table and boxes staged in LDS per workgroup when they are
//      small); the children of every surviving group are then tested the
//      same way. Survivors are compacted with a wavefront ballot + mbcnt
//      prefix count into a per-wave LDS ring of (group, point) items, which
//      is consumed 64 items per round whatever their level, or, for blocks,
//      into a list of (block, point) pairs.
//   2. crossing-number test (paper Sec. III-A) on every surviving
//      (block, point) pair, edge-parallel: each pair's ring is cut into
//      chunks of a few edges, the chunks of all pairs of the tile are dealt
//      across the 64 lanes, and each chunk's crossing parity is folded into
//      its pair with an LDS xor.
//   3. result: for every pair with odd parity, atomic min of the block index
//      into the point's LDS slot; one coalesced store per tile.
// A point whose candidates would overflow a per-wave list (only for heavily
// overlapping input) is finished by a per-lane depth-first walk instead,
// which gives the same exact answer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace bm {
namespace {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;
constexpr int kTile = kWave * kTilePts;  // points per wave tile
static_assert((1 << kSlotBits) == kTile, "slot field");
constexpr int kCap = kTile < 128 ? 256 : 2 * kTile;  // (node, point) items per list per wave
constexpr int kCapChunk = 256;                       // crossing-test chunks per window per wave

// Workgroups per CU the mapping kernels are compiled for (register budget):
// the 4-edge chunk form fits 7 (7 waves per SIMD); wider chunks hold more
// edges in registers.
__host__ __device__ constexpr int map_min_blocks(int chunk_shift) {
  return chunk_shift == 2 ? 7 : chunk_shift == 3 ? 5 : 4;
}

struct WaveLds {
  int2 pts[kTile];
  unsigned best[kTile];
  unsigned par[kWave];     // crossing parity of the pairs of one round
  uint4 pair[kWave];       // per pair of a round: first listed edge, edges, first chunk, point slot
  unsigned item[2][kCap];  // (node << kSlotBits | point slot) lists: the ring of group items and the pairs
                           // (the cover form keeps its pairs in the first)
  unsigned char ovf[kTile];
  unsigned char ch_q[kCapChunk];  // pair (within the round) of each chunk of a window
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Points, permutation entries and results are touched once per pass; they
// are loaded (and the mapping kernels' results stored) non-temporally so that
// they do not push the index's lines out of the caches (mapping kernel 5.60
// -> 5.17 ms, sort passes 1.87 -> 1.68 ms per 100M points). The sort passes'
// stores stay ordinary: their runs are merged in the caches.
__device__ __forceinline__ int2 ld_once(const int2* p) {
  int2 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}
__device__ __forceinline__ int ld_once(const int* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void st_once(int* p, const int v) { __builtin_nontemporal_store(v, p); }

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0ull; }

__device__ __forceinline__ unsigned wave_incl_scan(unsigned v, int lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned t = __shfl_up(v, o);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ bool in_box(const int4& b, int2 p) {
  return b.x <= p.x && p.x < b.y && b.z <= p.y && p.y < b.w;
}

// Crossing of the ray from p towards +x with the edge a -> b.
// Takes part when exactly one end is strictly above p; counts when the edge
// meets the line y = p.y strictly right of p. With the x-range known:
// p.x < min(a.x, b.x) always crosses, p.x >= max(a.x, b.x) never does, and
// in between the sign of the 64-bit cross product
//   c = (a.x - p.x)(b.y - p.y) - (b.x - p.x)(a.y - p.y)
// decides (c > 0 for an upward edge, c < 0 for a downward one). There p lies
// inside the edge's box, so every factor is below 2^31 in magnitude and c
// fits in int64.
__device__ __forceinline__ unsigned crosses(int2 a, int2 b, int2 p) {
  const bool a_up = a.y > p.y, b_up = b.y > p.y;
  const int xlo = min(a.x, b.x), xhi = max(a.x, b.x);
  unsigned r = (a_up != b_up) & (p.x < xlo);
  const bool amb = (a_up != b_up) & (p.x >= xlo) & (p.x < xhi);
  if (amb) {
    const long long c = (long long)(a.x - p.x) * (long long)(b.y - p.y) -
                        (long long)(b.x - p.x) * (long long)(a.y - p.y);
    r = b_up ? (c > 0) : (c < 0);
  }
  return r;
}

__device__ __forceinline__ int4 node_box(const KIndex& ix, int e) {
  return e >= ix.leaf_base ? ix.leaf[e - ix.leaf_base].box : ix.grp[e].box;
}

// Setup of one (leaf, point) pair, p inside the leaf's box: the class of p's
// cell in the leaf's cell map (kCellOut, kCellIn or kCellTest), the leaf's
// block index, and for kCellTest the slab holding p.y as a range
// [first, first + len) of `ent` (len = 0 otherwise). The record's box and
// header are read first; the cell word and the slab offsets, which depend on
// them, come from the same 128-byte line.
__device__ __forceinline__ unsigned pair_setup(const KIndex& ix, const int leaf, const int2 p, unsigned& first,
                                               unsigned& len, unsigned& bid) {
  const LeafRec* r = ix.leaf + leaf;  // 128-byte records: leaf << 7 needs more than 32 bits above 2^25 leaves
  const int4 bx = r->box;
  const int4 meta = *reinterpret_cast<const int4*>(&r->ent);  // ent (2 words, below 2^31), leaf_id, packed
  const unsigned ent = (unsigned)meta.x;
  bid = (unsigned)meta.z;
  const int packed = meta.w;
  const int sh = packed & 0xff, logK = (packed >> 8) & 0xff;
  const unsigned dy = (unsigned)p.y - (unsigned)bx.z;
  const unsigned col = ((unsigned)p.x - (unsigned)bx.x) >> cell_shift((unsigned)(bx.y - bx.x));
  const unsigned row = dy >> cell_shift((unsigned)(bx.w - bx.z));
  const unsigned cls = (r->cell[row] >> (2u * col)) & 3u;
  const unsigned b = dy >> sh;
  unsigned o0, o1;
  if (packed & kLeafExtOff) {
    const unsigned nq = ((1u << logK) + 1u + 3u) >> 2;
    const unsigned* o = reinterpret_cast<const unsigned*>(ix.ent + (ent - nq));
    o0 = o[b];
    o1 = o[b + 1];
  } else {
    o0 = r->off[b];
    o1 = r->off[b + 1];
  }
  first = ent + o0;
  len = cls >= kCellTest ? o1 - o0 : 0u;
  return cls;
}

// Crossing parity of a point against one leaf (point inside the leaf box).
__device__ unsigned leaf_parity(const KIndex& ix, int leaf, int2 p) {
  unsigned first, len, bid;
  const unsigned cls = pair_setup(ix, leaf, p, first, len, bid);
  unsigned acc = cls == kCellIn ? 1u : 0u;
  for (unsigned j = 0; j < len; ++j) {
    const int4 e = ix.ent[first + j];
    acc ^= crosses(make_int2(e.x, e.y), make_int2(e.z, e.w), p);
  }
  return acc;
}

// Depth-first walk of the whole hierarchy for one point: used only for points
// whose candidate lists overflowed. Stackless: a node's parent link gives the
// way back up.
__device__ unsigned walk_point(const KIndex& ix, int2 p) {
  unsigned best = 0xFFFFFFFFu;
  int e = 0, end = ix.g0, par = -1;
  for (;;) {
    if (e >= end) {
      if (par < 0) break;
      e = par + 1;
      par = ix.parent[par];
      end = par < 0 ? ix.g0 : ix.grp[par].child.y;
      continue;
    }
    if (in_box(node_box(ix, e), p)) {
      if (e >= ix.leaf_base) {
        const int leaf = e - ix.leaf_base;
        if (leaf_parity(ix, leaf, p)) best = min(best, (unsigned)ix.leaf[leaf].leaf_id);
        ++e;
      } else {
        const int4 c = ix.grp[e].child;
        par = e;
        e = c.x;
        end = c.y;
      }
    } else {
      ++e;
    }
  }
  return best;
}

// Append item (node, point slot) to list `dst` (wave-uniform count `cnt`) for
// every lane where `pred` holds; all 64 lanes must be active. Items that do
// not fit mark their point for the depth-first fallback.
__device__ __forceinline__ void emit(WaveLds& S, int dst, bool pred, unsigned node, int plane,
                                     unsigned& cnt) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const unsigned k = (unsigned)__popcll(m);
  const unsigned slot = cnt + lanes_below(m);
  const unsigned it = (node << kSlotBits) | (unsigned)plane;
  if (cnt + k <= (unsigned)kCap) {  // wave-uniform: every new item fits
    if (pred) S.item[dst][slot] = it;
  } else if (pred) {
    if (slot < (unsigned)kCap)
      S.item[dst][slot] = it;
    else
      S.ovf[plane] = 1;
  }
  cnt += k;
}

// The plain path keeps the (group, point) items of all levels in one ring,
// S.item[0] (kCap entries), consumed 64 per round in FIFO order whatever
// their level, so the rounds run full; (leaf, point) pairs go to S.item[1].
// emit_ring appends to the ring at `tail`; slots [tail, lim) are free. Items
// that do not fit mark their point for the depth-first fallback.
__device__ __forceinline__ void emit_ring(WaveLds& S, bool pred, unsigned node, int plane, unsigned& tail,
                                          const unsigned lim) {
  const unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  const unsigned k = (unsigned)__popcll(m);
  const unsigned slot = tail + lanes_below(m);
  const unsigned it = (node << kSlotBits) | (unsigned)plane;
  if (tail + k <= lim) {  // wave-uniform: every new item fits
    if (pred) S.item[0][slot & (kCap - 1)] = it;
  } else if (pred) {
    if (slot < lim)
      S.item[0][slot & (kCap - 1)] = it;
    else
      S.ovf[plane] = 1;
  }
  tail = min(tail + k, lim);
}

// Two candidates per lane in one append (to the ring, or to list `dst` for
// emit2): all lanes' first items, then their second items. The order of a
// list does not change any result.
__device__ __forceinline__ void emit2_ring(WaveLds& S, const bool p1, const unsigned n1, const bool p2,
                                           const unsigned n2, const int plane, unsigned& tail, const unsigned lim) {
  const unsigned long long m1 = __ballot(p1), m2 = __ballot(p2);
  if ((m1 | m2) == 0ull) return;
  const unsigned k1 = (unsigned)__popcll(m1), k = k1 + (unsigned)__popcll(m2);
  const unsigned s1 = tail + lanes_below(m1), s2 = tail + k1 + lanes_below(m2);
  const unsigned i1 = (n1 << kSlotBits) | (unsigned)plane, i2 = (n2 << kSlotBits) | (unsigned)plane;
  if (tail + k <= lim) {  // wave-uniform: every new item fits
    if (p1) S.item[0][s1 & (kCap - 1)] = i1;
    if (p2) S.item[0][s2 & (kCap - 1)] = i2;
  } else {
    if (p1) {
      if (s1 < lim) S.item[0][s1 & (kCap - 1)] = i1; else S.ovf[plane] = 1;
    }
    if (p2) {
      if (s2 < lim) S.item[0][s2 & (kCap - 1)] = i2; else S.ovf[plane] = 1;
    }
  }
  tail = min(tail + k, lim);
}

__device__ __forceinline__ void emit2(WaveLds& S, const int dst, const bool p1, const unsigned n1, const bool p2,
                                      const unsigned n2, const int plane, unsigned& cnt) {
  const unsigned long long m1 = __ballot(p1), m2 = __ballot(p2);
  if ((m1 | m2) == 0ull) return;
  const unsigned k1 = (unsigned)__popcll(m1), k = k1 + (unsigned)__popcll(m2);
  const unsigned s1 = cnt + lanes_below(m1), s2 = cnt + k1 + lanes_below(m2);
  const unsigned i1 = (n1 << kSlotBits) | (unsigned)plane, i2 = (n2 << kSlotBits) | (unsigned)plane;
  if (cnt + k <= (unsigned)kCap) {  // wave-uniform: every new item fits
    if (p1) S.item[dst][s1] = i1;
    if (p2) S.item[dst][s2] = i2;
  } else {
    if (p1) {
      if (s1 < (unsigned)kCap) S.item[dst][s1] = i1; else S.ovf[plane] = 1;
    }
    if (p2) {
      if (s2 < (unsigned)kCap) S.item[dst][s2] = i2; else S.ovf[plane] = 1;
    }
  }
  cnt += k;
}

// Children of one group per lane (ci = child record, gb = group box, pp =
// the lane's point), in a round whose lanes may hold groups of different
// levels: every child whose half-open box holds pp is emitted; children that
// are leaves (the group's first child id is at least leaf_base) become pairs,
// other children items of the ring. With a slot table only the children
// flagged in both the x-slot and the y-slot of pp are tested (a table row
// holds one 64-bit word per 64 children); otherwise all of them, 64 at a
// time. Called with all 64 lanes active; `has` masks lanes without an item.
__device__ __forceinline__ void expand_mixed(const KIndex& ix, WaveLds& S, bool has, const int4 ci,
                                             const int4 gb, const int2 pp, int pl, unsigned& tail,
                                             const unsigned lim, unsigned& pcnt) {
  // The boxes a step tests start at byte ((n - sub) << shift) + adj from
  // ix.grp, a 32-bit offset: group n's record (32 bytes), or the copy of
  // leaf n's box (16 bytes) in the array that follows the group records.
  const bool leaves = ci.x >= ix.leaf_base;
  const char* recs = reinterpret_cast<const char*>(ix.grp);
  const unsigned sub = leaves ? (unsigned)ix.leaf_base : 0u;
  const unsigned shift = leaves ? 4u : 5u;
  const unsigned adj = leaves ? ix.lbox_off : 0u;
  const char* masks = reinterpret_cast<const char*>(ix.slot_mask);  // below 2^29 words
  const int m = has ? ci.y - ci.x : 0;
  // children in windows of 128 (two 64-bit candidate words, lo then hi), so
  // that a lane's candidates of both words are taken in one loop
  for (int base = 0; wave_any(base < m); base += 128) {
    unsigned long long lo = 0ull, hi = 0ull;
    if (base < m) {
      const int mm = min(128, m - base);
      lo = mm >= 64 ? ~0ull : ((1ull << mm) - 1ull);
      hi = mm <= 64 ? 0ull : mm == 128 ? ~0ull : ((1ull << (mm - 64)) - 1ull);
      if (ci.z >= 0) {  // slot table: S x-rows then S y-rows of W words
        const int logS = ci.w & 0xff, shx = (ci.w >> 8) & 0xff, shy = (ci.w >> 16) & 0xff;
        const unsigned W = (unsigned)ci.w >> 24;
        const unsigned S_ = 1u << logS;
        const unsigned sx = ((unsigned)pp.x - (unsigned)gb.x) >> shx;
        const unsigned sy = ((unsigned)pp.y - (unsigned)gb.z) >> shy;
        if (pp.x < gb.x || pp.y < gb.z || sx >= S_ || sy >= S_) {
          lo = hi = 0ull;
        } else {
          const unsigned w = (unsigned)base >> 6;
          const unsigned ox = ((unsigned)ci.z + sx * W + w) << 3, oy = ((unsigned)ci.z + (S_ + sy) * W + w) << 3;
          lo &= *reinterpret_cast<const unsigned long long*>(masks + ox) &
                *reinterpret_cast<const unsigned long long*>(masks + oy);
          if (mm > 64)
            hi &= *reinterpret_cast<const unsigned long long*>(masks + ox + 8) &
                  *reinterpret_cast<const unsigned long long*>(masks + oy + 8);
        }
      }
    }
    const unsigned c0 = (unsigned)(ci.x + base);
    // two candidates per lane and step: box tests, then the appends
    auto step = [&](const bool h1, const unsigned n1, const bool h2, const unsigned n2) {
      const int4 bx1 = *reinterpret_cast<const int4*>(recs + (((n1 - sub) << shift) + adj));
      const int4 bx2 = *reinterpret_cast<const int4*>(recs + (((n2 - sub) << shift) + adj));
      const bool in1 = h1 && in_box(bx1, pp), in2 = h2 && in_box(bx2, pp);
      emit2_ring(S, in1 && !leaves, n1, in2 && !leaves, n2, pl, tail, lim);
      emit2(S, 1, in1 && leaves, n1, in2 && leaves, n2, pl, pcnt);
    };
    if (!wave_any(hi != 0ull)) {  // every lane's candidates in the first word
      while (wave_any(lo != 0ull)) {
        const bool h1 = lo != 0ull;
        const unsigned n1 = h1 ? c0 + (unsigned)__builtin_ctzll(lo) : sub;
        lo &= lo - 1ull;
        const bool h2 = lo != 0ull;
        const unsigned n2 = h2 ? c0 + (unsigned)__builtin_ctzll(lo) : sub;
        lo &= lo - 1ull;
        step(h1, n1, h2, n2);
      }
    } else {
      while (wave_any((lo | hi) != 0ull)) {
        bool a = lo != 0ull;
        unsigned long long v = a ? lo : hi;
        const bool h1 = v != 0ull;
        const unsigned n1 = h1 ? c0 + (a ? 0u : 64u) + (unsigned)__builtin_ctzll(v) : sub;
        v &= v - 1ull;
        lo = a ? v : lo;
        hi = a ? hi : v;
        a = lo != 0ull;
        v = a ? lo : hi;
        const bool h2 = v != 0ull;
        const unsigned n2 = h2 ? c0 + (a ? 0u : 64u) + (unsigned)__builtin_ctzll(v) : sub;
        v &= v - 1ull;
        lo = a ? v : lo;
        hi = a ? hi : v;
        step(h1, n1, h2, n2);
      }
    }
  }
}

// The root's level-0 boxes and slot table, staged in LDS once per workgroup
// when they are small (at most 64 level-0 entries and a one-word table: 3 KB,
// which leaves room for the 7 workgroups per CU the registers allow).
// Every point of every tile starts at the root, so its table rows and boxes
// then come from LDS rather than from the caches (mapping kernel 3.42 ->
// 3.24 ms per 100M points on the 220,900-block grid, 4.30 -> 4.19 ms per
// 2^26 points on the 8M-block quadtree).
struct RootLds {
  int4 box[64];
  unsigned long long row[256];  // S x-rows, then S y-rows (S <= 128)
  int ok;
};

__device__ __forceinline__ void stage_root(const KIndex& ix, RootLds& R) {
  const int4 rc = ix.root_child;
  const int m = rc.y - rc.x;
  const int logS = rc.w & 0xff;
  const bool ok = rc.z >= 0 && m >= 1 && m <= 64 && ((unsigned)rc.w >> 24) == 1u && logS <= 7;
  if (ok) {
    const bool leaves = rc.x >= ix.leaf_base;
    const char* recs = reinterpret_cast<const char*>(ix.grp);
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      const unsigned n = (unsigned)(rc.x + i);
      R.box[i] = leaves ? *reinterpret_cast<const int4*>(recs + (((n - (unsigned)ix.leaf_base) << 4) + ix.lbox_off))
                        : ix.grp[n].box;
    }
    for (int i = threadIdx.x; i < (2 << logS); i += blockDim.x) R.row[i] = ix.slot_mask[rc.z + i];
  }
  if (threadIdx.x == 0) R.ok = ok ? 1 : 0;
  __syncthreads();
}

// The root's children for the lane's point, from LDS (see expand_mixed).
__device__ __forceinline__ void expand_root(const KIndex& ix, WaveLds& S, const RootLds& R, const bool has,
                                            const int2 pp, const int pl, unsigned& tail, const unsigned lim,
                                            unsigned& pcnt) {
  if (!R.ok) {
    expand_mixed(ix, S, has, ix.root_child, ix.root_box, pp, pl, tail, lim, pcnt);
    return;
  }
  const int4 ci = ix.root_child, gb = ix.root_box;
  const bool leaves = ci.x >= ix.leaf_base;
  const int m = ci.y - ci.x;
  const int logS = ci.w & 0xff, shx = (ci.w >> 8) & 0xff, shy = (ci.w >> 16) & 0xff;
  const unsigned S_ = 1u << logS;
  const unsigned sx = ((unsigned)pp.x - (unsigned)gb.x) >> shx, sy = ((unsigned)pp.y - (unsigned)gb.z) >> shy;
  unsigned long long lo = 0ull;
  if (has && !(pp.x < gb.x || pp.y < gb.z || sx >= S_ || sy >= S_))
    lo = (m >= 64 ? ~0ull : ((1ull << m) - 1ull)) & R.row[sx] & R.row[S_ + sy];
  const unsigned c0 = (unsigned)ci.x;
  while (wave_any(lo != 0ull)) {
    const bool h1 = lo != 0ull;
    const unsigned k1 = h1 ? (unsigned)__builtin_ctzll(lo) : 0u;
    lo &= lo - 1ull;
    const bool h2 = lo != 0ull;
    const unsigned k2 = h2 ? (unsigned)__builtin_ctzll(lo) : 0u;
    lo &= lo - 1ull;
    const bool in1 = h1 && in_box(R.box[k1], pp), in2 = h2 && in_box(R.box[k2], pp);
    emit2_ring(S, in1 && !leaves, c0 + k1, in2 && !leaves, c0 + k2, pl, tail, lim);
    emit2(S, 1, in1 && leaves, c0 + k1, in2 && leaves, c0 + k2, pl, pcnt);
  }
}

// Crossing-number test on the cnt (leaf, point) pairs of list `cur`, 64 pairs
// per round; odd pairs atomic-min their block index into the point's slot of
// S.best. A pair whose point lies in an In or Out cell of the leaf's cell map
// is decided by the map (parity 1 or 0) and needs no edges. Any other pair
// only needs the ring edges listed for the y-slab holding its point (every
// pair passed the leaf's box test, so the point lies in the ring's
// y-extent); that list is cut into chunks of kChunk edges and all chunks of
// the round are dealt across the lanes. The edge list is padded at its end,
// so a chunk's loads never leave it. All 64 lanes take part.
template <int kChunkShift>
__device__ __forceinline__ void pip_rounds(const KIndex& ix, WaveLds& S, const int lane, const int cur,
                                           const unsigned cnt) {
  constexpr int kChunk = 1 << kChunkShift;
  for (unsigned r = 0; r < cnt; r += kWave) {
    const unsigned q = r + lane;
    const bool has = q < cnt;
    unsigned first = 0, len = 0, bid = 0, cls = kCellOut;
    const unsigned it = has ? S.item[cur][q] : 0u;
    const int pl = (int)(it & (kTile - 1));
    if (has) cls = pair_setup(ix, (int)(it >> kSlotBits) - ix.leaf_base, S.pts[pl], first, len, bid);
    const unsigned nch = (len + kChunk - 1) >> kChunkShift;
    const unsigned incl = wave_incl_scan(nch, lane);
    const unsigned start = incl - nch;
    const unsigned total = __shfl(incl, kWave - 1);
    S.pair[lane] = make_uint4(first, len, start, (unsigned)pl);
    S.par[lane] = cls == kCellIn ? 1u : 0u;
    for (unsigned w = 0; w < total; w += kCapChunk) {
      const unsigned a = max(start, w), b = min(start + nch, w + (unsigned)kCapChunk);
      for (unsigned c = a; c < b; ++c) S.ch_q[c - w] = (unsigned char)lane;
      wave_sync();
      const unsigned nw = min((unsigned)kCapChunk, total - w);
      for (unsigned c = lane; c < nw; c += kWave) {
        const unsigned pq = S.ch_q[c];
        const uint4 pr = S.pair[pq];
        const unsigned k0 = (w + c - pr.z) << kChunkShift;
        const unsigned ne = min((unsigned)kChunk, pr.y - k0);
        const int4* e = ix.ent + (pr.x + k0);
        int4 ev[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) ev[u] = e[u];
        const int2 pp = S.pts[pr.w];
        unsigned acc = 0;
#pragma unroll
        for (int u = 0; u < kChunk; ++u)
          acc ^= ((unsigned)u < ne) ? crosses(make_int2(ev[u].x, ev[u].y), make_int2(ev[u].z, ev[u].w), pp) : 0u;
        if (acc) atomicXor(&S.par[pq], 1u);
      }
      wave_sync();
    }
    if (has && (S.par[lane] & 1u)) atomicMin(&S.best[pl], bid);
    wave_sync();
  }
}

// The whole path for one tile of up to kTile points (point j * 64 + lane on
// lane `lane`, given in registers as pt[j]); all 64 lanes of the wave take
// part. Writes the result of point i < nvalid to out[i], one coalesced store
// per tile. With several points per lane the candidate lists of a level hold
// the items of all of them, so its rounds of 64 items run nearly full.
template <int kChunkShift>
__device__ __forceinline__ void map_tile_pts(const KIndex& ix, WaveLds& S, const RootLds& R, const int lane,
                                             const int2 (&pt)[kTilePts], const int nvalid,
                                             int* __restrict__ out);

template <int kChunkShift>
__device__ __forceinline__ void map_tile(const KIndex& ix, WaveLds& S, const RootLds& R, const int lane,
                                         const int2* __restrict__ xy, const int nvalid, int* __restrict__ out) {
  int2 pt[kTilePts];
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    pt[j] = i < nvalid ? ld_once(xy + i) : make_int2(0, 0);
  }
  map_tile_pts<kChunkShift>(ix, S, R, lane, pt, nvalid, out);
}

template <int kChunkShift>
__device__ __forceinline__ void map_tile_pts(const KIndex& ix, WaveLds& S, const RootLds& R, const int lane,
                                             const int2 (&pt)[kTilePts], const int nvalid,
                                             int* __restrict__ out) {
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    S.pts[i] = pt[j];
    S.best[i] = 0xFFFFFFFFu;
    S.ovf[i] = 0;
  }
  wave_sync();

  // ---- the root's children (level 0), one item per point
  static_assert((kCap & (kCap - 1)) == 0 && kCap >= 2 * kWave, "ring of a power-of-two size");
  unsigned head = 0, tail = 0, pcnt = 0;
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    expand_root(ix, S, R, i < nvalid, S.pts[i], i, tail, head + kCap, pcnt);
  }
  wave_sync();

  // ---- groups of every level, 64 items per round in FIFO order
  while (head < tail) {
    const unsigned q = head + lane;
    const bool has = q < tail;
    const unsigned it = has ? S.item[0][q & (kCap - 1)] : 0u;  // lanes without an item read group 0
    head += min((unsigned)kWave, tail - head);
    wave_sync();  // this round's slots are free from here on
    const GroupRec* g =
        reinterpret_cast<const GroupRec*>(reinterpret_cast<const char*>(ix.grp) + ((it >> kSlotBits) << 5));
    const int pl = (int)(it & (kTile - 1));
    expand_mixed(ix, S, has, g->child, g->box, S.pts[pl], pl, tail, head + kCap, pcnt);
    wave_sync();
  }
  const int cur = 1;
  const unsigned cnt = min(pcnt, (unsigned)kCap);

  pip_rounds<kChunkShift>(ix, S, lane, cur, cnt);

#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    if (i < nvalid) {
      unsigned best = S.best[i];
      if (S.ovf[i]) best = min(best, walk_point(ix, S.pts[i]));
      st_once(out + i, (int)best);
    }
  }
  wave_sync();
}

// ---- cell cover (the fast approach) -------------------------------------
// The trie entry of the cell holding p: interior (block index), boundary
// (cell number) or kCoverEmpty (also for points off the covered square).
__device__ __forceinline__ uint32_t cover_lookup(const KCover& cv, const int2 p) {
  if (p.x < cv.ox || p.y < cv.oy) return kCoverEmpty;
  const unsigned dx = (unsigned)p.x - (unsigned)cv.ox, dy = (unsigned)p.y - (unsigned)cv.oy;
  if (((dx | dy) >> cv.log_side) != 0u) return kCoverEmpty;
  int shift = cv.log_side;
  unsigned node = 0;
  for (int t = 0; t < cv.n_levels; ++t) {
    const int bits = t == cv.n_levels - 1 ? cv.last_bits : 4;
    shift -= bits;
    const unsigned m = (1u << bits) - 1u;
    const uint32_t v = cv.ent[node + (((dx >> shift) & m) | (((dy >> shift) & m) << bits))];
    if ((v >> 30) != 1u) return v;
    node = v & kCoverPayload;
  }
  return kCoverEmpty;  // the last trie level holds no node entries
}

// One tile through the cover: a point in an interior or empty cell takes the
// trie's answer; a point in a boundary cell takes the cell's centre answer
// (approx) or becomes a (leaf, point) pair for every listed block whose box
// holds it, resolved by the same crossing-test rounds as the plain path.
template <int kChunkShift>
__device__ __forceinline__ void cover_tile(const KIndex& ix, const KCover& cv, WaveLds& S, const int lane,
                                           const int2* __restrict__ xy, const int nvalid, int* __restrict__ out,
                                           const bool approx) {
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    S.pts[i] = i < nvalid ? ld_once(xy + i) : make_int2(0, 0);
    S.best[i] = 0xFFFFFFFFu;
    S.ovf[i] = 0;
  }
  wave_sync();
  unsigned cnt = 0;
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    const int2 p = S.pts[i];
    const uint32_t v = i < nvalid ? cover_lookup(cv, p) : kCoverEmpty;
    const uint32_t tag = v >> 30, pay = v & kCoverPayload;
    if (tag == 0u) S.best[i] = pay;
    if (tag == 2u && approx) S.best[i] = (unsigned)cv.cell_rep[pay];
    unsigned k = 0, k1 = 0;
    if (tag == 2u && !approx) {
      k = cv.cell_off[pay];
      k1 = cv.cell_off[pay + 1];
    }
    for (; wave_any(k < k1); ++k) {
      const bool h = k < k1;
      const unsigned leaf = h ? cv.cell_leaf[k] : 0u;  // lanes without one read leaf 0
      const int4 bx = ix.leaf[leaf].box;
      emit(S, 0, h && in_box(bx, p), (unsigned)ix.leaf_base + leaf, i, cnt);
    }
  }
  cnt = min(cnt, (unsigned)kCap);
  wave_sync();
  pip_rounds<kChunkShift>(ix, S, lane, 0, cnt);
#pragma unroll
  for (int j = 0; j < kTilePts; ++j) {
    const int i = j * kWave + lane;
    if (i < nvalid) {
      unsigned best = S.best[i];
      if (S.ovf[i]) best = min(best, walk_point(ix, S.pts[i]));
      st_once(out + i, (int)best);
    }
  }
  wave_sync();
}

template <int kChunkShift>
__global__ __launch_bounds__(kBlock, map_min_blocks(kChunkShift)) void cover_map_kernel(
    const KIndex ix, const KCover cv, const int2* __restrict__ xy, const long long n, int* __restrict__ out,
    const int approx) {
  __shared__ WaveLds wl[kWavesPerBlock];
  const int lane = threadIdx.x & (kWave - 1);
  WaveLds& S = wl[threadIdx.x / kWave];
  const long long ntiles = (n + kTile - 1) / kTile;
  const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
  for (long long t = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < ntiles;
       t += nwaves) {
    const long long i0 = t * kTile;
    cover_tile<kChunkShift>(ix, cv, S, lane, xy + i0, (int)min((long long)kTile, n - i0), out + i0, approx != 0);
  }
}

// Plain form: the waves of the grid stride over the tiles.
template <int kChunkShift>
__global__ __launch_bounds__(kBlock, map_min_blocks(kChunkShift)) void map_kernel(const KIndex ix, const int2* __restrict__ xy,
                                                     const long long n, int* __restrict__ out) {
  __shared__ WaveLds wl[kWavesPerBlock];
  __shared__ RootLds R;
  stage_root(ix, R);
  const int lane = threadIdx.x & (kWave - 1);
  WaveLds& S = wl[threadIdx.x / kWave];
  const long long ntiles = (n + kTile - 1) / kTile;
  const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
  for (long long t = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < ntiles;
       t += nwaves) {
    const long long i0 = t * kTile;
    map_tile<kChunkShift>(ix, S, R, lane, xy + i0, (int)min((long long)kTile, n - i0), out + i0);
  }
}

// Batched form. The batch table holds `nb` (xy, out, n) entries in device
// memory. batch_prefix_kernel writes meta[0] = nb, clears the work counter
// meta[1] and writes meta[2 + b] = number of work units (`unit` points each,
// a multiple of 64) before batch b. nb comes from hdr[0] when hdr is given
// (the graph form stages it with the table), else from nb_arg. Persistent
// waves of batch_map_kernel then take units from the counter until none is
// left, so batches of very uneven size balance across the machine.
__global__ __launch_bounds__(1024) void batch_prefix_kernel(const long long* __restrict__ hdr,
                                                            const long long nb_arg,
                                                            const BatchEntry* __restrict__ tab,
                                                            long long* __restrict__ meta,
                                                            const int unit) {
  __shared__ long long part[1024];
  const long long nb = hdr ? hdr[0] : nb_arg;
  long long* prefix = meta + 2;
  long long carry = 0;
  if (threadIdx.x == 0) {
    meta[0] = nb;
    meta[1] = 0;
    prefix[0] = 0;
  }
  for (long long base = 0; base < nb; base += 1024) {
    const long long b = base + threadIdx.x;
    const long long n = b < nb ? (long long)tab[b].n : 0;
    part[threadIdx.x] = n > 0 ? (n + unit - 1) / unit : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan
      const long long t = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (b < nb) prefix[b + 1] = carry + part[threadIdx.x];
    carry += part[1023];
    __syncthreads();
  }
}

// Offset form of the batched call: batch b is points [off[b], off[b+1]) of
// one concatenated xy array, its results the same range of out. The
// descriptor table is written here, on the device: from the arguments, or,
// when hdr is given, from the header the graph form stages (nb, xy, out, off).
// A batch whose offsets decrease, start below 0 or end beyond max_points
// (max_points < 0: no bound) gets n = 0 and is skipped.
__global__ __launch_bounds__(256) void batch_offsets_kernel(const OffsetHeader* __restrict__ hdr,
                                                            const long long nb_arg, const int32_t* xy_arg,
                                                            int32_t* out_arg, const long long* off_arg,
                                                            const long long max_points,
                                                            BatchEntry* __restrict__ tab) {
  const long long nb = hdr ? hdr->nb : nb_arg;
  const int32_t* xy = hdr ? hdr->xy : xy_arg;
  int32_t* out = hdr ? hdr->out : out_arg;
  const long long* off = hdr ? hdr->off : off_arg;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += stride) {
    const long long o0 = off[b], o1 = off[b + 1];
    const bool ok = o0 >= 0 && o1 >= o0 && (max_points < 0 || o1 <= max_points);
    tab[b] = BatchEntry{xy + 2 * (ok ? o0 : 0), out + (ok ? o0 : 0), ok ? o1 - o0 : 0};
  }
}

template <int kChunkShift>
__global__ __launch_bounds__(kBlock, map_min_blocks(kChunkShift)) void batch_map_kernel(const KIndex ix, const BatchEntry* __restrict__ tab,
                                                           long long* __restrict__ meta, const int unit) {
  __shared__ WaveLds wl[kWavesPerBlock];
  __shared__ RootLds R;
  stage_root(ix, R);
  const int lane = threadIdx.x & (kWave - 1);
  WaveLds& S = wl[threadIdx.x / kWave];
  const long long nb = meta[0];
  const long long* prefix = meta + 2;
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(meta + 1);
  const long long total = prefix[nb];
  for (;;) {
    unsigned long long u = 0;
    if (lane == 0) u = atomicAdd(counter, 1ull);
    u = __shfl(u, 0);
    if ((long long)u >= total) break;
    // batch holding unit u: the last b with prefix[b] <= u
    long long lo = 0, hi = nb - 1;
    while (lo < hi) {
      const long long mid = (lo + hi + 1) >> 1;
      if (prefix[mid] <= (long long)u) lo = mid; else hi = mid - 1;
    }
    const BatchEntry d = tab[lo];
    const int2* bxy = reinterpret_cast<const int2*>(d.xy);
    const long long p0 = ((long long)u - prefix[lo]) * unit;
    const long long p1 = min(p0 + unit, (long long)d.n);
    for (long long i0 = p0; i0 < p1; i0 += kTile)
      map_tile<kChunkShift>(ix, S, R, lane, bxy + i0, (int)min((long long)kTile, p1 - i0), d.out + i0);
  }
}

// ---- spatial binning ------------------------------------------------------
// Points arrive in any order; a wave maps 64 of them together, and its tree
// nodes, slab lists and cache lines are shared only when those points are
// close. Before mapping, each chunk of points is therefore counting-sorted by
// the Morton index of its cell in a 2^kBB x 2^kBB grid of bins over the root
// box (points outside fall in the nearest border cell), and each bin is then
// re-sorted, in pieces, by the Morton index of its sub-cell: together a
// Z-order on a 1024 x 1024 grid (kBB = 5, 32 x 32 sub-cells per bin) or a
// 4096 x 4096 grid (kBB = 6, 64 x 64). The mapping kernel then maps the
// sorted copy and stores its results in sorted order, coalesced; two passes
// bring them back to the points' original positions: the first undoes the
// re-sort of each piece through LDS, the second gathers every original
// position's result from the runs its scatter block wrote. (Storing each result
// through the permutation from the mapping kernel instead costs a partial
// cache line per 4-byte result: mapping kernel 4.61 -> 3.79 ms per 100M
// points on the 220,900-block grid, 6.11 -> 4.53 ms per 2^26 points on the
// 8M-block quadtree without those stores.) Each point's result depends on
// that point alone, so the order does not change any output. kBB is 5 for an
// index that fits the last-level cache (shorter sort passes) and 6 for a
// larger one (finer order, so that the points of one block share a tile and
// its lines are read from HBM fewer times: 8M-block quadtree 8.19 -> 7.58 ms
// per 2^26 points with 64 x 64 sub-cells in 8,192-point pieces, against 16 x
// 16 in 2,048). A large index's 4,096 bins are adaptive (SortMap: a 32 x 32
// grid of coarse cells, each cut into 4^d bins where its blocks are dense),
// and a bin's sub-cells are those of its own square: where blocks are small
// and points crowd, a uniform bin holds up to millions of a chunk's points,
// cut into hundreds of pieces that each hold a few points of every block, so
// a tile touched a block per point (quadtree mapping kernel 4.19 -> 3.68 ms
// per 2^26-point chunk; the coarse-cell table is read from LDS, so finding the
// bin costs the sort passes almost nothing). With 64 x 64 sub-cells a piece
// holds 6,144 points, so that a refine block's LDS (76 KB) lets two run on a
// CU (8,192-point pieces: sort passes 0.96 -> 1.08 ms, mapping 3.74 -> 3.68
// ms per quadtree chunk).
template <int kBB>
struct Bins {
  static constexpr int kN = 1 << (2 * kBB);          // bins
  static constexpr int kSubBits = kBB == 5 ? 5 : 6;  // per axis
  static constexpr int kSubs = 1 << (2 * kSubBits);  // sub-cells per bin
  static constexpr int kRefThreads = kBB == 5 ? 256 : 512;  // refinement: threads per piece
  static constexpr int kRefPer = kBB == 5 ? 16 : 12;        // refinement: points per thread
};
constexpr int kBins = 1 << 12;  // the most bins of any grid: per-chunk stride of the bin arrays
constexpr int kBinThreads = 1024;  // threads per block of the count and scatter passes
constexpr int kBinPer = 16;        // points per thread: all loaded before any LDS atomic
constexpr long long kBinBlockPts = (long long)kBinThreads * kBinPer;

__device__ __forceinline__ unsigned spread6(unsigned v) {
  v &= 63u;
  v = (v | (v << 4)) & 0x0F0Fu;
  v = (v | (v << 2)) & 0x3333u;
  v = (v | (v << 1)) & 0x5555u;
  return v;
}

template <int kBB>
__device__ __forceinline__ unsigned bin_of(const int2 p, const int4 rb, const int shx, const int shy) {
  const long long dx = (long long)p.x - rb.x, dy = (long long)p.y - rb.z;
  const long long top = (1 << kBB) - 1;
  const unsigned cx = (unsigned)min(top, max(0ll, dx >> shx));
  const unsigned cy = (unsigned)min(top, max(0ll, dy >> shy));
  return spread6(cx) | (spread6(cy) << 1);
}

// The adaptive bins (SortMap) of a large index. cell_bin: the bin of p, from
// the coarse-cell table C (staged in LDS); points outside the square are
// clamped onto it, as bin_of clamps onto the grid. map_sub_of: p's sub-cell
// (64 x 64, Morton) of its bin's square sq.
__device__ __forceinline__ unsigned cell_bin(const int2 p, const uint32_t* __restrict__ C, const SortMap& sm) {
  const long long top = (1ll << sm.log_side) - 1;
  const unsigned ox = (unsigned)min(top, max(0ll, (long long)p.x - sm.org.x));
  const unsigned oy = (unsigned)min(top, max(0ll, (long long)p.y - sm.org.y));
  const int cs = sm.log_side - kSortCoarseBits;
  const unsigned e = C[((oy >> cs) << kSortCoarseBits) | (ox >> cs)];
  const int fs = cs - (int)(e >> 16);
  const unsigned m = (1u << (e >> 16)) - 1u;
  return (e & 0xFFFFu) + (spread6((ox >> fs) & m) | (spread6((oy >> fs) & m) << 1));
}

__device__ __forceinline__ unsigned map_sub_of(const int2 p, const SortMap& sm, const int4 sq) {
  const long long top = (1ll << sq.z) - 1;
  const long long dx = (long long)p.x - sm.org.x - (long long)(unsigned)sq.x;
  const long long dy = (long long)p.y - sm.org.y - (long long)(unsigned)sq.y;
  const unsigned cx = (unsigned)(min(top, max(0ll, dx)) >> (sq.z - 6));
  const unsigned cy = (unsigned)(min(top, max(0ll, dy)) >> (sq.z - 6));
  return spread6(cx) | (spread6(cy) << 1);
}

// The coarse-cell table in LDS (C[1] and nothing staged for uniform bins).
template <bool kAd>
__device__ __forceinline__ void stage_cells(const SortMap& sm, uint32_t* C) {
  if constexpr (kAd)
    for (int i = threadIdx.x; i < kSortCells; i += blockDim.x) C[i] = sm.cell[i];
}

// Exclusive prefix sum over a block of kThreads threads; `wsum` holds one
// entry per wave. Every thread of the block must call it.
template <int kThreads>
__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned* wsum) {
  constexpr int kW = kThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  unsigned inc = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned t = __shfl_up(inc, o);
    if (lane >= o) inc += t;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  if (w == 0) {
    unsigned s = lane < kW ? wsum[lane] : 0u;
#pragma unroll
    for (int o = 1; o < kW; o <<= 1) {
      const unsigned t = __shfl_up(s, o);
      if (lane >= o) s += t;
    }
    if (lane < kW) wsum[lane] = s;  // inclusive prefix over waves
  }
  __syncthreads();
  return (w ? wsum[w - 1] : 0u) + inc - v;
}

// Both passes give block b the kBinBlockPts points starting at b * kBinBlockPts,
// thread t the points t, t + kBinThreads, ... of that range, and load all of a
// thread's points before the first LDS atomic, so the loads of a block are in
// flight together rather than one per loop trip.
template <int kBB, bool kAd>
__device__ __forceinline__ void bin_load(const int2* __restrict__ xy, const long long n, const int4 rb,
                                         const int shx, const int shy, const SortMap& sm,
                                         const uint32_t* __restrict__ C, int2 (&p)[kBinPer],
                                         unsigned (&b)[kBinPer]) {
  const long long lo = (long long)blockIdx.x * kBinBlockPts + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBinPer; ++k) {
    const long long i = lo + (long long)k * kBinThreads;
    p[k] = i < n ? ld_once(xy + i) : make_int2(0, 0);
  }
#pragma unroll
  for (int k = 0; k < kBinPer; ++k)
    b[k] = lo + (long long)k * kBinThreads < n ? (kAd ? cell_bin(p[k], C, sm) : bin_of<kBB>(p[k], rb, shx, shy))
                                               : (unsigned)Bins<kBB>::kN;
}

// Each block counts the bins of its range in LDS and adds the counts to the
// chunk's per-bin totals.
template <int kBB, bool kAd>
__global__ __launch_bounds__(kBinThreads) void bin_count_kernel(const int2* __restrict__ xy, const long long m,
                                                                const long long chunk, const int4 rb, const int shx,
                                                                const int shy, const SortMap sm,
                                                                unsigned* __restrict__ tot) {
  constexpr int kNB = Bins<kBB>::kN;
  __shared__ unsigned h[kNB];
  __shared__ uint32_t C[kAd ? kSortCells : 1];
  const long long c0 = (long long)blockIdx.y * chunk, n = min(chunk, m - c0);
  if ((long long)blockIdx.x * kBinBlockPts >= n) return;
  xy += c0;
  tot += (size_t)blockIdx.y * kBins;
  if constexpr (kAd) {
    stage_cells<kAd>(sm, C);
    __syncthreads();
  }
  int2 p[kBinPer];
  unsigned b[kBinPer];
  bin_load<kBB, kAd>(xy, n, rb, shx, shy, sm, C, p, b);
  for (int i = threadIdx.x; i < kNB; i += kBinThreads) h[i] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kBinPer; ++k)
    if (b[k] < (unsigned)kNB) atomicAdd(&h[b[k]], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kNB; i += kBinThreads)
    if (h[i]) atomicAdd(&tot[i], h[i]);
}

// The refinement pass cuts every bin into pieces of kRefThreads * kRefPer points.

constexpr int kPStride = kBins + 64;  // pstart entries per chunk

// Block c handles chunk c. cursor[bin] = first sorted position of the bin in
// the chunk (exclusive scan of tot); tot is cleared for the next use. With
// `pstart`, also the bins' first piece numbers (exclusive scan of
// ceil(tot / piece size)) and, in pstart[kN], the number of pieces.
template <int kBB>
__global__ __launch_bounds__(kBinThreads) void bin_scan_kernel(unsigned* __restrict__ tot,
                                                               unsigned* __restrict__ cursor,
                                                               unsigned* __restrict__ pstart) {
  constexpr int kNB = Bins<kBB>::kN, kPer = kNB / kBinThreads;
  constexpr unsigned kRefPts = Bins<kBB>::kRefThreads * Bins<kBB>::kRefPer;
  tot += (size_t)blockIdx.x * kBins;
  cursor += (size_t)blockIdx.x * kBins;
  if (pstart) pstart += (size_t)blockIdx.x * kPStride;
  __shared__ unsigned wsum[kBinThreads / kWave];
  unsigned v[kPer], mine = 0, pcs = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    v[k] = tot[threadIdx.x * kPer + k];
    mine += v[k];
    pcs += (v[k] + kRefPts - 1) / kRefPts;
  }
  unsigned run = block_exclusive_scan<kBinThreads>(mine, wsum);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    cursor[threadIdx.x * kPer + k] = run;
    tot[threadIdx.x * kPer + k] = 0;
    run += v[k];
  }
  if (pstart) {
    __syncthreads();  // wsum is reused
    unsigned pr = block_exclusive_scan<kBinThreads>(pcs, wsum);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      pstart[threadIdx.x * kPer + k] = pr;
      pr += (v[k] + kRefPts - 1) / kRefPts;
    }
    if (threadIdx.x == kBinThreads - 1) pstart[kNB] = pr;
  }
}

__global__ __launch_bounds__(1024) void bin_zero_kernel(unsigned* __restrict__ tot, const long long count) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x)
    tot[i] = 0;
}

// The scatter pass gives each block kScatPts points (kScatPer per thread).
// A block ranks its points by bin in LDS, reserves one run of every bin it
// uses from the bin cursors, lays the points out in LDS in bin order, and
// then stores them with consecutive threads on consecutive positions of the
// runs, so a wave's stores touch a few cache lines rather than one per lane:
// sorted[pos] = point. For the unscatter pass the block also records, in the
// same (bin) order and at the same offsets of its own range, each point's
// position in the chunk's sorted order (spos, int) and its offset in the
// block's range of points (sidx, u16). (The order inside a bin varies from
// run to run; no output depends on it.)
constexpr int kScatPer = 12;
constexpr long long kScatPts = (long long)kBinThreads * kScatPer;

template <int kBB, bool kAd>
__global__ __launch_bounds__(kBinThreads) void bin_scatter_kernel(const int2* __restrict__ xy, const long long m,
                                                                  const long long chunk, const int4 rb, const int shx,
                                                                  const int shy, const SortMap sm,
                                                                  unsigned* __restrict__ cursor,
                                                                  int2* __restrict__ sorted, int* __restrict__ spos,
                                                                  unsigned short* __restrict__ sidx) {
  static_assert(kScatPts <= 65536, "offsets in a scatter block fit 16 bits");
  __shared__ int2 sx[kScatPts];
  __shared__ unsigned short si[kScatPts];
  constexpr int kNB = Bins<kBB>::kN;
  __shared__ unsigned h[kNB];  // counts, then first local position of each bin
  __shared__ unsigned d[kNB];  // first position in the chunk minus first local position
  __shared__ unsigned wsum[kBinThreads / kWave];
  __shared__ uint32_t C[kAd ? kSortCells : 1];
  const long long c0 = (long long)blockIdx.y * chunk, n = min(chunk, m - c0);
  const long long lo = (long long)blockIdx.x * kScatPts;
  if (lo >= n) return;
  xy += c0;
  cursor += (size_t)blockIdx.y * kBins;
  sorted += c0;
  spos += c0;
  sidx += c0;
  if constexpr (kAd) {
    stage_cells<kAd>(sm, C);
    __syncthreads();
  }
  int2 p[kScatPer];
  unsigned b[kScatPer], r[kScatPer];
#pragma unroll
  for (int k = 0; k < kScatPer; ++k) {
    const long long i = lo + threadIdx.x + (long long)k * kBinThreads;
    p[k] = i < n ? ld_once(xy + i) : make_int2(0, 0);
  }
#pragma unroll
  for (int k = 0; k < kScatPer; ++k)
    b[k] = lo + threadIdx.x + (long long)k * kBinThreads < n
               ? (kAd ? cell_bin(p[k], C, sm) : bin_of<kBB>(p[k], rb, shx, shy))
               : (unsigned)kNB;
  for (int i = threadIdx.x; i < kNB; i += kBinThreads) h[i] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScatPer; ++k) r[k] = b[k] < (unsigned)kNB ? atomicAdd(&h[b[k]], 1u) : 0u;
  __syncthreads();
  // local starts (exclusive scan of the counts) and the global runs
  constexpr int kQ = kNB / kBinThreads;
  unsigned v[kQ], mine = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    v[q] = h[threadIdx.x * kQ + q];
    mine += v[q];
  }
  unsigned run = block_exclusive_scan<kBinThreads>(mine, wsum);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int bin = threadIdx.x * kQ + q;
    if (v[q]) d[bin] = atomicAdd(&cursor[bin], v[q]) - run;
    h[bin] = run;
    run += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kScatPer; ++k)
    if (b[k] < (unsigned)kNB) {
      const unsigned j = h[b[k]] + r[k];
      sx[j] = p[k];
      si[j] = (unsigned short)(threadIdx.x + k * kBinThreads);
    }
  __syncthreads();
  const int cnt = (int)min((long long)kScatPts, n - lo);
  for (int j = threadIdx.x; j < cnt; j += kBinThreads) {
    const int2 q = sx[j];
    const unsigned pos = d[kAd ? cell_bin(q, C, sm) : bin_of<kBB>(q, rb, shx, shy)] + (unsigned)j;
    sorted[pos] = q;
    spos[lo + j] = (int)pos;
    sidx[lo + j] = si[j];
  }
}

// Refinement: after the scatter, cursor[bin] is the end of the bin. Block
// (i, c) takes piece i of chunk c (the bin found by a binary search of
// pstart) and sorts its points in place by the Morton index of their
// sub-cell of the bin's cell, through LDS; rof[base + j] records the offset
// in the piece that the point at offset j came from, for the unrefine pass.
// Bin and sub-cell together order the chunk along a Z-curve, so the mapping
// kernel's tiles of points are spatially tighter. Blocks beyond the last
// piece exit at once.
template <int kBB>
__device__ __forceinline__ unsigned sub_of(const int2 p, const int4 rb, const int shx, const int shy) {
  constexpr int kSubBits = Bins<kBB>::kSubBits;
  const long long dx = (long long)p.x - rb.x, dy = (long long)p.y - rb.z;
  const long long top = (1ll << (kBB + kSubBits)) - 1;
  const unsigned cx = (unsigned)min(top, max(0ll, dx >> (shx - kSubBits))) & ((1u << kSubBits) - 1);
  const unsigned cy = (unsigned)min(top, max(0ll, dy >> (shy - kSubBits))) & ((1u << kSubBits) - 1);
  return spread6(cx) | (spread6(cy) << 1);
}

// The piece that block (piece, chunk) of the refine and unrefine passes
// takes: [base, base + cnt) of the chunk's sorted order; false for blocks
// beyond the chunk's last piece. Every thread of the block must call it.
template <int kBB>
__device__ __forceinline__ bool piece_range(const unsigned* __restrict__ cursor, const unsigned* __restrict__ pstart,
                                            int* the_bin, unsigned& base, int& cnt) {
  constexpr int kNB = Bins<kBB>::kN;
  constexpr unsigned kRefPts = Bins<kBB>::kRefThreads * Bins<kBB>::kRefPer;
  const unsigned piece = blockIdx.x;
  if (piece >= pstart[kNB]) return false;
  if (threadIdx.x == 0) {  // the last bin whose first piece is <= piece
    int lo = 0, hi = kNB - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pstart[mid] <= piece) lo = mid; else hi = mid - 1;
    }
    *the_bin = lo;
  }
  __syncthreads();
  const int b = *the_bin;
  const unsigned start = b ? cursor[b - 1] : 0u, end = cursor[b];
  base = start + (piece - pstart[b]) * kRefPts;
  cnt = (int)min(kRefPts, end - base);
  return true;
}

template <int kBB, bool kAd>
__global__ __launch_bounds__(Bins<kBB>::kRefThreads) void bin_refine_kernel(int2* __restrict__ sorted,
                                                                 unsigned short* __restrict__ rof,
                                                                 const long long chunk,
                                                                 const unsigned* __restrict__ cursor,
                                                                 const unsigned* __restrict__ pstart, const int4 rb,
                                                                 const int shx, const int shy, const SortMap sm) {
  constexpr int kSubs = Bins<kBB>::kSubs, kRefPer = Bins<kBB>::kRefPer;
  constexpr int kRefThreads = Bins<kBB>::kRefThreads;
  constexpr int kRefPts = kRefThreads * kRefPer;
  static_assert(kRefPts <= 65536, "offsets in a piece fit 16 bits");
  __shared__ int2 sx[kRefPts];
  __shared__ unsigned short so[kRefPts];
  __shared__ unsigned h[kSubs];
  __shared__ unsigned wsum[kRefThreads / kWave];
  __shared__ int the_bin;
  static_assert(kSubs % kRefThreads == 0, "whole sub-cell counts per thread");
  constexpr int kQ = kSubs / kRefThreads;
  sorted += (long long)blockIdx.y * chunk;  // block (piece, chunk)
  rof += (long long)blockIdx.y * chunk;
  cursor += (size_t)blockIdx.y * kBins;
  pstart += (size_t)blockIdx.y * kPStride;
  for (int i = threadIdx.x; i < kSubs; i += kRefThreads) h[i] = 0;
  unsigned base;
  int cnt;
  if (!piece_range<kBB>(cursor, pstart, &the_bin, base, cnt)) return;
  const int4 sq = kAd ? sm.sq[the_bin] : make_int4(0, 0, 0, 0);
  int2 p[kRefPer];
  unsigned key[kRefPer], r[kRefPer];
#pragma unroll
  for (int k = 0; k < kRefPer; ++k) {
    const int j = threadIdx.x + k * kRefThreads;
    p[k] = j < cnt ? ld_once(sorted + base + j) : make_int2(0, 0);
  }
#pragma unroll
  for (int k = 0; k < kRefPer; ++k) {
    key[k] = threadIdx.x + k * kRefThreads < cnt
                 ? (kAd ? map_sub_of(p[k], sm, sq) : sub_of<kBB>(p[k], rb, shx, shy))
                 : (unsigned)kSubs;
    r[k] = key[k] < (unsigned)kSubs ? atomicAdd(&h[key[k]], 1u) : 0u;
  }
  __syncthreads();
  unsigned v[kQ], mine = 0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    v[q] = h[threadIdx.x * kQ + q];
    mine += v[q];
  }
  unsigned run = block_exclusive_scan<kRefThreads>(mine, wsum);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {  // each thread rewrites only its own sub-cells
    h[threadIdx.x * kQ + q] = run;
    run += v[q];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRefPer; ++k)
    if (key[k] < (unsigned)kSubs) {
      const unsigned j = h[key[k]] + r[k];
      sx[j] = p[k];
      so[j] = (unsigned short)(threadIdx.x + k * kRefThreads);
    }
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += kRefThreads) {
    sorted[base + j] = sx[j];
    rof[base + j] = so[j];
  }
}

// Unrefine: the inverse of the refine pass on the results, piece by piece
// and in place: the result at offset j goes back to offset rof[base + j].
template <int kBB>
__global__ __launch_bounds__(Bins<kBB>::kRefThreads) void bin_unrefine_kernel(int* __restrict__ res,
                                                                   const unsigned short* __restrict__ rof,
                                                                   const long long chunk,
                                                                   const unsigned* __restrict__ cursor,
                                                                   const unsigned* __restrict__ pstart) {
  constexpr int kRefPer = Bins<kBB>::kRefPer, kRefThreads = Bins<kBB>::kRefThreads;
  constexpr int kRefPts = kRefThreads * kRefPer;
  __shared__ int sr[kRefPts];
  __shared__ int the_bin;
  res += (long long)blockIdx.y * chunk;
  rof += (long long)blockIdx.y * chunk;
  cursor += (size_t)blockIdx.y * kBins;
  pstart += (size_t)blockIdx.y * kPStride;
  unsigned base;
  int cnt;
  if (!piece_range<kBB>(cursor, pstart, &the_bin, base, cnt)) return;
  int v[kRefPer];
  unsigned o[kRefPer];
#pragma unroll
  for (int k = 0; k < kRefPer; ++k) {
    const int j = threadIdx.x + k * kRefThreads;
    v[k] = j < cnt ? ld_once(res + base + j) : 0;
    o[k] = j < cnt ? (unsigned)__builtin_nontemporal_load(rof + base + j) : 0u;
  }
#pragma unroll
  for (int k = 0; k < kRefPer; ++k)
    if (threadIdx.x + k * kRefThreads < cnt) sr[o[k]] = v[k];
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += kRefThreads) res[base + j] = sr[j];
}

// Unscatter: the inverse of the scatter pass on the results. Block (b, c)
// takes the kScatPts points of scatter block b of chunk c: consecutive
// threads read the results at the positions the scatter block recorded
// (spos, in bin order, so a wave's loads follow a few runs), place each at
// its point's offset in LDS (sidx), and store the block's range of out
// coalesced.
__global__ __launch_bounds__(kBinThreads) void unscatter_kernel(const int* __restrict__ res, const int* __restrict__ spos,
                                                               const unsigned short* __restrict__ sidx,
                                                               const long long m, const long long chunk,
                                                               int* __restrict__ out) {
  __shared__ int sv[kScatPts];
  const long long c0 = (long long)blockIdx.y * chunk, n = min(chunk, m - c0);
  const long long lo = (long long)blockIdx.x * kScatPts;
  if (lo >= n) return;
  res += c0;
  spos += c0 + lo;
  sidx += c0 + lo;
  out += c0 + lo;
  const int cnt = (int)min((long long)kScatPts, n - lo);
  int q[kScatPer];
  unsigned t[kScatPer];
#pragma unroll
  for (int k = 0; k < kScatPer; ++k) {
    const int j = threadIdx.x + k * kBinThreads;
    q[k] = j < cnt ? ld_once(spos + j) : 0;
    t[k] = j < cnt ? (unsigned)__builtin_nontemporal_load(sidx + j) : 0u;
  }
  int v[kScatPer];
#pragma unroll
  for (int k = 0; k < kScatPer; ++k) v[k] = res[q[k]];
#pragma unroll
  for (int k = 0; k < kScatPer; ++k)
    if (threadIdx.x + k * kBinThreads < cnt) sv[t[k]] = v[k];
  __syncthreads();
  for (int j = threadIdx.x; j < cnt; j += kBinThreads) st_once(out + j, sv[j]);
}

// Sorted form: as the plain form, over the sorted copy of a round of sort
// passes; results in sorted order (the unrefine and unscatter passes bring
// them to the points' original positions). Each wave loads its next tile's
// points while it maps the current one.
template <int kChunkShift>
__global__ __launch_bounds__(kBlock, map_min_blocks(kChunkShift)) void map_sorted_kernel(
    const KIndex ix, const int2* __restrict__ xy, const long long n, int* __restrict__ out) {
  __shared__ WaveLds wl[kWavesPerBlock];
  __shared__ RootLds R;
  stage_root(ix, R);
  const int lane = threadIdx.x & (kWave - 1);
  WaveLds& S = wl[threadIdx.x / kWave];
  const long long ntiles = (n + kTile - 1) / kTile;
  const long long nwaves = (long long)gridDim.x * kWavesPerBlock;
  int2 np[kTilePts];
  auto fetch = [&](const long long t) {
#pragma unroll
    for (int j = 0; j < kTilePts; ++j) {
      const long long i = t * kTile + j * kWave + lane;
      np[j] = i < n ? ld_once(xy + i) : make_int2(0, 0);
    }
  };
  long long t = (long long)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
  if (t < ntiles) fetch(t);
  for (; t < ntiles; t += nwaves) {
    int2 pt[kTilePts];
#pragma unroll
    for (int j = 0; j < kTilePts; ++j) pt[j] = np[j];
    if (t + nwaves < ntiles) fetch(t + nwaves);
    map_tile_pts<kChunkShift>(ix, S, R, lane, pt, (int)min((long long)kTile, n - t * kTile), out + t * kTile);
  }
}

// Points per block: counts[b] += |{i : ids[i] == b}| for b < nb, and
// counts[nb] += the ids outside [0, nb) (-1: no block). Lanes holding the same
// id add it with one atomic (up to kAggRounds distinct ids per wave step;
// the rest add one by one), which matters when points of one block arrive
// together.
constexpr int kAggRounds = 4;

__global__ __launch_bounds__(256) void count_kernel(const int* __restrict__ ids, const long long n, const int nb,
                                                    unsigned long long* __restrict__ counts) {
  const int lane = threadIdx.x & (kWave - 1);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < n; base += stride) {
    const long long i = base + threadIdx.x;
    bool active = i < n;
    const int id = active ? ids[i] : -1;
    const unsigned b = (id >= 0 && id < nb) ? (unsigned)id : (unsigned)nb;
    for (int r = 0; r < kAggRounds; ++r) {
      const unsigned long long act = __ballot(active);
      if (act == 0ull) break;
      const int leader = __builtin_ctzll(act);
      const unsigned bl = __shfl(b, leader);
      const unsigned long long same = __ballot(active && b == bl);
      if (lane == leader) atomicAdd(&counts[bl], (unsigned long long)__popcll(same));
      if (b == bl) active = false;
    }
    if (active) atomicAdd(&counts[b], 1ull);
  }
}

// Bucketed count for large calls: ids are counting-sorted by bucket id >> 13
// (at most kBins buckets of 8192 ids; the binning passes above with a
// different key), then each slice of a bucket is counted in an LDS histogram
// into its own row of partial counts, and the rows are summed. No two
// threads then add to one global counter.
constexpr int kCntShift = 13;
constexpr int kCntIds = 1 << kCntShift;

// Block b takes ids b * kBinBlockPts + t + k * kBinThreads; a thread loads
// its kBinPer ids before its first LDS atomic. Ids outside [0, nb) get
// bucket kBins (none).
__device__ __forceinline__ void cnt_load(const int* __restrict__ ids, const long long n, const int nb,
                                         int (&id)[kBinPer]) {
  const long long lo = (long long)blockIdx.x * kBinBlockPts + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kBinPer; ++k) {
    const long long i = lo + (long long)k * kBinThreads;
    id[k] = i < n ? ld_once(ids + i) : -1;
  }
#pragma unroll
  for (int k = 0; k < kBinPer; ++k)
    if (id[k] >= nb) id[k] = -1;
}

__global__ __launch_bounds__(kBinThreads) void cnt_bucket_count_kernel(const int* __restrict__ ids,
                                                                       const long long n, const int nb,
                                                                       unsigned* __restrict__ tot,
                                                                       unsigned long long* __restrict__ counts) {
  __shared__ unsigned h[kBins];
  __shared__ unsigned other;
  int id[kBinPer];
  cnt_load(ids, n, nb, id);
  for (int i = threadIdx.x; i < kBins; i += kBinThreads) h[i] = 0;
  if (threadIdx.x == 0) other = 0;
  __syncthreads();
  const long long lo = (long long)blockIdx.x * kBinBlockPts + threadIdx.x;
  unsigned mine = 0;  // this thread's ids in range of the call but not of [0, nb)
#pragma unroll
  for (int k = 0; k < kBinPer; ++k) {
    if (id[k] >= 0)
      atomicAdd(&h[id[k] >> kCntShift], 1u);
    else if (lo + (long long)k * kBinThreads < n)
      ++mine;
  }
  if (mine) atomicAdd(&other, mine);
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += kBinThreads)
    if (h[i]) atomicAdd(&tot[i], h[i]);
  if (threadIdx.x == 0 && other) atomicAdd(&counts[nb], (unsigned long long)other);
}

__global__ __launch_bounds__(kBinThreads) void cnt_bucket_scatter_kernel(const int* __restrict__ ids,
                                                                         const long long n, const int nb,
                                                                         unsigned* __restrict__ cursor,
                                                                         int* __restrict__ sorted) {
  __shared__ unsigned cur[kBins];
  int id[kBinPer];
  cnt_load(ids, n, nb, id);
  for (int i = threadIdx.x; i < kBins; i += kBinThreads) cur[i] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kBinPer; ++k)
    if (id[k] >= 0) atomicAdd(&cur[id[k] >> kCntShift], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kBins; i += kBinThreads)
    if (cur[i]) cur[i] = atomicAdd(&cursor[i], cur[i]);
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kBinPer; ++k)
    if (id[k] >= 0) sorted[atomicAdd(&cur[id[k] >> kCntShift], 1u)] = id[k];
}

// Block (bucket b = blockIdx.x, slice s = blockIdx.y) counts its slice of the
// bucket's segment [end[b-1], end[b]) of `sorted` into part[s][b * 8192 + k].
__global__ __launch_bounds__(1024) void cnt_slice_kernel(const int* __restrict__ sorted,
                                                         const unsigned* __restrict__ end, const int nb,
                                                         unsigned* __restrict__ part, const long long part_stride) {
  __shared__ unsigned h[kCntIds];
  for (int i = threadIdx.x; i < kCntIds; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int b = blockIdx.x, sl = blockIdx.y, ns = gridDim.y;
  const long long s0 = b ? end[b - 1] : 0, s1 = end[b];
  const long long len = s1 - s0, per = (len + ns - 1) / ns;
  const long long lo = s0 + (long long)sl * per, hi = min(s1, lo + per);
  for (long long i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&h[sorted[i] & (kCntIds - 1)], 1u);
  __syncthreads();
  const long long base = (long long)b * kCntIds;
  unsigned* row = part + (long long)sl * part_stride + base;
  for (int i = threadIdx.x; i < kCntIds; i += blockDim.x)
    if (base + i < nb) row[i] = h[i];
}

// counts[id] += sum over slices of part[s][id], for id < nb.
__global__ __launch_bounds__(256) void cnt_reduce_kernel(const unsigned* __restrict__ part, const int ns,
                                                         const long long part_stride, const int nb,
                                                         unsigned long long* __restrict__ counts) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x; id < nb; id += stride) {
    unsigned long long t = 0;
    for (int sl = 0; sl < ns; ++sl) t += part[(long long)sl * part_stride + id];
    counts[id] += t;
  }
}

// Per-point join of a per-block attribute (App. A gives each point its
// block's FIPS code): out[i] = table[ids[i]] for ids in [0, nb), else fill.
// kVec: ids and out 16-byte aligned, four ids per thread (one 16-byte load,
// four gathers from the table, two 16-byte stores); the last n % 4 ids, or
// all of them without kVec, one per thread.
template <bool kVec>
__global__ __launch_bounds__(256) void join_kernel(const int* __restrict__ ids, const long long n,
                                                   const long long* __restrict__ table, const int nb,
                                                   const long long fill, long long* __restrict__ out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long done = 0;
  if (kVec) {
    const long long n4 = n >> 2;
    const int4* ids4 = reinterpret_cast<const int4*>(ids);
    longlong2* out2 = reinterpret_cast<longlong2*>(out);
    for (long long q = t0; q < n4; q += stride) {
      int4 v;
      v.x = __builtin_nontemporal_load(&ids4[q].x);
      v.y = __builtin_nontemporal_load(&ids4[q].y);
      v.z = __builtin_nontemporal_load(&ids4[q].z);
      v.w = __builtin_nontemporal_load(&ids4[q].w);
      longlong2 a, b;
      a.x = ((unsigned)v.x < (unsigned)nb) ? table[v.x] : fill;
      a.y = ((unsigned)v.y < (unsigned)nb) ? table[v.y] : fill;
      b.x = ((unsigned)v.z < (unsigned)nb) ? table[v.z] : fill;
      b.y = ((unsigned)v.w < (unsigned)nb) ? table[v.w] : fill;
      out2[2 * q] = a;
      out2[2 * q + 1] = b;
    }
    done = n4 << 2;
  }
  for (long long i = done + t0; i < n; i += stride) {
    const int id = ld_once(ids + i);
    out[i] = ((unsigned)id < (unsigned)nb) ? table[id] : fill;
  }
}

// Quantiser: q = rint(v * 2^22) + 2^30 per axis; invalid input -> (-1, -1).
// The product by a power of two is exact, so rint is the only rounding.
__global__ __launch_bounds__(256) void quantize_kernel(const double2* __restrict__ ll,
                                                       const long long n, int2* __restrict__ xy) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 v = ll[i];
    const bool ok = (fabs(v.x) <= 180.0) && (fabs(v.y) <= 90.0);  // false for NaN
    const long long qx = (long long)rint(v.x * 4194304.0) + 1073741824ll;
    const long long qy = (long long)rint(v.y * 4194304.0) + 1073741824ll;
    xy[i] = ok ? make_int2((int)qx, (int)qy) : make_int2(-1, -1);
  }
}

}  // namespace

// Workgroups of kKernel that fit on one CU at once (registers and LDS),
// asked once per kernel.
template <auto kKernel>
static int resident_blocks() {
  static const int r = [] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kKernel, kBlock, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    return nb;
  }();
  return r;
}

// Grid of a mapping launch: enough workgroups for every wave to have a tile,
// at most blocks_per_cu per CU, and never more per CU than can be resident
// (with a static tile split a workgroup that waits for a free CU finishes
// last and stretches the launch).
template <auto kKernel>
static long long grid_blocks(long long n, const Tuning& t, int num_cu) {
  const long long tiles = (n + kTile - 1) / kTile;
  long long blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  const long long cap = (long long)num_cu * std::min(t.blocks_per_cu, resident_blocks<kKernel>());
  if (blocks > cap) blocks = cap;
  return blocks < 1 ? 1 : blocks;
}

template <int kShift>
static void launch_plain(const KIndex& ix, const int2* p, long long n, int* out, const Tuning& t, int num_cu,
                         hipStream_t stream) {
  const dim3 grid((unsigned)grid_blocks<map_kernel<kShift>>(n, t, num_cu));
  hipLaunchKernelGGL(map_kernel<kShift>, grid, dim3(kBlock), 0, stream, ix, p, n, out);
}

template <int kShift>
static void launch_sorted(const KIndex& ix, const int2* p, long long n, int* out, const Tuning& t, int num_cu,
                          hipStream_t stream) {
  const dim3 grid((unsigned)grid_blocks<map_sorted_kernel<kShift>>(n, t, num_cu));
  hipLaunchKernelGGL(map_sorted_kernel<kShift>, grid, dim3(kBlock), 0, stream, ix, p, n, out);
}

// Shifts of the sort grid over the root box, and whether the refine pass
// runs (the root box at least 1024 units a side).
struct SortGrid {
  int shx = 0, shy = 0;
  bool refine = false;
};

template <int kBB>
static SortGrid sort_grid(const int4 rb) {
  SortGrid g;
  while (((1ll << kBB) << g.shx) < (long long)rb.y - rb.x) ++g.shx;
  while (((1ll << kBB) << g.shy) < (long long)rb.w - rb.z) ++g.shy;
  g.refine = g.shx >= Bins<kBB>::kSubBits && g.shy >= Bins<kBB>::kSubBits;
  return g;
}

// Blocks per chunk of the refine and unrefine passes: at most chunk / piece
// size + bins pieces per chunk.
template <int kBB>
static unsigned piece_blocks(const long long chunk) {
  return (unsigned)(chunk / ((long long)Bins<kBB>::kRefThreads * Bins<kBB>::kRefPer) + Bins<kBB>::kN);
}

constexpr SortMap kNoSortMap{nullptr, nullptr, {0, 0}, 0, 0};

// Does a round refine its bins? Always with adaptive bins (their squares are
// at least 64 units wide), else when the grid's cells are.
template <int kBB>
static bool refines(const int4 rb, const SortMap& sm) {
  return sm.cell != nullptr || sort_grid<kBB>(rb).refine;
}

// One round of sort passes over the nc chunks of m points at p: count, scan,
// scatter and (when the bins allow) refine; kAd: the index's adaptive bins
// instead of the uniform grid.
template <int kBB, bool kAd>
static void sort_passes_in(const int4 rb, const SortMap& sm, const int2* p, const long long m, const long long chunk,
                           const unsigned nc, unsigned* tot, unsigned* cursor, unsigned* pstart, int2* sorted,
                           int* spos, unsigned short* sidx, unsigned short* rof, hipStream_t stream) {
  const SortGrid g = sort_grid<kBB>(rb);
  const bool refine = kAd || g.refine;
  hipLaunchKernelGGL((bin_count_kernel<kBB, kAd>), dim3((unsigned)((chunk + kBinBlockPts - 1) / kBinBlockPts), nc),
                     dim3(kBinThreads), 0, stream, p, m, chunk, rb, g.shx, g.shy, sm, tot);
  hipLaunchKernelGGL(bin_scan_kernel<kBB>, dim3(nc), dim3(kBinThreads), 0, stream, tot, cursor,
                     refine ? pstart : nullptr);
  hipLaunchKernelGGL((bin_scatter_kernel<kBB, kAd>), dim3((unsigned)((chunk + kScatPts - 1) / kScatPts), nc),
                     dim3(kBinThreads), 0, stream, p, m, chunk, rb, g.shx, g.shy, sm, cursor, sorted, spos, sidx);
  if (refine)
    hipLaunchKernelGGL((bin_refine_kernel<kBB, kAd>), dim3(piece_blocks<kBB>(chunk), nc),
                       dim3(Bins<kBB>::kRefThreads), 0, stream, sorted, rof, chunk, cursor, pstart, rb, g.shx, g.shy,
                       sm);
}

template <int kBB>
static void sort_passes(const int4 rb, const SortMap& sm, const int2* p, const long long m, const long long chunk,
                        const unsigned nc, unsigned* tot, unsigned* cursor, unsigned* pstart, int2* sorted, int* spos,
                        unsigned short* sidx, unsigned short* rof, hipStream_t stream) {
  if constexpr (kBB == 6) {
    static_assert(Bins<6>::kN == kSortMapBins, "adaptive bins fill the 64 x 64 grid's bin arrays");
    if (sm.cell) {
      sort_passes_in<kBB, true>(rb, sm, p, m, chunk, nc, tot, cursor, pstart, sorted, spos, sidx, rof, stream);
      return;
    }
  }
  sort_passes_in<kBB, false>(rb, sm, p, m, chunk, nc, tot, cursor, pstart, sorted, spos, sidx, rof, stream);
}

// The results of a round (res, in sorted order) back to the points'
// original positions: unrefine (when the refine pass ran), then unscatter
// into out.
template <int kBB>
static void unsort_passes(const int4 rb, const SortMap& sm, const long long m, const long long chunk,
                          const unsigned nc, const unsigned* cursor, const unsigned* pstart, const int* spos,
                          const unsigned short* sidx, const unsigned short* rof, int* res, int* out,
                          hipStream_t stream) {
  if (refines<kBB>(rb, sm))
    hipLaunchKernelGGL(bin_unrefine_kernel<kBB>, dim3(piece_blocks<kBB>(chunk), nc), dim3(Bins<kBB>::kRefThreads), 0,
                       stream, res, rof, chunk, cursor, pstart);
  hipLaunchKernelGGL(unscatter_kernel, dim3((unsigned)((chunk + kScatPts - 1) / kScatPts), nc), dim3(kBinThreads), 0,
                     stream, res, spos, sidx, m, chunk, out);
}

// Scratch of a pre-sorted call that sorts `super` points per round in chunks
// of `chunk`: per chunk the sort's bin totals, cursors and piece starts; then
// per point of a round the sorted copy (int2), the scatter pass's position
// and offset records (int, u16), the result in sorted order (int) and the
// refine pass's offset record (u16): 20 bytes per point.
struct PresortPlan {
  long long chunk = 0, super = 0, max_nc = 0;
  size_t hist_bytes = 0, sorted_off = 0, spos_off = 0, sidx_off = 0, res_off = 0, rof_off = 0, bytes = 0;
};

static size_t round256(size_t v) { return (v + 255) / 256 * 256; }

static PresortPlan presort_plan(long long chunk, long long super) {
  PresortPlan pl;
  pl.chunk = chunk;
  pl.super = super;
  pl.max_nc = (super + chunk - 1) / chunk;
  pl.hist_bytes = round256(sizeof(unsigned) * (size_t)pl.max_nc * (2 * (size_t)kBins + kPStride));
  pl.sorted_off = pl.hist_bytes;
  pl.spos_off = pl.sorted_off + round256((size_t)super * sizeof(int2));
  pl.sidx_off = pl.spos_off + round256((size_t)super * sizeof(int));
  pl.res_off = pl.sidx_off + round256((size_t)super * sizeof(unsigned short));
  pl.rof_off = pl.res_off + round256((size_t)super * sizeof(int));
  pl.bytes = pl.rof_off + round256((size_t)super * sizeof(unsigned short));
  return pl;
}

static bool wants_presort(const KIndex& ix, int64_t n, const Tuning& t) {
  return t.presort && n >= kPresortMin && ix.root_box.x < ix.root_box.y && ix.root_box.z < ix.root_box.w;
}

size_t map_scratch_bytes(const KIndex& ix, int64_t n, const Tuning& t) {
  if (!wants_presort(ix, n, t)) return 0;
  const long long super = std::min<long long>(n, kPresortSuper);
  return presort_plan(std::min<long long>(super, ix.presort_chunk), super).bytes;
}

// The spatially sorted pipeline shared by the hierarchical path and the
// cover path: through scratch (20 bytes per point, up to kPresortSuper points
// at a time), every sort pass runs once over all chunks of a round (chunk =
// blockIdx.y), one launch of map_round(sorted, m, res) maps the round's
// sorted copy, and the unrefine and unscatter passes put its results in
// place. The scratch is stream-ordered memory, or the caller's workspace:
// then the call sorts as many points per round as the workspace holds (in
// chunks no larger), and maps unsorted (map_plain(xy, n, out)) when it holds
// fewer than kPresortMin.
template <class MapRound, class MapPlain>
static hipError_t launch_presorted(const KIndex& ix, const int32_t* xy, int64_t n, int32_t* out, bool presort,
                                   hipStream_t stream, LaunchTimer* timer, void* ws, size_t ws_bytes,
                                   MapRound map_round, MapPlain map_plain) {
  const int2* p = reinterpret_cast<const int2*>(xy);
  auto mark = [&](int slot) {
    if (timer && timer->n < LaunchTimer::kMax) {
      (void)hipEventRecord(timer->ev[timer->n], stream);
      timer->tag[timer->n++] = slot;
    }
  };
  PresortPlan pl;
  if (presort) {
    long long super = std::min<long long>(n, kPresortSuper);
    pl = presort_plan(std::min<long long>(super, ix.presort_chunk), super);
    if (ws) {
      while (pl.bytes > ws_bytes && super >= 2 * kPresortMin) {
        super = super / 2;
        pl = presort_plan(std::min<long long>(super, ix.presort_chunk), super);
      }
      presort = pl.bytes <= ws_bytes;
    }
  }
  if (!presort) {
    mark(0);
    map_plain(p, (long long)n, out);
    mark(1);
    return hipGetLastError();
  }
  const long long chunk = pl.chunk, super = pl.super, max_nc = pl.max_nc;
  void* scratch = ws;
  hipError_t e = hipSuccess;
  if (!ws) {
    e = hipMallocAsync(&scratch, pl.bytes, stream);
    if (e != hipSuccess) return e;
  }
  char* base = static_cast<char*>(scratch);
  unsigned* tot = reinterpret_cast<unsigned*>(base);
  unsigned* cursor = tot + max_nc * kBins;
  unsigned* pstart = cursor + max_nc * kBins;
  int2* sorted = reinterpret_cast<int2*>(base + pl.sorted_off);
  int* spos = reinterpret_cast<int*>(base + pl.spos_off);
  unsigned short* sidx = reinterpret_cast<unsigned short*>(base + pl.sidx_off);
  int* res = reinterpret_cast<int*>(base + pl.res_off);
  unsigned short* rof = reinterpret_cast<unsigned short*>(base + pl.rof_off);
  hipLaunchKernelGGL(bin_zero_kernel, dim3((unsigned)std::min<long long>(max_nc * 4, 1024)), dim3(1024), 0, stream,
                     tot, max_nc * kBins);
  for (long long s0 = 0; s0 < n && e == hipSuccess; s0 += super) {
    const long long m = std::min(super, (long long)n - s0);  // the first round is the largest
    const unsigned nc = (unsigned)((m + chunk - 1) / chunk);
    mark(2);
    if (ix.presort_bin_bits == 6)
      sort_passes<6>(ix.root_box, ix.sort_map, p + s0, m, chunk, nc, tot, cursor, pstart, sorted, spos, sidx, rof,
                     stream);
    else
      sort_passes<5>(ix.root_box, kNoSortMap, p + s0, m, chunk, nc, tot, cursor, pstart, sorted, spos, sidx, rof,
                     stream);
    mark(0);
    map_round(sorted, m, res);
    mark(1);
    mark(3);
    if (ix.presort_bin_bits == 6)
      unsort_passes<6>(ix.root_box, ix.sort_map, m, chunk, nc, cursor, pstart, spos, sidx, rof, res, out + s0,
                       stream);
    else
      unsort_passes<5>(ix.root_box, kNoSortMap, m, chunk, nc, cursor, pstart, spos, sidx, rof, res, out + s0,
                       stream);
    e = hipGetLastError();
  }
  mark(4);
  if (ws) return e;
  const hipError_t e2 = hipFreeAsync(scratch, stream);
  return e != hipSuccess ? e : e2;
}

hipError_t launch_map(const KIndex& ix, const int32_t* xy, int64_t n, int32_t* out,
                      const Tuning& t, int num_cu, hipStream_t stream, LaunchTimer* timer, void* ws,
                      size_t ws_bytes) {
  auto map_round = [&](const int2* sp, long long m, int* res) {
    switch (t.edge_chunk) {
      case 8: launch_sorted<3>(ix, sp, m, res, t, num_cu, stream); break;
      case 16: launch_sorted<4>(ix, sp, m, res, t, num_cu, stream); break;
      default: launch_sorted<2>(ix, sp, m, res, t, num_cu, stream); break;
    }
  };
  auto map_plain = [&](const int2* pp, long long m, int* o) {
    switch (t.edge_chunk) {
      case 8: launch_plain<3>(ix, pp, m, o, t, num_cu, stream); break;
      case 16: launch_plain<4>(ix, pp, m, o, t, num_cu, stream); break;
      default: launch_plain<2>(ix, pp, m, o, t, num_cu, stream); break;
    }
  };
  return launch_presorted(ix, xy, n, out, wants_presort(ix, n, t), stream, timer, ws, ws_bytes, map_round,
                          map_plain);
}

template <int kShift>
static void launch_batch_map(const KIndex& ix, const BatchEntry* tab, long long* meta, const Tuning& t, int num_cu,
                             hipStream_t stream) {
  const int per_cu = std::max(1, std::min(t.blocks_per_cu, resident_blocks<batch_map_kernel<kShift>>()));
  hipLaunchKernelGGL(batch_map_kernel<kShift>, dim3((unsigned)(num_cu * per_cu)), dim3(kBlock), 0, stream, ix, tab,
                     meta, t.tile_points);
}

hipError_t launch_batch_offsets(const OffsetHeader* hdr, long long nb, const int32_t* xy, int32_t* out,
                                const int64_t* off, long long max_points, long long max_nb, BatchEntry* tab,
                                int num_cu, hipStream_t stream) {
  const long long blocks = std::max<long long>(1, std::min<long long>((max_nb + 255) / 256, (long long)num_cu * 4));
  hipLaunchKernelGGL(batch_offsets_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, hdr, nb, xy, out,
                     reinterpret_cast<const long long*>(off), max_points, tab);
  return hipGetLastError();
}

hipError_t launch_batches(const KIndex& ix, const long long* hdr, long long nb, const BatchEntry* tab,
                          long long* meta, const Tuning& t, int num_cu, hipStream_t stream) {
  hipLaunchKernelGGL(batch_prefix_kernel, dim3(1), dim3(1024), 0, stream, hdr, nb, tab, meta, t.tile_points);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  switch (t.edge_chunk) {
    case 4: launch_batch_map<2>(ix, tab, meta, t, num_cu, stream); break;
    case 16: launch_batch_map<4>(ix, tab, meta, t, num_cu, stream); break;
    default: launch_batch_map<3>(ix, tab, meta, t, num_cu, stream); break;
  }
  return hipGetLastError();
}

template <int kShift>
static void launch_cover_t(const KIndex& ix, const KCover& cv, const int2* p, long long n, int* out, bool approx,
                           const Tuning& t, int num_cu, hipStream_t stream) {
  const dim3 grid((unsigned)grid_blocks<cover_map_kernel<kShift>>(n, t, num_cu));
  hipLaunchKernelGGL(cover_map_kernel<kShift>, grid, dim3(kBlock), 0, stream, ix, cv, p, n, out, approx ? 1 : 0);
}

// The cover path maps the points in their own order. (Through the spatial
// sort of the hierarchical path its kernel is 1.2 ms faster per 100M points,
// but the sort and unsort passes cost 1.65 ms.)
hipError_t launch_cover(const KIndex& ix, const KCover& cv, const int32_t* xy, int64_t n, int32_t* out, bool approx,
                        const Tuning& t, int num_cu, hipStream_t stream) {
  const int2* p = reinterpret_cast<const int2*>(xy);
  switch (t.edge_chunk) {
    case 8: launch_cover_t<3>(ix, cv, p, n, out, approx, t, num_cu, stream); break;
    case 16: launch_cover_t<4>(ix, cv, p, n, out, approx, t, num_cu, stream); break;
    default: launch_cover_t<2>(ix, cv, p, n, out, approx, t, num_cu, stream); break;
  }
  return hipGetLastError();
}

hipError_t launch_count(const int32_t* ids, int64_t n, int32_t nb, unsigned long long* counts, int num_cu,
                        hipStream_t stream) {
  const long long nbk = ((long long)nb + kCntIds - 1) / kCntIds;
  if (n >= kPresortMin && nbk >= 1 && nbk <= kBins) {
    // bucketed: no contended global atomics
    const int ns = (int)std::max<long long>(1, std::min<long long>(64, (4LL * num_cu + nbk - 1) / nbk));
    const long long part_stride = nbk * kCntIds;
    const size_t bytes = sizeof(unsigned) * (2 * (size_t)kBins + (size_t)ns * part_stride) + sizeof(int) * (size_t)n;
    void* scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, bytes, stream);
    if (e != hipSuccess) return e;
    unsigned* tot = static_cast<unsigned*>(scratch);
    unsigned* cursor = tot + kBins;
    unsigned* part = cursor + kBins;
    int* sorted = reinterpret_cast<int*>(part + (size_t)ns * part_stride);
    const unsigned nblk = (unsigned)((n + kBinBlockPts - 1) / kBinBlockPts);
    hipLaunchKernelGGL(bin_zero_kernel, dim3(4), dim3(1024), 0, stream, tot, (long long)kBins);
    hipLaunchKernelGGL(cnt_bucket_count_kernel, dim3(nblk), dim3(kBinThreads), 0, stream,
                       reinterpret_cast<const int*>(ids), (long long)n, nb, tot, counts);
    hipLaunchKernelGGL(bin_scan_kernel<6>, dim3(1), dim3(kBinThreads), 0, stream, tot, cursor, nullptr);
    hipLaunchKernelGGL(cnt_bucket_scatter_kernel, dim3(nblk), dim3(kBinThreads), 0, stream,
                       reinterpret_cast<const int*>(ids), (long long)n, nb, cursor, sorted);
    hipLaunchKernelGGL(cnt_slice_kernel, dim3((unsigned)nbk, (unsigned)ns), dim3(1024), 0, stream, sorted, cursor, nb,
                       part, part_stride);
    const long long rb = std::min<long long>(((long long)nb + 255) / 256, (long long)num_cu * 8);
    hipLaunchKernelGGL(cnt_reduce_kernel, dim3((unsigned)std::max<long long>(1, rb)), dim3(256), 0, stream, part, ns,
                       part_stride, nb, counts);
    e = hipGetLastError();
    const hipError_t e2 = hipFreeAsync(scratch, stream);
    return e != hipSuccess ? e : e2;
  }
  long long blocks = (n + 255) / 256;
  const long long cap = (long long)num_cu * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(count_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ids, (long long)n, nb, counts);
  return hipGetLastError();
}

hipError_t launch_join(const int32_t* ids, int64_t n, const int64_t* table, int32_t nb, int64_t fill, int64_t* out,
                       int num_cu, hipStream_t stream) {
  const bool vec = ((reinterpret_cast<uintptr_t>(ids) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  long long blocks = ((vec ? (n + 3) / 4 : n) + 255) / 256;
  const long long cap = (long long)num_cu * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  if (vec)
    hipLaunchKernelGGL(join_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const int*>(ids), (long long)n, reinterpret_cast<const long long*>(table), nb,
                       (long long)fill, reinterpret_cast<long long*>(out));
  else
    hipLaunchKernelGGL(join_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, stream,
                       reinterpret_cast<const int*>(ids), (long long)n, reinterpret_cast<const long long*>(table), nb,
                       (long long)fill, reinterpret_cast<long long*>(out));
  return hipGetLastError();
}

hipError_t launch_quantize(const double* lonlat, int64_t n, int32_t* xy, int num_cu,
                           hipStream_t stream) {
  long long blocks = (n + 255) / 256;
  const long long cap = (long long)num_cu * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)blocks), dim3(256), 0, stream,
                     reinterpret_cast<const double2*>(lonlat), (long long)n,
                     reinterpret_cast<int2*>(xy));
  return hipGetLastError();
}

}  // namespace bm
