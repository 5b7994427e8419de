// Internal declarations shared by the blockmap host code and kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/blockmap.h"

namespace bm {

// Device view of an index. Every entity of every level is a node with a
// global id: level 0 occupies [0, g0), the next level follows, and the
// blocks ("leaves") come last, [leaf_base, leaf_base + n_leaves). The
// children of a group node form one contiguous id range, and consecutive
// groups own consecutive ranges.
//
// Records are sized and aligned so that each sits within one cache line: a
// group's box beside its child record, a leaf's box beside what the crossing
// test needs. Filter steps test leaf boxes from a compact copy (16 bytes per
// leaf, after the group records; KIndex::lbox_off).
struct alignas(32) GroupRec {
  int4 box;    // half-open (xmin, xmax, ymin, ymax), the union of the children's boxes
  int4 child;  // (first child, end of children, offset of the slot table in
               // slot_mask or -1, log2 slot count | x shift << 8 | y shift << 16 |
               // words per slot row << 24)
};

// A block's ring is reached through y-slabs: its y-extent [ymin, ymax) is cut
// into K = 2^logK slabs of height 2^sh, and slab s lists, as ready vertex
// pairs (a.x, a.y, b.x, b.y), the ring edges whose y-span overlaps it.
//
// The record also holds a map of the block's box cut into 16 x 16 cells of
// 2^sx x 2^sy units (the smallest power-of-two sides with 16 cells covering
// each side; kLeafCells, cell_shift): 2 bits per cell, row r in cell[r], column
// c in bits 2c..2c+1. A cell whose closed rectangle meets no ring edge
// (horizontal edges included) gives every point in it the same answer, found
// once at index build: kCellOut (no point of the cell is in the block) or
// kCellIn (every point is); other cells are kCellTest (run the crossing test).
// A (block, point) pair whose point lies in an In or Out cell needs none of
// the block's edges.
constexpr int kLeafCells = 16;
constexpr unsigned kCellOut = 0, kCellIn = 1, kCellTest = 2;
struct alignas(128) LeafRec {
  int4 box;
  long long ent;       // index in `ent` of the leaf's first listed edge
  int leaf_id;         // block index as given by the caller
  int packed;          // sh | logK << 8 | kLeafExtOff when the offsets are not inline
  unsigned char off[32];  // inline slab offsets (K + 1 <= 32, all <= 255), relative to ent
  uint32_t cell[kLeafCells];  // cell classes, 2 bits per cell
};
constexpr int kLeafExtOff = 1 << 24;  // offsets are K + 1 uint32 stored in the int4s before ent
static_assert(sizeof(GroupRec) == 32 && sizeof(LeafRec) == 128, "record sizes");
static_assert(offsetof(LeafRec, ent) == 16 && offsetof(LeafRec, leaf_id) == 24 && offsetof(LeafRec, packed) == 28,
              "the kernels read ent, leaf_id and packed as one int4");
static_assert(offsetof(LeafRec, cell) == 64, "cell map in the record's second half");

// Shift of the cell side along an axis of extent w >= 1 units: the smallest
// s >= 0 with kLeafCells << s >= w (the same on host and device).
__host__ __device__ inline int cell_shift(const unsigned w) {
  const int bits = w > 1u ? 32 - __builtin_clz(w - 1u) : 0;  // ceil(log2 w)
  return bits > 4 ? bits - 4 : 0;
}

// A wavefront maps a tile of 64 * kTilePts points (kTilePts per lane).
// Kernel-side limits: a candidate item packs a node id with the point's slot
// in the tile (kSlotBits), and edge-list positions are 32-bit. The device copy
// of `ent` carries kEntPad zero entries at its end, so a crossing-test chunk
// may load past its list.
#ifndef BM_TILE_PTS
#define BM_TILE_PTS 1
#endif
constexpr int kTilePts = BM_TILE_PTS;
static_assert(kTilePts == 1 || kTilePts == 2 || kTilePts == 4, "1, 2 or 4 points per lane");
constexpr int kSlotBits = kTilePts == 4 ? 8 : kTilePts == 2 ? 7 : 6;
constexpr long long kMaxNodes = 1ll << (32 - kSlotBits);
constexpr long long kMaxEnt = (1ll << 31) - 64;
constexpr long long kMaxSlotWords = 1ll << 29;    // slot-table words (byte offsets below 2^32)
constexpr int kEntPad = 16;

// Adaptive sort bins of a large index (built in index.cpp, used by the
// spatial sort of map_kernels.hip): a 32 x 32 grid of coarse cells over the
// square of side 2^log_side whose low corner is org; coarse cell c is cut
// into a 2^d x 2^d grid of bins, d = 0..kSortMaxDepth chosen so that the bins
// hold about equally many blocks (by box centre), kSortMapBins bins at most,
// numbered along a Z-curve (coarse cells in Z-order, the bins of a cell in
// Z-order). cell[c] = first bin | d << 16; sq[bin] = (x0, y0, log side, 0) of
// the bin's square, as offsets from org.
constexpr int kSortCoarseBits = 5;
constexpr int kSortCells = 1 << (2 * kSortCoarseBits);
constexpr int kSortMapBins = 4096;
constexpr int kSortMaxDepth = 6;
struct SortMap {
  const uint32_t* cell;  // [kSortCells]; null: uniform bins
  const int4* sq;        // [kSortMapBins]
  int2 org;
  int32_t log_side;      // >= kSortCoarseBits + kSortMaxDepth + 6: every bin square is >= 64 wide
  int32_t n_bins;        // bins in use (host side)
};

struct KIndex {
  const GroupRec* grp;        // [leaf_base]
  const LeafRec* leaf;        // [n_leaves]
  const int4* ent;            // slab edge lists (and out-of-line slab offsets)
  const unsigned long long* slot_mask;  // per table: S x-slot masks, then S y-slot masks
  const int32_t* parent;      // [n_nodes] parent node, -1 on level 0 (fallback walk)
  int32_t n_levels;           // group levels above the leaves
  int32_t g0;                 // nodes on level 0
  int32_t leaf_base;          // first leaf node id
  int32_t n_leaves;
  int4 root_child;            // the virtual root: its children are level 0
  int4 root_box;              // union of the level-0 boxes
  uint32_t lbox_off;          // bytes from grp to the leaf boxes (int4 per leaf): the group
                              // records and the leaf boxes share one allocation below 2^31
                              // bytes, so 32-bit offsets reach every box a filter step tests
  long long presort_chunk;    // points per spatial-sort chunk (host side)
  int32_t presort_bin_bits;   // bins per axis of the sort: 2^5 or 2^6 (host side)
  SortMap sort_map;           // with 2^6: the adaptive bins, when the extent allows them
};

// Cell cover (cover.cpp): a radix trie over non-overlapping square cells of
// the plane, origin (ox, oy), side 2^log_side. Trie level t consumes `bits`
// quadtree levels (4, the last level last_bits), i.e. a node of 4^bits entries
// indexed by (x digit | y digit << bits). An entry is an interior cell (tag 0,
// payload = block index), a child node (tag 1, payload = the child's first
// entry), a boundary cell (tag 2, payload = cell number) or empty (all ones:
// outside every block).
struct CoverShape {
  int32_t ox, oy;
  int32_t log_side;
  int32_t n_levels;
  int32_t last_bits;
  int32_t cell_log2;  // side of the finest cells: log_side - 4 * (n_levels - 1) - last_bits
};
constexpr uint32_t kCoverInterior = 0u << 30, kCoverNode = 1u << 30, kCoverBoundary = 2u << 30;
constexpr uint32_t kCoverEmpty = 0xFFFFFFFFu, kCoverPayload = (1u << 30) - 1;

struct KCover {
  const uint32_t* ent;        // trie entries, root node first
  const uint32_t* cell_off;   // [cells + 1]: boundary cell c lists cell_leaf[cell_off[c] .. cell_off[c+1])
  const uint32_t* cell_leaf;  // leaf positions in the index's leaf array
  const int32_t* cell_rep;    // per boundary cell: the answer at its centre (approximate mode)
  int32_t ox, oy, log_side, n_levels, last_bits;
};

// One batch of the batched form, as laid out in device memory (identical to
// the public bm_batch).
struct BatchEntry {
  const int32_t* xy;
  int32_t* out;
  int64_t n;
};

// Header of an offset-form batched call as the graph form stages it in
// device memory: batch b is points [off[b], off[b+1]) of xy, results into the
// same range of out. nb comes first, where the prefix kernel reads it.
struct OffsetHeader {
  long long nb;
  const int32_t* xy;
  int32_t* out;
  const long long* off;
};

// Calls of at least kPresortMin points are spatially sorted in chunks of
// KIndex::presort_chunk points before mapping (when Tuning::presort is set),
// up to kPresortSuper points (all their chunks) per round of sort passes.
// Each chunk is sorted on its own, so a chunk is one pass over the plane in
// Z-order. The chunk is 2^24 points while the index fits the 256 MB
// last-level cache (220,900-block grid, 100M points per call: 5.32 / 5.23 /
// 5.26 ms with 2^23 / 2^24 / 2^25-point chunks); above that each chunk reads
// the part of the index it touches from HBM, and 2^26-point chunks read it
// fewer times per point (8M-block quadtree: 10.1 -> 8.4 ms per 2^26 points).
// The sort's bin grid has 32 x 32 bins for the smaller indexes (each bin then
// re-sorted by 32 x 32 sub-cells in pieces of 4,096 points; 2,048 / 8,192
// points: 5.36 / 5.33 ms) and 4,096 bins (64 x 64 sub-cells) for the
// larger ones: a 64 x 64 grid (the quadtree: 7.58 ms per 2^26 points, against
// 8.63 with 32 x 32 bins), or the adaptive bins of SortMap when the index's
// extent allows them.
constexpr long long kPresortMin = 1 << 20;
constexpr long long kPresortChunk = 1 << 24;
constexpr long long kPresortChunkBigIndex = 1 << 26;
constexpr long long kPresortBigIndex = 256ll << 20;
constexpr long long kPresortSuper = 1 << 27;

struct Tuning {
  int edge_chunk;     // 4, 8 or 16
  int blocks_per_cu;  // 1..8
  int tile_points;    // batched form: points per unit of work taken from the counter (multiple of 64)
  int presort;        // 0 / 1: spatial sort of large calls (uses stream-ordered scratch)
};

Tuning tuning_from(const bm_tuning* t);

// Optional event marks around the launches of one mapping call: tag 0 opens
// and tag 1 closes a mapping-kernel launch; tag 2 opens a round's sort
// passes and tag 3 its unsort passes (each closed by the next mark); tag 4
// ends the call.
struct LaunchTimer {
  static constexpr int kMax = 1024;
  hipEvent_t ev[kMax];
  int tag[kMax];
  int n = 0;
};

// Launchers (map_kernels.hip). Return hipSuccess or the launch error.
// launch_map takes its pre-sort scratch from stream-ordered memory, or, when
// ws is given, from the ws_bytes there (never allocating; with less than
// map_scratch_bytes it sorts fewer points per round, or none).
hipError_t launch_map(const KIndex& ix, const int32_t* xy, int64_t n, int32_t* out,
                      const Tuning& t, int num_cu, hipStream_t stream, LaunchTimer* timer = nullptr,
                      void* ws = nullptr, size_t ws_bytes = 0);
// Scratch bytes a call of n points uses at full speed (0 when it is not
// pre-sorted).
size_t map_scratch_bytes(const KIndex& ix, int64_t n, const Tuning& t);
// Offset form of the batched call: writes the descriptor table of nb batches
// (from hdr when given, else from the arguments) into tab; max_nb bounds nb
// (the launch shape); max_points < 0: no bound on the offsets.
hipError_t launch_batch_offsets(const OffsetHeader* hdr, long long nb, const int32_t* xy, int32_t* out,
                                const int64_t* off, long long max_points, long long max_nb, BatchEntry* tab,
                                int num_cu, hipStream_t stream);
// Batched form: meta must hold nb + 3 int64 (nb, work counter, prefix).
hipError_t launch_batches(const KIndex& ix, const long long* hdr, long long nb, const BatchEntry* tab,
                          long long* meta, const Tuning& t, int num_cu, hipStream_t stream);
hipError_t launch_quantize(const double* lonlat, int64_t n, int32_t* xy, int num_cu,
                           hipStream_t stream);
// Per-point join: out[i] = table[ids[i]] for ids in [0, nb), else fill.
hipError_t launch_join(const int32_t* ids, int64_t n, const int64_t* table, int32_t nb, int64_t fill, int64_t* out,
                       int num_cu, hipStream_t stream);
// Points per block into counts[0 .. nb] (the last slot: ids outside [0, nb)).
hipError_t launch_count(const int32_t* ids, int64_t n, int32_t nb, unsigned long long* counts, int num_cu,
                        hipStream_t stream);
// Cover form: every point looked up in the cell trie; boundary cells resolved
// by the crossing test over their listed blocks, or (approx) by the cell's
// stored answer.
hipError_t launch_cover(const KIndex& ix, const KCover& cv, const int32_t* xy, int64_t n, int32_t* out,
                        bool approx, const Tuning& t, int num_cu, hipStream_t stream);

// Cover construction and access (cover.cpp).
int cover_create(const bm_index* index, const bm_index_desc* desc, const bm_cover_cfg* cfg, bm_cover** out);
int cover_build_file(const bm_index_desc* desc, const bm_cover_cfg* cfg, const char* path);
void cover_destroy(bm_cover* cv);
const KCover& cover_view(const bm_cover* cv);
const bm_index* cover_index(const bm_cover* cv);
int cover_device(const bm_cover* cv);
const bm_cover_info& cover_info(const bm_cover* cv);

// Thread-local error text + code helper.
int fail(int code, const std::string& msg);
void clear_error();
const char* error_text();

}  // namespace bm

struct bm_index {
  bm::KIndex k;
  int device;
  int num_cu;
  int64_t n_blocks;
  int64_t n_nodes;
  int64_t n_verts;   // ring vertices as given (for reporting)
  int64_t n_masks;
  int64_t n_ent;
  int64_t bytes;
  void* allocs[16];
  int n_allocs;
};
