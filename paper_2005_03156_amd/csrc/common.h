// Internal declarations shared by the blockmap host code and kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include <string>

#include "../../include/blockmap.h"

namespace bm {

// Device view of an index. Every entity of every level is a node with a
// global id: level 0 occupies [0, g0), the next level follows, and the
// blocks ("leaves") come last, [leaf_base, leaf_base + n_leaves). The
// children of a group node form one contiguous id range, and consecutive
// groups own consecutive ranges.
struct KIndex {
  const int4* box;           // [n_nodes] half-open (xmin, xmax, ymin, ymax)
  // [leaf_base] per group node: (first child, end of children, offset of the
  // group's slot table in `slot_mask` or -1, packed table shape: log2 of the
  // slot count | x shift << 8 | y shift << 16)
  const int4* child;
  const unsigned long long* slot_mask;  // per table: S x-slot masks, then S y-slot masks
  const int32_t* parent;     // [n_nodes] parent node, -1 on level 0
  const int64_t* vert_off;   // [n_leaves + 1] ring offsets into verts (leaf order)
  const int32_t* leaf_id;    // [n_leaves] block index of each leaf as given by the caller
  const int2* verts;         // rings, each closed by a stored copy of its first vertex
  int32_t n_levels;          // group levels above the leaves
  int32_t g0;                // nodes on level 0
  int32_t leaf_base;         // first leaf node id
  int32_t n_leaves;
  int4 root_child;           // the virtual root: its children are level 0
  int4 root_box;             // union of the level-0 boxes
};

// One batch of the batched form, as laid out in device memory (identical to
// the public bm_batch).
struct BatchEntry {
  const int32_t* xy;
  int32_t* out;
  int64_t n;
};

struct Tuning {
  int edge_chunk;     // 4, 8 or 16
  int blocks_per_cu;  // 1..8
  int tile_points;    // batched form: points per unit of work taken from the counter (multiple of 64)
};

Tuning tuning_from(const bm_tuning* t);

// Launchers (map_kernels.hip). Return hipSuccess or the launch error.
hipError_t launch_map(const KIndex& ix, const int32_t* xy, int64_t n, int32_t* out,
                      const Tuning& t, int num_cu, hipStream_t stream);
// Batched form: meta must hold nb + 3 int64 (nb, work counter, prefix).
hipError_t launch_batches(const KIndex& ix, const long long* hdr, long long nb, const BatchEntry* tab,
                          long long* meta, const Tuning& t, int num_cu, hipStream_t stream);
hipError_t launch_quantize(const double* lonlat, int64_t n, int32_t* xy, int num_cu,
                           hipStream_t stream);

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
  int64_t n_verts_stored;
  int64_t n_masks;
  int64_t bytes;
  void* allocs[12];
  int n_allocs;
};
