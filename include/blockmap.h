/*
 * blockmap -- map points onto the blocks of a polygon partition on an AMD
 * Instinct MI355X (gfx950).
 *
 * The operation (paper: "Fast Mapping onto Census Blocks", Sec. III and
 * Sec. III-A): for every query point, find the block whose polygon contains
 * it. Candidates are narrowed with a hierarchy of bounding boxes (groups of
 * blocks, groups of groups, ...), and every surviving block is decided with
 * the crossing-number test: the number of times a ray from the point towards
 * +x crosses the block's boundary is odd exactly when the point is inside.
 *
 * Exactness. Coordinates are integers and every decision is exact:
 *   - an edge (a -> b) takes part when exactly one end lies strictly above the
 *     point (a.y > p.y differs from b.y > p.y); horizontal edges never do;
 *   - it counts when it meets the point's horizontal line strictly to the
 *     right of the point, decided with exact 64-bit integer products;
 *   - so a point on a boundary belongs to the block on its right (and, on a
 *     horizontal boundary, to the block above it). In a gap-free partition of
 *     the plane every point lies in exactly one block;
 *   - bounding boxes are half-open, [xmin, xmax) x [ymin, ymax), which never
 *     drops a containing block;
 *   - when several blocks contain a point (overlapping input) the answer is
 *     the smallest block index; when none does it is -1.
 *
 * All entry points return a status code (BM_OK on success); no C++ exception
 * crosses this interface. bm_last_error() gives a description of the last
 * failure on the calling thread.
 */
#ifndef BLOCKMAP_H
#define BLOCKMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The HIP stream type, declared exactly as the HIP runtime declares it. */
typedef struct ihipStream_t* hipStream_t;

enum {
  BM_OK = 0,
  BM_EINVAL = 1,     /* bad argument: null pointer, negative size, bad descriptor */
  BM_ERANGE = 2,     /* a vertex coordinate outside [0, 2^31 - 1], or an index too large */
  BM_ENOMEM = 3,     /* a device or host allocation failed */
  BM_EHIP = 4,       /* the HIP runtime reported an error */
  BM_EBUSY = 5,      /* the server queue is full */
  BM_ETIMEDOUT = 6,  /* a wait ran out of time */
  BM_EIO = 7         /* a file could not be read or written */
};

/* ------------------------------------------------------------------------ */
/* Index: the blocks and their group hierarchy, resident in device memory.  */
/* ------------------------------------------------------------------------ */

typedef struct bm_index bm_index;

/* Host-side description of a partition and its hierarchy (paper Sec. III-B:
 * state -> county -> block, here any number of group levels).
 *
 *   n_blocks      number of blocks. Block b keeps the index b in every result.
 *                 Blocks plus the groups of all levels: at most 2^26
 *                 (67,108,864) nodes.
 *   vert_off      [n_blocks + 1] int64, vert_off[0] = 0, non-decreasing: ring b
 *                 is verts_xy[2*vert_off[b] .. 2*vert_off[b+1]).
 *   verts_xy      interleaved (x, y) int32 vertices, each coordinate in
 *                 [0, 2^31 - 1]. A ring is closed implicitly from its last
 *                 vertex to its first; a stored closing copy of the first
 *                 vertex is harmless. Every ring has at least 3 and at most
 *                 2^24 vertices.
 *                 Holes or several parts can be joined into one ring by a
 *                 bridge walked once each way (its crossings cancel).
 *   n_levels      number of group levels above the blocks (0 = no hierarchy).
 *   n_groups      [n_levels] group count per level, coarse to fine (each >= 1).
 *   parent        [n_levels] arrays: parent[l][i] in [0, n_groups[l]) is the
 *                 level-l group of entity i of level l+1 (of block i for
 *                 l = n_levels - 1). Groups may be empty. Any grouping gives
 *                 the same result; a spatially tight one is faster. A level
 *                 whose groups hold fewer than 4 entities on average is left
 *                 out of the index (the level above adopts its entities)
 *                 unless a group would then hold more than 256.
 *   keep_all_levels  nonzero: keep every level given, thin ones included
 *                 (each point then passes every level of the hierarchy;
 *                 results are the same either way). Zero-initialise it when
 *                 unused.
 *
 * The descriptor and its arrays are only read during bm_index_create. */
typedef struct {
  int64_t n_blocks;
  const int64_t* vert_off;
  const int32_t* verts_xy;
  int32_t n_levels;
  const int64_t* n_groups;
  const int32_t* const* parent;
  int32_t keep_all_levels;
} bm_index_desc;

/* Validate the descriptor, derive the half-open boxes of every block and
 * group (a group's box is the smallest box holding its children's boxes) and
 * copy everything to the current HIP device. *out receives the handle, owned
 * by the caller until bm_index_destroy. Synchronous.
 * Errors: BM_EINVAL (null pointer, bad sizes or offsets, ring with fewer than
 * 3 or more than 2^24 vertices, parent out of range), BM_ERANGE (coordinate outside
 * [0, 2^31 - 1], more than 2^26 nodes, or slab edge lists of 2^31 or more
 * entries), BM_ENOMEM, BM_EHIP. */
int bm_index_create(const bm_index_desc* desc, bm_index** out);

/* Free the device copy. Null is accepted. The caller must make sure no work
 * that uses the index is still queued on any stream. */
void bm_index_destroy(bm_index* index);

typedef struct {
  int64_t n_blocks;
  int64_t n_vertices;      /* ring vertices as given */
  int64_t n_nodes;         /* groups on all levels plus blocks */
  int64_t device_bytes;    /* device memory held by the index */
  int32_t n_levels;        /* group levels kept in the index */
  int32_t device;          /* HIP device ordinal holding the index */
  int64_t top_groups;      /* entities on the coarsest level */
  int32_t sort_bins;       /* bins of the spatial pre-sort (bm_tuning.presort) */
  int32_t sort_adaptive;   /* 1: those bins adapt to where the blocks are dense (an index over
                              256 MB); 0: a uniform 32 x 32 or 64 x 64 grid of bins */
} bm_index_info;

int bm_index_get_info(const bm_index* index, bm_index_info* info);

/* Save / load the index as a flat binary file (the host-side arrays that
 * bm_index_create derives), so a large index need not be rebuilt.
 * bm_index_load places the index on the current device.
 * Errors: BM_EINVAL, BM_EIO (open/read/write failure or a malformed file),
 * BM_ENOMEM, BM_EHIP. */
int bm_index_save(const bm_index* index, const char* path);
int bm_index_load(const char* path, bm_index** out);

/* Build the index on the host only and write it to `path` in the format of
 * bm_index_save (no device needed; load it later with bm_index_load).
 * Errors: those of bm_index_create except BM_EHIP, and BM_EIO. */
int bm_index_build_file(const bm_index_desc* desc, const char* path);

/* ------------------------------------------------------------------------ */
/* Plain mapping.                                                           */
/* ------------------------------------------------------------------------ */

/* out_ids[i] = smallest block index whose ring contains point i, or -1.
 *   xy       device pointer, n interleaved (x, y) int32 points (any values).
 *   out_ids  device pointer, n int32, written by the call (caller-owned).
 *   stream   HIP stream the work is queued on (0 = default stream).
 * Asynchronous: results are ready when the stream reaches this point. The
 * index must live on the current device. n == 0 is a no-op. xy and out_ids
 * must not overlap. The index is read-only, so calls on different streams may
 * run at the same time. Calls of 2^20 points or more use stream-ordered
 * scratch for the spatial pre-sort (see bm_tuning.presort).
 * Errors: BM_EINVAL (null index, n < 0, null buffers when n > 0, index on
 * another device), BM_EHIP (launch failure). */
int map_points(const bm_index* index, const int32_t* xy, int64_t n, int32_t* out_ids,
               hipStream_t stream);

/* Longitude/latitude doubles (paper Sec. II) to the int32 fixed point the
 * index uses: per axis q = rint(v * 2^22) + 2^30 (rint rounds half to even;
 * the offset is added after rounding, so the result is exact). Resolution
 * 2^-22 degree. NaN, infinities, |lon| > 180 or |lat| > 90 give (-1, -1),
 * which lies outside every block of an index built from quantised vertices.
 *   lonlat  device pointer, n (lon, lat) pairs;  xy  device pointer, n pairs.
 * Asynchronous on stream. Errors: BM_EINVAL, BM_EHIP. */
int bm_quantize_lonlat(const double* lonlat, int64_t n, int32_t* xy, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Launch shape. Never changes results, only speed.                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int32_t edge_chunk;       /* ring edges per crossing-test work item: 4, 8 or 16 */
  int32_t blocks_per_cu;    /* workgroups per compute unit (1..8), capped at what fits */
  int32_t tile_points;      /* batched form: points per unit of work (multiple of 64, <= 2^20) */
  int32_t presort;          /* 1: a call of at least 2^20 points is first sorted along a Z-curve
                               (Morton bins over the index, refined by Morton sub-cells: a
                               1024 x 1024 grid, or, for an index over 256 MB, 4,096 bins that
                               are smaller where the blocks are, each cut into 64 x 64) in
                               chunks of 2^24 points (2^26 for an index over 256 MB), so that
                               nearby points are mapped together, and the results, computed in
                               sorted order, are put back in the points' order; it uses
                               20 bytes of stream-ordered device scratch (hipMallocAsync) per
                               point, for at most 2^27 points at a time (2.7 GB). 0: off */
} bm_tuning;

/* Out-of-range fields are replaced by their defaults. */

/* Fill *t with the defaults used when a tuning pointer is null. */
int bm_tuning_default(bm_tuning* t);

/* map_points without allocating, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no hipMalloc, hipFree or other allocation. Same
 * arguments and results as map_points; n may be at most 2^22 (4,194,304)
 * points, else BM_ERANGE. A call of 2^20 points or more is pre-sorted through
 * a fixed 81 MiB array of device memory that every device the library runs
 * on holds until the process ends; the array is shared by all calls on a
 * device and keeps the last call's contents (each call clears what it needs
 * cleared). Calls that overlap on one device (other streams, other threads)
 * race on it: order them on one stream, or use map_points.
 * Errors: BM_EINVAL (as map_points), BM_ERANGE (n > 2^22), BM_EHIP. */
int map_points_noalloc(const bm_index* index, const int32_t* xy, int64_t n, int32_t* out_ids,
                       hipStream_t stream);

/* As map_points, with an explicit launch shape (t may be null). */
int map_points_tuned(const bm_index* index, const int32_t* xy, int64_t n, int32_t* out_ids,
                     const bm_tuning* t, hipStream_t stream);

/* Pick a launch shape by timing candidates on a sample of points (device
 * pointer, n >= 64) with this index: edge_chunk and blocks_per_cu (6 shapes)
 * and presort (on or off, for samples of 2^20 points or more) by timing
 * map_points_tuned on the sample; then tile_points (3 sizes) by timing the
 * batched form on the sample cut into 16 batches. The batched form uses
 * edge_chunk, blocks_per_cu and tile_points; it never pre-sorts (its batches
 * are mapped in their own order), so presort only matters to
 * map_points_tuned. The choice is cached per (device architecture, index
 * shape, size class) in the file named by the environment variable
 * BM_TUNE_CACHE (default $HOME/.cache/blockmap_tune.txt; unreadable or
 * unwritable cache files are ignored). Runs and synchronises on `stream`.
 * Errors: BM_EINVAL, BM_EHIP. */
int bm_autotune(const bm_index* index, const int32_t* sample_xy, int64_t n, bm_tuning* out,
                hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Batched form: many independent point batches of uneven size in one      */
/* persistent launch (the data-parallel split of the paper's Sec. V, on one */
/* device). Results are identical to one map_points call per batch.         */
/* ------------------------------------------------------------------------ */

/* One batch: device pointers to n interleaved (x, y) points and n outputs. */
typedef struct {
  const int32_t* xy;
  int32_t* out_ids;
  int64_t n;
} bm_batch;

/* Map nb batches that lie back to back in one array, with one persistent
 * kernel: batch b is points [batch_off[b], batch_off[b+1]) of xy (device,
 * interleaved (x, y) int32) and its results the same range of out_ids
 * (device int32). batch_off is a DEVICE array of nb + 1 int64; a batch whose
 * offsets decrease or start below 0 is skipped. The result equals one
 * map_points call per batch, and so map_points over the concatenation. Work
 * units of tuning->tile_points points are taken from a device counter by the
 * resident waves, so uneven batches balance. Uses 32 * nb + 24 bytes of
 * stream-ordered scratch (hipMallocAsync / hipFreeAsync on `stream`) for the
 * descriptor table and the work-unit prefix. Asynchronous.
 * Errors: BM_EINVAL (null pointer, nb < 0), BM_ENOMEM, BM_EHIP. */
int bm_map_batches(const bm_index* index, const int32_t* xy, const int64_t* batch_off, int64_t nb,
                   int32_t* out_ids, const bm_tuning* t, hipStream_t stream);

/* The same over batches anywhere in memory: `batches` is a DEVICE array of nb
 * descriptors (the caller keeps it alive until the stream has passed this
 * call); their pointers must be valid device pointers for n points, and a
 * descriptor with n <= 0 is skipped. Batches must not overlap each other's
 * outputs. Uses nb + 3 int64 of stream-ordered scratch.
 * Errors: BM_EINVAL (null index or table, nb < 0), BM_ENOMEM, BM_EHIP. */
int bm_map_batch_table(const bm_index* index, const bm_batch* batches, int64_t nb, const bm_tuning* t,
                       hipStream_t stream);

/* Both forms as captured HIP graphs, for repeated use. The plan owns a
 * device descriptor table for up to max_batches batches, the work-unit
 * prefix and pinned staging copies; two graphs are captured once at creation
 * and replayed by the run calls, which only rewrite a staging copy:
 *   bm_batch_plan_run: the offset form (xy, batch_off and out_ids as for
 *     bm_map_batches; nb <= max_batches). The graph uploads a 32-byte header
 *     (nb and the three pointers), writes the descriptor table on the device,
 *     takes the prefix and runs the persistent kernel. A batch whose offsets
 *     decrease, start below 0 or end beyond max_points is skipped, so a run
 *     never touches xy or out_ids past max_points points.
 *   bm_batch_plan_run_table: the descriptor form with the table given on the
 *     HOST (checked there: n >= 0, non-null pointers when n > 0); the graph
 *     uploads the whole table.
 * A run waits for the previous run of the same plan to finish before
 * touching the staging copies; different plans are independent.
 * Errors: BM_EINVAL (null plan, nb outside [0, max_batches], bad
 * descriptors, max_points < 0), BM_ENOMEM, BM_EHIP. */
typedef struct bm_batch_plan bm_batch_plan;

int bm_batch_plan_create(const bm_index* index, int64_t max_points, int64_t max_batches, const bm_tuning* t,
                         bm_batch_plan** out);
int bm_batch_plan_run(bm_batch_plan* plan, const int32_t* xy, const int64_t* batch_off, int64_t nb,
                      int32_t* out_ids, hipStream_t stream);
int bm_batch_plan_run_table(bm_batch_plan* plan, const bm_batch* batches, int64_t nb, hipStream_t stream);
void bm_batch_plan_destroy(bm_batch_plan* plan);

/* ------------------------------------------------------------------------ */
/* Served form: a request loop with continuous batching over a resident     */
/* index. Requests (host buffers) queue FIFO; a dispatcher thread packs the  */
/* head of the queue into a device batch as soon as a batch slot and enough  */
/* pool memory are free (admission by memory), copies it in, maps it and     */
/* copies it back on one of several streams, so batches overlap on the      */
/* device; a completion thread scatters results and frees memory. Results    */
/* are those of map_points on each request alone.                           */
/* ------------------------------------------------------------------------ */

typedef struct bm_server bm_server;

enum {
  BM_SERVER_FAIL_ALLOC = 1,     /* force the pool allocation to fail (failure-path tests) */
  BM_SERVER_ONE_PER_BATCH = 2   /* no coalescing: one request piece per batch (with one slot and
                                   one stream this is the plain kernel request by request) */
};

typedef struct {
  int64_t mem_budget_bytes;  /* device pool (and pinned host pool) for in-flight batches; each
                                point in flight takes 12 bytes (+256-byte alignment per batch),
                                and a batch of 2^20 points or more also its pre-sort scratch
                                (about 20 bytes per point more) */
  int64_t max_batch_points;  /* points per device batch; larger requests are split */
  int32_t max_slots;         /* batches in flight at once (1..64) */
  int32_t n_streams;         /* streams the batches are spread over (1..16) */
  int32_t coalesce_us;       /* a batch smaller than max_batch_points may wait this long for
                                more arrivals (0 = dispatch at once) */
  int32_t queue_capacity;    /* queued request pieces before submit returns BM_EBUSY */
  int32_t flags;             /* BM_SERVER_* */
  bm_tuning tuning;          /* launch shape of the mapping kernel */
  int32_t copy_threads;      /* host threads (1..64, the server's own two included) that pack
                                request pieces into the pinned pool and results out of it */
  int64_t direct_min_points; /* pieces of at least this many points whose caller buffers are
                                page-locked are copied by DMA directly, not packed (>= 1) */
} bm_server_cfg;

int bm_server_cfg_default(bm_server_cfg* cfg);

/* Allocates the pools, streams and two threads. The index must live on the
 * current device and outlive the server. The server allocates nothing per
 * batch: a batch's points, results and mapping scratch all come from the
 * pool. After a device error it fails the queued requests and dispatches no
 * more (submit then returns that error).
 * Errors: BM_EINVAL (budget below one full batch, fields out of range),
 * BM_ENOMEM, BM_EHIP. */
int bm_server_create(const bm_index* index, const bm_server_cfg* cfg, bm_server** out);

/* Queue a request: n points at host address xy, results to host address out
 * (both must stay valid until the request is waited for). *ticket identifies
 * it. Buffers in page-locked memory (hipHostMalloc) are copied by DMA
 * directly; others are packed through the server's pinned pool. Returns BM_EBUSY when the queue is full (nothing is queued then), or the
 * error of an earlier device failure. */
int bm_server_submit(bm_server* srv, const int32_t* xy, int64_t n, int32_t* out, uint64_t* ticket);

/* Wait for a request (timeout_us < 0: no limit) until every piece of it has
 * been retired, so no copy into its buffers is pending afterwards. BM_OK, or
 * the error of a failed piece, consumes the ticket; BM_ETIMEDOUT leaves it
 * pending; an unknown ticket gives BM_EINVAL. */
int bm_server_wait(bm_server* srv, uint64_t ticket, int64_t timeout_us);

typedef struct {
  int64_t completed;          /* requests finished */
  int64_t points;             /* their points */
  int64_t batches;            /* device batches dispatched */
  int64_t rejected;           /* submits refused with BM_EBUSY */
  double mean_requests_per_batch;
  double p50_us, p99_us, mean_us, max_us;  /* submit-to-completion latency */
  double points_per_s;        /* points / (last completion - first submit) */
} bm_server_stats_t;

int bm_server_stats(bm_server* srv, bm_server_stats_t* out);
/* The same (an earlier name). */
int bm_server_get_stats(bm_server* srv, bm_server_stats_t* out);
int bm_server_reset_stats(bm_server* srv);

/* Load harness: submit reqs[i] at arrival_us[i] microseconds after the call
 * (busy-waiting for the time; retrying while the queue is full), then wait
 * for all of them. Latencies are in bm_server_get_stats. */
typedef struct {
  const int32_t* xy;
  int32_t* out_ids;
  int64_t n;
} bm_request;

int bm_server_run_trace(bm_server* srv, const bm_request* reqs, int64_t nreq, const double* arrival_us);

/* Stop the threads after the batches in flight finish; requests still queued
 * are dropped. No call on the server may be running. */
void bm_server_destroy(bm_server* srv);

/* Measurement aid: as map_points_tuned, but with HIP events recorded on
 * `stream` around each launch of the mapping kernel and each phase of the
 * spatial pre-sort (the sort passes before a mapping launch, and the passes
 * after it that put the results, computed in sorted order, back in the
 * points' order); waits for the stream and returns the summed durations. */
typedef struct {
  double map_ms;          /* mapping-kernel launches */
  double sort_ms;         /* sort passes (0 when not sorted) */
  int32_t map_launches;
  int32_t sort_launches;  /* rounds of sort passes */
  double unsort_ms;       /* passes that put the results in the points' order */
  int32_t unsort_launches;
} bm_launch_times;

int map_points_timed(const bm_index* index, const int32_t* xy, int64_t n, int32_t* out_ids,
                     const bm_tuning* t, hipStream_t stream, bm_launch_times* times);

/* ---- Cell cover: the fast approach (paper Sec. IV, true-hit filtering) ----
 *
 * A cover cuts the plane into non-overlapping square cells of a quadtree over
 * the index's root box and indexes them with a radix trie that consumes four
 * quadtree levels (4 bits of each coordinate, a 256-way node) per trie level,
 * as the paper's F4 trie does; the last trie level takes the remaining 1-4
 * quadtree levels. A cell that no block edge enters lies wholly inside one
 * block (an interior cell, which stores that block) or outside every block
 * (empty); a point there gets its answer from the trie alone. Cells an edge
 * enters are split down to side 2^cell_log2 and become boundary cells, which
 * list every block that can hold one of their points and store the answer at
 * their centre.
 *
 * Exact mode returns exactly what map_points returns. Approximate mode skips
 * the crossing test: a point in a boundary cell gets the exact answer at the
 * centre of that cell, so every answer is exact at the point itself or at a
 * point no farther than 2^(cell_log2 - 1) * sqrt(2) from it (the paper's
 * user-defined precision); points in interior and empty cells are exact. */
typedef struct bm_cover bm_cover;

typedef struct {
  int32_t cell_log2; /* side of the finest (boundary) cells = 2^cell_log2 coordinate units, 1..30;
                        0 = automatic: about 1/64 of the median block's box side, but no finer
                        than the total ring length / 2^26 (bounds the number of boundary cells) */
  int32_t threads;   /* host threads for the build; 0 = all */
} bm_cover_cfg;

typedef struct {
  int32_t origin_x, origin_y; /* low corner of the covered square */
  int32_t log2_side;          /* the square's side is 2^log2_side */
  int32_t trie_levels;
  int32_t last_level_bits;    /* quadtree levels in the last trie level (the others: 4) */
  int32_t cell_log2;          /* finest cell side 2^cell_log2 */
  int64_t trie_entries;       /* 4-byte entries over all trie nodes */
  int64_t interior_entries, node_entries, boundary_cells, empty_entries;
  int64_t cell_leaves;        /* listed blocks over all boundary cells */
  int64_t device_bytes;       /* device memory held by the cover (the index not counted) */
  double build_seconds;       /* host build time, including the copy of the index to the host */
} bm_cover_info;

/* Build the cover of `index` on the host (threads as configured; cfg may be
 * null) and copy it to the index's device. Synchronous. `desc` must be the
 * descriptor the index was built from (only its rings are read, during the
 * call): the index keeps just the edges that can cross a ray, and a cell's
 * uniformity depends on every edge, horizontal ones too. The cover refers to
 * the index for the crossing tests: the index must outlive it.
 * Errors: BM_EINVAL (null pointer, cell_log2 out of range, a descriptor whose
 * rings do not match the index), BM_ERANGE (more than 2^30 trie entries or
 * cells: raise cell_log2), BM_ENOMEM, BM_EHIP. */
int bm_cover_create(const bm_index* index, const bm_index_desc* desc, const bm_cover_cfg* cfg, bm_cover** out);

/* Free the cover's device memory (null accepted); no queued work may use it. */
void bm_cover_destroy(bm_cover* cover);

int bm_cover_get_info(const bm_cover* cover, bm_cover_info* info);

/* Host-only: build the index and its cover from a descriptor and write the
 * cover to `path` ("BMCOV001", then the shape as 6 int32 (origin x, y, log2
 * side, trie levels, last-level bits, cell_log2), 4 int64 entry counts
 * (interior, node, boundary, empty), and the arrays trie entries (uint32),
 * cell offsets (uint32), cell blocks (uint32 leaf positions in the index
 * file's leaf order) and cell centre answers (int32), each as an int64
 * length followed by the data). No GPU is needed. */
int bm_cover_build_file(const bm_index_desc* desc, const bm_cover_cfg* cfg, const char* path);

/* Map n points (device xy, as map_points) through the cover into out_ids
 * (device, n int32). approx = 0: exact, identical to map_points; approx = 1:
 * boundary cells answer with their centre's block (see above). Asynchronous
 * on `stream`; `stream` must belong to the cover's device.
 * Errors: BM_EINVAL (null pointer, n < 0, approx not 0/1, or another device
 * current than the cover's), BM_EHIP. */
int map_points_cover(const bm_cover* cover, const int32_t* xy, int64_t n, int32_t* out_ids, int32_t approx,
                     hipStream_t stream);

/* Points per block: the count the mapping feeds into the paper's purpose,
 * merging demographic data by block (Sec. I-II). For ids[0..n) (device, as
 * written by map_points), adds to counts[b] (device, n_blocks + 1 uint64) the
 * number of ids equal to b, for b in [0, n_blocks), and to counts[n_blocks]
 * the number of the others (-1: no block). Counts accumulate: clear them first
 * for a fresh count. Asynchronous on `stream`. Calls of 2^20 ids or more use
 * stream-ordered scratch (hipMallocAsync) of about 4 bytes per id plus
 * 32 KiB per 8192 blocks per slice.
 * Errors: BM_EINVAL (null buffer, n < 0, n_blocks outside [0, 2^31 - 2]), BM_EHIP. */
int bm_count_per_block(const int32_t* ids, int64_t n, int64_t n_blocks, uint64_t* counts, hipStream_t stream);

/* Per-point join of a per-block attribute: App. A ends by giving each point
 * the FIPS code of its block, the key on which the census tables of Sec. I-II
 * are merged. For ids[0..n) (device, as written by map_points) and table
 * (device, n_blocks int64, e.g. numeric block FIPS codes), writes out[i] =
 * table[ids[i]] when ids[i] is in [0, n_blocks), else fill (device, n int64,
 * caller-owned; must not overlap ids or table). Asynchronous on `stream`; no
 * scratch. table may be null when n_blocks = 0.
 * Errors: BM_EINVAL (null buffer, n < 0, n_blocks outside [0, 2^31 - 2]), BM_EHIP. */
int bm_join_per_block(const int32_t* ids, int64_t n, const int64_t* table, int64_t n_blocks, int64_t fill,
                      int64_t* out, hipStream_t stream);

/* Error text for the last failing call on this thread ("" if none). */
const char* bm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BLOCKMAP_H */
