// C-ABI entry points of libblockmap: argument checks, error text, launches.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <exception>
#include <new>
#include <string>

#include "common.h"
#include "trace.h"

namespace bm {

int index_create(const bm_index_desc* d, bm_index** out);
void index_destroy(bm_index* ix);
int index_save(const bm_index* ix, const char* path);
int index_load(const char* path, bm_index** out);
int index_build_file(const bm_index_desc* d, const char* path);

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void clear_error() { g_err.clear(); }

const char* error_text() { return g_err.c_str(); }

Tuning tuning_from(const bm_tuning* t) {
  Tuning r{4, 8, 2048, 1};
  if (t) {
    if (t->presort == 0 || t->presort == 1) r.presort = t->presort;
    if (t->edge_chunk == 4 || t->edge_chunk == 8 || t->edge_chunk == 16) r.edge_chunk = t->edge_chunk;
    if (t->blocks_per_cu >= 1 && t->blocks_per_cu <= 8) r.blocks_per_cu = t->blocks_per_cu;
    if (t->tile_points >= 64 && t->tile_points <= (1 << 20) && t->tile_points % 64 == 0)
      r.tile_points = t->tile_points;
  }
  return r;
}

static int check_device(const bm_index* ix, const char* who) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(BM_EHIP, std::string(who) + ": hipGetDevice: " + hipGetErrorString(e));
  if (dev != ix->device)
    return fail(BM_EINVAL, std::string(who) + ": the index lives on device " + std::to_string(ix->device) +
                               " but device " + std::to_string(dev) + " is current");
  return BM_OK;
}

}  // namespace bm

using namespace bm;

#define BM_GUARD(who)                                      \
  catch (const std::bad_alloc&) {                          \
    return fail(BM_ENOMEM, std::string(who) + ": out of host memory"); \
  }                                                        \
  catch (const std::exception& ex) {                       \
    return fail(BM_EINVAL, std::string(who) + ": " + ex.what()); \
  }                                                        \
  catch (...) {                                            \
    return fail(BM_EINVAL, std::string(who) + ": unknown error"); \
  }

extern "C" {

__attribute__((visibility("default"))) int bm_index_create(const bm_index_desc* desc, bm_index** out) {
  try {
    const TraceRange trace_range("bm_index_create");
    clear_error();
    return index_create(desc, out);
  }
  BM_GUARD("bm_index_create")
}

__attribute__((visibility("default"))) void bm_index_destroy(bm_index* index) {
  try {
    index_destroy(index);
  } catch (...) {
  }
}

__attribute__((visibility("default"))) int bm_index_get_info(const bm_index* ix, bm_index_info* info) {
  if (!ix || !info) return fail(BM_EINVAL, "bm_index_get_info: null argument");
  info->n_blocks = ix->n_blocks;
  info->n_vertices = ix->n_verts;
  info->n_nodes = ix->n_nodes;
  info->device_bytes = ix->bytes;
  info->n_levels = ix->k.n_levels;
  info->device = ix->device;
  info->top_groups = ix->k.g0;
  info->sort_adaptive = ix->k.sort_map.cell ? 1 : 0;
  info->sort_bins = ix->k.sort_map.cell ? ix->k.sort_map.n_bins : 1 << (2 * ix->k.presort_bin_bits);
  return BM_OK;
}

__attribute__((visibility("default"))) int bm_index_save(const bm_index* index, const char* path) {
  try {
    clear_error();
    return index_save(index, path);
  }
  BM_GUARD("bm_index_save")
}

__attribute__((visibility("default"))) int bm_index_build_file(const bm_index_desc* desc, const char* path) {
  try {
    clear_error();
    return index_build_file(desc, path);
  }
  BM_GUARD("bm_index_build_file")
}

__attribute__((visibility("default"))) int bm_index_load(const char* path, bm_index** out) {
  try {
    const TraceRange trace_range("bm_index_load");
    clear_error();
    return index_load(path, out);
  }
  BM_GUARD("bm_index_load")
}

__attribute__((visibility("default"))) int bm_tuning_default(bm_tuning* t) {
  if (!t) return fail(BM_EINVAL, "bm_tuning_default: null argument");
  const Tuning d = tuning_from(nullptr);
  t->edge_chunk = d.edge_chunk;
  t->blocks_per_cu = d.blocks_per_cu;
  t->tile_points = d.tile_points;
  t->presort = d.presort;
  return BM_OK;
}

__attribute__((visibility("default"))) int map_points_tuned(const bm_index* index, const int32_t* xy, int64_t n,
                                                           int32_t* out_ids, const bm_tuning* t,
                                                           hipStream_t stream) {
  try {
    const TraceRange trace_range("map_points");
    if (!index) return fail(BM_EINVAL, "map_points: null index");
    if (n < 0) return fail(BM_EINVAL, "map_points: n < 0");
    if (n == 0) return BM_OK;
    if (!xy || !out_ids) return fail(BM_EINVAL, "map_points: null buffer");
    int rc = check_device(index, "map_points");
    if (rc != BM_OK) return rc;
    hipError_t e = launch_map(index->k, xy, n, out_ids, tuning_from(t), index->num_cu, stream);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("map_points: launch: ") + hipGetErrorString(e));
    return BM_OK;
  }
  BM_GUARD("map_points")
}

__attribute__((visibility("default"))) int bm_cover_create(const bm_index* index, const bm_index_desc* desc,
                                                          const bm_cover_cfg* cfg, bm_cover** out) {
  try {
    const TraceRange trace_range("bm_cover_create");
    if (index) {
      const int rc = check_device(index, "bm_cover_create");
      if (rc != BM_OK) return rc;
    }
    return cover_create(index, desc, cfg, out);
  }
  BM_GUARD("bm_cover_create")
}

__attribute__((visibility("default"))) void bm_cover_destroy(bm_cover* cover) { cover_destroy(cover); }

__attribute__((visibility("default"))) int bm_cover_get_info(const bm_cover* cover, bm_cover_info* info) {
  if (!cover || !info) return fail(BM_EINVAL, "bm_cover_get_info: null argument");
  *info = cover_info(cover);
  return BM_OK;
}

__attribute__((visibility("default"))) int bm_cover_build_file(const bm_index_desc* desc, const bm_cover_cfg* cfg,
                                                              const char* path) {
  try {
    return cover_build_file(desc, cfg, path);
  }
  BM_GUARD("bm_cover_build_file")
}

__attribute__((visibility("default"))) int map_points_cover(const bm_cover* cover, const int32_t* xy, int64_t n,
                                                           int32_t* out_ids, int32_t approx, hipStream_t stream) {
  try {
    const TraceRange trace_range("map_points_cover");
    if (!cover) return fail(BM_EINVAL, "map_points_cover: null cover");
    if (n < 0) return fail(BM_EINVAL, "map_points_cover: n < 0");
    if (approx != 0 && approx != 1) return fail(BM_EINVAL, "map_points_cover: approx must be 0 or 1");
    if (n == 0) return BM_OK;
    if (!xy || !out_ids) return fail(BM_EINVAL, "map_points_cover: null buffer");
    const bm_index* index = cover_index(cover);
    int rc = check_device(index, "map_points_cover");
    if (rc != BM_OK) return rc;
    hipError_t e = launch_cover(index->k, cover_view(cover), xy, n, out_ids, approx != 0, tuning_from(nullptr),
                                index->num_cu, stream);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("map_points_cover: launch: ") + hipGetErrorString(e));
    return BM_OK;
  }
  BM_GUARD("map_points_cover")
}

__attribute__((visibility("default"))) int bm_count_per_block(const int32_t* ids, int64_t n, int64_t n_blocks,
                                                             uint64_t* counts, hipStream_t stream) {
  try {
    const TraceRange trace_range("bm_count_per_block");
    if (n < 0 || n_blocks < 0 || n_blocks > INT32_MAX - 1) return fail(BM_EINVAL, "bm_count_per_block: bad size");
    if (!counts || (n > 0 && !ids)) return fail(BM_EINVAL, "bm_count_per_block: null buffer");
    if (n == 0) return BM_OK;
    int dev = 0, num_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = launch_count(ids, n, (int32_t)n_blocks, reinterpret_cast<unsigned long long*>(counts),
                                std::max(1, num_cu), stream);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("bm_count_per_block: launch: ") + hipGetErrorString(e));
    return BM_OK;
  }
  BM_GUARD("bm_count_per_block")
}

__attribute__((visibility("default"))) int bm_join_per_block(const int32_t* ids, int64_t n, const int64_t* table,
                                                            int64_t n_blocks, int64_t fill, int64_t* out,
                                                            hipStream_t stream) {
  try {
    const TraceRange trace_range("bm_join_per_block");
    if (n < 0 || n_blocks < 0 || n_blocks > INT32_MAX - 1) return fail(BM_EINVAL, "bm_join_per_block: bad size");
    if (n > 0 && (!ids || !out || (n_blocks > 0 && !table)))
      return fail(BM_EINVAL, "bm_join_per_block: null buffer");
    if (n == 0) return BM_OK;
    int dev = 0, num_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = launch_join(ids, n, table, (int32_t)n_blocks, fill, out, std::max(1, num_cu), stream);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("bm_join_per_block: launch: ") + hipGetErrorString(e));
    return BM_OK;
  }
  BM_GUARD("bm_join_per_block")
}

__attribute__((visibility("default"))) int map_points_timed(const bm_index* index, const int32_t* xy, int64_t n,
                                                           int32_t* out_ids, const bm_tuning* t, hipStream_t stream,
                                                           bm_launch_times* times) {
  try {
    const TraceRange trace_range("map_points_timed");
    if (!index || !times) return fail(BM_EINVAL, "map_points_timed: null argument");
    if (n < 0) return fail(BM_EINVAL, "map_points_timed: n < 0");
    if (n > 0 && (!xy || !out_ids)) return fail(BM_EINVAL, "map_points_timed: null buffer");
    int rc = check_device(index, "map_points_timed");
    if (rc != BM_OK) return rc;
    LaunchTimer* tm = new (std::nothrow) LaunchTimer();
    if (!tm) return fail(BM_ENOMEM, "map_points_timed: out of host memory");
    hipError_t e = hipSuccess;
    int made = 0;
    for (; made < LaunchTimer::kMax && e == hipSuccess; ++made) e = hipEventCreate(&tm->ev[made]);
    if (e == hipSuccess && n > 0) e = launch_map(index->k, xy, n, out_ids, tuning_from(t), index->num_cu, stream, tm);
    if (e == hipSuccess && tm->n > 0) e = hipEventSynchronize(tm->ev[tm->n - 1]);
    double map_ms = 0, sort_ms = 0, unsort_ms = 0;
    int maps = 0, sorts = 0, unsorts = 0;
    for (int i = 0; e == hipSuccess && i + 1 < tm->n; ++i) {
      float ms = 0;
      e = hipEventElapsedTime(&ms, tm->ev[i], tm->ev[i + 1]);
      if (tm->tag[i] == 0 && tm->tag[i + 1] == 1) { map_ms += ms; ++maps; }
      if (tm->tag[i] == 2) { sort_ms += ms; ++sorts; }
      if (tm->tag[i] == 3) { unsort_ms += ms; ++unsorts; }
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(tm->ev[i]);
    delete tm;
    if (e != hipSuccess) return fail(BM_EHIP, std::string("map_points_timed: ") + hipGetErrorString(e));
    times->map_ms = map_ms;
    times->sort_ms = sort_ms;
    times->map_launches = maps;
    times->sort_launches = sorts;
    times->unsort_ms = unsort_ms;
    times->unsort_launches = unsorts;
    return BM_OK;
  }
  BM_GUARD("map_points_timed")
}

__attribute__((visibility("default"))) int map_points(const bm_index* index, const int32_t* xy, int64_t n,
                                                     int32_t* out_ids, hipStream_t stream) {
  return map_points_tuned(index, xy, n, out_ids, nullptr, stream);
}

__attribute__((visibility("default"))) int bm_quantize_lonlat(const double* lonlat, int64_t n, int32_t* xy,
                                                             hipStream_t stream) {
  try {
    const TraceRange trace_range("bm_quantize_lonlat");
    if (n < 0) return fail(BM_EINVAL, "bm_quantize_lonlat: n < 0");
    if (n == 0) return BM_OK;
    if (!lonlat || !xy) return fail(BM_EINVAL, "bm_quantize_lonlat: null buffer");
    int dev = 0, cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e = launch_quantize(lonlat, n, xy, cu > 0 ? cu : 256, stream);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("bm_quantize_lonlat: launch: ") + hipGetErrorString(e));
    return BM_OK;
  }
  BM_GUARD("bm_quantize_lonlat")
}

__attribute__((visibility("default"))) const char* bm_last_error(void) { return error_text(); }

}  // extern "C"
