// Batched form: one persistent launch over a table of point batches, eager
// (bm_map_batches over offsets into one concatenated array, bm_map_batch_table
// over a device table of descriptors) or as captured HIP graphs
// (bm_batch_plan_*: one per form), and the launch-shape autotuner.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "trace.h"

using namespace bm;

namespace {

// Device table layout: [header: nb (int64), padding to 32 bytes][nb entries]
constexpr size_t kHdrBytes = 32;

int check_batches(const bm_batch* b, int64_t nb, const char* who) {
  if (nb < 0) return fail(BM_EINVAL, std::string(who) + ": nb < 0");
  if (nb > 0 && !b) return fail(BM_EINVAL, std::string(who) + ": null batch table");
  for (int64_t i = 0; i < nb; ++i) {
    if (b[i].n < 0) return fail(BM_EINVAL, std::string(who) + ": batch " + std::to_string(i) + " has n < 0");
    if (b[i].n > 0 && (!b[i].xy || !b[i].out_ids))
      return fail(BM_EINVAL, std::string(who) + ": batch " + std::to_string(i) + " has a null pointer");
  }
  return BM_OK;
}

int hip_fail(hipError_t e, const std::string& what) {
  return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP, what + ": " + hipGetErrorString(e));
}

int current_is(const bm_index* ix, const char* who) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, std::string(who) + ": hipGetDevice");
  if (dev != ix->device) return fail(BM_EINVAL, std::string(who) + ": index lives on another device");
  return BM_OK;
}

}  // namespace

struct bm_batch_plan {
  const bm_index* index = nullptr;
  int64_t max_batches = 0;
  int64_t max_points = 0;
  Tuning tuning{};
  size_t table_bytes = 0;
  char* d_table = nullptr;              // header + entries
  OffsetHeader* d_off = nullptr;        // the offset form's header
  long long* d_meta = nullptr;          // [max_batches + 3]: nb, work counter, prefix
  char* h_staging = nullptr;            // pinned copy of the table
  OffsetHeader* h_off = nullptr;        // pinned copy of the offset form's header
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr, graph_off = nullptr;
  hipGraphExec_t exec = nullptr, exec_off = nullptr;
  hipEvent_t done = nullptr;
  bool ran = false;
};

static void plan_free(bm_batch_plan* p) {
  if (!p) return;
  if (p->done) (void)hipEventSynchronize(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->exec_off) (void)hipGraphExecDestroy(p->exec_off);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->graph_off) (void)hipGraphDestroy(p->graph_off);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->done) (void)hipEventDestroy(p->done);
  if (p->d_table) (void)hipFree(p->d_table);
  if (p->d_off) (void)hipFree(p->d_off);
  if (p->d_meta) (void)hipFree(p->d_meta);
  if (p->h_staging) (void)hipHostFree(p->h_staging);
  if (p->h_off) (void)hipHostFree(p->h_off);
  delete p;
}

// Replays wait for the previous one to have read the staged table or header.
static int plan_wait(bm_batch_plan* p, const char* who) {
  if (!p->ran) return BM_OK;
  const hipError_t e = hipEventSynchronize(p->done);
  return e == hipSuccess ? BM_OK : hip_fail(e, std::string(who) + ": wait");
}

static int plan_launch(bm_batch_plan* p, hipGraphExec_t exec, hipStream_t stream, const char* who) {
  hipError_t e = hipGraphLaunch(exec, stream);
  if (e == hipSuccess) e = hipEventRecord(p->done, stream);
  if (e != hipSuccess) return hip_fail(e, std::string(who) + ": launch");
  p->ran = true;
  return BM_OK;
}

extern "C" {

__attribute__((visibility("default"))) int bm_map_batch_table(const bm_index* index, const bm_batch* batches,
                                                             int64_t nb, const bm_tuning* t, hipStream_t stream) {
  try {
    const bm::TraceRange trace_range("bm_map_batch_table");
    clear_error();
    if (!index) return fail(BM_EINVAL, "bm_map_batch_table: null index");
    if (nb < 0) return fail(BM_EINVAL, "bm_map_batch_table: nb < 0");
    if (nb == 0) return BM_OK;
    if (!batches) return fail(BM_EINVAL, "bm_map_batch_table: null batch table");
    int rc = current_is(index, "bm_map_batch_table");
    if (rc != BM_OK) return rc;
    const Tuning tu = tuning_from(t);
    void* meta = nullptr;
    hipError_t e = hipMallocAsync(&meta, sizeof(long long) * (size_t)(nb + 3), stream);
    if (e != hipSuccess) return hip_fail(e, "bm_map_batch_table: hipMallocAsync");
    e = launch_batches(index->k, nullptr, nb, reinterpret_cast<const BatchEntry*>(batches),
                       static_cast<long long*>(meta), tu, index->num_cu, stream);
    hipError_t e2 = hipFreeAsync(meta, stream);
    if (e != hipSuccess) return hip_fail(e, "bm_map_batch_table");
    if (e2 != hipSuccess) return hip_fail(e2, "bm_map_batch_table: hipFreeAsync");
    return BM_OK;
  } catch (...) {
    return fail(BM_EINVAL, "bm_map_batch_table: unexpected error");
  }
}

__attribute__((visibility("default"))) int bm_map_batches(const bm_index* index, const int32_t* xy,
                                                         const int64_t* batch_off, int64_t nb, int32_t* out_ids,
                                                         const bm_tuning* t, hipStream_t stream) {
  try {
    const bm::TraceRange trace_range("bm_map_batches");
    clear_error();
    if (!index) return fail(BM_EINVAL, "bm_map_batches: null index");
    if (nb < 0) return fail(BM_EINVAL, "bm_map_batches: nb < 0");
    if (nb == 0) return BM_OK;
    if (!xy || !batch_off || !out_ids) return fail(BM_EINVAL, "bm_map_batches: null pointer");
    int rc = current_is(index, "bm_map_batches");
    if (rc != BM_OK) return rc;
    const Tuning tu = tuning_from(t);
    // scratch: the descriptor table, then the prefix kernel's meta
    const size_t tab_bytes = (sizeof(BatchEntry) * (size_t)nb + 255) / 256 * 256;
    void* scratch = nullptr;
    hipError_t e = hipMallocAsync(&scratch, tab_bytes + sizeof(long long) * (size_t)(nb + 3), stream);
    if (e != hipSuccess) return hip_fail(e, "bm_map_batches: hipMallocAsync");
    BatchEntry* tab = static_cast<BatchEntry*>(scratch);
    long long* meta = reinterpret_cast<long long*>(static_cast<char*>(scratch) + tab_bytes);
    e = launch_batch_offsets(nullptr, nb, xy, out_ids, batch_off, -1, nb, tab, index->num_cu, stream);
    if (e == hipSuccess) e = launch_batches(index->k, nullptr, nb, tab, meta, tu, index->num_cu, stream);
    hipError_t e2 = hipFreeAsync(scratch, stream);
    if (e != hipSuccess) return hip_fail(e, "bm_map_batches");
    if (e2 != hipSuccess) return hip_fail(e2, "bm_map_batches: hipFreeAsync");
    return BM_OK;
  } catch (...) {
    return fail(BM_EINVAL, "bm_map_batches: unexpected error");
  }
}

__attribute__((visibility("default"))) int bm_batch_plan_create(const bm_index* index, int64_t max_points,
                                                               int64_t max_batches, const bm_tuning* t,
                                                               bm_batch_plan** out) {
  try {
    clear_error();
    if (!index || !out) return fail(BM_EINVAL, "bm_batch_plan_create: null argument");
    *out = nullptr;
    if (max_batches < 1 || max_batches > (1 << 26)) return fail(BM_EINVAL, "bm_batch_plan_create: max_batches out of range");
    if (max_points < 0) return fail(BM_EINVAL, "bm_batch_plan_create: max_points < 0");
    int rc = current_is(index, "bm_batch_plan_create");
    if (rc != BM_OK) return rc;
    bm_batch_plan* p = new (std::nothrow) bm_batch_plan();
    if (!p) return fail(BM_ENOMEM, "bm_batch_plan_create: out of host memory");
    p->index = index;
    p->max_batches = max_batches;
    p->max_points = max_points;
    p->tuning = tuning_from(t);
    p->table_bytes = kHdrBytes + sizeof(BatchEntry) * (size_t)max_batches;
    hipError_t e = hipMalloc((void**)&p->d_table, p->table_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_off, sizeof(OffsetHeader));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_meta, sizeof(long long) * (size_t)(max_batches + 3));
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_staging, p->table_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&p->h_off, sizeof(OffsetHeader), hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) {
      plan_free(p);
      return hip_fail(e, "bm_batch_plan_create");
    }
    memset(p->h_staging, 0, p->table_bytes);
    memset(p->h_off, 0, sizeof(OffsetHeader));
    BatchEntry* tab = reinterpret_cast<BatchEntry*>(p->d_table + kHdrBytes);
    // table form: upload the staged table, prefix (also clears the counter), map
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ec = hipMemcpyAsync(p->d_table, p->h_staging, p->table_bytes, hipMemcpyHostToDevice, p->cap);
      if (ec == hipSuccess)
        ec = launch_batches(index->k, reinterpret_cast<const long long*>(p->d_table), 0, tab, p->d_meta, p->tuning,
                            index->num_cu, p->cap);
      e = hipStreamEndCapture(p->cap, &p->graph);
      if (ec != hipSuccess) e = ec;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    // offset form: upload the staged header, write the table on the device, prefix, map
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t ec = hipMemcpyAsync(p->d_off, p->h_off, sizeof(OffsetHeader), hipMemcpyHostToDevice, p->cap);
      if (ec == hipSuccess)
        ec = launch_batch_offsets(p->d_off, 0, nullptr, nullptr, nullptr, max_points, max_batches, tab,
                                  index->num_cu, p->cap);
      if (ec == hipSuccess)
        ec = launch_batches(index->k, reinterpret_cast<const long long*>(p->d_off), 0, tab, p->d_meta, p->tuning,
                            index->num_cu, p->cap);
      e = hipStreamEndCapture(p->cap, &p->graph_off);
      if (ec != hipSuccess) e = ec;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec_off, p->graph_off, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      plan_free(p);
      return hip_fail(e, "bm_batch_plan_create: graph capture");
    }
    *out = p;
    return BM_OK;
  } catch (...) {
    return fail(BM_ENOMEM, "bm_batch_plan_create: unexpected error");
  }
}

__attribute__((visibility("default"))) int bm_batch_plan_run(bm_batch_plan* p, const int32_t* xy,
                                                            const int64_t* batch_off, int64_t nb, int32_t* out_ids,
                                                            hipStream_t stream) {
  try {
    const bm::TraceRange trace_range("bm_batch_plan_run");
    clear_error();
    if (!p) return fail(BM_EINVAL, "bm_batch_plan_run: null plan");
    if (nb < 0 || nb > p->max_batches) return fail(BM_EINVAL, "bm_batch_plan_run: nb outside [0, max_batches]");
    if (nb > 0 && (!xy || !batch_off || !out_ids)) return fail(BM_EINVAL, "bm_batch_plan_run: null pointer");
    int rc = current_is(p->index, "bm_batch_plan_run");
    if (rc == BM_OK) rc = plan_wait(p, "bm_batch_plan_run");
    if (rc != BM_OK) return rc;
    *p->h_off = OffsetHeader{nb, xy, out_ids, reinterpret_cast<const long long*>(batch_off)};
    return plan_launch(p, p->exec_off, stream, "bm_batch_plan_run");
  } catch (...) {
    return fail(BM_EINVAL, "bm_batch_plan_run: unexpected error");
  }
}

__attribute__((visibility("default"))) int bm_batch_plan_run_table(bm_batch_plan* p, const bm_batch* batches,
                                                                  int64_t nb, hipStream_t stream) {
  try {
    const bm::TraceRange trace_range("bm_batch_plan_run_table");
    clear_error();
    if (!p) return fail(BM_EINVAL, "bm_batch_plan_run_table: null plan");
    if (nb > p->max_batches) return fail(BM_EINVAL, "bm_batch_plan_run_table: more batches than the plan holds");
    int rc = check_batches(batches, nb, "bm_batch_plan_run_table");
    if (rc == BM_OK) rc = current_is(p->index, "bm_batch_plan_run_table");
    if (rc == BM_OK) rc = plan_wait(p, "bm_batch_plan_run_table");
    if (rc != BM_OK) return rc;
    memcpy(p->h_staging, &nb, sizeof nb);
    if (nb > 0) memcpy(p->h_staging + kHdrBytes, batches, sizeof(BatchEntry) * (size_t)nb);
    return plan_launch(p, p->exec, stream, "bm_batch_plan_run_table");
  } catch (...) {
    return fail(BM_EINVAL, "bm_batch_plan_run_table: unexpected error");
  }
}

__attribute__((visibility("default"))) void bm_batch_plan_destroy(bm_batch_plan* p) {
  try {
    plan_free(p);
  } catch (...) {
  }
}

// ------------------------------------------------------------- autotune ----

static std::string cache_path() {
  const char* e = getenv("BM_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/blockmap_tune.txt";
}

__attribute__((visibility("default"))) int bm_autotune(const bm_index* index, const int32_t* xy, int64_t n,
                                                      bm_tuning* out, hipStream_t stream) {
  try {
    const bm::TraceRange trace_range("bm_autotune");
    clear_error();
    if (!index || !xy || !out) return fail(BM_EINVAL, "bm_autotune: null argument");
    if (n < 64) return fail(BM_EINVAL, "bm_autotune: need at least 64 sample points");
    int rc = current_is(index, "bm_autotune");
    if (rc != BM_OK) return rc;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDeviceProperties(&prop, index->device);
    if (e != hipSuccess) return hip_fail(e, "bm_autotune: hipGetDeviceProperties");
    char key[256];
    const int size_class = (int)std::floor(std::log2((double)n));
    snprintf(key, sizeof key, "%s|blocks=%lld|verts=%lld|levels=%d|top=%d|n=2^%d", prop.gcnArchName,
             (long long)index->n_blocks, (long long)index->n_verts, index->k.n_levels, index->k.g0,
             size_class);
    const std::string path = cache_path();
    if (FILE* f = fopen(path.c_str(), "r")) {
      char line[512];
      while (fgets(line, sizeof line, f)) {
        char k2[256];
        int a, b, c, d;
        if (sscanf(line, "%255s %d %d %d %d", k2, &a, &b, &c, &d) == 5 && strcmp(k2, key) == 0) {
          fclose(f);
          bm_tuning t{a, b, c, d};
          const Tuning v = tuning_from(&t);
          out->edge_chunk = v.edge_chunk;
          out->blocks_per_cu = v.blocks_per_cu;
          out->tile_points = v.tile_points;
          out->presort = v.presort;
          return BM_OK;
        }
      }
      fclose(f);
    }
    // the sample split into 16 batches for the batched-form timings
    const int64_t per = (n + 15) / 16;
    BatchEntry htab[16];
    int nbt = 0;
    int32_t* dout = nullptr;
    BatchEntry* dtab = nullptr;
    long long* dmeta = nullptr;
    e = hipMalloc((void**)&dout, sizeof(int32_t) * (size_t)n);
    if (e == hipSuccess) e = hipMalloc((void**)&dtab, sizeof htab);
    if (e == hipSuccess) e = hipMalloc((void**)&dmeta, sizeof(long long) * 24);
    if (e == hipSuccess) {
      for (int64_t s0 = 0; s0 < n; s0 += per, ++nbt) htab[nbt] = BatchEntry{xy + 2 * s0, dout + s0, std::min(per, n - s0)};
      e = hipMemcpy(dtab, htab, sizeof(BatchEntry) * nbt, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      if (dout) (void)hipFree(dout);
      if (dtab) (void)hipFree(dtab);
      if (dmeta) (void)hipFree(dmeta);
      return hip_fail(e, "bm_autotune: setup");
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    auto time_it = [&](const Tuning& t, bool batched, float* ms) -> hipError_t {
      hipError_t r = hipSuccess;
      for (int rep = 0; rep < 3 && r == hipSuccess; ++rep) {
        if (rep == 1) r = hipEventRecord(e0, stream);
        if (r != hipSuccess) break;
        if (!batched) {
          r = launch_map(index->k, xy, n, dout, t, index->num_cu, stream);
        } else {
          r = launch_batches(index->k, nullptr, nbt, dtab, dmeta, t, index->num_cu, stream);
        }
      }
      if (r == hipSuccess) r = hipEventRecord(e1, stream);
      if (r == hipSuccess) r = hipEventSynchronize(e1);
      if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
      return r;
    };
    Tuning best = tuning_from(nullptr);
    float best_ms = 1e30f;
    const int chunks[2] = {4, 8};
    const int bpcs[3] = {4, 6, 8};
    for (int c : chunks)
      for (int b : bpcs) {
        Tuning t{c, b, best.tile_points, 1};
        float ms = 0;
        e = time_it(t, false, &ms);
        if (e != hipSuccess) break;
        if (ms < best_ms) { best_ms = ms; best = t; }
      }
    if (e == hipSuccess && n >= kPresortMin) {  // is the spatial pre-sort worth it here?
      Tuning t = best;
      t.presort = 0;
      float ms = 0;
      e = time_it(t, false, &ms);
      if (e == hipSuccess && ms < best_ms) { best_ms = ms; best = t; }
    }
    if (e == hipSuccess) {
      const int units[3] = {512, 2048, 8192};
      float bu = 1e30f;
      int keep = best.tile_points;
      for (int u : units) {
        Tuning t = best;
        t.tile_points = u;
        float ms = 0;
        e = time_it(t, true, &ms);
        if (e != hipSuccess) break;
        if (ms < bu) { bu = ms; keep = u; }
      }
      best.tile_points = keep;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(dout);
    (void)hipFree(dtab);
    (void)hipFree(dmeta);
    if (e != hipSuccess) return hip_fail(e, "bm_autotune: timing");
    out->edge_chunk = best.edge_chunk;
    out->blocks_per_cu = best.blocks_per_cu;
    out->tile_points = best.tile_points;
    out->presort = best.presort;
    if (FILE* f = fopen(path.c_str(), "a")) {
      fprintf(f, "%s %d %d %d %d\n", key, best.edge_chunk, best.blocks_per_cu, best.tile_points, best.presort);
      fclose(f);
    }
    return BM_OK;
  } catch (...) {
    return fail(BM_EINVAL, "bm_autotune: unexpected error");
  }
}

}  // extern "C"
