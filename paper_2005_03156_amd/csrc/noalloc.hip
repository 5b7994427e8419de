// Allocation-free form of map_points, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). A call of at least 2^20 points is spatially pre-sorted,
// which needs scratch (the sort's histograms, the sorted copy, the records
// that bring the results back to the points' order, and the results in
// sorted order: 20 bytes per point); here it comes from `scratch` below, a
// fixed array of kNoAllocBytes in device memory that every device the library
// runs on holds until the process ends. Calls on one device share that
// device's array.
//
// Host code never hands the array's name to a kernel: on the host that name
// is a stand-in, not a device address. Its device address is looked up once
// per device, with that device current (hipGetSymbolAddress), and only that
// address is used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.h"
#include "trace.h"

namespace bm {
namespace {

constexpr long long kNoAllocMaxPoints = 1ll << 22;
// one round of sort passes over kNoAllocMaxPoints points in one chunk: 20 B
// per point plus 1 MiB, more than the chunk's histograms and alignment need
constexpr size_t kNoAllocBytes = (size_t)kNoAllocMaxPoints * 20 + (1u << 20);

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

}  // namespace
}  // namespace bm

static __device__ __align__(256) unsigned char scratch[bm::kNoAllocBytes];

using namespace bm;

extern "C" {

__attribute__((visibility("default"))) int map_points_noalloc(const bm_index* index, const int32_t* xy, int64_t n,
                                                             int32_t* out_ids, hipStream_t stream) {
  try {
    const TraceRange trace_range("map_points_noalloc");
    if (!index) return fail(BM_EINVAL, "map_points_noalloc: null index");
    if (n < 0) return fail(BM_EINVAL, "map_points_noalloc: n < 0");
    if (n > kNoAllocMaxPoints)
      return fail(BM_ERANGE, "map_points_noalloc: n = " + std::to_string(n) + " is more than the " +
                                 std::to_string(kNoAllocMaxPoints) +
                                 " points its fixed device scratch serves per call; split the call, or use "
                                 "map_points");
    if (n == 0) return BM_OK;
    if (!xy || !out_ids) return fail(BM_EINVAL, "map_points_noalloc: null buffer");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("map_points_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    if (dev != index->device)
      return fail(BM_EINVAL, "map_points_noalloc: the index lives on device " + std::to_string(index->device) +
                                 " but device " + std::to_string(dev) + " is current");
    if (dev < 0 || dev >= kMaxDevices) return fail(BM_EINVAL, "map_points_noalloc: device number out of range");
    void* ws = nullptr;
    {
      std::lock_guard<std::mutex> g(g_mu);
      if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
          return fail(BM_EHIP, std::string("map_points_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch[dev] = p;
      }
      ws = g_scratch[dev];
    }
    e = launch_map(index->k, xy, n, out_ids, tuning_from(nullptr), index->num_cu, stream, nullptr, ws,
                   kNoAllocBytes);
    if (e != hipSuccess) return fail(BM_EHIP, std::string("map_points_noalloc: launch: ") + hipGetErrorString(e));
    return BM_OK;
  } catch (...) {
    return fail(BM_EINVAL, "map_points_noalloc: unexpected error");
  }
}

}  // extern "C"
