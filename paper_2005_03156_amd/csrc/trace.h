// roctx ranges on the host timeline around the library's entry points and the
// served form's device batches (shown by rocprofv3 --marker-trace; without a
// profiler attached a range costs a function call).
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace bm {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

inline void trace_push(const char* name) { roctxRangePushA(name); }
inline void trace_pop() { roctxRangePop(); }

}  // namespace bm
