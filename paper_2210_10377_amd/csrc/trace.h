// Named ranges around the library's entry points for the ROCm tracer (rocprofv3
// --marker-trace shows them beside the kernels they enqueue).  Costs one call each when
// no tracer is attached.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace lbm {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace lbm
