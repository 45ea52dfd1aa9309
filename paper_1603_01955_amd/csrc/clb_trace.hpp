// Host-side trace ranges: each long-running entry point opens a roctx range
// named after itself, so that `rocprofv3 --marker-trace` shows where host
// time goes (queueing, graph recording, the synchronising reads) beside the
// kernels it enqueued.  Without a profiler attached a range costs a call
// into an empty stub.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace clb {

struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace clb
