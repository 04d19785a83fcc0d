// roctx ranges around the library's device work, for timelines taken with
// `rocprofv3 --marker-trace`: each entry point that launches kernels (and
// each chunk the server enqueues) opens a range named after it.  Without a
// profiler attached a range costs a call into the roctx library.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

namespace tbpm {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace tbpm
