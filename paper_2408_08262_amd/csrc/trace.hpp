// Named host ranges for timeline tools (rocprofv3 --marker-trace): the
// setup, its levels and phases, the solves and the V-cycles.  Without a
// tool attached a range costs a function call.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>

namespace airg {

struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    TraceRange(const char *fmt, int k) {
        char buf[48];
        std::snprintf(buf, sizeof buf, fmt, k);
        roctxRangePushA(buf);
    }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

inline void trace_push(const char *name) { roctxRangePushA(name); }
inline void trace_pop() { roctxRangePop(); }

}  // namespace airg
