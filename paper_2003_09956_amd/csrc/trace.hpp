// Named ranges on the ROCm tracing timeline (rocprofv3 --marker-trace): one
// per library call on the calling host thread, one per chunk of iterations
// that a solve queues, and one per served request from its submission to its
// completion (a start/stop range, since requests overlap).  With no tracing
// tool attached every call returns at once.
#pragma once

#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>

namespace modap_host {

class TraceRange {
public:
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

inline uint64_t trace_start(const char *name) { return roctxRangeStartA(name); }
inline void trace_stop(uint64_t id) { roctxRangeStop(id); }

}  // namespace modap_host
