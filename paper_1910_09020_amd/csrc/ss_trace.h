// Named ranges on the host timeline (roctx): rocprofv3 --marker-trace records
// them beside the kernels and copies; without a tool attached a range costs a
// call into the roctx library and nothing else.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace ss {

class TraceRange {
public:
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace ss
