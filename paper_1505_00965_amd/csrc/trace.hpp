// Named host-side ranges for profilers (ROCTx): a tracer such as
// `rocprofv3 --marker-trace` shows each mlmc_run and each of its driver
// iterations as a range on the host timeline; without a tracer attached the
// calls return at once.
#pragma once
#include <rocprofiler-sdk-roctx/roctx.h>

namespace mlmc {

struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

}  // namespace mlmc
