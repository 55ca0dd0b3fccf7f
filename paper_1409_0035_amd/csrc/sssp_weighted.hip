// Weighted single-source shortest paths (integer arc lengths >= 1).
#include "internal.h"

namespace ccg {

size_t sssp_weighted_batched_scratch(int64_t n) { return 1024 + (size_t)n * 0; }
size_t sssp_weighted_plain_scratch(int64_t n) { return 1024 + (size_t)n * 0; }

void sssp_weighted_batched(hipStream_t, const DevGraph&, bool, const int32_t*, int32_t, int32_t*, int32_t, void*,
                           size_t, DevFlags*, LevelCounters*, LevelCounters*, TravStats*) {
    throw HipError{hipErrorNotSupported, "weighted traversal not built yet"};
}
void sssp_weighted_plain(hipStream_t, const DevGraph&, bool, const int32_t*, int32_t, int32_t*, int32_t, void*, size_t,
                         DevFlags*, LevelCounters*, LevelCounters*, TravStats*) {
    throw HipError{hipErrorNotSupported, "weighted traversal not built yet"};
}

}  // namespace ccg
