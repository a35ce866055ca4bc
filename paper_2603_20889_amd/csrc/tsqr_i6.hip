// Kernel instances of the TSQR fold for n = 64 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np64_r5(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<64, 5>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
}  // namespace qless
