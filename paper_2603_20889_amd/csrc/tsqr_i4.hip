// Kernel instances of the TSQR fold for n = 24, 32, 40 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np24_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<24, 16>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np32_r12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<32, 12>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np40_r10(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<40, 10>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
}  // namespace qless
