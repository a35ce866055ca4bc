// Kernel instances of the TSQR fold for n = 24, 32, 40 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np24_r21(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<24, 21>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np32_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<32, 16>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np40_r12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<40, 12>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
}  // namespace qless
