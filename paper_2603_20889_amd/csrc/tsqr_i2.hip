// Kernel instances of the TSQR fold for n = 5, 6, 7, 8 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np5_r12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<5, 12>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np6_r10(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<6, 10>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np7_r9(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<7, 9>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np8_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<8, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
}  // namespace qless
