// Kernel instances of the TSQR fold on the FP64 matrix cores (n = 32, 48,
// 64; 64-row panels, one row per lane).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np32_r1(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<32, 1>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np48_r1(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<48, 1>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np64_r1(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<64, 1>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
}  // namespace qless
