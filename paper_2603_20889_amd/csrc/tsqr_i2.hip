// Kernel instances of the TSQR fold for n = 5, 6, 7, 8 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np5_r6(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<5, 6>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np5_r6(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<5, 6>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np6_r6(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<6, 6>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np6_r6(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<6, 6>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np7_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<7, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np7_r4(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<7, 4>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np8_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<8, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np8_r4(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<8, 4>(Y, k, n, stage, R, ldr, s);
}
}  // namespace qless
