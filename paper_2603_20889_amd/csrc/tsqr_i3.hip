// Kernel instances of the TSQR fold for n = 10, 12, 14, 16 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np10_r6(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<10, 6>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np10_r6(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<10, 6>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np12_r5(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<12, 5>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np12_r5(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<12, 5>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np14_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<14, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np14_r4(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<14, 4>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np16_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<16, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np16_r4(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<16, 4>(Y, k, n, stage, R, ldr, s);
}
}  // namespace qless
