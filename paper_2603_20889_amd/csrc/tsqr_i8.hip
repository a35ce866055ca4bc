// Alternative panel heights (rows per lane) of the TSQR fold, selectable per n
// through qless_tune_set; the autotuner times them against the defaults.
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np5_r12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<5, 12>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np5_r12(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<5, 12>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np6_r10(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<6, 10>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np6_r10(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<6, 10>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np7_r9(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<7, 9>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np7_r9(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<7, 9>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np8_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<8, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np8_r8(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<8, 8>(Y, k, n, stage, R, ldr, s);
}
}  // namespace qless
