// Kernel instances of the TSQR fold for n = 1, 2, 3, 4 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np1_r32(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<1, 32>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np1_r32(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<1, 32>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np2_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<2, 16>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np2_r16(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<2, 16>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np3_r12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<3, 12>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np3_r12(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<3, 12>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np4_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<4, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np4_r8(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<4, 8>(Y, k, n, stage, R, ldr, s);
}
}  // namespace qless
