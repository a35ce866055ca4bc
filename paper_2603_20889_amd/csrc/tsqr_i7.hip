// Alternative panel heights (rows per lane) of the TSQR fold, selectable per n
// through qless_tune_set; the autotuner times them against the defaults.
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np1_r64(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<1, 64>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np1_r64(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<1, 64>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np2_r32(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<2, 32>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np2_r32(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<2, 32>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np3_r21(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<3, 21>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np3_r21(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<3, 21>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np4_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<4, 16>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np4_r16(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<4, 16>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np16_r2(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<16, 2>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np16_r2(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<16, 2>(Y, k, n, stage, R, ldr, s);
}
hipError_t launch_fold_np32_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<32, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np64_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<64, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np16_r3(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<16, 3>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_tree_np16_r3(const double* Y, int64_t k, int n, double* stage, double* R, int64_t ldr,
                               hipStream_t s) {
    return tsqr_detail::launch_tree_block<16, 3>(Y, k, n, stage, R, ldr, s);
}
}  // namespace qless
