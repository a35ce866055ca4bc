// Alternative panel heights (rows per lane) of the TSQR fold, selectable per n
// through qless_tune_set; the autotuner times them against the defaults.
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np1_r32(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<1, 32>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np2_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<2, 16>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np4_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<4, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np8_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<8, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np16_r2(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<16, 2>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np32_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<32, 8>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np64_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<64, 4>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np8_r5(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<8, 5>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
hipError_t launch_fold_np16_r3(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<16, 3>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
}  // namespace qless
