// Alternative panel heights (rows per lane) selectable by the autotuner.
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np1_r32(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<1, 32>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np2_r16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<2, 16>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np4_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<4, 8>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np8_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<8, 4>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np16_r2(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<16, 2>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np32_r8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<32, 8>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
hipError_t launch_fold_np64_r4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* R, int64_t ldr, double* slots, unsigned long long* counters,
                               int fan_in, unsigned long long tag, hipStream_t s) {
    return tsqr_detail::launch_fused<64, 4>(X, m, n, ldx, rpw, nw, R, ldr, slots, counters, fan_in, tag, s);
}
}  // namespace qless
