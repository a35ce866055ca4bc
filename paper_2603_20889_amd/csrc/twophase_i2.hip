// Instances of the two-phase stage-1 fold over [Y X] (twophase_kernels.h), one
// file per group of widths so that they compile in parallel.
#include "twophase_kernels.h"

namespace qless {
hipError_t launch_cat_np10_r6(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<10, 6>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np12_r5(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<12, 5>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np14_r4(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<14, 4>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np16_r4(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<16, 4>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np24_r21(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<24, 21>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np32_r16(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<32, 16>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
}  // namespace qless
