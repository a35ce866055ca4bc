// Instances of the two-phase stage-1 fold over [Y X] (twophase_kernels.h), one
// file per group of widths so that they compile in parallel.
#include "twophase_kernels.h"

namespace qless {
hipError_t launch_cat_np1_r32(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<1, 32>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np2_r16(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<2, 16>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np3_r12(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<3, 12>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np4_r8(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<4, 8>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np5_r6(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<5, 6>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np6_r6(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<6, 6>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np7_r4(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<7, 4>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np8_r4(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<8, 4>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
}  // namespace qless
