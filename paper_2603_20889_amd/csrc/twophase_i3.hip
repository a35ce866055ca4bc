// Instances of the two-phase stage-1 fold over [Y X] (twophase_kernels.h), one
// file per group of widths so that they compile in parallel.
#include "twophase_kernels.h"

namespace qless {
hipError_t launch_cat_np40_r12(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<40, 12>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np48_r16(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<48, 16>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np56_r8(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<56, 8>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
hipError_t launch_cat_np64_r12(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, double* out,
                          int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
    return tsqr_detail::launch_cat_fold<64, 12>(s, m, rpw, nw, out, ldo, ostride, normalise, st);
}
}  // namespace qless
