// Kernel instances of the TSQR fold for n = 64 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
hipError_t launch_fold_np64_r7(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                               double* Y, int64_t ldy, int64_t ystride, int normalise, hipStream_t s) {
    return tsqr_detail::launch_fold<64, 7>(X, m, n, ldx, rpw, nw, Y, ldy, ystride, normalise, s);
}
}  // namespace qless
