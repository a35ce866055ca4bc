// Kernel instances of the TSQR fold on the FP64 matrix cores (n = 32, 48,
// 64; 64-row panels, one row per lane).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(32, 1)
QLESS_DEFINE_FOLD(48, 1)
QLESS_DEFINE_FOLD(64, 1)
}  // namespace qless
