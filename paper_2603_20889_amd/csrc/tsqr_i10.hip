// Kernel instances of the TSQR fold in the 4 x 16 column-group layout (n = 32,
// 48, 64; one file per group so the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(32, 24)
QLESS_DEFINE_FOLD(48, 16)
QLESS_DEFINE_FOLD(64, 12)
}  // namespace qless
