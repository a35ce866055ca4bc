// Kernel instances of the TSQR fold for n = 24, 32, 40 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(24, 21)
QLESS_DEFINE_FOLD(32, 16)
QLESS_DEFINE_FOLD(40, 12)
}  // namespace qless
