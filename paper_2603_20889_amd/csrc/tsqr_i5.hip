// Kernel instances of the TSQR fold for n = 48, 56 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(48, 10)
QLESS_DEFINE_FOLD(56, 8)
}  // namespace qless
