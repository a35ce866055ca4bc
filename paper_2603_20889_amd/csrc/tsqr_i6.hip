// Kernel instances of the TSQR fold for n = 64 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(64, 7)
}  // namespace qless
