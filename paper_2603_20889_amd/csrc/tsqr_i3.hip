// Kernel instances of the TSQR fold for n = 10, 12, 14, 16 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(10, 6)
QLESS_DEFINE_FOLD(12, 5)
QLESS_DEFINE_FOLD(14, 4)
QLESS_DEFINE_FOLD(16, 4)
QLESS_DEFINE_TREE(10, 6)
QLESS_DEFINE_TREE(12, 5)
QLESS_DEFINE_TREE(14, 4)
QLESS_DEFINE_TREE(16, 4)
}  // namespace qless
