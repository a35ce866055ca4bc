// Kernel instances of the TSQR fold for n = 1, 2, 3, 4 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(1, 32)
QLESS_DEFINE_FOLD(2, 16)
QLESS_DEFINE_FOLD(3, 12)
QLESS_DEFINE_FOLD(4, 8)
QLESS_DEFINE_TREE(1, 32)
QLESS_DEFINE_TREE(2, 16)
QLESS_DEFINE_TREE(3, 12)
QLESS_DEFINE_TREE(4, 8)
}  // namespace qless
