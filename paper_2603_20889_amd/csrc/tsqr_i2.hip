// Kernel instances of the TSQR fold for n = 5, 6, 7, 8 (one file per group so
// the instances compile in parallel).
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(5, 6)
QLESS_DEFINE_FOLD(6, 6)
QLESS_DEFINE_FOLD(7, 4)
QLESS_DEFINE_FOLD(8, 4)
QLESS_DEFINE_TREE(5, 6)
QLESS_DEFINE_TREE(6, 6)
QLESS_DEFINE_TREE(7, 4)
QLESS_DEFINE_TREE(8, 4)
}  // namespace qless
