// Alternative panel heights (rows per lane) of the TSQR fold, selectable per n
// through qless_tune_set; the autotuner times them against the defaults.
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(1, 64)
QLESS_DEFINE_FOLD(2, 32)
QLESS_DEFINE_FOLD(3, 21)
QLESS_DEFINE_FOLD(4, 16)
QLESS_DEFINE_FOLD(16, 2)
QLESS_DEFINE_FOLD(32, 8)
QLESS_DEFINE_FOLD(64, 4)
QLESS_DEFINE_FOLD(16, 3)
QLESS_DEFINE_TREE(1, 64)
QLESS_DEFINE_TREE(2, 32)
QLESS_DEFINE_TREE(3, 21)
QLESS_DEFINE_TREE(4, 16)
QLESS_DEFINE_TREE(16, 2)
QLESS_DEFINE_TREE(16, 3)
}  // namespace qless
