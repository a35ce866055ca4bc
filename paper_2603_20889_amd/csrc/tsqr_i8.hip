// Alternative panel heights (rows per lane) of the TSQR fold, selectable per n
// through qless_tune_set; the autotuner times them against the defaults.
#include "tsqr_kernels.h"

namespace qless {
QLESS_DEFINE_FOLD(5, 12)
QLESS_DEFINE_FOLD(6, 10)
QLESS_DEFINE_FOLD(7, 9)
QLESS_DEFINE_FOLD(8, 8)
QLESS_DEFINE_TREE(5, 12)
QLESS_DEFINE_TREE(6, 10)
QLESS_DEFINE_TREE(7, 9)
QLESS_DEFINE_TREE(8, 8)
}  // namespace qless
