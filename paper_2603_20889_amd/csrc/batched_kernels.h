// Device side of the batched Q-less TSQR (paper Alg. 2 per matrix): the
// per-tile and per-group folds and the instance switch shared by the stage-1
// kernel (batched_stage.hip) and the tree kernel (batched_tree.hip).
#pragma once

#include "tsqr_kernels.h"

namespace qless {
namespace batch_detail {

constexpr int kFanIn = 16;     // stacked triangles per tree group
constexpr int kBatchWpb = 2;   // wavefronts per workgroup of the batched kernels
// LDS staging buffer per wavefront for the staged instances (n <= 8): every
// one of them streams panels of 2048 doubles (16 KB).  It shares the
// wavefront's LDS region with the running triangle: a tile of width <= 8
// needs at most 44 doubles of triangle, so the buffer starts at double 64,
// and a wider tile (no staging) uses the whole region for its triangle.
constexpr int kStageDoubles = 2048;
constexpr int kStageOffset = 64;

// Padded widths of the batched kernels and their rows per lane (the
// single-matrix defaults of those widths), in four classes compiled as four
// kernels: one kernel holding every width would take the registers of the
// widest (and spill), starving the narrow ones of occupancy.
//   class 0: n <= 8 (lane-private folds, LDS-staged panels)
//   class 1: n = 9..16 (cross-lane fold)
//   class 2: n = 17..32, class 3: n = 33..64 (column-group fold)
constexpr int kBatchClasses = 4;

constexpr int batch_class(int np) { return np <= 8 ? 0 : np <= 16 ? 1 : np <= 32 ? 2 : 3; }

// Rows per lane of the batched instance of each padded width; the host plan
// cuts tiles into whole panels of these instances.  The single-matrix
// defaults, except the 8 x 8 column-group fold for 48 and 64: in one kernel
// with 40 and 56 the 4 x 16 fold would spill.
constexpr int batch_rpl(int np) {
    return np == 1 ? 32 : np == 2 ? 16 : np == 4 ? 8 : np == 8 ? 4 : np == 16 ? 4 : np == 24 ? 21 : np == 32 ? 16
         : np == 40 ? 12 : np == 48 ? 10 : np == 56 ? 8 : 7;
}

#define QLESS_BATCH_SWITCH_0(np, CALL)             \
    switch (np) {                                  \
        case 1: CALL(1, batch_rpl(1)); break;      \
        case 2: CALL(2, batch_rpl(2)); break;      \
        case 4: CALL(4, batch_rpl(4)); break;      \
        default: CALL(8, batch_rpl(8)); break;     \
    }
#define QLESS_BATCH_SWITCH_1(np, CALL) { CALL(16, batch_rpl(16)); }
#define QLESS_BATCH_SWITCH_2(np, CALL)             \
    switch (np) {                                  \
        case 24: CALL(24, batch_rpl(24)); break;   \
        default: CALL(32, batch_rpl(32)); break;   \
    }
#define QLESS_BATCH_SWITCH_3(np, CALL)             \
    switch (np) {                                  \
        case 40: CALL(40, batch_rpl(40)); break;   \
        case 48: CALL(48, batch_rpl(48)); break;   \
        case 56: CALL(56, batch_rpl(56)); break;   \
        default: CALL(64, batch_rpl(64)); break;   \
    }

// Fold tile t of matrix M (rows [t*tile_rows, ...)) and write its triangle to
// the matrix's level-0 slot, or, for a matrix of one tile, its final R
// (stacking the previous R in with accumulate).
template <int NP, int RPL>
__device__ __forceinline__ void batch_stage_tile(const BatchMat& M, int t, double* __restrict__ Rw,
                                                 double* __restrict__ slots, double* stage, int lane) {
    using namespace tsqr_detail;
    zero_r<NP>(Rw, lane);
    const int64_t r0 = (int64_t)t * M.tile_rows;
    const int64_t r1 = (r0 + M.tile_rows < M.m) ? r0 + M.tile_rows : M.m;
    fold_rows<NP, RPL>(M.X, M.n, M.ldx, r0, r1, Rw, lane, staged_instance<NP, RPL>() ? stage : nullptr);
    if (M.ntiles == 1) {
        if (M.accumulate) fold_rows<NP, RPL>(M.R, M.n, M.ldr, 0, M.n, Rw, lane);
        store_r<NP>(Rw, M.n, M.R, M.ldr, true, lane);
    } else {
        store_r<NP>(Rw, M.n, slots + M.slot_base + (int64_t)t * M.n * M.n, M.n, false, lane);
    }
}

// Fold tree group G of matrix M: its gsize stacked triangles go to the next
// level's slot, or, for the root, to the matrix's R.
template <int NP, int RPL>
__device__ __forceinline__ void batch_tree_group(const BatchMat& M, const BatchGroup& G, double* __restrict__ Rw,
                                                 double* __restrict__ slots, int lane) {
    using namespace tsqr_detail;
    zero_r<NP>(Rw, lane);
    fold_rows<NP, RPL>(slots + G.src, M.n, M.n, 0, (int64_t)G.gsize * M.n, Rw, lane);
    if (G.dst < 0) {
        if (M.accumulate) fold_rows<NP, RPL>(M.R, M.n, M.ldr, 0, M.n, Rw, lane);
        store_r<NP>(Rw, M.n, M.R, M.ldr, true, lane);
    } else {
        store_r<NP>(Rw, M.n, slots + G.dst, M.n, false, lane);
    }
}

}  // namespace batch_detail
}  // namespace qless
