// Stage 1 of the batched Q-less TSQR: one persistent launch over the row
// tiles of every matrix (longest first).  Wavefront w of the fixed grid
// takes tiles w, w + W, w + 2W, ...; each tile is folded with the
// single-matrix code of its padded width (one switch per tile).
#include "batched_kernels.h"

namespace qless {
namespace batch_detail {

template <int CLS>
__global__ void __launch_bounds__(64 * kBatchWpb) __attribute__((amdgpu_waves_per_eu(2)))
batched_stage_kernel(const BatchMat* __restrict__ mats, const int2* __restrict__ tiles, int64_t ntiles,
                     int64_t nwaves, double* __restrict__ slots, int region_doubles, int staged) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (SGPR)
    const int64_t w = (int64_t)blockIdx.x * kBatchWpb + wib;
    if (w >= nwaves) return;
    double* Rw = lds + (size_t)wib * region_doubles;
    double* stage = staged ? Rw + kStageOffset : nullptr;
    for (int64_t t = w; t < ntiles; t += nwaves) {
        const int2 tl = tiles[t];
        const BatchMat M = mats[tl.x];
#define QLESS_STAGE_CALL(NP, RPL) batch_stage_tile<NP, RPL>(M, tl.y, Rw, slots, stage, lane)
        if constexpr (CLS == 0) QLESS_BATCH_SWITCH_0(M.np, QLESS_STAGE_CALL)
        else if constexpr (CLS == 1) QLESS_BATCH_SWITCH_1(M.np, QLESS_STAGE_CALL)
        else if constexpr (CLS == 2) QLESS_BATCH_SWITCH_2(M.np, QLESS_STAGE_CALL)
        else QLESS_BATCH_SWITCH_3(M.np, QLESS_STAGE_CALL)
#undef QLESS_STAGE_CALL
    }
}

}  // namespace batch_detail

// Stage 1 over the tiles [0, ntiles) of one width class (all of the same
// class, longest first).
hipError_t launch_batched_stage(int cls, const BatchMat* mats, const int2* tiles, int64_t ntiles, int64_t nwaves,
                                double* slots, int r_doubles, bool staged, hipStream_t s) {
    using namespace batch_detail;
    int region = r_doubles;
    if (staged && region < kStageOffset + kStageDoubles) region = kStageOffset + kStageDoubles;
    const size_t lds = (size_t)kBatchWpb * region * sizeof(double);
    const dim3 grid((unsigned)ceil_div(nwaves, kBatchWpb)), block(64 * kBatchWpb);
    const int st = staged ? 1 : 0;
    switch (cls) {
        case 0: hipLaunchKernelGGL(batched_stage_kernel<0>, grid, block, lds, s, mats, tiles, ntiles, nwaves, slots, region, st); break;
        case 1: hipLaunchKernelGGL(batched_stage_kernel<1>, grid, block, lds, s, mats, tiles, ntiles, nwaves, slots, region, st); break;
        case 2: hipLaunchKernelGGL(batched_stage_kernel<2>, grid, block, lds, s, mats, tiles, ntiles, nwaves, slots, region, st); break;
        default: hipLaunchKernelGGL(batched_stage_kernel<3>, grid, block, lds, s, mats, tiles, ntiles, nwaves, slots, region, st); break;
    }
    return hipGetLastError();
}

}  // namespace qless
