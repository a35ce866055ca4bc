// Tree levels of the batched Q-less TSQR: one launch per level over the
// groups of all matrices at that level (fan-in kFanIn stacked triangles).
#include "batched_kernels.h"

namespace qless {
namespace batch_detail {

template <int CLS>
__global__ void __launch_bounds__(64 * kBatchWpb) __attribute__((amdgpu_waves_per_eu(2)))
batched_tree_kernel(const BatchMat* __restrict__ mats, const BatchGroup* __restrict__ groups, int64_t ngroups,
                    int64_t nwaves, double* __restrict__ slots, int r_doubles) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * kBatchWpb + wib;
    if (w >= nwaves) return;
    double* Rw = lds + (size_t)wib * r_doubles;
    for (int64_t q = w; q < ngroups; q += nwaves) {
        const BatchGroup G = groups[q];
        const BatchMat M = mats[G.mat];
#define QLESS_TREE_CALL(NP, RPL) batch_tree_group<NP, RPL>(M, G, Rw, slots, lane)
        if constexpr (CLS == 0) QLESS_BATCH_SWITCH_0(M.np, QLESS_TREE_CALL)
        else if constexpr (CLS == 1) QLESS_BATCH_SWITCH_1(M.np, QLESS_TREE_CALL)
        else if constexpr (CLS == 2) QLESS_BATCH_SWITCH_2(M.np, QLESS_TREE_CALL)
        else QLESS_BATCH_SWITCH_3(M.np, QLESS_TREE_CALL)
#undef QLESS_TREE_CALL
    }
}

}  // namespace batch_detail

// One tree level of one width class: its groups [0, ngroups).
hipError_t launch_batched_tree(int cls, const BatchMat* mats, const BatchGroup* groups, int64_t ngroups,
                               int64_t nwaves, double* slots, int r_doubles, hipStream_t s) {
    using namespace batch_detail;
    const size_t lds = (size_t)kBatchWpb * r_doubles * sizeof(double);
    const dim3 grid((unsigned)ceil_div(nwaves, kBatchWpb)), block(64 * kBatchWpb);
    switch (cls) {
        case 0: hipLaunchKernelGGL(batched_tree_kernel<0>, grid, block, lds, s, mats, groups, ngroups, nwaves, slots, r_doubles); break;
        case 1: hipLaunchKernelGGL(batched_tree_kernel<1>, grid, block, lds, s, mats, groups, ngroups, nwaves, slots, r_doubles); break;
        case 2: hipLaunchKernelGGL(batched_tree_kernel<2>, grid, block, lds, s, mats, groups, ngroups, nwaves, slots, r_doubles); break;
        default: hipLaunchKernelGGL(batched_tree_kernel<3>, grid, block, lds, s, mats, groups, ngroups, nwaves, slots, r_doubles); break;
    }
    return hipGetLastError();
}

}  // namespace qless
