// Tree levels of the batched Q-less TSQR: one launch per level over the
// groups of all matrices at that level (fan-in kFanIn stacked triangles).
#include "batched_kernels.h"

namespace qless {
namespace batch_detail {

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
        QLESS_BATCH_SWITCH(M.np, QLESS_TREE_CALL)
#undef QLESS_TREE_CALL
    }
}

}  // namespace batch_detail

hipError_t launch_batched_tree(const BatchMat* mats, const BatchGroup* groups, int64_t ngroups, int64_t nwaves,
                               double* slots, int r_doubles, hipStream_t s) {
    using namespace batch_detail;
    const size_t lds = (size_t)kBatchWpb * r_doubles * sizeof(double);
    hipLaunchKernelGGL(batched_tree_kernel, dim3((unsigned)ceil_div(nwaves, kBatchWpb)), dim3(64 * kBatchWpb), lds, s,
                       mats, groups, ngroups, nwaves, slots, r_doubles);
    return hipGetLastError();
}

}  // namespace qless
