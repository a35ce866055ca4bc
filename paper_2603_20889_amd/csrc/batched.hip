// Batched Q-less TSQR: many independent tall-skinny matrices of uneven m and
// n in ONE persistent launch (paper Alg. 2 applied per matrix).
//
// The host plan cuts every matrix into row tiles (about tile_bytes each) and
// orders all tiles longest first.  A fixed grid of wavefronts pulls tiles
// from a device queue (one atomic counter).  A wavefront folds its tile into
// an R with the same per-n code as qless_tsqr_r, writes it to the matrix's
// level-0 slot and increments the counter of its group of kFanIn siblings;
// the wavefront that completes a group folds the group's stacked triangles
// (the tree step of Alg. 2) into the next level, and the one that completes
// the root writes the matrix's sign-normalised R.  No wavefront ever waits
// for another, so the grid drains whatever the residency; counters reset
// themselves, so the launch can be replayed from a captured graph with no
// memset in between.  Optionally the previous contents of a matrix's R are
// stacked into its root (R([R_old; X])), which is how a caller keeps a
// running R over chunks of rows.
#include <algorithm>
#include <new>
#include <vector>

#include "tsqr_kernels.h"

struct qless_batch_plan {
    std::vector<qless::BatchMat> mats;
    std::vector<int2> tiles;
    int np_max = 1;
    int64_t slot_doubles = 0;
    int64_t counter_ints = 0;
    size_t off_tiles = 0, off_counters = 0, off_slots = 0, bytes = 0;
    int64_t nwaves = 0;
};

namespace qless {
namespace {

constexpr int kFanIn = 16;
constexpr int kBatchWpb = 2;  // wavefronts per workgroup of the batched kernel

__device__ __forceinline__ int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <int NP, int RPL>
__device__ __forceinline__ void batch_tile(const BatchMat& M, int t, double* __restrict__ Rw, double* __restrict__ slots,
                           int* __restrict__ counters, int lane) {
    using namespace tsqr_detail;
    const int n = M.n;
    const int64_t nn = (int64_t)n * n;
    zero_r<NP>(Rw, lane);
    const int64_t r0 = (int64_t)t * M.tile_rows;
    const int64_t r1 = (r0 + M.tile_rows < M.m) ? r0 + M.tile_rows : M.m;
    fold_rows<NP, RPL>(M.X, n, M.ldx, r0, r1, Rw, lane);
    int64_t count = M.ntiles, idx = t, sbase = M.slot_base, cbase = M.cnt_base;
    while (true) {
        if (count == 1) {
            if (M.accumulate) fold_rows<NP, RPL>(M.R, n, M.ldr, 0, n, Rw, lane);
            store_r<NP>(Rw, n, M.R, M.ldr, true, lane);
            return;
        }
        store_r<NP>(Rw, n, slots + sbase + idx * nn, n, false, lane);
        __threadfence();
        const int64_t g = idx / kFanIn;
        const int64_t gsize = (count - g * kFanIn < kFanIn) ? count - g * kFanIn : kFanIn;
        int old = 0;
        if (lane == 0)
            old = __hip_atomic_fetch_add(counters + cbase + g, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old != gsize - 1) return;     // a sibling is still running; it will continue the tree
        if (lane == 0) __hip_atomic_store(counters + cbase + g, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        zero_r<NP>(Rw, lane);
        fold_rows<NP, RPL>(slots + sbase + g * kFanIn * nn, n, n, 0, gsize * n, Rw, lane);
        sbase += count * nn;
        cbase += cdiv(count, kFanIn);
        idx = g;
        count = cdiv(count, kFanIn);
    }
}

// queue[0]: next tile, queue[1]: wavefronts finished (both reset by the last wavefront)
__global__ void __launch_bounds__(64 * kBatchWpb) __attribute__((amdgpu_waves_per_eu(2)))
batched_kernel(const BatchMat* __restrict__ mats, const int2* __restrict__ tiles, int64_t ntiles, int64_t nwaves,
               double* __restrict__ slots, int* __restrict__ counters, int* __restrict__ queue, int np_max) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (SGPR)
    const int64_t w = (int64_t)blockIdx.x * kBatchWpb + wib;
    if (w >= nwaves) return;
    double* Rw = lds + (size_t)wib * (np_max * (np_max + 1) / 2 + np_max);
    while (true) {
        int t = 0;
        if (lane == 0) t = __hip_atomic_fetch_add(queue, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = __builtin_amdgcn_readfirstlane(t);
        if (t >= ntiles) break;
        const int2 tl = tiles[t];
        const BatchMat M = mats[tl.x];
        switch (M.np) {
            case 1: batch_tile<1, 64>(M, tl.y, Rw, slots, counters, lane); break;
            case 2: batch_tile<2, 32>(M, tl.y, Rw, slots, counters, lane); break;
            case 4: batch_tile<4, 16>(M, tl.y, Rw, slots, counters, lane); break;
            case 8: batch_tile<8, 8>(M, tl.y, Rw, slots, counters, lane); break;
            case 16: batch_tile<16, 4>(M, tl.y, Rw, slots, counters, lane); break;
            case 32: batch_tile<32, 12>(M, tl.y, Rw, slots, counters, lane); break;
            default: batch_tile<64, 5>(M, tl.y, Rw, slots, counters, lane); break;
        }
    }
    // the last wavefront to leave resets the queue for the next launch
    if (lane == 0) {
        const int done = __hip_atomic_fetch_add(queue + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (int)nwaves - 1) {
            __hip_atomic_store(queue, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(queue + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

int batch_np(int64_t n) {
    int np = 1;
    while (np < n) np <<= 1;
    return np;
}

int64_t batch_panel_rows(int np) {
    switch (np) {
        case 1: return 64 * 64;
        case 2: return 64 * 32;
        case 4: return 64 * 16;
        case 8: return 64 * 8;
        case 16: return 64 * 4;
        case 32: return 8 * 12;
        default: return 8 * 5;
    }
}

}  // namespace

int batch_plan_create(const qless_matrix_desc* d, int32_t count, int64_t tile_bytes, int waves_per_cu,
                      qless_batch_plan** out) {
    if (out == nullptr || d == nullptr || count < 1) return QLESS_ERR_ARG;
    *out = nullptr;
    if (tile_bytes <= 0) tile_bytes = 4 << 20;
    if (waves_per_cu <= 0) waves_per_cu = 8;
    for (int32_t i = 0; i < count; ++i) {
        if (d[i].n < 1 || d[i].m < 0) return QLESS_ERR_ARG;
        if (d[i].n > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
        if (d[i].R == nullptr || d[i].ldr < d[i].n) return QLESS_ERR_ARG;
        if (d[i].m > 0 && (d[i].X == nullptr || d[i].ldx < d[i].n)) return QLESS_ERR_ARG;
    }
    qless_batch_plan* p = new (std::nothrow) qless_batch_plan;
    if (!p) return QLESS_ERR_ARG;
    int64_t slots = 0, cnts = 0;
    std::vector<std::pair<int64_t, int2>> order;
    for (int32_t i = 0; i < count; ++i) {
        BatchMat M{};
        M.X = d[i].X;
        M.R = d[i].R;
        M.m = d[i].m;
        M.ldx = d[i].m > 0 ? d[i].ldx : d[i].n;
        M.ldr = d[i].ldr;
        M.n = (int)d[i].n;
        M.np = batch_np(d[i].n);
        M.accumulate = d[i].accumulate ? 1 : 0;
        const int64_t panel = batch_panel_rows(M.np);
        int64_t tr = tile_bytes / (8 * d[i].n);
        tr = std::max<int64_t>(panel, tr / panel * panel);
        M.tile_rows = tr;
        M.ntiles = (int)std::max<int64_t>(1, ceil_div(d[i].m, tr));
        M.slot_base = slots;
        M.cnt_base = cnts;
        for (int64_t c = M.ntiles; c > 1; c = ceil_div(c, kFanIn)) {
            slots += c * d[i].n * d[i].n;
            cnts += ceil_div(c, kFanIn);
        }
        p->np_max = std::max(p->np_max, M.np);
        p->mats.push_back(M);
        for (int t = 0; t < M.ntiles; ++t) {
            const int64_t rows = std::min<int64_t>(tr, std::max<int64_t>(0, d[i].m - (int64_t)t * tr));
            order.push_back({rows * d[i].n, make_int2(i, t)});
        }
    }
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int64_t, int2>& a, const std::pair<int64_t, int2>& b) { return a.first > b.first; });
    p->tiles.reserve(order.size());
    for (auto& o : order) p->tiles.push_back(o.second);
    p->slot_doubles = slots;
    p->counter_ints = cnts + 2;
    p->off_tiles = align_up(p->mats.size() * sizeof(BatchMat), 256);
    p->off_counters = p->off_tiles + align_up(p->tiles.size() * sizeof(int2), 256);
    p->off_slots = p->off_counters + align_up((size_t)p->counter_ints * sizeof(int), 256);
    p->bytes = p->off_slots + align_up((size_t)std::max<int64_t>(slots, 1) * sizeof(double), 256);
    const DeviceInfo& di = current_device_info();
    p->nwaves = std::min<int64_t>((int64_t)p->tiles.size(), (int64_t)di.num_cus * waves_per_cu);
    *out = p;
    return QLESS_OK;
}

int batch_plan_upload(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s) {
    if (p == nullptr) return QLESS_ERR_ARG;
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) || work_bytes < p->bytes)
        return QLESS_ERR_WORKSPACE;
    char* b = static_cast<char*>(work);
    hipError_t e = hipMemcpyAsync(b, p->mats.data(), p->mats.size() * sizeof(BatchMat), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b + p->off_tiles, p->tiles.data(), p->tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(b + p->off_counters, 0, (size_t)p->counter_ints * sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the plan's host arrays may be reused right after
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int batch_run(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s) {
    if (p == nullptr) return QLESS_ERR_ARG;
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) || work_bytes < p->bytes)
        return QLESS_ERR_WORKSPACE;
    char* b = static_cast<char*>(work);
    int* counters = reinterpret_cast<int*>(b + p->off_counters);
    int* queue = counters + (p->counter_ints - 2);
    const size_t lds = (size_t)kBatchWpb * (p->np_max * (p->np_max + 1) / 2 + p->np_max) * sizeof(double);
    const int64_t blocks = ceil_div(p->nwaves, kBatchWpb);
    hipLaunchKernelGGL(batched_kernel, dim3((unsigned)blocks), dim3(64 * kBatchWpb), lds, s,
                       reinterpret_cast<const BatchMat*>(b), reinterpret_cast<const int2*>(b + p->off_tiles),
                       (int64_t)p->tiles.size(), p->nwaves, reinterpret_cast<double*>(b + p->off_slots), counters,
                       queue, p->np_max);
    return hipGetLastError() == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

size_t batch_plan_bytes(const qless_batch_plan* p) { return p ? p->bytes : 0; }
int64_t batch_plan_tiles(const qless_batch_plan* p) { return p ? (int64_t)p->tiles.size() : 0; }

}  // namespace qless
