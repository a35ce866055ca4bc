// Running Q-less TSQR over chunks of rows with the partial tree state kept on
// the device (Alg. 2 with its first stage spread over several calls): the
// state holds the stage-1 triangles of the k1 workgroups of the TSQR plan
// for the whole row count; each chunk is streamed by the same k0 wavefronts,
// every workgroup starting from its own triangle in the state and writing it
// back, and only the finishing call runs the tree.  Folding a matrix chunk by
// chunk thus costs one stage-1 launch per chunk and one tree in all -- the
// per-request state of the served form (Sec. 1's least squares in a single
// pass over the data, with the data arriving in pieces).
#include <algorithm>

#include "tsqr_kernels.h"

namespace qless {
namespace {

__global__ void __launch_bounds__(256) zero_fill_kernel(double* __restrict__ p, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

bool state_sizes_ok(int64_t m_total, int64_t n) { return m_total >= 0 && n >= 1 && n <= QLESS_MAX_N; }

// The plan of the whole row count, without tuning overrides: the state's
// layout must not change between the calls of one running factorisation.
TsqrPlan state_plan(int64_t m_total, int64_t n) {
    return make_tsqr_plan(m_total, n, current_device_info().num_cus, false);
}

size_t state_bytes(const TsqrPlan& p, int64_t n) {
    const size_t tri = align_up((size_t)std::max<int64_t>(p.k1, 1) * (size_t)(n * n) * sizeof(double), 256);
    return p.k1 > 1 ? std::max(p.work_bytes, tri + p.ybytes_b) : tri;
}

int check_state(const void* state, size_t have, size_t need) {
    if (state == nullptr || (reinterpret_cast<uintptr_t>(state) & 255u) != 0 || have < need) return QLESS_ERR_WORKSPACE;
    return QLESS_OK;
}

}  // namespace
}  // namespace qless

using namespace qless;

extern "C" {

size_t qless_tsqr_state_bytes(int64_t m_total, int64_t n) {
    if (!state_sizes_ok(m_total, n)) return 0;
    return state_bytes(state_plan(m_total, n), n);
}

int qless_tsqr_state_init(void* state, size_t bytes, int64_t m_total, int64_t n, hipStream_t stream) {
    if (!state_sizes_ok(m_total, n)) return n > QLESS_MAX_N ? QLESS_ERR_UNSUPPORTED : QLESS_ERR_ARG;
    const TsqrPlan p = state_plan(m_total, n);
    int st = check_state(state, bytes, state_bytes(p, n));
    if (st != QLESS_OK) return st;
    const int64_t count = std::max<int64_t>(p.k1, 1) * n * n;
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(count, 256), 1024);
    hipLaunchKernelGGL(zero_fill_kernel, dim3(blocks), dim3(256), 0, stream, static_cast<double*>(state), count);
    return hipGetLastError() == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_tsqr_state_fold(const double* X, int64_t m, int64_t ldx, void* state, size_t bytes, int64_t m_total,
                          int64_t n, hipStream_t stream) {
    if (!state_sizes_ok(m_total, n)) return n > QLESS_MAX_N ? QLESS_ERR_UNSUPPORTED : QLESS_ERR_ARG;
    if (m < 0 || (m > 0 && (X == nullptr || ldx < n))) return QLESS_ERR_ARG;
    const TsqrPlan p = state_plan(m_total, n);
    int st = check_state(state, bytes, state_bytes(p, n));
    if (st != QLESS_OK) return st;
    if (m == 0) return QLESS_OK;
    FoldFn fn = find_fold(p.npad, p.rows_per_lane);
    if (fn == nullptr) return QLESS_ERR_HIP;
    // the chunk over the plan's k0 wavefronts, whole panels per wavefront
    int64_t rpw = ceil_div(m, p.k0);
    const int64_t unit = tsqr_panel_rows(p.npad, p.rows_per_lane);
    rpw = ceil_div(rpw, unit) * unit;
    double* tri = static_cast<double*>(state);
    const FoldArgs a{X, m, (int)n, ldx, rpw, p.k0, tri, n, n * n, 0, tri};
    return fn(a, stream) == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_tsqr_state_finish(void* state, size_t bytes, int64_t m_total, int64_t n, double* R, int64_t ldr,
                            hipStream_t stream) {
    if (!state_sizes_ok(m_total, n)) return n > QLESS_MAX_N ? QLESS_ERR_UNSUPPORTED : QLESS_ERR_ARG;
    if (R == nullptr || ldr < n) return QLESS_ERR_ARG;
    const TsqrPlan p = state_plan(m_total, n);
    int st = check_state(state, bytes, state_bytes(p, n));
    if (st != QLESS_OK) return st;
    double* tri = static_cast<double*>(state);
    hipError_t e;
    if (p.k1 <= 1) {
        FoldFn fn = find_fold(p.npad, p.rows_per_lane);
        if (fn == nullptr) return QLESS_ERR_HIP;
        e = fn(FoldArgs{tri, n, (int)n, n, n, 1, R, ldr, 0, 1, nullptr}, stream);
    } else {
        const size_t tri_bytes = align_up((size_t)p.k1 * (size_t)(n * n) * sizeof(double), 256);
        double* dst = reinterpret_cast<double*>(static_cast<char*>(state) + tri_bytes);
        e = launch_tsqr_tree(p, tri, dst, p.k1, n, R, ldr, stream);
    }
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

}  // extern "C"
