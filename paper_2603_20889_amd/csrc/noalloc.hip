// qless_tsqr_r_noalloc: the Q-less TSQR of qless_tsqr_r for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).  The stacked triangles of the
// stage-1 workgroups and of the tree levels -- the only scratch the TSQR
// launches use -- live in a library-owned device array instead of a caller
// workspace.  The array is a module global, so every GPU the library runs on
// holds its own copy until the process ends; its device address is looked up
// once per device on the first call made with that device current.
#include <mutex>

#include "qless_internal.h"

namespace qless {
namespace {

// 64 MiB: the largest TSQR plan on a 256-CU device (n = 64: 1024 stage-1
// workgroups, two stacked buffers of 1024 triangles of 64 x 64 doubles).
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr on failure).
void* scratch_address() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace qless

using namespace qless;

extern "C" {

size_t qless_noalloc_scratch_bytes(void) { return kScratchBytes; }

int qless_tsqr_r_noalloc(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                         hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const TsqrPlan plan = make_tsqr_plan(m, n, current_device_info().num_cus);
    if (plan.work_bytes > kScratchBytes) return QLESS_ERR_WORKSPACE;
    void* work = scratch_address();
    if (work == nullptr) return QLESS_ERR_HIP;
    // Every stacked triangle the launches read was written by an earlier
    // launch of the same call, so nothing needs clearing first.
    return launch_tsqr(X, m, n, ldx, R, ldr, work, plan, stream) == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

}  // extern "C"
