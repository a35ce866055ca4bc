// R of a matrix wider than one TSQR panel (n > 64): block classical
// Gram-Schmidt with reorthogonalisation (BCGS2) over column panels of width
// w <= 64.  Sec. 4.6 notes that Q-less TSQR runs out of on-chip room beyond
// 64 columns and that variants which store Q, like block Gram-Schmidt, are
// the choice there.  For panel j (columns c0 .. c0 + w - 1), with Q the
// orthonormal columns of the earlier panels:
//   V = X_j;  B1 = Q^T V;  V -= Q B1;  B2 = Q^T V;  V -= Q B2   (twice: BCGS2)
//   R_jj = Q-less TSQR of V (qless_tsqr_r's launches);  Q_j = V R_jj^{-1}
//   (the streaming explicit-Q pass);  R[0:c0, c0:c0+w] = B1 + B2.
// The four cross products are plain library GEMMs (rocBLAS); the panel
// factorisation and the explicit Q are this library's kernels.  Q is the
// explicit orthonormal factor of X (m x n), written as a by-product.
#include <mutex>
#include <vector>

#include <rocblas/rocblas.h>

#include "qless_internal.h"

namespace qless {
namespace {

std::mutex g_blas_mu;
std::vector<rocblas_handle> g_blas;

// rocBLAS handle of the current device (created on first use).
rocblas_handle blas_handle() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    std::lock_guard<std::mutex> g(g_blas_mu);
    if ((int)g_blas.size() <= dev) g_blas.resize(dev + 1, nullptr);
    if (g_blas[dev] == nullptr) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
        g_blas[dev] = h;
    }
    return g_blas[dev];
}

struct WideWork {
    double* V = nullptr;      // m x w panel being orthogonalised (ld w)
    double* B1 = nullptr;     // w x n, column-major view of the p x w product Q^T V
    double* B2 = nullptr;
    double* Rinv = nullptr;   // w x w
    int* iw = nullptr;        // status of the current panel's R_jj inverse
    int* gw = nullptr;        // first failing column over all panels
    void* tsqr = nullptr;     // workspace of the panel TSQR
    size_t tsqr_bytes = 0;
    size_t bytes = 0;
};

WideWork wide_layout(int64_t m, int64_t n, int64_t w, void* base) {
    WideWork k;
    char* b = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t nb) -> char* {
        char* p = b ? b + off : nullptr;
        off += align_up(nb, 256);
        return p;
    };
    k.V = reinterpret_cast<double*>(take((size_t)(m * w) * sizeof(double)));
    k.B1 = reinterpret_cast<double*>(take((size_t)(w * n) * sizeof(double)));
    k.B2 = reinterpret_cast<double*>(take((size_t)(w * n) * sizeof(double)));
    k.Rinv = reinterpret_cast<double*>(take((size_t)(w * w) * sizeof(double)));
    k.iw = reinterpret_cast<int*>(take(sizeof(int)));
    k.gw = reinterpret_cast<int*>(take(sizeof(int)));
    k.tsqr_bytes = make_tsqr_plan(m, w, current_device_info().num_cus, false).work_bytes;
    k.tsqr = take(k.tsqr_bytes);
    k.bytes = off;
    return k;
}

// Zeros below the diagonal of R (n x n, ld ldr).
__global__ void __launch_bounds__(256) zero_lower_kernel(double* __restrict__ R, int64_t n, int64_t ldr) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / n, c = e - i * n;
        if (c < i) R[i * ldr + c] = 0.0;
    }
}

// R[i][c0 + c] = B1[i][c] + B2[i][c] for i < p, c < w; B1, B2 hold the p x w
// products column-major as w x p (element (i, c) at c + i * w).
__global__ void __launch_bounds__(256) add_blocks_kernel(const double* __restrict__ B1, const double* __restrict__ B2,
                                                         int64_t p, int64_t w, double* __restrict__ R, int64_t ldr,
                                                         int64_t c0) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < p * w; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / w, c = e - i * w;
        R[i * ldr + c0 + c] = B1[c + i * w] + B2[c + i * w];
    }
}

// info bookkeeping: *g = 0 at the start; after a panel at column c0, the
// first non-zero panel status j becomes c0 + j.
__global__ void set_zero_kernel(int* __restrict__ g) {
    if (threadIdx.x == 0) *g = 0;
}

__global__ void note_panel_kernel(const int* __restrict__ panel_info, int* __restrict__ g, int64_t c0) {
    if (threadIdx.x == 0 && *g == 0 && *panel_info != 0) *g = (int)(c0 + *panel_info);
}

unsigned grid_for(int64_t count) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 256), 2048)); }

// Row-major M (rows x cols, ld) is column-major cols x rows with the same ld:
// C = A B in row-major terms is C^T = B^T A^T column-major.
//   Bc (w x p) = V^T Q  <=>  B = Q^T V        : gemm(N, T, w, p, m) of Vc (w x m) and Qc (p x m)
//   Vc (w x m) -= Bc Qc  <=>  V -= Q B          : gemm(N, N, w, m, p)
rocblas_status cross(rocblas_handle h, const double* V, int64_t m, int64_t w, const double* Q, int64_t ldq, int64_t p,
                     double* Bc) {
    const double one = 1.0, zero = 0.0;
    return rocblas_dgemm_64(h, rocblas_operation_none, rocblas_operation_transpose, w, p, m, &one, V, w, Q, ldq, &zero,
                            Bc, w);
}

rocblas_status subtract(rocblas_handle h, double* V, int64_t m, int64_t w, const double* Q, int64_t ldq, int64_t p,
                        const double* Bc) {
    const double mone = -1.0, one = 1.0;
    return rocblas_dgemm_64(h, rocblas_operation_none, rocblas_operation_none, w, m, p, &mone, Bc, w, Q, ldq, &one, V,
                            w);
}

}  // namespace
}  // namespace qless

using namespace qless;

extern "C" {

size_t qless_wide_workspace_bytes(int64_t m, int64_t n, int64_t panel) {
    if (m < 1 || n < 1 || m < n || panel < 1 || panel > QLESS_MAX_N) return 0;
    return wide_layout(m, n, std::min(panel, n), nullptr).bytes;
}

int qless_wide_r(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, double* Q, int64_t ldq,
                 int64_t panel, int32_t* info, void* work, size_t work_bytes, hipStream_t stream) {
    if (X == nullptr || R == nullptr || Q == nullptr || m < 1 || n < 1 || m < n || ldx < n || ldr < n || ldq < n ||
        panel < 1)
        return QLESS_ERR_ARG;
    if (panel > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
    const int64_t w = std::min(panel, n);
    const WideWork k = wide_layout(m, n, w, work);
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) != 0 || work_bytes < k.bytes)
        return QLESS_ERR_WORKSPACE;
    rocblas_handle h = blas_handle();
    if (h == nullptr || rocblas_set_stream(h, stream) != rocblas_status_success) return QLESS_ERR_HIP;
    const int cus = current_device_info().num_cus;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(zero_lower_kernel, dim3(grid_for(n * n)), dim3(256), 0, stream, R, n, ldr);
    hipLaunchKernelGGL(set_zero_kernel, dim3(1), dim3(64), 0, stream, k.gw);
    e = hipGetLastError();
    for (int64_t c0 = 0; c0 < n && e == hipSuccess; c0 += w) {
        const int64_t wj = std::min(w, n - c0);
        // V = X_j (rows of wj doubles, packed)
        e = hipMemcpy2DAsync(k.V, (size_t)wj * sizeof(double), X + c0, (size_t)ldx * sizeof(double),
                             (size_t)wj * sizeof(double), (size_t)m, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) break;
        if (c0 > 0) {
            if (cross(h, k.V, m, wj, Q, ldq, c0, k.B1) != rocblas_status_success ||
                subtract(h, k.V, m, wj, Q, ldq, c0, k.B1) != rocblas_status_success ||
                cross(h, k.V, m, wj, Q, ldq, c0, k.B2) != rocblas_status_success ||
                subtract(h, k.V, m, wj, Q, ldq, c0, k.B2) != rocblas_status_success) {
                e = hipErrorUnknown;
                break;
            }
            hipLaunchKernelGGL(add_blocks_kernel, dim3(grid_for(c0 * wj)), dim3(256), 0, stream, k.B1, k.B2, c0, wj,
                               R, ldr, c0);
            e = hipGetLastError();
            if (e != hipSuccess) break;
        }
        // R_jj (diagonal >= 0) and Q_j = V R_jj^{-1}
        double* Rjj = R + c0 * ldr + c0;
        const TsqrPlan plan = make_tsqr_plan(m, wj, cus, false);
        e = launch_tsqr(k.V, m, wj, wj, Rjj, ldr, k.tsqr, plan, stream);
        if (e == hipSuccess) e = launch_trinv(Rjj, ldr, (int)wj, k.Rinv, k.iw, stream);
        if (e == hipSuccess) e = launch_apply_right(k.V, m, wj, wj, k.Rinv, true, Q + c0, ldq, k.iw, stream);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(note_panel_kernel, dim3(1), dim3(64), 0, stream, k.iw, k.gw, c0);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess && info) e = launch_copy_int(k.gw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

}  // extern "C"
