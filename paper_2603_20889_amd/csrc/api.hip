// C-ABI of libqless: argument validation, workspace sizing and dispatch.
// Every entry point validates on the host before any HIP call that could
// launch work, so argument errors are testable without a GPU.
#include <algorithm>
#include <mutex>
#include <string.h>
#include <vector>

#include "qless_internal.h"

namespace qless {

// ------------------------------------------------------------ device info

const DeviceInfo& current_device_info() {
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> g(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    DeviceInfo& d = cache[dev];
    if (d.device < 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;  // MI355X
        d.num_cus = cus;
        d.device = dev;
    }
    return d;
}

// ----------------------------------------------------------------- timing

namespace {
struct TimingSlot {
    std::vector<hipEvent_t> begin, end;
    size_t used = 0;
    double total_ms = 0.0;
    int64_t count = 0;
};
bool g_timing = false;
TimingSlot g_slots[kTimeSlots];
const char* const g_slot_names[kTimeSlots] = {"tsqr_stage1", "gram"};
}  // namespace

void timing_begin(int which, hipStream_t stream) {
    if (!g_timing) return;
    TimingSlot& s = g_slots[which];
    if (s.used == s.begin.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
        s.begin.push_back(a);
        s.end.push_back(b);
    }
    (void)hipEventRecord(s.begin[s.used], stream);
}

void timing_end(int which, hipStream_t stream) {
    if (!g_timing) return;
    TimingSlot& s = g_slots[which];
    if (s.used >= s.begin.size()) return;
    (void)hipEventRecord(s.end[s.used], stream);
    ++s.used;
}

static void timing_collect(TimingSlot& s) {
    for (size_t i = 0; i < s.used; ++i) {
        float ms = 0.0f;
        if (hipEventSynchronize(s.end[i]) == hipSuccess &&
            hipEventElapsedTime(&ms, s.begin[i], s.end[i]) == hipSuccess) {
            s.total_ms += ms;
            ++s.count;
        }
    }
    s.used = 0;
}

// Workspace of the Gram-based forms: k partial Gram matrices, C, seven n x n
// work matrices, one n-vector and an int status word, each 256-byte aligned.
struct GramWork {
    double* Cpart = nullptr;
    double* C = nullptr;
    double *A1 = nullptr, *A2 = nullptr, *A3 = nullptr, *A4 = nullptr;
    double *A5 = nullptr, *A6 = nullptr, *A7 = nullptr;   // shifted CholQR3 only
    double* vec = nullptr;
    int* iw = nullptr;
    void* tsqr_work = nullptr;   // workspace of the n x n TSQR of Z (SVQB R mode)
    size_t tsqr_bytes = 0;
    size_t bytes = 0;
};

GramWork gram_work_layout(const GramPlan& gp, int64_t n, void* base) {
    GramWork w;
    char* b = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t nbytes) -> char* {
        char* p = b ? b + off : nullptr;
        off += align_up(nbytes, 256);
        return p;
    };
    const size_t sq = (size_t)(n * n) * sizeof(double);
    w.Cpart = reinterpret_cast<double*>(take(gp.part_bytes));
    w.C = reinterpret_cast<double*>(take(sq));
    w.A1 = reinterpret_cast<double*>(take(sq));
    w.A2 = reinterpret_cast<double*>(take(sq));
    w.A3 = reinterpret_cast<double*>(take(sq));
    w.A4 = reinterpret_cast<double*>(take(sq));
    w.A5 = reinterpret_cast<double*>(take(sq));
    w.A6 = reinterpret_cast<double*>(take(sq));
    w.A7 = reinterpret_cast<double*>(take(sq));
    w.vec = reinterpret_cast<double*>(take((size_t)n * sizeof(double)));
    w.iw = reinterpret_cast<int*>(take(sizeof(int)));
    w.tsqr_bytes = make_tsqr_plan(n, n, current_device_info().num_cus).work_bytes;
    w.tsqr_work = take(w.tsqr_bytes);
    w.bytes = off;
    return w;
}

// Shift of the shifted Cholesky-QR (Fukaya et al., SIAM J. Sci. Comput. 42,
// 2020): C += s I with s = 11 (m n + n (n + 1)) u ||X||^2, u = 2^-53, where
// ||X||^2 is taken as ||X||_F^2 = trace C (an upper bound of ||X||_2^2).  One
// thread: n <= 64 additions in a fixed order.
__global__ void __launch_bounds__(64) shift_diag_kernel(double* __restrict__ C, int n, double size_term) {
    if (threadIdx.x != 0) return;
    double tr = 0.0;
    for (int j = 0; j < n; ++j) tr = tr + C[j * n + j];
    const double shift = 11.0 * size_term * 0x1p-53 * tr;
    for (int j = 0; j < n; ++j) C[j * n + j] = C[j * n + j] + shift;
}

}  // namespace qless

using namespace qless;

extern "C" {

const char* qless_status_string(int status) {
    switch (status) {
        case QLESS_OK: return "QLESS_OK";
        case QLESS_ERR_ARG: return "QLESS_ERR_ARG: invalid argument";
        case QLESS_ERR_UNSUPPORTED: return "QLESS_ERR_UNSUPPORTED: n exceeds QLESS_MAX_N (64)";
        case QLESS_ERR_WORKSPACE: return "QLESS_ERR_WORKSPACE: workspace missing, misaligned or too small";
        case QLESS_ERR_HIP: return "QLESS_ERR_HIP: HIP runtime or launch failure";
        default: return "unknown qless status";
    }
}

const char* qless_version(void) { return "qless 0.1 gfx950"; }

// Workspace of qless_gram: the partials of either Gram kernel and C.
static size_t gram_only_work_bytes(int64_t m, int64_t n) {
    const int cus = current_device_info().num_cus;
    const size_t plain = make_gram_plan(m, n, cus).part_bytes;
    const size_t dd = make_gram_dd_plan(m, n, cus).part_bytes;
    return std::max(plain, dd) + align_up((size_t)(n * n) * sizeof(double), 256);
}

// Workspace of cholqr2_dd_r: the double-double Gram partials, C (hi, lo),
// R1 (hi, lo), M = R1^{-1}, the plain Gram pass (partials, C2), R2, R2^{-1}
// and the status word.
struct DdWork {
    GramDdPlan dp;
    GramPlan gp;
    double *part = nullptr, *Chi = nullptr, *Clo = nullptr, *R1h = nullptr, *R1l = nullptr, *M = nullptr;
    double *gpart = nullptr, *C2 = nullptr, *R2 = nullptr, *R2i = nullptr;
    int* iw = nullptr;
    size_t bytes = 0;
};

static DdWork cholqr2_dd_layout(int64_t m, int64_t n, void* base) {
    DdWork w;
    const int cus = current_device_info().num_cus;
    w.dp = make_gram_dd_plan(m, n, cus);
    w.gp = make_gram_plan(m, n, cus);
    char* b = static_cast<char*>(base);
    size_t off = 0;
    auto take = [&](size_t nb) -> char* {
        char* p = b ? b + off : nullptr;
        off += align_up(nb, 256);
        return p;
    };
    const size_t sq = (size_t)(n * n) * sizeof(double);
    w.part = reinterpret_cast<double*>(take(w.dp.part_bytes));
    w.Chi = reinterpret_cast<double*>(take(sq));
    w.Clo = reinterpret_cast<double*>(take(sq));
    w.R1h = reinterpret_cast<double*>(take(sq));
    w.R1l = reinterpret_cast<double*>(take(sq));
    w.M = reinterpret_cast<double*>(take(sq));
    w.gpart = reinterpret_cast<double*>(take(w.gp.part_bytes));
    w.C2 = reinterpret_cast<double*>(take(sq));
    w.R2 = reinterpret_cast<double*>(take(sq));
    w.R2i = reinterpret_cast<double*>(take(sq));
    w.iw = reinterpret_cast<int*>(take(sizeof(int)));
    w.bytes = off;
    return w;
}

// Workspace of qless_q_from_r: R^{-1} (n x n) and an int status word.
static size_t q_from_r_work_bytes(int64_t n) { return align_up((size_t)(n * n) * sizeof(double), 256) + 256; }

static int check_work(const void* work, size_t have, size_t need) {
    if (need == 0) return QLESS_OK;
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) != 0 || have < need)
        return QLESS_ERR_WORKSPACE;
    return QLESS_OK;
}

size_t qless_workspace_bytes(int method, int64_t m, int64_t n) {
    if (n < 1 || n > QLESS_MAX_N || m < 0) return 0;
    const DeviceInfo& d = current_device_info();
    switch (method) {
        case QLESS_METHOD_TSQR: return make_tsqr_plan(m, n, d.num_cus).work_bytes;
        case QLESS_METHOD_TSQR_UPDATE: return make_tsqr_update_plan(m, n, d.num_cus).work_bytes;
        case QLESS_METHOD_CHOLQR2:
        case QLESS_METHOD_SVQB:
        case QLESS_METHOD_SHIFTED_CHOLQR3: return gram_work_layout(make_gram_plan(m, n, d.num_cus), n, nullptr).bytes;
        case QLESS_METHOD_Q_FROM_R: return q_from_r_work_bytes(n);
        case QLESS_METHOD_GRAM: return gram_only_work_bytes(m, n);
        case QLESS_METHOD_CHOLQR2_DD: return cholqr2_dd_layout(m, n, nullptr).bytes;
        default: return 0;
    }
}

int qless_tsqr_r(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, void* work,
                 size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const DeviceInfo& d = current_device_info();
    TsqrPlan plan = make_tsqr_plan(m, n, d.num_cus);
    st = check_work(work, work_bytes, plan.work_bytes);
    if (st != QLESS_OK) return st;
    return launch_tsqr(X, m, n, ldx, R, ldr, work, plan, stream) == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_tsqr_r_update(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, void* work,
                        size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const DeviceInfo& d = current_device_info();
    TsqrPlan plan = make_tsqr_update_plan(m, n, d.num_cus);
    st = check_work(work, work_bytes, plan.work_bytes);
    if (st != QLESS_OK) return st;
    return launch_tsqr_update(X, m, n, ldx, R, ldr, work, plan, stream) == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int cholqr2_r(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, int32_t* info,
              void* work, size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const DeviceInfo& d = current_device_info();
    GramPlan gp = make_gram_plan(m, n, d.num_cus);
    GramWork gw = gram_work_layout(gp, n, work);
    st = check_work(work, work_bytes, gw.bytes);
    if (st != QLESS_OK) return st;
    const int ni = (int)n;
    hipError_t e = launch_gram(X, m, n, ldx, nullptr, false, gw.Cpart, gw.C, gp, stream); // C = X^T X
    if (e == hipSuccess) e = launch_chol_inv(gw.C, ni, gw.A1, gw.A2, gw.iw, 0, stream);  // R1, R1^{-1}
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, gw.A2, true, gw.Cpart, gw.C, gp, stream); // (X/R1)^T (X/R1)
    if (e == hipSuccess) e = launch_chol_inv(gw.C, ni, gw.A3, gw.A4, gw.iw, ni, stream); // R2
    if (e == hipSuccess) e = launch_trmm_out(gw.A3, gw.A1, ni, R, ldr, gw.iw, stream);   // R = R2 R1
    if (e == hipSuccess && info) e = launch_copy_int(gw.iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int svqb(const double* X, int64_t m, int64_t n, int64_t ldx, int out, double* Z_or_R, int64_t ldz,
         double* sigma, double trunc_tol, int32_t* info, void* work, size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, Z_or_R, ldz);
    if (st != QLESS_OK) return st;
    if (out != QLESS_SVQB_R && out != QLESS_SVQB_QZ) return QLESS_ERR_ARG;
    if (!(trunc_tol > 0.0)) trunc_tol = (double)n * 2.220446049250313e-16;
    const DeviceInfo& d = current_device_info();
    GramPlan gp = make_gram_plan(m, n, d.num_cus);
    GramWork gw = gram_work_layout(gp, n, work);
    st = check_work(work, work_bytes, gw.bytes);
    if (st != QLESS_OK) return st;
    const int ni = (int)n;
    double* U1 = gw.A1;
    double* D1 = gw.A2;
    double* Zt = gw.A3;
    double* lam1 = gw.vec;
    double* zdst = (out == QLESS_SVQB_QZ) ? Z_or_R : Zt;
    const int64_t zld = (out == QLESS_SVQB_QZ) ? ldz : n;
    hipError_t e = launch_gram(X, m, n, ldx, nullptr, false, gw.Cpart, gw.C, gp, stream);
    if (e == hipSuccess)
        e = launch_svqb_eig(gw.C, ni, trunc_tol, 1, U1, lam1, D1, sigma, nullptr, 0, gw.iw, stream);
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, D1, false, gw.Cpart, gw.C, gp, stream);
    if (e == hipSuccess)
        e = launch_svqb_eig(gw.C, ni, trunc_tol, 0, U1, lam1, nullptr, nullptr, zdst, zld, gw.iw, stream);
    if (e == hipSuccess && out == QLESS_SVQB_R) {
        TsqrPlan tp = make_tsqr_plan(n, n, d.num_cus);
        e = launch_tsqr(Zt, n, n, n, Z_or_R, ldz, gw.tsqr_work, tp, stream);
    }
    if (e == hipSuccess && info) e = launch_copy_int(gw.iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_gram(const double* X, int64_t m, int64_t n, int64_t ldx, double* C, int64_t ldc, double* C_lo, void* work,
               size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, C, ldc);
    if (st != QLESS_OK) return st;
    st = check_work(work, work_bytes, gram_only_work_bytes(m, n));
    if (st != QLESS_OK) return st;
    const int cus = current_device_info().num_cus;
    hipError_t e;
    if (C_lo != nullptr) {
        e = launch_gram_dd(X, m, n, ldx, static_cast<double*>(work), C, C_lo, ldc, make_gram_dd_plan(m, n, cus), stream);
    } else {
        const GramPlan gp = make_gram_plan(m, n, cus);
        double* Cw = reinterpret_cast<double*>(static_cast<char*>(work) + gram_only_work_bytes(m, n) -
                                               align_up((size_t)(n * n) * sizeof(double), 256));
        e = launch_gram(X, m, n, ldx, nullptr, false, static_cast<double*>(work), Cw, gp, stream);
        if (e == hipSuccess)
            e = hipMemcpy2DAsync(C, (size_t)ldc * sizeof(double), Cw, (size_t)n * sizeof(double),
                                 (size_t)n * sizeof(double), (size_t)n, hipMemcpyDeviceToDevice, stream);
    }
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int cholqr2_dd_r(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, int32_t* info, void* work,
                 size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const DdWork w = cholqr2_dd_layout(m, n, work);
    st = check_work(work, work_bytes, w.bytes);
    if (st != QLESS_OK) return st;
    const int ni = (int)n;
    hipError_t e = launch_gram_dd(X, m, n, ldx, w.part, w.Chi, w.Clo, n, w.dp, stream);        // C1 in dd
    if (e == hipSuccess) e = launch_chol_dd(w.Chi, w.Clo, ni, w.R1h, w.R1l, w.M, w.iw, stream);   // R1, R1^{-1}
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, w.M, true, w.gpart, w.C2, w.gp, stream);   // (X/R1)^T (X/R1)
    if (e == hipSuccess) e = launch_chol_inv(w.C2, ni, w.R2, w.R2i, w.iw, ni, stream);            // R2
    if (e == hipSuccess) e = launch_trmm_dd(w.R2, w.R1h, w.R1l, ni, R, ldr, w.iw, stream);        // R = R2 R1
    if (e == hipSuccess && info) e = launch_copy_int(w.iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int svqb_q(const double* X, int64_t m, int64_t n, int64_t ldx, double* Q, int64_t ldq, double* Z, int64_t ldz,
           double* sigma, double trunc_tol, int32_t* info, void* work, size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, Z, ldz);
    if (st != QLESS_OK) return st;
    if ((m > 0 && Q == nullptr) || ldq < n) return QLESS_ERR_ARG;
    if (!(trunc_tol > 0.0)) trunc_tol = (double)n * 2.220446049250313e-16;
    const DeviceInfo& d = current_device_info();
    GramPlan gp = make_gram_plan(m, n, d.num_cus);
    GramWork gw = gram_work_layout(gp, n, work);
    st = check_work(work, work_bytes, gw.bytes);
    if (st != QLESS_OK) return st;
    const int ni = (int)n;
    double* U1 = gw.A1;
    double* D1 = gw.A2;
    double* Dq = gw.A4;
    hipError_t e = launch_gram(X, m, n, ldx, nullptr, false, gw.Cpart, gw.C, gp, stream);
    if (e == hipSuccess)
        e = launch_svqb_eig(gw.C, ni, trunc_tol, 1, U1, gw.vec, D1, sigma, nullptr, 0, gw.iw, stream);
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, D1, false, gw.Cpart, gw.C, gp, stream);
    if (e == hipSuccess)
        e = launch_svqb_eig(gw.C, ni, trunc_tol, 0, U1, gw.vec, nullptr, nullptr, Z, ldz, gw.iw, stream, D1, Dq);
    if (e == hipSuccess) e = launch_apply_right(X, m, n, ldx, Dq, false, Q, ldq, nullptr, stream);
    if (e == hipSuccess && info) e = launch_copy_int(gw.iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_q_from_r(const double* X, int64_t m, int64_t n, int64_t ldx, const double* R, int64_t ldr, double* Q,
                   int64_t ldq, int32_t* info, void* work, size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    if ((m > 0 && Q == nullptr) || ldq < n) return QLESS_ERR_ARG;
    st = check_work(work, work_bytes, q_from_r_work_bytes(n));
    if (st != QLESS_OK) return st;
    double* Rinv = static_cast<double*>(work);
    int* iw = reinterpret_cast<int*>(static_cast<char*>(work) + align_up((size_t)(n * n) * sizeof(double), 256));
    hipError_t e = launch_trinv(R, ldr, (int)n, Rinv, iw, stream);
    if (e == hipSuccess) e = launch_apply_right(X, m, n, ldx, Rinv, true, Q, ldq, iw, stream);
    if (e == hipSuccess && info) e = launch_copy_int(iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int shifted_cholqr3_r(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr, int32_t* info,
                      void* work, size_t work_bytes, hipStream_t stream) {
    int st = check_matrix_args(X, m, n, ldx, R, ldr);
    if (st != QLESS_OK) return st;
    const DeviceInfo& d = current_device_info();
    GramPlan gp = make_gram_plan(m, n, d.num_cus);
    GramWork gw = gram_work_layout(gp, n, work);
    st = check_work(work, work_bytes, gw.bytes);
    if (st != QLESS_OK) return st;
    const int ni = (int)n;
    const double size_term = (double)m * (double)n + (double)n * (double)(n + 1);
    double *R1 = gw.A1, *R1i = gw.A2, *R2 = gw.A3, *R2i = gw.A4, *M3 = gw.A5, *R3 = gw.A6, *R3i = gw.A7;
    hipError_t e = launch_gram(X, m, n, ldx, nullptr, false, gw.Cpart, gw.C, gp, stream);   // C = X^T X
    if (e == hipSuccess) {
        hipLaunchKernelGGL(shift_diag_kernel, dim3(1), dim3(64), 0, stream, gw.C, ni, size_term);   // C + s I
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = launch_chol_inv(gw.C, ni, R1, R1i, gw.iw, 0, stream);
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, R1i, true, gw.Cpart, gw.C, gp, stream);  // Y = X R1^{-1}
    if (e == hipSuccess) e = launch_chol_inv(gw.C, ni, R2, R2i, gw.iw, ni, stream);
    if (e == hipSuccess) e = launch_trmm_out(R1i, R2i, ni, M3, n, gw.iw, stream);             // R1^{-1} R2^{-1}
    if (e == hipSuccess) e = launch_gram(X, m, n, ldx, M3, true, gw.Cpart, gw.C, gp, stream);   // Y R2^{-1}
    if (e == hipSuccess) e = launch_chol_inv(gw.C, ni, R3, R3i, gw.iw, 2 * ni, stream);
    if (e == hipSuccess) e = launch_trmm_out(R2, R1, ni, M3, n, gw.iw, stream);                // R2 R1
    if (e == hipSuccess) e = launch_trmm_out(R3, M3, ni, R, ldr, gw.iw, stream);               // R = R3 R2 R1
    if (e == hipSuccess && info) e = launch_copy_int(gw.iw, info, stream);
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_lstsq_finish(const double* Rt, int64_t n, int64_t ldr, double* x, double* resid, int32_t* info,
                       hipStream_t stream) {
    if (Rt == nullptr || x == nullptr || n < 1 || ldr < n + 1) return QLESS_ERR_ARG;
    if (n + 1 > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
    return launch_lstsq(Rt, (int)n, ldr, x, resid, info, stream) == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

int qless_tune_set(int64_t n, int32_t waves_per_cu, int32_t fan_in, int32_t rows_per_lane) {
    return tsqr_tune_set(n, waves_per_cu, fan_in, rows_per_lane);
}

int qless_tune_get(int64_t n, int32_t* waves_per_cu, int32_t* fan_in, int32_t* rows_per_lane) {
    return tsqr_tune_get(n, waves_per_cu, fan_in, rows_per_lane);
}

int qless_batch_plan_create(const qless_matrix_desc* descs, int32_t count, int64_t tile_bytes, int32_t waves_per_cu,
                            qless_batch_plan** plan) {
    return batch_plan_create(descs, count, tile_bytes, waves_per_cu, plan);
}

void qless_batch_plan_destroy(qless_batch_plan* plan) { batch_plan_destroy(plan); }

size_t qless_batch_plan_workspace_bytes(const qless_batch_plan* plan) { return batch_plan_bytes(plan); }

int64_t qless_batch_plan_tiles(const qless_batch_plan* plan) { return batch_plan_tiles(plan); }

int qless_batch_plan_upload(const qless_batch_plan* plan, void* work, size_t work_bytes, hipStream_t stream) {
    return batch_plan_upload(plan, work, work_bytes, stream);
}

int qless_tsqr_r_batched(const qless_batch_plan* plan, void* work, size_t work_bytes, hipStream_t stream) {
    return batch_run(plan, work, work_bytes, stream);
}

int qless_timing_enable(int on) {
    g_timing = (on != 0);
    return QLESS_OK;
}

int qless_timing_reset(void) {
    for (auto& s : g_slots) {
        timing_collect(s);
        s.total_ms = 0.0;
        s.count = 0;
    }
    return QLESS_OK;
}

int qless_timing_read(const char* kernel, double* total_ms, int64_t* count) {
    if (kernel == nullptr || total_ms == nullptr || count == nullptr) return QLESS_ERR_ARG;
    for (int i = 0; i < kTimeSlots; ++i)
        if (strcmp(kernel, g_slot_names[i]) == 0) {
            timing_collect(g_slots[i]);
            *total_ms = g_slots[i].total_ms;
            *count = g_slots[i].count;
            return QLESS_OK;
        }
    return QLESS_ERR_ARG;
}

}  // extern "C"
