// Host side of the one-pass two-phase orthogonalisation (qless_two_phase_r):
// plan, the stage-1 fold over [Y X], the tree of qless_tsqr_r and the split
// of the (p+n) x (p+n) R into B = R12 and R = R22.
#include <algorithm>

#include "twophase_kernels.h"

namespace qless {

// Kernel instances (twophase_i*.hip): launch_cat_np<NP>_r<RPL>.  The TSQR
// plan of a call is made for the same (NP, RPL), so that its rows per
// wavefront, workgroup size and tree match what the kernel writes.
#define QLESS_CAT_INSTANCES(X)                                                                   \
    X(1, 32) X(2, 16) X(3, 12) X(4, 8) X(5, 6) X(6, 6) X(7, 4) X(8, 4) X(10, 6) X(12, 5) X(14, 4) \
    X(16, 4) X(24, 21) X(32, 16) X(40, 12) X(48, 16) X(56, 8) X(64, 12)
#define QLESS_CAT_DECL(NP, RPL)                                                                         \
    hipError_t launch_cat_np##NP##_r##RPL(const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw, \
                                          double* out, int64_t ldo, int64_t ostride, int normalise, hipStream_t st);
QLESS_CAT_INSTANCES(QLESS_CAT_DECL)
#undef QLESS_CAT_DECL

namespace {

// Rows per lane of the two-phase instance of a padded width (0: none).
int cat_rpl(int npad) {
    switch (npad) {
#define QLESS_CAT_RPL(NP, RPL) \
    case NP: return RPL;
        QLESS_CAT_INSTANCES(QLESS_CAT_RPL)
#undef QLESS_CAT_RPL
        default: return 0;
    }
}

hipError_t launch_cat(int npad, int rpl, const tsqr_detail::CatSrc& s, int64_t m, int64_t rpw, int64_t nw,
                      double* out, int64_t ldo, int64_t ostride, int normalise, hipStream_t st) {
#define QLESS_CAT_CASE(NP, RPL) \
    if (npad == NP && rpl == RPL) return launch_cat_np##NP##_r##RPL(s, m, rpw, nw, out, ldo, ostride, normalise, st);
    QLESS_CAT_INSTANCES(QLESS_CAT_CASE)
#undef QLESS_CAT_CASE
    return hipErrorInvalidValue;
}

// The plan of a two-phase call: the untuned TSQR plan of width w, made for
// the two-phase instance of its padded width.
TsqrPlan cat_plan(int64_t m, int64_t w) {
    const int cus = current_device_info().num_cus;
    const TsqrPlan p0 = make_tsqr_plan(m, w, cus, false);
    return make_tsqr_plan(m, w, cus, false, cat_rpl(p0.npad));
}

// B (p x n, ld ldb) = rows 0..p-1, columns p.. of Rf; R (n x n, ld ldr) =
// the trailing block, zeros below the diagonal (Rf: w x w, ld w).
__global__ void __launch_bounds__(256)
split_two_phase_kernel(const double* __restrict__ Rf, int p, int n, double* __restrict__ B, int64_t ldb,
                       double* __restrict__ R, int64_t ldr) {
    const int w = p + n;
    for (int e = threadIdx.x; e < p * n; e += blockDim.x) {
        const int a = e / n, c = e - a * n;
        B[(int64_t)a * ldb + c] = Rf[a * w + p + c];
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e - i * n;
        R[(int64_t)i * ldr + c] = c >= i ? Rf[(p + i) * w + p + c] : 0.0;
    }
}

bool two_phase_sizes_ok(int64_t m, int64_t p, int64_t n) { return m >= 0 && p >= 0 && n >= 1; }

size_t two_phase_work(const TsqrPlan& plan, int64_t w) {
    return align_up((size_t)(w * w) * sizeof(double), 256) + plan.work_bytes;
}

}  // namespace
}  // namespace qless

using namespace qless;

extern "C" {

size_t qless_two_phase_workspace_bytes(int64_t m, int64_t p, int64_t n) {
    if (!two_phase_sizes_ok(m, p, n) || p + n > QLESS_MAX_N) return 0;
    return two_phase_work(cat_plan(m, p + n), p + n);
}

int qless_two_phase_r(const double* Y, int64_t p, int64_t ldy, const double* X, int64_t m, int64_t n, int64_t ldx,
                      double* B, int64_t ldb, double* R, int64_t ldr, void* work, size_t work_bytes,
                      hipStream_t stream) {
    if (!two_phase_sizes_ok(m, p, n)) return QLESS_ERR_ARG;
    if (p + n > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
    if (R == nullptr || ldr < n) return QLESS_ERR_ARG;
    if (m > 0 && (X == nullptr || ldx < n)) return QLESS_ERR_ARG;
    if (p > 0 && (B == nullptr || ldb < n)) return QLESS_ERR_ARG;
    if (p > 0 && m > 0 && (Y == nullptr || ldy < p)) return QLESS_ERR_ARG;
    const int64_t w = p + n;
    const TsqrPlan plan = cat_plan(m, w);
    // the kernel addresses a panel with 32-bit byte offsets
    const int64_t ld_max = std::max(p > 0 ? ldy : 0, m > 0 ? ldx : n);
    if (m > 0 && tsqr_panel_rows(plan.npad, plan.rows_per_lane) * ld_max * 8 >= 0x7FFFFFFF)
        return QLESS_ERR_UNSUPPORTED;
    const size_t need = two_phase_work(plan, w);
    if (work == nullptr || (reinterpret_cast<uintptr_t>(work) & 255u) != 0 || work_bytes < need)
        return QLESS_ERR_WORKSPACE;
    double* Rf = static_cast<double*>(work);
    double* tree = reinterpret_cast<double*>(static_cast<char*>(work) + align_up((size_t)(w * w) * sizeof(double), 256));
    const tsqr_detail::CatSrc s{p > 0 ? Y : nullptr, p > 0 ? ldy : 0, (int)p, X, m > 0 ? ldx : n, (int)n};
    hipError_t e;
    timing_begin(kTimeTsqrStage1, stream);
    if (plan.k1 == 1) {
        e = launch_cat(plan.npad, plan.rows_per_lane, s, m, plan.rows_per_wave, plan.k0, Rf, w, 0, 1, stream);
        timing_end(kTimeTsqrStage1, stream);
    } else {
        double* src = tree;
        double* dst = reinterpret_cast<double*>(reinterpret_cast<char*>(tree) + plan.ybytes_a);
        e = launch_cat(plan.npad, plan.rows_per_lane, s, m, plan.rows_per_wave, plan.k0, src, w, w * w, 0, stream);
        timing_end(kTimeTsqrStage1, stream);
        if (e == hipSuccess) e = launch_tsqr_tree(plan, src, dst, plan.k1, w, Rf, w, stream);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(split_two_phase_kernel, dim3(1), dim3(256), 0, stream, Rf, (int)p, (int)n, B, ldb, R, ldr);
        e = hipGetLastError();
    }
    return e == hipSuccess ? QLESS_OK : QLESS_ERR_HIP;
}

}  // extern "C"
