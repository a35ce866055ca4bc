// Host side of the Q-less TSQR (paper Alg. 2): launch plan (stage-1
// wavefront count, rows per wavefront, tree levels, workspace) and the
// stage-1 + tree launch sequence.  The kernels are in tsqr_kernels.h and are
// instantiated per padded column count in tsqr_i*.hip.
#include "tsqr_kernels.h"

namespace qless {

hipError_t launch_fold_np1(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np2(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np3(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np4(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np5(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np6(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np7(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np8(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np10(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np12(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np14(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np16(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np24(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np32(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np40(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np48(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np56(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);
hipError_t launch_fold_np64(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw, double* Y,
                          int64_t ldy, int fin, hipStream_t s);

namespace {

// Padded column counts with a kernel instance, and their panel rows per lane.
struct Instance {
    int npad;
    int rpl;
};

Instance instance_for(int64_t n) {
    static const int pads[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 24, 32, 40, 48, 56, 64};
    int np = 64;
    for (int p : pads)
        if (n <= p) { np = p; break; }
    // n <= 16: RPL full rows per lane; n > 16: RPL rows of NP/8 columns per lane
    int rpl = np <= 16 ? 64 / np : np == 64 ? 7 : 64 / (np / 8);
    return {np, rpl};
}

hipError_t dispatch_fold(int np, const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                         double* Y, int64_t ldy, int fin, hipStream_t s) {
    switch (np) {
#define QLESS_CASE(NP, RPL) \
    case NP: return launch_fold_np##NP(X, m, n, ldx, rpw, nw, Y, ldy, fin, s);
        QLESS_CASE(1, 64) QLESS_CASE(2, 32) QLESS_CASE(3, 21) QLESS_CASE(4, 16)
        QLESS_CASE(5, 12) QLESS_CASE(6, 10) QLESS_CASE(7, 9) QLESS_CASE(8, 8)
        QLESS_CASE(10, 6) QLESS_CASE(12, 5) QLESS_CASE(14, 4) QLESS_CASE(16, 4)
        QLESS_CASE(24, 21) QLESS_CASE(32, 16) QLESS_CASE(40, 12) QLESS_CASE(48, 10)
        QLESS_CASE(56, 9) QLESS_CASE(64, 7)
#undef QLESS_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

TsqrPlan make_tsqr_plan(int64_t m, int64_t n, int num_cus) {
    TsqrPlan p;
    Instance in = instance_for(n);
    p.npad = in.npad;
    p.rows_per_lane = in.rpl;
    const int64_t panel = (int64_t)(in.npad <= 16 ? kWave : tsqr_detail::kRG2) * in.rpl;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * 8;
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, panel) * panel;
    // Small inputs (up to four panels) go to one wavefront: a tree launch
    // would cost more than folding the few extra panels.
    if (m <= 4 * panel) rpw = ceil_div(m > 0 ? m : 1, panel) * panel;
    p.rows_per_wave = rpw;
    p.k0 = m > 0 ? ceil_div(m, rpw) : 1;
    p.fan_in = 16;
    int levels = 0;
    for (int64_t k = p.k0; k > 1; k = ceil_div(k, p.fan_in)) ++levels;
    p.levels = levels;
    const size_t blk = (size_t)n * (size_t)n * sizeof(double);
    p.ybytes_a = align_up((size_t)p.k0 * blk, 256);
    p.ybytes_b = align_up((size_t)ceil_div(p.k0, p.fan_in) * blk, 256);
    p.work_bytes = levels == 0 ? 256 : p.ybytes_a + p.ybytes_b;
    return p;
}

hipError_t launch_tsqr(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                       void* work, const TsqrPlan& plan, hipStream_t stream) {
    if (plan.levels > 0 && work == nullptr) return hipErrorInvalidValue;  // the tree needs its buffers
    double* ya = static_cast<double*>(work);
    double* yb = reinterpret_cast<double*>(static_cast<char*>(work) + plan.ybytes_a);
    const int ni = (int)n;
    hipError_t e;
    timing_begin(kTimeTsqrStage1, stream);
    if (plan.levels == 0) {
        e = dispatch_fold(plan.npad, X, m, ni, ldx, plan.rows_per_wave, 1, R, ldr, 1, stream);
        timing_end(kTimeTsqrStage1, stream);
        return e;
    }
    e = dispatch_fold(plan.npad, X, m, ni, ldx, plan.rows_per_wave, plan.k0, ya, n, 0, stream);
    timing_end(kTimeTsqrStage1, stream);
    if (e != hipSuccess) return e;
    int64_t k = plan.k0;
    double* src = ya;
    double* dst = yb;
    const int64_t rpw = (int64_t)plan.fan_in * n;
    for (int l = 0; l < plan.levels; ++l) {
        const int64_t kn = ceil_div(k, plan.fan_in);
        const bool last = (kn == 1);
        e = dispatch_fold(plan.npad, src, k * n, ni, n, rpw, kn, last ? R : dst, last ? ldr : n,
                          last ? 1 : 0, stream);
        if (e != hipSuccess) return e;
        k = kn;
        double* t = src;
        src = dst;
        dst = t;
    }
    return hipSuccess;
}

}  // namespace qless
