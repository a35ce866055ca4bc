// Host side of the Q-less TSQR (paper Alg. 2): launch plan (stage-1
// wavefront count, rows per wavefront, tree levels, workspace) and the
// stage-1 + tree launch sequence.  The kernels are in tsqr_kernels.h and are
// instantiated per padded column count in tsqr_i*.hip.
#include "tsqr_kernels.h"

namespace qless {

// Kernel instances (tsqr_i*.hip): launch_fold_np<NP>_r<RPL>.
#define QLESS_DECL(NP, RPL)                                                                              \
    hipError_t launch_fold_np##NP##_r##RPL(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, \
                                           int64_t nw, double* Y, int64_t ldy, int64_t ystride,         \
                                           int normalise, hipStream_t s);
#define QLESS_INSTANCES(X)                                                                          \
    X(1, 64) X(2, 32) X(3, 21) X(4, 16) X(5, 12) X(6, 10) X(7, 9) X(8, 8) X(10, 6) X(12, 5)          \
    X(14, 4) X(16, 4) X(24, 21) X(32, 16) X(40, 12) X(48, 10) X(56, 8) X(64, 7)                     \
    X(1, 32) X(2, 16) X(4, 8) X(8, 4) X(16, 2) X(32, 8) X(64, 4) X(8, 5) X(16, 3)
QLESS_INSTANCES(QLESS_DECL)
#undef QLESS_DECL

namespace {

typedef hipError_t (*FoldFn)(const double*, int64_t, int, int64_t, int64_t, int64_t, double*, int64_t, int64_t, int,
                              hipStream_t);

struct Instance {
    int npad;
    int rpl;
    FoldFn fn;
};

const Instance kInstances[] = {
#define QLESS_ENTRY(NP, RPL) {NP, RPL, launch_fold_np##NP##_r##RPL},
    QLESS_INSTANCES(QLESS_ENTRY)
#undef QLESS_ENTRY
};

int npad_for(int64_t n) {
    static const int pads[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 24, 32, 40, 48, 56, 64};
    for (int p : pads)
        if (n <= p) return p;
    return 64;
}

// Default instance of a padded width: n <= 16 keeps RPL = 64/NP full rows per
// lane (64 doubles); wider layouts keep about 64 doubles of RPL x NP/8.
const Instance* find_instance(int np, int rpl) {
    const Instance* def = nullptr;
    for (const Instance& in : kInstances) {
        if (in.npad != np) continue;
        if (in.rpl == rpl) return &in;
        if (!def) def = &in;   // the first listed instance of a width is its default
    }
    return def;
}

// Launch-parameter overrides per column count (set by the autotuner).
struct Tuning {
    int waves_per_cu = 0, fan_in = 0, rpl = 0;
};
Tuning g_tuning[QLESS_MAX_N + 1];

}  // namespace

int tsqr_tune_set(int64_t n, int waves_per_cu, int fan_in, int rpl) {
    if (n < 1 || n > QLESS_MAX_N || waves_per_cu < 0 || waves_per_cu > 32 || fan_in < 0 || fan_in == 1 ||
        fan_in > 256 || rpl < 0)
        return QLESS_ERR_ARG;
    if (rpl != 0) {
        const Instance* in = find_instance(npad_for(n), rpl);
        if (!in || in->rpl != rpl) return QLESS_ERR_UNSUPPORTED;
    }
    g_tuning[n] = Tuning{waves_per_cu, fan_in, rpl};
    return QLESS_OK;
}

int tsqr_tune_get(int64_t n, int* waves_per_cu, int* fan_in, int* rpl) {
    if (n < 1 || n > QLESS_MAX_N) return QLESS_ERR_ARG;
    const Tuning& t = g_tuning[n];
    const Instance* in = find_instance(npad_for(n), t.rpl);
    if (waves_per_cu) *waves_per_cu = t.waves_per_cu ? t.waves_per_cu : 8;
    if (fan_in) *fan_in = t.fan_in ? t.fan_in : 16;
    if (rpl) *rpl = in->rpl;
    return QLESS_OK;
}

TsqrPlan make_tsqr_plan(int64_t m, int64_t n, int num_cus) {
    TsqrPlan p;
    const Tuning t = (n >= 1 && n <= QLESS_MAX_N) ? g_tuning[n] : Tuning{};
    const Instance* in = find_instance(npad_for(n), t.rpl);
    p.npad = in->npad;
    p.rows_per_lane = in->rpl;
    const int64_t panel = (int64_t)(in->npad <= 16 ? kWave : tsqr_detail::kRG2) * in->rpl;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * (t.waves_per_cu ? t.waves_per_cu : 8);
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, panel) * panel;
    // Small inputs (up to four panels) go to one wavefront: a tree launch
    // would cost more than folding the few extra panels.
    if (m <= 4 * panel) rpw = ceil_div(m > 0 ? m : 1, panel) * panel;
    p.rows_per_wave = rpw;
    p.k0 = m > 0 ? ceil_div(m, rpw) : 1;
    p.fan_in = t.fan_in ? t.fan_in : 16;
    int levels = 0;
    for (int64_t k = p.k0; k > 1; k = ceil_div(k, p.fan_in)) ++levels;
    p.levels = levels;
    // two stacked buffers used in turn: level l reads one and writes the other
    const size_t blk = (size_t)n * (size_t)n * sizeof(double);
    p.ybytes_a = align_up((size_t)p.k0 * blk, 256);
    p.ybytes_b = align_up((size_t)ceil_div(p.k0, p.fan_in) * blk, 256);
    p.work_bytes = levels == 0 ? 256 : p.ybytes_a + p.ybytes_b;
    return p;
}

hipError_t launch_tsqr(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                       void* work, const TsqrPlan& plan, hipStream_t stream) {
    if (plan.levels > 0 && work == nullptr) return hipErrorInvalidValue;  // the tree needs its buffers
    const Instance* in = find_instance(plan.npad, plan.rows_per_lane);
    if (!in) return hipErrorInvalidValue;
    const int ni = (int)n;
    const int64_t nn = n * n;
    hipError_t e;
    timing_begin(kTimeTsqrStage1, stream);
    if (plan.levels == 0) {
        e = in->fn(X, m, ni, ldx, plan.rows_per_wave, 1, R, ldr, 0, 1, stream);
        timing_end(kTimeTsqrStage1, stream);
        return e;
    }
    double* src = static_cast<double*>(work);
    double* dst = reinterpret_cast<double*>(static_cast<char*>(work) + plan.ybytes_a);
    e = in->fn(X, m, ni, ldx, plan.rows_per_wave, plan.k0, src, n, nn, 0, stream);
    timing_end(kTimeTsqrStage1, stream);
    // tree (Alg. 2, second call, repeated): wavefront g of a level folds the
    // fan_in triangles g*fan_in .. of the previous level, read as one tall
    // (fan_in*n) x n matrix.
    const int64_t rpw = (int64_t)plan.fan_in * n;
    for (int64_t k = plan.k0; e == hipSuccess && k > 1;) {
        const int64_t kn = ceil_div(k, plan.fan_in);
        if (kn == 1) {
            e = in->fn(src, k * n, ni, n, rpw, 1, R, ldr, 0, 1, stream);
        } else {
            e = in->fn(src, k * n, ni, n, rpw, kn, dst, n, nn, 0, stream);
            double* t = src;
            src = dst;
            dst = t;
        }
        k = kn;
    }
    return e;
}

}  // namespace qless
