// Host side of the Q-less TSQR (paper Alg. 2): launch plan (stage-1
// wavefront count, rows per wavefront, tree levels, workspace) and the
// stage-1 + tree launch sequence.  The kernels are in tsqr_kernels.h and are
// instantiated per padded column count in tsqr_i*.hip.
#include <algorithm>

#include "tsqr_kernels.h"

namespace qless {


// Kernel instances (tsqr_i*.hip): launch_fold_np<NP>_r<RPL>.
#define QLESS_DECL(NP, RPL) hipError_t launch_fold_np##NP##_r##RPL(const FoldArgs& a, hipStream_t s);
#define QLESS_INSTANCES(X)                                                                          \
    X(1, 32) X(2, 16) X(3, 12) X(4, 8) X(5, 6) X(6, 6) X(7, 4) X(8, 4) X(10, 6) X(12, 5)              \
    X(14, 4) X(16, 4) X(24, 21) X(32, 16) X(40, 12) X(48, 16) X(56, 8) X(64, 12)                    \
    X(1, 64) X(2, 32) X(3, 21) X(4, 16) X(5, 12) X(6, 10) X(7, 9) X(8, 8) X(16, 2) X(32, 8) X(64, 4)  \
    X(16, 3) X(32, 1) X(48, 1) X(64, 1) X(32, 24) X(48, 10) X(64, 7)
QLESS_INSTANCES(QLESS_DECL)
#undef QLESS_DECL
// One-workgroup last tree level, compiled for n <= 16 (launch_tree_np<NP>_r<RPL>).
#define QLESS_TREE_DECL(NP, RPL)                                                                            \
    hipError_t launch_tree_np##NP##_r##RPL(const double* Y, int64_t k, int n, double* R, int64_t ldr, hipStream_t s);
#define QLESS_TREE_INSTANCES(X)                                                                         \
    X(1, 32) X(2, 16) X(3, 12) X(4, 8) X(5, 6) X(6, 6) X(7, 4) X(8, 4) X(10, 6) X(12, 5) X(14, 4)      \
    X(16, 4) X(1, 64) X(2, 32) X(3, 21) X(4, 16) X(5, 12) X(6, 10) X(7, 9) X(8, 8) X(16, 2) X(16, 3)
QLESS_TREE_INSTANCES(QLESS_TREE_DECL)
#undef QLESS_TREE_DECL

namespace {

typedef hipError_t (*TreeFn)(const double*, int64_t, int, double*, int64_t, hipStream_t);

struct Instance {
    int npad;
    int rpl;
    FoldFn fn;
    TreeFn tree;   // one-workgroup last level (n <= 16), else null
    int wpb;       // wavefronts per workgroup of the instance's fold kernel
    int64_t panel; // rows of one panel (the unit rows_per_wave is rounded to)
};

const Instance kInstances[] = {
#define QLESS_ENTRY(NP, RPL)                                                                  \
    {NP, RPL, launch_fold_np##NP##_r##RPL, nullptr, tsqr_detail::waves_per_block<NP, RPL>(), \
     tsqr_detail::panel_rows<NP, RPL>()},
    QLESS_INSTANCES(QLESS_ENTRY)
#undef QLESS_ENTRY
};

struct TreeEntry {
    int npad;
    int rpl;
    TreeFn fn;
};

const TreeEntry kTrees[] = {
#define QLESS_TREE_ENTRY(NP, RPL) {NP, RPL, launch_tree_np##NP##_r##RPL},
    QLESS_TREE_INSTANCES(QLESS_TREE_ENTRY)
#undef QLESS_TREE_ENTRY
};

TreeFn find_tree(int np, int rpl) {
    for (const TreeEntry& t : kTrees)
        if (t.npad == np && t.rpl == rpl) return t.fn;
    return nullptr;
}

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
    if (fan_in) *fan_in = make_tsqr_plan(1, n, 1).fan_in;
    if (rpl) *rpl = in->rpl;
    return QLESS_OK;
}

FoldFn find_fold(int npad, int rpl) {
    const Instance* in = find_instance(npad, rpl);
    return (in && in->npad == npad && in->rpl == rpl) ? in->fn : nullptr;
}

int64_t tsqr_panel_rows(int npad, int rpl) {
    const Instance* in = find_instance(npad, rpl);
    return in ? in->panel : 0;
}

TsqrPlan make_tsqr_plan(int64_t m, int64_t n, int num_cus, bool tuned, int rpl) {
    TsqrPlan p;
    const Tuning t = (tuned && n >= 1 && n <= QLESS_MAX_N) ? g_tuning[n] : Tuning{};
    const Instance* in = find_instance(npad_for(n), rpl ? rpl : t.rpl);
    p.npad = in->npad;
    p.rows_per_lane = in->rpl;
    const int64_t panel = in->panel;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * (t.waves_per_cu ? t.waves_per_cu : 8);
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, panel) * panel;
    // Small inputs (up to four panels) go to one wavefront: a tree launch
    // would cost more than folding the few extra panels.
    if (m <= 4 * panel) rpw = ceil_div(m > 0 ? m : 1, panel) * panel;
    p.rows_per_wave = rpw;
    p.k0 = m > 0 ? ceil_div(m, rpw) : 1;
    p.wpb = in->wpb;
    // Each launch leaves one triangle per workgroup.  Tree for n <= 16:
    // fan-in levels of one panel per wavefront (fan_in = panel / n) until the
    // remaining triangles fit two panels per wavefront of the one-workgroup
    // last level, which then writes R (two panels there cost less than one
    // more launch).  Wider n: fan-in 4 levels throughout -- a wavefront's
    // fold of 4n stacked rows is short, and the level keeps enough
    // wavefronts busy (at n = 64, fan-in 16 took 1.4 ms of tree, 4 took 0.8).
    p.block_tree = find_tree(in->npad, in->rpl) != nullptr;
    p.tree_rows = p.block_tree ? 2 * panel : 0;
    p.fan_in = t.fan_in ? t.fan_in : (p.block_tree ? (int)std::max<int64_t>(2, panel / n) : 4);
    p.k1 = ceil_div(p.k0, p.wpb);
    int levels = 0;
    int64_t k = p.k1;
    while (k > 1) {
        ++levels;
        if (p.block_tree && k * n <= (int64_t)tsqr_detail::kTreeWaves * p.tree_rows) break;
        k = ceil_div(ceil_div(k, p.fan_in), p.wpb);
    }
    p.levels = levels;
    // two stacked buffers used in turn: level l reads one and writes the other
    // (the last level's per-wavefront triangles go to the buffer not read)
    const size_t blk = (size_t)n * (size_t)n * sizeof(double);
    const size_t ybytes = align_up((size_t)std::max<int64_t>(p.k1, tsqr_detail::kTreeWaves) * blk, 256);
    p.ybytes_a = ybytes;
    p.ybytes_b = ybytes;
    p.work_bytes = levels == 0 ? 256 : p.ybytes_a + p.ybytes_b;
    return p;
}

namespace {

// Tree of Alg. 2 over the k >= 2 stacked triangles in src (the other buffer,
// dst, takes intermediate levels): wavefront g of a level folds the fan_in
// triangles g*fan_in .. of the previous level, read as one tall
// (fan_in*n) x n matrix, and each workgroup leaves one triangle; the last
// level writes R with a non-negative diagonal.
hipError_t launch_tree(const Instance* in, const TsqrPlan& plan, double* src, double* dst, int64_t k, int64_t n,
                       double* R, int64_t ldr, hipStream_t stream) {
    const int ni = (int)n;
    const int64_t nn = n * n;
    const int64_t rpw = (int64_t)plan.fan_in * n;
    TreeFn tree = plan.block_tree ? find_tree(plan.npad, plan.rows_per_lane) : nullptr;
    hipError_t e = hipSuccess;
    while (e == hipSuccess && k > 1) {
        if (tree && k * n <= (int64_t)tsqr_detail::kTreeWaves * plan.tree_rows) return tree(src, k, ni, R, ldr, stream);
        const int64_t nw = ceil_div(k, plan.fan_in);
        const int64_t kn = ceil_div(nw, plan.wpb);
        if (kn == 1) {
            e = in->fn(FoldArgs{src, k * n, ni, n, rpw, nw, R, ldr, 0, 1, nullptr}, stream);
        } else {
            e = in->fn(FoldArgs{src, k * n, ni, n, rpw, nw, dst, n, nn, 0, nullptr}, stream);
            double* t = src;
            src = dst;
            dst = t;
        }
        k = kn;
    }
    return e;
}

// Upper triangle of R (ld ldr) into an n x n slot (ld n), zeros below.
__global__ void copy_upper_kernel(const double* __restrict__ R, int64_t ldr, int n, double* __restrict__ out) {
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e - i * n;
        out[e] = c >= i ? R[(int64_t)i * ldr + c] : 0.0;
    }
}

}  // namespace

hipError_t launch_tsqr_tree(const TsqrPlan& plan, double* src, double* dst, int64_t k, int64_t n, double* R,
                            int64_t ldr, hipStream_t stream) {
    const Instance* in = find_instance(plan.npad, plan.rows_per_lane);
    if (!in) return hipErrorInvalidValue;
    return launch_tree(in, plan, src, dst, k, n, R, ldr, stream);
}

hipError_t launch_tsqr(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                       void* work, const TsqrPlan& plan, hipStream_t stream) {
    if (plan.levels > 0 && work == nullptr) return hipErrorInvalidValue;  // the tree needs its buffers
    const Instance* in = find_instance(plan.npad, plan.rows_per_lane);
    if (!in) return hipErrorInvalidValue;
    const int64_t nn = n * n;
    hipError_t e;
    timing_begin(kTimeTsqrStage1, stream);
    if (plan.k1 == 1) {
        e = in->fn(FoldArgs{X, m, (int)n, ldx, plan.rows_per_wave, plan.k0, R, ldr, 0, 1, nullptr}, stream);
        timing_end(kTimeTsqrStage1, stream);
        return e;
    }
    double* src = static_cast<double*>(work);
    double* dst = reinterpret_cast<double*>(static_cast<char*>(work) + plan.ybytes_a);
    e = in->fn(FoldArgs{X, m, (int)n, ldx, plan.rows_per_wave, plan.k0, src, n, nn, 0, nullptr}, stream);
    timing_end(kTimeTsqrStage1, stream);
    if (e != hipSuccess) return e;
    return launch_tree(in, plan, src, dst, plan.k1, n, R, ldr, stream);
}

TsqrPlan make_tsqr_update_plan(int64_t m, int64_t n, int num_cus) {
    TsqrPlan p = make_tsqr_plan(m, n, num_cus);
    // the previous R joins the stage-1 triangles as one more, so there is
    // always a tree and both stacked buffers hold k1 + 1 triangles
    const size_t blk = (size_t)n * (size_t)n * sizeof(double);
    const size_t ybytes = align_up((size_t)std::max<int64_t>(p.k1 + 1, tsqr_detail::kTreeWaves) * blk, 256);
    p.ybytes_a = ybytes;
    p.ybytes_b = ybytes;
    p.work_bytes = 2 * ybytes;
    if (p.levels == 0) p.levels = 1;
    return p;
}

hipError_t launch_tsqr_update(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                              void* work, const TsqrPlan& plan, hipStream_t stream) {
    if (work == nullptr) return hipErrorInvalidValue;
    const Instance* in = find_instance(plan.npad, plan.rows_per_lane);
    if (!in) return hipErrorInvalidValue;
    const int64_t nn = n * n;
    double* src = static_cast<double*>(work);
    double* dst = reinterpret_cast<double*>(static_cast<char*>(work) + plan.ybytes_a);
    int64_t k = 0;
    hipError_t e = hipSuccess;
    if (m > 0) {
        timing_begin(kTimeTsqrStage1, stream);
        e = in->fn(FoldArgs{X, m, (int)n, ldx, plan.rows_per_wave, plan.k0, src, n, nn, 0, nullptr}, stream);
        timing_end(kTimeTsqrStage1, stream);
        k = plan.k1;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(copy_upper_kernel, dim3(1), dim3(256), 0, stream, R, ldr, (int)n, src + k * nn);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ++k;
    if (k == 1) {   // no new rows: R([R]) is R with its diagonal made non-negative
        return in->fn(FoldArgs{src, n, (int)n, n, n, 1, R, ldr, 0, 1, nullptr}, stream);
    }
    return launch_tree(in, plan, src, dst, k, n, R, ldr, stream);
}

}  // namespace qless
