// Q-less Householder TSQR for gfx950 (paper Alg. 2-4).
//
// Stage 1 (Alg. 2, first call; Alg. 3): the rows of X are split into k
// contiguous blocks, one per wavefront.  A wavefront streams its block in
// panels of 64*RPL rows -- lane l holds rows l, l+64, ..., l+64*(RPL-1) of the
// panel, full rows in registers -- and keeps the running triangle R of the
// rows seen so far in LDS.  Each panel W is folded in by the structured
// Householder QR of [R; W] (Alg. 4 without the column pairing): for column j
// the reflector pivots on R_jj and spans column j of W, so it has length
// 64*RPL + 1 and touches only row j of R and the panel.  Dot products over the
// panel rows are per-lane partial sums followed by a 64-lane butterfly; the
// reflector scalars are computed redundantly in every lane.  Q and the
// reflectors are never stored.  At the end the wavefront writes its R_i
// (n x n) into the stacked buffer Y.
//
// Stage 2 (Alg. 2, second call): the stacked triangles are reduced by a tree
// of the same kernel -- each wavefront of a level treats fan_in consecutive
// R_i as a tall (fan_in*n) x n matrix -- until one remains; the last launch
// writes R with its diagonal made non-negative.
#include "qless_internal.h"

namespace qless {
namespace {

// Rows of R in LDS: wavefront-private n x n row-major triangle (padded size).
template <int NP>
struct Tri {
    static constexpr int kElems = NP * NP;
};

// Fold one panel (registers x) into R (LDS, wavefront-private).
// Columns >= n of the padded instance hold zeros and stay zero.
template <int NP, int RPL>
__device__ __forceinline__ void fold_panel(double (&x)[RPL][NP], double* __restrict__ Rw) {
    constexpr int CH = 16;  // trailing columns reduced per butterfly batch
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const double alpha = Rw[j * NP + j];
        double u0 = 0.0, gamma = 0.0;
        bool active = false;
#pragma unroll
        for (int c0 = j; c0 < NP; c0 += CH) {
            double p[CH];
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const int c = c0 + t;
                if (c < NP) {
                    double s = 0.0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) s = fma(x[i][j], x[i][c], s);
                    p[t] = wave_sum_f64(s);
                }
            }
            if (c0 == j) {
                // p[0] = squared norm of the panel part of column j.
                const double s = p[0];
                active = (s != 0.0);
                if (active) {
                    const double nrm = sqrt(fma(alpha, alpha, s));
                    const double beta = (alpha >= 0.0) ? -nrm : nrm;
                    u0 = alpha - beta;                         // pivot entry of the reflector
                    gamma = 1.0 / (nrm * (nrm + fabs(alpha)));  // 2 / (u^T u)
                    Rw[j * NP + j] = beta;
                }
            }
            if (active) {
#pragma unroll
                for (int t = 0; t < CH; ++t) {
                    const int c = c0 + t;
                    if (c > j && c < NP) {
                        const double rjc = Rw[j * NP + c];
                        const double coef = gamma * fma(u0, rjc, p[t]);  // gamma * (u^T col_c)
#pragma unroll
                        for (int i = 0; i < RPL; ++i) x[i][c] = fma(-coef, x[i][j], x[i][c]);
                        Rw[j * NP + c] = fma(-coef, u0, rjc);
                    }
                }
            }
        }
    }
}

template <int NP>
constexpr int waves_per_block() {
    return (NP * NP * 8 * 4 <= 65536) ? 4 : 2;
}

// One kernel for stage 1 and every tree level.
//   X: rows [0, m) of a row-major matrix with leading dimension ldx, n columns.
//   Wavefront w owns rows [w*rows_per_wave, min(m, (w+1)*rows_per_wave)).
//   final == 0: write R_w (n x n, ld n) to Y + w*n*n.
//   final != 0: (single wavefront) write sign-normalised R to Y with ld ldy.
template <int NP, int RPL>
__global__ void __launch_bounds__(64 * waves_per_block<NP>())
tsqr_fold_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                 int64_t nwaves, double* __restrict__ Y, int64_t ldy, int final_write) {
    constexpr int WPB = waves_per_block<NP>();
    __shared__ double Rsh[WPB][NP * NP];
    const int lane = lane_id();
    const int wib = threadIdx.x >> 6;
    const int64_t w = (int64_t)blockIdx.x * WPB + wib;
    if (w >= nwaves) return;
    double* Rw = Rsh[wib];
    for (int e = lane; e < NP * NP; e += kWave) Rw[e] = 0.0;
    __builtin_amdgcn_wave_barrier();

    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    for (int64_t base = r_begin; base < r_end; base += (int64_t)kWave * RPL) {
        double x[RPL][NP];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int64_t row = base + lane + (int64_t)kWave * i;
            const bool ok = row < r_end;
            const double* xr = X + (ok ? row : 0) * ldx;
#pragma unroll
            for (int c = 0; c < NP; ++c) x[i][c] = (ok && c < n) ? xr[c] : 0.0;
        }
        fold_panel<NP, RPL>(x, Rw);
    }

    if (lane < n) {
        const int r = lane;
        double sgn = 1.0;
        if (final_write && Rw[r * NP + r] < 0.0) sgn = -1.0;
        double* out = final_write ? Y + (int64_t)r * ldy : Y + w * (int64_t)n * n + (int64_t)r * n;
        for (int c = 0; c < n; ++c) {
            double v = (c >= r) ? Rw[r * NP + c] : 0.0;
            out[c] = final_write ? sgn * v + 0.0 : v;
        }
    }
}

template <int NP, int RPL>
hipError_t launch_fold(const double* X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                       int64_t nwaves, double* Y, int64_t ldy, int final_write, hipStream_t stream) {
    constexpr int WPB = waves_per_block<NP>();
    const int64_t blocks = ceil_div(nwaves, WPB);
    hipLaunchKernelGGL((tsqr_fold_kernel<NP, RPL>), dim3((unsigned)blocks), dim3(64 * WPB), 0, stream,
                       X, m, n, ldx, rows_per_wave, nwaves, Y, ldy, final_write);
    return hipGetLastError();
}

// Padded column counts with a kernel instance, and their panel rows per lane.
struct Instance {
    int npad;
    int rpl;
};

Instance instance_for(int64_t n) {
    static const int pads[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64};
    int np = 64;
    for (int p : pads)
        if (n <= p) { np = p; break; }
    int rpl = np <= 8 ? 8 : np <= 16 ? 4 : np <= 32 ? 2 : 1;
    return {np, rpl};
}

hipError_t dispatch_fold(int np, const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                         double* Y, int64_t ldy, int fin, hipStream_t s) {
    switch (np) {
#define QLESS_CASE(NP, RPL) \
    case NP: return launch_fold<NP, RPL>(X, m, n, ldx, rpw, nw, Y, ldy, fin, s);
        QLESS_CASE(1, 8) QLESS_CASE(2, 8) QLESS_CASE(3, 8) QLESS_CASE(4, 8)
        QLESS_CASE(5, 8) QLESS_CASE(6, 8) QLESS_CASE(7, 8) QLESS_CASE(8, 8)
        QLESS_CASE(10, 4) QLESS_CASE(12, 4) QLESS_CASE(14, 4) QLESS_CASE(16, 4)
        QLESS_CASE(20, 2) QLESS_CASE(24, 2) QLESS_CASE(28, 2) QLESS_CASE(32, 2)
        QLESS_CASE(40, 1) QLESS_CASE(48, 1) QLESS_CASE(56, 1) QLESS_CASE(64, 1)
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
    const int64_t panel = (int64_t)kWave * in.rpl;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * 8;
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, panel) * panel;
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
