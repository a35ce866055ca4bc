// Gram kernels for the Q-less Cholesky-QR2 and SVQB2 forms (paper Sec. 3.1).
//
//   pass 1  (tsmttsm):               C = X^T X
//   pass 2  (tsmRttsmR / tsmmttsmm): C = (X M)^T (X M) with M = R1^{-1}
//                                    (CholQR2) or M = U1 L1^{-1/2} (SVQB2),
//                                    never storing X M.
//
// Layout: a wavefront splits its 64 lanes into G = 64/NP row groups of NP
// lanes; lane (g, i) owns column i of the rows of group g.  X is staged
// through a wavefront-private LDS slab loaded with coalesced row-major reads
// (lane (g, i) loads exactly its own entries), so every lane can read a
// whole row as a broadcast.  Lane (g, i) then forms y_i = sum_k x_k M_ki
// (M column i in registers), writes it back to LDS, and accumulates
// acc_c += y_i y_c for every c: row i of the wavefront's partial Gram
// matrix.  At the end the G groups are summed and each wavefront writes its
// n x n partial to the workspace; gram_sum adds the partials in a fixed order
// (no atomics, so results are reproducible bit for bit).
#include "tsqr_kernels.h"

namespace qless {
namespace {

template <int NP>
struct GramShape {
    static constexpr int G = kWave / NP;            // row groups per wavefront
    static constexpr int SR = 512 / NP;             // rows per LDS slab (512 elements)
    static constexpr int LD = NP >= 8 ? NP + 2 : NP; // padded row stride in LDS
    static constexpr int PER_LANE = SR / G;         // rows per lane per slab (= 8)
};

template <int NP, bool HAS_M>
__global__ void __launch_bounds__(256)
gram_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
            int64_t nwaves, const double* __restrict__ M, double* __restrict__ Cpart) {
    using S = GramShape<NP>;
    __shared__ double slab[4][2][S::SR * S::LD];
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (SGPR)
    const int64_t w = (int64_t)blockIdx.x * 4 + wib;
    if (w >= nwaves) return;
    const int g = lane / NP;
    const int i = lane % NP;
    double* xs = slab[wib][0];
    double* ys = slab[wib][1];

    double mcol[NP];
    if (HAS_M) {
#pragma unroll
        for (int k = 0; k < NP; ++k) mcol[k] = (k < n && i < n) ? M[(int64_t)k * n + i] : 0.0;
    }
    double acc[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) acc[c] = 0.0;

    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    for (int64_t base = r_begin; base < r_end; base += S::SR) {
        // coalesced load: lane (g, i) fetches rows g + G*t, column i
#pragma unroll
        for (int t = 0; t < S::PER_LANE; ++t) {
            const int r = g + S::G * t;
            const int64_t row = base + r;
            double v = 0.0;
            if (row < r_end && i < n) v = X[row * ldx + i];
            xs[r * S::LD + i] = v;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int t = 0; t < S::PER_LANE; ++t) {
            const int r = g + S::G * t;
            const double* xr = xs + r * S::LD;
            if (HAS_M) {
                double y = 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k) y = fma(xr[k], mcol[k], y);
                ys[r * S::LD + i] = y;
            }
        }
        __builtin_amdgcn_wave_barrier();
        const double* src = HAS_M ? ys : xs;
#pragma unroll
        for (int t = 0; t < S::PER_LANE; ++t) {
            const int r = g + S::G * t;
            const double* yr = src + r * S::LD;
            const double yi = yr[i];
#pragma unroll
            for (int c = 0; c < NP; ++c) acc[c] = fma(yi, yr[c], acc[c]);
        }
        __builtin_amdgcn_wave_barrier();
    }

    // sum the G row groups: lanes i, i + NP, i + 2NP, ...
#pragma unroll
    for (int c = 0; c < NP; ++c) {
        double v = acc[c];
#pragma unroll
        for (int d = NP; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
        acc[c] = v;
    }
    if (g == 0 && i < n) {
        double* out = Cpart + w * (int64_t)n * n + (int64_t)i * n;
#pragma unroll
        for (int c = 0; c < NP; ++c)
            if (c < n) out[c] = acc[c];
    }
}

// Row layout for n <= 8: each lane holds RPL full rows of a 64*RPL-row panel
// (the TSQR stage-1 loads), forms y = x M one row at a time (M from LDS,
// broadcast reads) and accumulates the n(n+1)/2 products y_a y_b of the upper
// triangle in registers.  Nothing crosses lanes until the end, where one
// transposed butterfly sums all accumulators over the wavefront.
template <int NP, int RPL, bool HAS_M>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
gram_rows_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                 int64_t nwaves, const double* __restrict__ M, double* __restrict__ Cpart) {
    constexpr int K = NP * (NP + 1) / 2;
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    __shared__ double Ms[NP * NP];
    const int lane = lane_id();
    if (HAS_M) {
        for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
            const int k = e / NP, c = e % NP;
            Ms[e] = (k < n && c < n) ? M[(int64_t)k * n + c] : 0.0;
        }
        __syncthreads();
    }
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nwaves) return;
    double acc[K];
#pragma unroll
    for (int t = 0; t < K; ++t) acc[t] = 0.0;
    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    const bool fast = (n == NP) && (PANEL * ldx * 8 < 0x7FFFFFFF);
    for (int64_t base = r_begin; base < r_end; base += PANEL) {
        double x[RPL][NP];
        if (fast && base + PANEL <= r_end) tsqr_detail::load_panel_1d_fast<NP, RPL>(x, X, ldx, base, lane);
        else tsqr_detail::load_panel_1d_tail<NP, RPL>(x, X, n, ldx, base, r_end, lane);
        if (HAS_M) {
            // y = x M for the lane's RPL rows, one column of M at a time so that
            // each M entry is read once from LDS and used for every row
            double y[RPL][NP];
#pragma unroll
            for (int c = 0; c < NP; ++c) {
#pragma unroll
                for (int i = 0; i < RPL; ++i) y[i][c] = 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double mkc = Ms[k * NP + c];
#pragma unroll
                    for (int i = 0; i < RPL; ++i) y[i][c] = fma(x[i][k], mkc, y[i][c]);
                }
                asm volatile("" ::: "memory");   // keep the M reads of later columns here (register pressure)
            }
#pragma unroll
            for (int i = 0; i < RPL; ++i)
#pragma unroll
                for (int c = 0; c < NP; ++c) x[i][c] = y[i][c];
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            int t = 0;
#pragma unroll
            for (int a = 0; a < NP; ++a)
#pragma unroll
                for (int b = a; b < NP; ++b, ++t) acc[t] = fma(x[i][a], x[i][b], acc[t]);
        }
    }
    double tot[K];
    wave_sum_multi<K>(acc, tot, lane);
    if (lane < n) {
        // row `lane` of the symmetric partial
        double* out = Cpart + w * (int64_t)n * n + (int64_t)lane * n;
        int t = 0;
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int b = a; b < NP; ++b, ++t) {
                if (a == lane && b < n) out[b] = tot[t];
                if (b == lane && a < n) out[a] = tot[t];
            }
    }
}

// C = sum over w < k of Cpart[w] (n x n), in a fixed order: each of the
// PARTS threads of an entry sums a contiguous range of w sequentially, and
// the PARTS subtotals are added pairwise in LDS.
__global__ void __launch_bounds__(256)
gram_sum_kernel(const double* __restrict__ Cpart, int64_t k, int n, double* __restrict__ C) {
    __shared__ double sub[256];
    const int nn = n * n;
    const int parts = 256 / 64;  // 4 threads per entry, 64 entries per block
    const int e = blockIdx.x * 64 + (threadIdx.x % 64);
    const int part = threadIdx.x / 64;
    const int64_t chunk = ceil_div(k, parts);
    const int64_t w0 = part * chunk;
    const int64_t w1 = (w0 + chunk < k) ? w0 + chunk : k;
    double s = 0.0;
    if (e < nn)
        for (int64_t w = w0; w < w1; ++w) s += Cpart[w * nn + e];
    sub[threadIdx.x] = s;
    __syncthreads();
    if (part == 0 && e < nn) {
        double a = sub[threadIdx.x] + sub[threadIdx.x + 64];
        double b = sub[threadIdx.x + 128] + sub[threadIdx.x + 192];
        C[e] = a + b;
    }
}

template <int NP, bool HAS_M>
hipError_t launch_gram_t(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                         const double* M, double* Cpart, hipStream_t s) {
    if constexpr (NP <= 8) {
        // with the fused multiply, half the rows per lane leave room for y = x M
        constexpr int RPL = HAS_M ? (NP >= 32 ? 1 : 32 / NP) : 64 / NP;
        hipLaunchKernelGGL((gram_rows_kernel<NP, RPL, HAS_M>), dim3((unsigned)ceil_div(nw, 4)), dim3(256), 0, s,
                           X, m, n, ldx, rpw, nw, M, Cpart);
    } else {
        hipLaunchKernelGGL((gram_kernel<NP, HAS_M>), dim3((unsigned)ceil_div(nw, 4)), dim3(256), 0, s, X, m, n,
                           ldx, rpw, nw, M, Cpart);
    }
    return hipGetLastError();
}

int gram_npad(int64_t n) {
    int np = 1;
    while (np < n) np <<= 1;
    return np;
}

}  // namespace

GramPlan make_gram_plan(int64_t m, int64_t n, int num_cus) {
    GramPlan p;
    p.npad = gram_npad(n);
    const int64_t slab = p.npad <= 8 ? (int64_t)kWave * (64 / p.npad) : 512 / p.npad;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * 8;
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, slab) * slab;
    p.rows_per_wave = rpw;
    p.k = m > 0 ? ceil_div(m, rpw) : 1;
    p.part_bytes = align_up((size_t)p.k * (size_t)(n * n) * sizeof(double), 256);
    return p;
}

hipError_t launch_gram(const double* X, int64_t m, int64_t n, int64_t ldx, const double* M, double* Cpart,
                       double* C, const GramPlan& plan, hipStream_t s) {
    const int ni = (int)n;
    hipError_t e = hipErrorInvalidValue;
    timing_begin(kTimeGram, s);
    const bool hm = (M != nullptr);
    switch (plan.npad) {
#define QLESS_GCASE(NP)                                                                              \
    case NP:                                                                                         \
        e = hm ? launch_gram_t<NP, true>(X, m, ni, ldx, plan.rows_per_wave, plan.k, M, Cpart, s)     \
               : launch_gram_t<NP, false>(X, m, ni, ldx, plan.rows_per_wave, plan.k, M, Cpart, s);   \
        break;
        QLESS_GCASE(1) QLESS_GCASE(2) QLESS_GCASE(4) QLESS_GCASE(8) QLESS_GCASE(16) QLESS_GCASE(32) QLESS_GCASE(64)
#undef QLESS_GCASE
        default: break;
    }
    timing_end(kTimeGram, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_sum_kernel, dim3((unsigned)ceil_div(n * n, 64)), dim3(256), 0, s, Cpart, plan.k, ni, C);
    return hipGetLastError();
}

}  // namespace qless
