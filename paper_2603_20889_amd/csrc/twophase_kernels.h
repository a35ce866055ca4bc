// Two-phase orthogonalisation in one streaming pass (the "two-phase problem"
// named in Sec. 2): orthogonalise X (m x n) against an m x p Y with
// orthonormal columns and factor what is left, Q R = (I - Y Y^T) X, together
// with B = Y^T X.
//
// One Q-less TSQR (Alg. 2-4) of the concatenation [Y X] gives both: its R is
// [[R11, R12], [0, R22]] with [Y X] = [Q1 Q2] R, and since Y = Q1 R11 has
// orthonormal columns, R11 = I (diagonal made non-negative), R12 = Q1^T X =
// Y^T X = B and Q2 R22 = X - Y B, so R22 = R((I - Y Y^T) X).  The kernel is
// the stage-1 fold of qless_tsqr_r with a panel loader that reads columns
// 0..p-1 of a row from Y and columns p..p+n-1 from X: [Y X] is never formed
// and Y and X are each read once.  The tree levels are those of qless_tsqr_r
// on the stacked (p+n) x (p+n) triangles.
#pragma once

#include "tsqr_kernels.h"

namespace qless {
namespace tsqr_detail {

// Row-major sources of [Y X]: Y (p columns, may be null when p == 0) and X.
struct CatSrc {
    const double* Y;
    int64_t ldy;
    int p;
    const double* X;
    int64_t ldx;
    int n;
};

// Full panels (all 64 RPL or 8 RPL rows present) through buffer loads, as
// the TSQR fold loads X: one resource per source, rebased at the panel, the
// row offset of a lane in a VGPR and the stripe offset in an SGPR.  Whether
// a column comes from Y or X is the same for every lane in the n <= 16
// layout; in the column-group layout it is the same for every lane of a
// column slot except the one slot that straddles column p, which takes both
// loads under complementary lane masks (G lanes per row group: 8 for the
// 8 x 8 layout, 16 for the 4 x 16 one).  Columns >= p + n are zero.  The
// host rejects leading dimensions for which a panel's byte offsets would not
// fit 31 bits.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cat_rsrc(const double* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(base), (short)0, 0x7FFFFFFF, 0x00020000);
}

__device__ __forceinline__ double cat_ld(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}

__device__ __forceinline__ f64x2 cat_ld2(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
    return __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
}

// Element c of a row: wave-uniform branches on the source.
__device__ __forceinline__ double cat_elem(const CatSrc& s, __amdgpu_buffer_rsrc_t ry, __amdgpu_buffer_rsrc_t rx,
                                           int vy, int vx, int sy, int sx, int c) {
    if (c < s.p) return cat_ld(ry, vy + c * 8, sy);
    if (c < s.p + s.n) return cat_ld(rx, vx + (c - s.p) * 8, sx);
    return 0.0;
}

template <int NP, int RPL>
__device__ __forceinline__ void load_cat_1d_fast(double (&x)[RPL][NP], const CatSrc& s, int64_t base, int lane) {
    const __amdgpu_buffer_rsrc_t ry = cat_rsrc(s.p > 0 ? s.Y + base * s.ldy : s.X);
    const __amdgpu_buffer_rsrc_t rx = cat_rsrc(s.X + base * s.ldx);
    const int vy = lane * (int)(s.ldy * 8), vx = lane * (int)(s.ldx * 8);
    const int sy = (int)(kWave * s.ldy * 8), sx = (int)(kWave * s.ldx * 8);
    const int w = s.p + s.n;
    // a row's columns back to back; two columns of one source in one 16-byte load
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
#pragma unroll
        for (int c = 0; c < NP; c += 2) {
            if (c + 1 < NP && c + 1 < s.p) {
                const f64x2 v = cat_ld2(ry, vy + c * 8, sy * i);
                x[i][c] = v[0];
                x[i][c + 1] = v[1];
            } else if (c + 1 < NP && c >= s.p && c + 1 < w) {
                const f64x2 v = cat_ld2(rx, vx + (c - s.p) * 8, sx * i);
                x[i][c] = v[0];
                x[i][c + 1] = v[1];
            } else {
                x[i][c] = cat_elem(s, ry, rx, vy, vx, sy * i, sx * i, c);
                if (c + 1 < NP) x[i][c + 1] = cat_elem(s, ry, rx, vy, vx, sy * i, sx * i, c + 1);
            }
        }
    }
}

template <int NP, int RPL, int G = kG2>
__device__ __forceinline__ void load_cat_2d_fast(double (&x)[RPL][NP / G], const CatSrc& s, int64_t base,
                                                 int lane) {
    constexpr int NC = NP / G;
    const int rg = lane / G, cg = lane % G;
    const __amdgpu_buffer_rsrc_t ry = cat_rsrc(s.p > 0 ? s.Y + base * s.ldy : s.X);
    const __amdgpu_buffer_rsrc_t rx = cat_rsrc(s.X + base * s.ldx);
    const int sy = (int)((kWave / G) * s.ldy * 8), sx = (int)((kWave / G) * s.ldx * 8);
    const int w = s.p + s.n;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
        const int c = cg + G * u;
        const int c0 = G * u;                          // first column of the slot (wave-uniform)
        if (c0 + G <= s.p) {                           // every lane reads Y
            const int vo = (int)((rg * s.ldy + c) * 8);
#pragma unroll
            for (int i = 0; i < RPL; ++i) x[i][u] = cat_ld(ry, vo, sy * i);
        } else if (c0 >= s.p) {                        // every lane reads X (or padding)
            const bool ok = c < w;
            const int vo = (int)((rg * s.ldx + (ok ? c - s.p : 0)) * 8);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const double v = cat_ld(rx, vo, sx * i);
                x[i][u] = ok ? v : 0.0;
            }
        } else {                                       // the slot across column p
            const bool fy = c < s.p, ok = c < w;
            const int vo = fy ? (int)((rg * s.ldy + c) * 8) : (int)((rg * s.ldx + (ok ? c - s.p : 0)) * 8);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                double v;
                if (fy) v = cat_ld(ry, vo, sy * i);
                else v = cat_ld(rx, vo, sx * i);
                x[i][u] = (fy || ok) ? v : 0.0;
            }
        }
    }
}


// The last, partial panel of a wavefront (rows_left < the panel's rows): a
// row past the end reads the panel's first row (in bounds) and is zeroed.
template <int NP, int RPL>
__device__ __forceinline__ void load_cat_1d_part(double (&x)[RPL][NP], const CatSrc& s, int64_t base,
                                                 int rows_left, int lane) {
    const __amdgpu_buffer_rsrc_t ry = cat_rsrc(s.p > 0 ? s.Y + base * s.ldy : s.X);
    const __amdgpu_buffer_rsrc_t rx = cat_rsrc(s.X + base * s.ldx);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int row = lane + kWave * i;
        const bool ok = row < rows_left;
        const int vy = (ok ? row : 0) * (int)(s.ldy * 8), vx = (ok ? row : 0) * (int)(s.ldx * 8);
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            double v = 0.0;
            if (c < s.p) v = cat_ld(ry, vy + c * 8, 0);
            else if (c < s.p + s.n) v = cat_ld(rx, vx + (c - s.p) * 8, 0);
            x[i][c] = ok ? v : 0.0;
        }
    }
}

template <int NP, int RPL, int G = kG2>
__device__ __forceinline__ void load_cat_2d_part(double (&x)[RPL][NP / G], const CatSrc& s, int64_t base,
                                                 int rows_left, int lane) {
    constexpr int NC = NP / G;
    const int rg = lane / G, cg = lane % G;
    const __amdgpu_buffer_rsrc_t ry = cat_rsrc(s.p > 0 ? s.Y + base * s.ldy : s.X);
    const __amdgpu_buffer_rsrc_t rx = cat_rsrc(s.X + base * s.ldx);
    const int w = s.p + s.n;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int row = rg + (kWave / G) * i;
        const bool ok = row < rows_left;
        const int r = ok ? row : 0;
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int c = cg + G * u;
            double v;
            if (c < s.p) v = cat_ld(ry, (int)((r * s.ldy + c) * 8), 0);
            else v = cat_ld(rx, (int)((r * s.ldx + (c < w ? c - s.p : 0)) * 8), 0);
            x[i][u] = (ok && c < w) ? v : 0.0;
        }
    }
}

// Lane-private fold (n <= 8) of the full panels [base, base + nfull*PANEL)
// read by the two-source loader: the structure of the TSQR fold's
// lane-private path (each lane folds its own rows into its own triangle in
// registers, panel p+1 loaded while panel p is folded, the 64 triangles
// combined once at the end by the cross-lane fold).
template <int NP, int RPL>
__device__ __forceinline__ void fold_cat_lane_private(const CatSrc& s, int64_t base, int64_t nfull,
                                                      double* __restrict__ Rw, double* __restrict__ Cw,
                                                      const LaneOrigins<NP>& org, int lane) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    double Rl[tri_size<NP>()];
#pragma unroll
    for (int e = 0; e < tri_size<NP>(); ++e) Rl[e] = 0.0;
    double xa[RPL][NP];
    if constexpr (double_buffered<NP, RPL>()) {
        double xb[RPL][NP];
        const int64_t last = base + (nfull - 1) * PANEL;
        load_cat_1d_fast<NP, RPL>(xa, s, base, lane);
        while (true) {
            load_cat_1d_fast<NP, RPL>(xb, s, base + PANEL < last ? base + PANEL : last, lane);
            LaneFoldStep<NP, RPL, 0>::run(xa, Rl);
            base += PANEL;
            if (base > last) break;
            load_cat_1d_fast<NP, RPL>(xa, s, base + PANEL < last ? base + PANEL : last, lane);
            LaneFoldStep<NP, RPL, 0>::run(xb, Rl);
            base += PANEL;
            if (base > last) break;
        }
    } else {
        for (int64_t p = 0; p < nfull; ++p, base += PANEL) {
            load_cat_1d_fast<NP, RPL>(xa, s, base, lane);
            LaneFoldStep<NP, RPL, 0>::run(xa, Rl);
        }
    }
    double xe[NP][NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int c = 0; c < NP; ++c) xe[i][c] = (c >= i) ? Rl[tri_row<NP>(i) + c - i] : 0.0;
    FoldStep<NP, NP, 0>::run(xe, Rw, Cw, org, lane);
}

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_cat(const CatSrc& s, int64_t r_begin, int64_t r_end,
                                              double* __restrict__ Rw, int lane) {
    if constexpr (NP <= 16) {
        constexpr int64_t PANEL = (int64_t)kWave * RPL;
        LaneOrigins<NP> org;
        org.init(lane);
        double* Cw = Rw + tri_size<NP>();
        int64_t base = r_begin;
        if constexpr (lane_private<NP>()) {
            // n <= 8: lane-private folds of the full panels, as in the TSQR fold
            const int64_t nfull = (r_end - r_begin) / PANEL;
            if (nfull >= kLanePrivateMin) {
                fold_cat_lane_private<NP, RPL>(s, base, nfull, Rw, Cw, org, lane);
                base += nfull * PANEL;
            }
        }
        for (; base + PANEL <= r_end; base += PANEL) {
            double x[RPL][NP];
            load_cat_1d_fast<NP, RPL>(x, s, base, lane);
            FoldStep<NP, RPL, 0>::run(x, Rw, Cw, org, lane);
        }
        if (base < r_end) {                       // the partial last panel
            double x[RPL][NP];
            load_cat_1d_part<NP, RPL>(x, s, base, (int)(r_end - base), lane);
            FoldStep<NP, RPL, 0>::run(x, Rw, Cw, org, lane);
        }
    } else if constexpr (g16_instance<NP, RPL>()) {
        // the 4 x 16 column-group layout (n = 48, 64), as in the TSQR fold
        constexpr int64_t PANEL = (int64_t)kRG4 * RPL;
        int64_t base = r_begin;
        for (; base + PANEL <= r_end; base += PANEL) {
            double x[RPL][NP / kG4];
            load_cat_2d_fast<NP, RPL, kG4>(x, s, base, lane);
            FoldStepG16<NP, RPL, 0>::run(x, Rw, lane);
        }
        if (base < r_end) {                       // the partial last panel
            double x[RPL][NP / kG4];
            load_cat_2d_part<NP, RPL, kG4>(x, s, base, (int)(r_end - base), lane);
            FoldStepG16<NP, RPL, 0>::run(x, Rw, lane);
        }
    } else {
        constexpr int64_t PANEL = (int64_t)kRG2 * RPL;
        int64_t base = r_begin;
        for (; base + PANEL <= r_end; base += PANEL) {
            double x[RPL][NP / kG2];
            load_cat_2d_fast<NP, RPL>(x, s, base, lane);
            FoldStep2D<NP, RPL, 0>::run(x, Rw, lane);
        }
        if (base < r_end) {                       // the partial last panel
            double x[RPL][NP / kG2];
            load_cat_2d_part<NP, RPL>(x, s, base, (int)(r_end - base), lane);
            FoldStep2D<NP, RPL, 0>::run(x, Rw, lane);
        }
    }
}

// Stage 1 over [Y X]: as tsqr_fold_kernel (one wavefront per contiguous row
// block, the workgroup's triangles combined in LDS in wavefront order, one
// triangle per workgroup written to out + blockIdx.x * ostride).
template <int NP, int RPL>
__global__ void __launch_bounds__((64 * waves_per_block<NP, RPL>())) __attribute__((amdgpu_waves_per_eu(2)))
tsqr_cat_fold_kernel(CatSrc s, int64_t m, int64_t rows_per_wave, int64_t nwaves, double* __restrict__ out,
                     int64_t ldo, int64_t ostride, int normalise) {
    constexpr int WPB = waves_per_block<NP, RPL>();
    constexpr int STRIDE = tri_size<NP>() + NP;
    __shared__ double Rsh[WPB][STRIDE];
    __shared__ int arrivals;
    if (threadIdx.x == 0) arrivals = 0;
    __syncthreads();
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w0 = (int64_t)blockIdx.x * WPB;
    const int64_t w = w0 + wib;
    if (w >= nwaves) return;
    const int nvalid = (int)(nwaves - w0 < WPB ? nwaves - w0 : WPB);
    const int width = s.p + s.n;
    double* Rw = Rsh[wib];
    zero_r<NP>(Rw, lane);
    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    if (r_begin < r_end) fold_rows_cat<NP, RPL>(s, r_begin, r_end, Rw, lane);
    if (nvalid > 1) {
        int old = 0;
        if (lane == 0) old = __hip_atomic_fetch_add(&arrivals, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old != nvalid - 1) return;
        fold_block_triangles<NP, RPL>(&Rsh[0][0], STRIDE, nvalid, width, lane);
        Rw = Rsh[0];
    }
    store_r<NP>(Rw, width, out + (int64_t)blockIdx.x * ostride, ldo, normalise != 0, lane);
}

template <int NP, int RPL>
hipError_t launch_cat_fold(const CatSrc& s, int64_t m, int64_t rows_per_wave, int64_t nwaves, double* out,
                           int64_t ldo, int64_t ostride, int normalise, hipStream_t stream) {
    constexpr int WPB = waves_per_block<NP, RPL>();
    hipLaunchKernelGGL((tsqr_cat_fold_kernel<NP, RPL>), dim3((unsigned)ceil_div(nwaves, WPB)), dim3(64 * WPB), 0,
                       stream, s, m, rows_per_wave, nwaves, out, ldo, ostride, normalise);
    return hipGetLastError();
}

}  // namespace tsqr_detail
}  // namespace qless
