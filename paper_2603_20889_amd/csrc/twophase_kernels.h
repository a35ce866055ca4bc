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

// Source of column c of [Y X]: its base pointer and row stride (null for a
// padding column c >= p + n).  Chosen once per column, not per element.
__device__ __forceinline__ const double* cat_col(const CatSrc& s, int c, int64_t& ld) {
    if (c < s.p) {
        ld = s.ldy;
        return s.Y + c;
    }
    ld = s.ldx;
    return c < s.p + s.n ? s.X + (c - s.p) : nullptr;
}

// Layout of n <= 16 (lane l holds rows base + l + 64 i, every column).
template <int NP, int RPL>
__device__ __forceinline__ void load_cat_1d(double (&x)[RPL][NP], const CatSrc& s, int64_t base, int64_t r_end,
                                            int lane) {
    const double* col[NP];
    int64_t ld[NP];
#pragma unroll
    for (int c = 0; c < NP; ++c) col[c] = cat_col(s, c, ld[c]);   // wave-uniform
    // a row's columns back to back, so that each cache line is fetched once
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int64_t row = base + lane + (int64_t)kWave * i;
#pragma unroll
        for (int c = 0; c < NP; ++c) x[i][c] = (col[c] != nullptr && row < r_end) ? col[c][row * ld[c]] : 0.0;
    }
}

// Layout of 16 < n <= 64 (lane (rg, cg) holds rows base + rg + 8 i, columns
// cg + 8 u).
template <int NP, int RPL>
__device__ __forceinline__ void load_cat_2d(double (&x)[RPL][NP / kG2], const CatSrc& s, int64_t base,
                                            int64_t r_end, int lane) {
    constexpr int NC = NP / kG2;
    const int rg = lane / kG2, cg = lane % kG2;
    const double* col[NC];
    int64_t ld[NC];
#pragma unroll
    for (int u = 0; u < NC; ++u) col[u] = cat_col(s, cg + kG2 * u, ld[u]);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const int64_t row = base + rg + (int64_t)kRG2 * i;
#pragma unroll
        for (int u = 0; u < NC; ++u) x[i][u] = (col[u] != nullptr && row < r_end) ? col[u][row * ld[u]] : 0.0;
    }
}

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_cat(const CatSrc& s, int64_t r_begin, int64_t r_end,
                                              double* __restrict__ Rw, int lane) {
    if constexpr (NP <= 16) {
        constexpr int64_t PANEL = (int64_t)kWave * RPL;
        LaneOrigins<NP> org;
        org.init(lane);
        double* Cw = Rw + tri_size<NP>();
        for (int64_t base = r_begin; base < r_end; base += PANEL) {
            double x[RPL][NP];
            load_cat_1d<NP, RPL>(x, s, base, r_end, lane);
            FoldStep<NP, RPL, 0>::run(x, Rw, Cw, org, lane);
        }
    } else {
        constexpr int64_t PANEL = (int64_t)kRG2 * RPL;
        for (int64_t base = r_begin; base < r_end; base += PANEL) {
            double x[RPL][NP / kG2];
            load_cat_2d<NP, RPL>(x, s, base, r_end, lane);
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
