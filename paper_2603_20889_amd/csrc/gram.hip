// Gram kernels for the Q-less Cholesky-QR2 and SVQB2 forms (paper Sec. 3.1).
//
//   pass 1  (tsmttsm):               C = X^T X
//   pass 2  (tsmRttsmR / tsmmttsmm): C = (X M)^T (X M) with M = R1^{-1}
//                                    (CholQR2) or M = U1 L1^{-1/2} (SVQB2),
//                                    never storing X M.
//
// n <= 8 (gram_rows_kernel): each lane holds full rows (the TSQR panel
// loads), forms y = x M on the VALU and accumulates the n(n+1)/2 products of
// the upper triangle; one transposed butterfly sums them at the end.
//
// n > 8 (gram_mfma_kernel): FP64 matrix cores, v_mfma_f64_16x16x4f64
// (D[16x16] += A[16x4] B[4x16]; lane l holds A[l%16][l/16] and B[l/16][l%16],
// and D[4v + l/16][l%16] in its v-th accumulator, as measured on gfx950).
// Columns are cut into NB = ceil(n/16) blocks of 16.  For a block of 16 rows
// the Gram operand of column block J and row quartet v is
//   y_J[v] = Y[r0 + 4v + l/16][16J + l%16],
// so tile (I, J) of C accumulates mfma(y_I[v], y_J[v]) over v and over the
// row blocks (upper tiles only; C is symmetric).  In pass 2, Y = X M is itself
// a product on the matrix cores: with A = X[r0 + l%16][4k + l/16] and
// B = M[4k + l/16][16J + l%16], the accumulator of column block J after the
// n/4 steps k holds exactly y_J[v] in its v-th register -- no transpose.
//
// Every wavefront writes its n x n partial to the workspace and gram_sum adds
// the partials in a fixed order (no atomics: results are reproducible bit for
// bit).
#include "tsqr_kernels.h"

namespace qless {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// Operands of U consecutive 16-row blocks [r0, r0 + 16U) for
// gram_mfma_kernel, from a buffer resource based at row r0 (lane offset in a
// VGPR, row stride and column in SGPR / immediate offsets).  For sub-block u
// (rows r0 + 16u ..):
//   pass 1: v[u][4J + q] = X[16u + 4q + hi][16J + lo]  (full 128-byte rows per load)
//   pass 2: v[u][k]      = X[16u + lo][4k + hi]         (A operand of Y = X M)
// Without GUARD (all 16U rows present and n a multiple of 16) the loads are
// unguarded.  With GUARD, the row and the column of each lane are clamped in
// bounds and what a clamped lane read is replaced by 0.  U is chosen so that a stage holds 16 to 32 doubles per lane;
// with two stages in registers, 8 KB or more per wavefront are in flight.
template <int NB>
constexpr int gram_sub_blocks() {
    return NB == 1 ? 8 : NB == 2 ? 4 : NB == 3 ? 2 : 1;
}

template <int NB>
struct GramStage {
    double v[gram_sub_blocks<NB>()][4 * NB];
};

template <int NB, bool HAS_M, bool GUARD>
__device__ __forceinline__ void gram_load_stage(GramStage<NB>& b, const double* __restrict__ X, int n, int64_t ldx,
                                                int64_t r0, int64_t r_end, int lo, int hi) {
    constexpr int U = gram_sub_blocks<NB>();
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + r0 * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
    const int row_bytes = (int)(ldx * 8);
    const int64_t rows_left = r_end - r0;
    if constexpr (HAS_M) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = 16 * u + lo;
            const bool rok = !GUARD || r < rows_left;
#pragma unroll
            for (int k = 0; k < 4 * NB; ++k) {
                const int c = 4 * k + hi;
                const bool ok = !GUARD || (rok && c < n);
                const int off =
                    GUARD ? (rok ? r : 0) * row_bytes + (c < n ? c : 0) * 8 : lo * row_bytes + hi * 8 + 32 * k;
                const double x = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, GUARD ? 0 : 16 * u * row_bytes, 0));
                b.v[u][k] = ok ? x : 0.0;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = 16 * u + 4 * q + hi;
                const bool rok = !GUARD || r < rows_left;
#pragma unroll
                for (int J = 0; J < NB; ++J) {
                    const int c = 16 * J + lo;
                    const bool ok = !GUARD || (rok && c < n);
                    const int off =
                        GUARD ? (rok ? r : 0) * row_bytes + (c < n ? c : 0) * 8 : hi * row_bytes + lo * 8 + 128 * J;
                    const double x = __builtin_bit_cast(
                        double,
                        __builtin_amdgcn_raw_buffer_load_b64(rs, off, GUARD ? 0 : (16 * u + 4 * q) * row_bytes, 0));
                    b.v[u][4 * J + q] = ok ? x : 0.0;
                }
            }
    }
}

// Number of accumulators: one per upper tile, and four partial sums of the
// single tile when NB == 1 so that consecutive products never wait for each
// other's result.
template <int NB>
constexpr int gram_accs() {
    return NB == 1 ? 4 : NB * (NB + 1) / 2;
}

// MK: 0 pass 1 (no M); 1 pass 2 with a dense M; 2 pass 2 with an upper
// triangular M (CholQR2's R1^{-1}), whose blocks below the diagonal are zero
// and are skipped: block (k, J) of M, rows 4k.., columns 16J.., is zero when
// 4k > 16J + 15.
template <int NB, int MK>
__device__ __forceinline__ void gram_stage(const GramStage<NB>& b, const double* __restrict__ Ms,
                                           f64x4 (&acc)[gram_accs<NB>()], int lo, int hi) {
    constexpr int NPAD = 16 * NB;
    constexpr int U = gram_sub_blocks<NB>();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        f64x4 y[NB];
        if constexpr (MK != 0) {
            // M stays in LDS: its operands are re-read for every block rather
            // than held in NB * 4NB registers
            asm volatile("" ::: "memory");
#pragma unroll
            for (int J = 0; J < NB; ++J) y[J] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 4 * NB; ++k)
#pragma unroll
                for (int J = 0; J < NB; ++J)
                    if (MK == 1 || k < 4 * (J + 1))
                        y[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(b.v[u][k], Ms[(4 * k + hi) * NPAD + 16 * J + lo],
                                                                   y[J], 0, 0, 0);
        } else {
#pragma unroll
            for (int J = 0; J < NB; ++J)
#pragma unroll
                for (int q = 0; q < 4; ++q) y[J][q] = b.v[u][4 * J + q];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if constexpr (NB == 1) {
                acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[0][q], y[0][q], acc[q], 0, 0, 0);
            } else {
                int t = 0;
#pragma unroll
                for (int I = 0; I < NB; ++I)
#pragma unroll
                    for (int J = I; J < NB; ++J, ++t)
                        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(y[I][q], y[J][q], acc[t], 0, 0, 0);
            }
        }
    }
}

// Rows [r_begin, r_end) of one wavefront, in stages of U 16-row blocks,
// double-buffered: the loads of stage s+1 are issued before stage s is
// multiplied (the last full stage is requested twice, so every iteration
// issues the same loads).  The partial stage at the end loads guarded.
template <int NB, int MK, bool GUARD>
__device__ __forceinline__ void gram_range(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                           int64_t r_end, const double* __restrict__ Ms,
                                           f64x4 (&acc)[gram_accs<NB>()], int lo, int hi) {
    constexpr int64_t STAGE = 16 * gram_sub_blocks<NB>();
    const int64_t nfull = (r_end - r_begin) / STAGE;
    if (nfull > 0) {
        const int64_t last = r_begin + (nfull - 1) * STAGE;   // start of the last full stage
        GramStage<NB> ba, bb;
        gram_load_stage<NB, MK != 0, GUARD>(ba, X, n, ldx, r_begin, r_end, lo, hi);
        for (int64_t r0 = r_begin;;) {
            gram_load_stage<NB, MK != 0, GUARD>(bb, X, n, ldx, r0 + STAGE < last ? r0 + STAGE : last, r_end, lo, hi);
            gram_stage<NB, MK>(ba, Ms, acc, lo, hi);
            r0 += STAGE;
            if (r0 > last) break;
            gram_load_stage<NB, MK != 0, GUARD>(ba, X, n, ldx, r0 + STAGE < last ? r0 + STAGE : last, r_end, lo, hi);
            gram_stage<NB, MK>(bb, Ms, acc, lo, hi);
            r0 += STAGE;
            if (r0 > last) break;
        }
    }
    const int64_t rt = r_begin + nfull * STAGE;
    if (rt < r_end) {
        GramStage<NB> bt;
        gram_load_stage<NB, MK != 0, true>(bt, X, n, ldx, rt, r_end, lo, hi);
        gram_stage<NB, MK>(bt, Ms, acc, lo, hi);
    }
}

// One wavefront per contiguous row range (gram_range).
template <int NB, int MK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
gram_mfma_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                 int64_t nwaves, const double* __restrict__ M, double* __restrict__ Cpart) {
    constexpr int NPAD = 16 * NB;
    constexpr int NA = gram_accs<NB>();
    __shared__ double Ms[MK != 0 ? NPAD * NPAD : 1];
    if constexpr (MK != 0) {
        for (int e = threadIdx.x; e < NPAD * NPAD; e += blockDim.x) {
            const int k = e / NPAD, c = e % NPAD;
            Ms[e] = (k < n && c < n) ? M[(int64_t)k * n + c] : 0.0;
        }
        __syncthreads();
    }
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * 4 + wib;
    if (w >= nwaves) return;
    const int lo = lane & 15, hi = lane >> 4;
    f64x4 acc[NA];
#pragma unroll
    for (int t = 0; t < NA; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    if (n == NPAD) gram_range<NB, MK, false>(X, n, ldx, r_begin, r_end, Ms, acc, lo, hi);
    else gram_range<NB, MK, true>(X, n, ldx, r_begin, r_end, Ms, acc, lo, hi);
    if constexpr (NB == 1) acc[0] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    // tile (I, J): this lane holds C[16I + 4v + hi][16J + lo]; the lower tiles
    // are the transposes of the upper ones
    double* out = Cpart + w * (int64_t)n * n;
    int t = 0;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = I; J < NB; ++J, ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * I + 4 * v + hi, j = 16 * J + lo;
                if (i < n && j < n) {
                    out[(int64_t)i * n + j] = acc[t][v];
                    if (I != J) out[(int64_t)j * n + i] = acc[t][v];
                }
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

// C = sum over w < k of Cpart[w] (n x n), in a fixed order.  A workgroup
// takes 16 entries; the 16 threads of an entry take the partials w = p,
// p + 16, ... (p = thread's part) with four running sums each, so many loads
// are in flight, and the parts are then added pairwise in LDS.  The order
// depends only on k, so the result is reproducible bit for bit.
constexpr int kSumParts = 16;
constexpr int kSumEntries = 256 / kSumParts;

__global__ void __launch_bounds__(256)
gram_sum_kernel(const double* __restrict__ Cpart, int64_t k, int n, double* __restrict__ C) {
    __shared__ double sub[kSumParts][kSumEntries];
    const int nn = n * n;
    const int j = threadIdx.x % kSumEntries;
    const int p = threadIdx.x / kSumEntries;
    const int e = blockIdx.x * kSumEntries + j;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < nn) {
        const double* src = Cpart + e;
        int64_t w = p;
        for (; w + 3 * kSumParts < k; w += 4 * kSumParts) {
            s0 += src[w * nn];
            s1 += src[(w + kSumParts) * nn];
            s2 += src[(w + 2 * kSumParts) * nn];
            s3 += src[(w + 3 * kSumParts) * nn];
        }
        for (; w < k; w += kSumParts) s0 += src[w * nn];
    }
    sub[p][j] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int h = kSumParts / 2; h > 0; h /= 2) {
        if (p < h) sub[p][j] += sub[p + h][j];
        __syncthreads();
    }
    if (p == 0 && e < nn) C[e] = sub[0][j];
}

template <int NP, bool HAS_M>
hipError_t launch_gram_rows(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                            const double* M, double* Cpart, hipStream_t s) {
    // with the fused multiply, half the rows per lane leave room for y = x M
    constexpr int RPL = HAS_M ? 32 / NP : 64 / NP;
    hipLaunchKernelGGL((gram_rows_kernel<NP, RPL, HAS_M>), dim3((unsigned)ceil_div(nw, 4)), dim3(256), 0, s, X, m, n,
                       ldx, rpw, nw, M, Cpart);
    return hipGetLastError();
}

template <int NB, int MK>
hipError_t launch_gram_mfma(const double* X, int64_t m, int n, int64_t ldx, int64_t rpw, int64_t nw,
                            const double* M, double* Cpart, hipStream_t s) {
    hipLaunchKernelGGL((gram_mfma_kernel<NB, MK>), dim3((unsigned)ceil_div(nw, 4)), dim3(256), 0, s, X, m, n, ldx,
                       rpw, nw, M, Cpart);
    return hipGetLastError();
}

// Kernel width: n <= 8 padded to a power of two (row layout); wider n to
// whole blocks of 16 columns (matrix cores).
int gram_npad(int64_t n) {
    if (n > 8) return (int)ceil_div(n, 16) * 16;
    int np = 1;
    while (np < n) np <<= 1;
    return np;
}

// ------------------------------------------------------- explicit Q = X M
//
// Q = X M, streamed once over X (read 8mn bytes, write 8mn with nontemporal
// stores: Q is not read back by this call), for the explicit
// Q that Sec. 1 says can be rebuilt from X and its Q-less R (M = R^{-1}), and
// for the Q of SVQB's X = Q Z (M = D1 D2).  Same loads and products as the
// Gram pass 2 above, but the rows of Y = X M are stored instead of being
// multiplied into a Gram matrix.  A non-zero *fail (a singular R) makes every
// row NaN instead.

// n > 8, matrix cores: lane l's accumulator v of column block J holds
// Y[r0 + 16u + 4v + l/16][16J + l%16]; the 16 lanes of a row write 128
// contiguous bytes.
template <int NB, int MK, bool GUARD>
__device__ __forceinline__ void apply_stage(const GramStage<NB>& b, const double* __restrict__ Ms,
                                            double* __restrict__ Q, int n, int64_t ldq, int64_t r0, int64_t r_end,
                                            int lo, int hi) {
    constexpr int NPAD = 16 * NB;
    constexpr int U = gram_sub_blocks<NB>();
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < U; ++u) {
        f64x4 y[NB];
#pragma unroll
        for (int J = 0; J < NB; ++J) y[J] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4 * NB; ++k)
#pragma unroll
            for (int J = 0; J < NB; ++J)
                if (MK == 1 || k < 4 * (J + 1))
                    y[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(b.v[u][k], Ms[(4 * k + hi) * NPAD + 16 * J + lo], y[J],
                                                               0, 0, 0);
#pragma unroll
        for (int J = 0; J < NB; ++J)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = r0 + 16 * u + 4 * v + hi;
                const int col = 16 * J + lo;
                if (!GUARD || (row < r_end && col < n)) __builtin_nontemporal_store(y[J][v], &Q[row * ldq + col]);
            }
    }
}

template <int NB, int MK, bool GUARD>
__device__ __forceinline__ void apply_range(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                            int64_t r_end, const double* __restrict__ Ms, double* __restrict__ Q,
                                            int64_t ldq, int lo, int hi) {
    constexpr int64_t STAGE = 16 * gram_sub_blocks<NB>();
    const int64_t nfull = (r_end - r_begin) / STAGE;
    if (nfull > 0) {
        const int64_t last = r_begin + (nfull - 1) * STAGE;
        GramStage<NB> ba, bb;
        gram_load_stage<NB, true, GUARD>(ba, X, n, ldx, r_begin, r_end, lo, hi);
        for (int64_t r0 = r_begin;;) {
            gram_load_stage<NB, true, GUARD>(bb, X, n, ldx, r0 + STAGE < last ? r0 + STAGE : last, r_end, lo, hi);
            apply_stage<NB, MK, GUARD>(ba, Ms, Q, n, ldq, r0, r_end, lo, hi);
            r0 += STAGE;
            if (r0 > last) break;
            gram_load_stage<NB, true, GUARD>(ba, X, n, ldx, r0 + STAGE < last ? r0 + STAGE : last, r_end, lo, hi);
            apply_stage<NB, MK, GUARD>(bb, Ms, Q, n, ldq, r0, r_end, lo, hi);
            r0 += STAGE;
            if (r0 > last) break;
        }
    }
    const int64_t rt = r_begin + nfull * STAGE;
    if (rt < r_end) {
        GramStage<NB> bt;
        gram_load_stage<NB, true, true>(bt, X, n, ldx, rt, r_end, lo, hi);
        apply_stage<NB, MK, true>(bt, Ms, Q, n, ldq, rt, r_end, lo, hi);
    }
}

// NaN rows [r_begin, r_end) of Q (the result of a failed call).
__device__ __forceinline__ void fill_nan_rows(double* __restrict__ Q, int n, int64_t ldq, int64_t r_begin,
                                              int64_t r_end, int lane) {
    for (int64_t r = r_begin; r < r_end; ++r)
        for (int c = lane; c < n; c += kWave) Q[r * ldq + c] = __builtin_nan("");
}

template <int NB, int MK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
apply_mfma_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                  int64_t nwaves, const double* __restrict__ M, double* __restrict__ Q, int64_t ldq,
                  const int* __restrict__ fail) {
    constexpr int NPAD = 16 * NB;
    __shared__ double Ms[NPAD * NPAD];
    for (int e = threadIdx.x; e < NPAD * NPAD; e += blockDim.x) {
        const int k = e / NPAD, c = e % NPAD;
        Ms[e] = (k < n && c < n) ? M[(int64_t)k * n + c] : 0.0;
    }
    __syncthreads();
    const int lane = lane_id();
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (w >= nwaves) return;
    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    if (fail != nullptr && *fail != 0) {
        fill_nan_rows(Q, n, ldq, r_begin, r_end, lane);
        return;
    }
    const int lo = lane & 15, hi = lane >> 4;
    if (n == NPAD) apply_range<NB, MK, false>(X, n, ldx, r_begin, r_end, Ms, Q, ldq, lo, hi);
    else apply_range<NB, MK, true>(X, n, ldx, r_begin, r_end, Ms, Q, ldq, lo, hi);
}

// n <= 8, row layout: each lane holds RPL full rows of a 64*RPL-row panel (the
// TSQR panel loads) and forms y = x M (M from LDS, broadcast reads).  Where
// Q's rows are contiguous (ldq == n) a full panel of Q is one contiguous
// block: the wavefront writes its rows into an LDS buffer and stores the
// block with consecutive lanes on consecutive 16-byte pieces (each store
// instruction covers 1 KB); otherwise each lane writes its own rows.
template <int NP, int RPL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
apply_rows_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                  int64_t nwaves, const double* __restrict__ M, double* __restrict__ Q, int64_t ldq,
                  const int* __restrict__ fail) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    constexpr int BLOCK = (int)PANEL * NP;          // doubles of one full panel of Q
    __shared__ double Ms[NP * NP];
    __shared__ __attribute__((aligned(16))) double qs[4][NP % 2 == 0 ? BLOCK : 2];
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {
        const int k = e / NP, c = e % NP;
        Ms[e] = (k < n && c < n) ? M[(int64_t)k * n + c] : 0.0;
    }
    __syncthreads();
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t w = (int64_t)blockIdx.x * 4 + wib;
    if (w >= nwaves) return;
    const int64_t r_begin = w * rows_per_wave;
    const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
    if (fail != nullptr && *fail != 0) {
        fill_nan_rows(Q, n, ldq, r_begin, r_end, lane);
        return;
    }
    const bool fast = (n == NP) && (PANEL * ldx * 8 < 0x7FFFFFFF);
    // contiguous, 16-byte aligned panels of Q: stored as blocks through LDS
    const bool block_store = (n == NP) && (ldq == NP) && (reinterpret_cast<uintptr_t>(Q) % 16 == 0);
    for (int64_t base = r_begin; base < r_end; base += PANEL) {
        double x[RPL][NP];
        const bool full = base + PANEL <= r_end;
        if (fast && full) tsqr_detail::load_panel_1d_fast<NP, RPL>(x, X, ldx, base, lane);
        else tsqr_detail::load_panel_1d_tail<NP, RPL>(x, X, n, ldx, base, r_end, lane);
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
        }
        if constexpr (NP % 2 == 0) {
            if (block_store && full) {
                double* st = qs[wib];
#pragma unroll
                for (int i = 0; i < RPL; ++i)
#pragma unroll
                    for (int c = 0; c < NP; ++c) st[(lane + kWave * i) * NP + c] = y[i][c];
                __builtin_amdgcn_wave_barrier();
                f64x2* dst = reinterpret_cast<f64x2*>(Q + base * ldq);
                const f64x2* src = reinterpret_cast<const f64x2*>(st);
#pragma unroll
                for (int f = lane; f < BLOCK / 2; f += kWave) __builtin_nontemporal_store(src[f], dst + f);
                __builtin_amdgcn_wave_barrier();   // the next panel overwrites the buffer
                continue;
            }
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int64_t row = base + lane + kWave * i;
            if (row < r_end) {
                double* q = Q + row * ldq;
#pragma unroll
                for (int c = 0; c < NP; ++c)
                    if (c < n) __builtin_nontemporal_store(y[i][c], &q[c]);
            }
        }
    }
}

}  // namespace

GramPlan make_gram_plan(int64_t m, int64_t n, int num_cus) {
    GramPlan p;
    p.npad = gram_npad(n);
    const int64_t slab = p.npad <= 8 ? (int64_t)kWave * (64 / p.npad) : 64;
    const int64_t max_waves = (int64_t)(num_cus > 0 ? num_cus : 1) * 8;
    int64_t rpw = ceil_div(m > 0 ? m : 1, max_waves);
    rpw = ceil_div(rpw, slab) * slab;
    p.rows_per_wave = rpw;
    p.k = m > 0 ? ceil_div(m, rpw) : 1;
    p.part_bytes = align_up((size_t)p.k * (size_t)(n * n) * sizeof(double), 256);
    return p;
}

hipError_t launch_gram(const double* X, int64_t m, int64_t n, int64_t ldx, const double* M, bool m_upper,
                       double* Cpart, double* C, const GramPlan& plan, hipStream_t s) {
    const int ni = (int)n;
    hipError_t e = hipErrorInvalidValue;
    timing_begin(kTimeGram, s);
    const bool hm = (M != nullptr);
    const int64_t rpw = plan.rows_per_wave, k = plan.k;
    switch (plan.npad) {
#define QLESS_GROWS(NP)                                                                           \
    case NP:                                                                                      \
        e = hm ? launch_gram_rows<NP, true>(X, m, ni, ldx, rpw, k, M, Cpart, s)                   \
               : launch_gram_rows<NP, false>(X, m, ni, ldx, rpw, k, M, Cpart, s);                 \
        break;
#define QLESS_GMFMA(NB)                                                                           \
    case 16 * NB:                                                                                 \
        e = !hm       ? launch_gram_mfma<NB, 0>(X, m, ni, ldx, rpw, k, M, Cpart, s)             \
            : m_upper ? launch_gram_mfma<NB, 2>(X, m, ni, ldx, rpw, k, M, Cpart, s)             \
                      : launch_gram_mfma<NB, 1>(X, m, ni, ldx, rpw, k, M, Cpart, s);            \
        break;
        QLESS_GROWS(1) QLESS_GROWS(2) QLESS_GROWS(4) QLESS_GROWS(8)
        QLESS_GMFMA(1) QLESS_GMFMA(2) QLESS_GMFMA(3) QLESS_GMFMA(4)
#undef QLESS_GROWS
#undef QLESS_GMFMA
        default: break;
    }
    timing_end(kTimeGram, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_sum_kernel, dim3((unsigned)ceil_div(n * n, kSumEntries)), dim3(256), 0, s, Cpart, plan.k, ni,
                       C);
    return hipGetLastError();
}

// Plan of the apply pass: the Gram pass's split of the rows over 8 wavefronts
// per CU, whole slabs per wavefront.
hipError_t launch_apply_right(const double* X, int64_t m, int64_t n, int64_t ldx, const double* M, bool m_upper,
                              double* Q, int64_t ldq, const int* fail, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    const GramPlan plan = make_gram_plan(m, n, current_device_info().num_cus);
    const int ni = (int)n;
    const int64_t rpw = plan.rows_per_wave, k = plan.k;
    const unsigned blocks = (unsigned)ceil_div(k, 4);
    switch (plan.npad) {
#define QLESS_AROWS(NP)                                                                                   \
    case NP:                                                                                              \
        hipLaunchKernelGGL((apply_rows_kernel<NP, 32 / NP>), dim3(blocks), dim3(256), 0, s, X, m, ni, ldx, rpw, \
                           k, M, Q, ldq, fail);                                                           \
        break;
#define QLESS_AMFMA(NB)                                                                                     \
    case 16 * NB:                                                                                           \
        if (m_upper)                                                                                        \
            hipLaunchKernelGGL((apply_mfma_kernel<NB, 2>), dim3(blocks), dim3(256), 0, s, X, m, ni, ldx, rpw, k, M, Q, \
                               ldq, fail);                                                                  \
        else                                                                                                \
            hipLaunchKernelGGL((apply_mfma_kernel<NB, 1>), dim3(blocks), dim3(256), 0, s, X, m, ni, ldx, rpw, k, M, Q, \
                               ldq, fail);                                                                  \
        break;
        QLESS_AROWS(1) QLESS_AROWS(2) QLESS_AROWS(4) QLESS_AROWS(8)
        QLESS_AMFMA(1) QLESS_AMFMA(2) QLESS_AMFMA(3) QLESS_AMFMA(4)
#undef QLESS_AROWS
#undef QLESS_AMFMA
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace qless
