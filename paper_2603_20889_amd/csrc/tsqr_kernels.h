// Q-less Householder TSQR kernels for gfx950 (paper Alg. 2-4).
//
// One kernel, tsqr_fold_kernel, serves both stages of Alg. 2.  Its
// wavefront w folds the rows [w*rows_per_wave, (w+1)*rows_per_wave) of a
// row-major matrix into an n x n triangle; the wavefronts of a workgroup
// combine theirs in LDS and the workgroup writes one triangle:
//   stage 1: the rows of X, split into k contiguous blocks; the triangles go
//            to a stacked buffer Y (rows of triangles, n columns);
//   tree   : the stacked buffer itself, fan_in triangles per wavefront,
//            level after level until one workgroup remains; that one writes
//            R with its diagonal made non-negative (for n <= 16 the last
//            level is tsqr_tree_block_kernel).
// Every level is its own launch: the end of a launch is what makes the
// triangles of one workgroup visible to the next level, so no workgroup
// ever synchronises with another (an agent-scope fence per wavefront costs
// an L2 write-back and invalidate on gfx950, which stalls the streaming of
// every other wavefront on that XCD).
//
// A wavefront streams its rows in panels and keeps the running triangle R of
// the rows seen so far in LDS (wavefront-private; broadcast reads, one-lane
// writes).  Each panel W is folded in by the structured Householder QR of
// [R; W] (Alg. 4 without the column pairing): the reflector of column j
// pivots on R_jj and spans column j of W, so it touches only row j of R and
// the panel.  Q and the reflectors are never stored.
//
// Register layouts of a panel:
//   n <= 16: lane l holds RPL full rows (l, l+64, ...); the K = n - j dot
//     products of step j are per-lane partial sums reduced over 64 lanes by
//     one transposed butterfly.  For n <= 8 the interior panels are instead
//     folded lane-privately (each lane its own triangle, no cross-lane
//     traffic) and, for contiguous rows, streamed through LDS with
//     direct-to-LDS nontemporal loads.
//   n > 16: 8 row groups x 8 column groups; lane (rg, cg) holds RPL rows of
//     the columns cg, cg+8, ...; the pivot column is broadcast inside the row
//     group and the sums run over the 8 row groups only.
#pragma once

#include "qless_internal.h"

namespace qless {
namespace tsqr_detail {

// R is kept in LDS as a packed upper triangle: row J holds columns J..NP-1
// starting at tri_row<NP>(J).
template <int NP>
__host__ __device__ constexpr int tri_row(int J) {
    return J * NP - J * (J - 1) / 2;
}

template <int NP>
constexpr int tri_size() {
    return NP * (NP + 1) / 2;
}


// A reflector is applied only where alpha^2 + s is at least this (2^-1000,
// about 9e-302); below it the column is left as it is.  Inputs in the
// documented range (|x| >= 1e-150) never come near it; what does is the
// roundoff residue of a block with fewer rows than columns, which shrinks by
// a factor of about u per column (a one-row block at n = 21 reaches 1e-300
// by its last columns), and whose square would pass a subnormal to the
// reciprocal square-root estimate (flushed to zero there: inf, then NaN).
// Leaving such a residue in the panel changes R by far less than one unit
// in the last place of any entry.
constexpr double kTinySq = 0x1p-1000;

__device__ __forceinline__ bool reflector_needed(double alpha, double s) {
    return s != 0.0 && fma(alpha, alpha, s) >= kTinySq;
}

// Scalars of the reflector that maps (alpha, x) with |x|^2 = s > 0 to
// (beta, 0): nrm = sqrt(alpha^2 + s), beta = -sign(alpha) nrm (sign(+0) = +),
// u0 = alpha - beta (its pivot entry) and gamma = 2 / (u^T u) =
// 1 / (nrm (nrm + |alpha|)).  The square root and the reciprocal start from
// the hardware estimates (v_rsq_f64, v_rcp_f64) and take two Newton steps
// each, which leaves a few units in the last place -- far inside the
// tolerance -- at a third of the instructions of the IEEE-rounded sequences.
__device__ __forceinline__ void reflector_scalars(double alpha, double s, double& beta, double& u0, double& gamma) {
    const double q = fma(alpha, alpha, s);
    const double h = 0.5 * q;
    double y = __builtin_amdgcn_rsq(q);          // ~ q^{-1/2}
#pragma unroll
    for (int it = 0; it < 2; ++it) {              // y <- y (3/2 - q y^2 / 2)
        const double e = fma(-h, y * y, 0.5);
        y = fma(y, e, y);
    }
    const double nrm = q * y;
    beta = (alpha >= 0.0) ? -nrm : nrm;
    u0 = alpha - beta;
    const double d = nrm * (nrm + fabs(alpha));
    double r = __builtin_amdgcn_rcp(d);           // ~ 1/d
#pragma unroll
    for (int it = 0; it < 2; ++it) {              // r <- r (2 - d r)
        const double e = fma(-d, r, 1.0);
        r = fma(r, e, r);
    }
    gamma = r;
}

// Fold one panel for NP <= 16: the column loop is a compile-time recursion so
// that every register index is a constant.  Step J forms the K = NP - J
// partial dot products of column J with columns J..NP-1 in each lane, sums
// all K over the wavefront in one transposed butterfly, and applies the
// reflector; the scalars (norm, beta, gamma) are wave-uniform.
// Per-lane value index after the transposed butterfly: byte K-1 of the
// packed words is red_origin(K, lane), the value whose wavefront total this
// lane holds when K values are summed.
template <int NP>
struct LaneOrigins {
    uint32_t w[(NP + 3) / 4];
    __device__ __forceinline__ void init(int lane) {
#pragma unroll
        for (int q = 0; q < (NP + 3) / 4; ++q) w[q] = 0u;
#pragma unroll
        for (int K = 1; K <= NP; ++K) w[(K - 1) >> 2] |= (uint32_t)red_origin(K, lane) << (8 * ((K - 1) & 3));
    }
    template <int K>
    __device__ __forceinline__ int get() const {
        return (int)((w[(K - 1) >> 2] >> (8 * ((K - 1) & 3))) & 0xFFu);
    }
};

// Step J of the fold (n <= 16).  The K = NP - J partial dot products of
// column J with columns J..NP-1 are summed over the wavefront by one
// transposed butterfly, after which every lane holds the total of one value
// v.  Each lane then finishes the work of its own value: the update
// coefficient of column J+v and the new R_{J,J+v} (R_JJ = beta for v = 0),
// written back to LDS, and the coefficients are shared through LDS
// broadcast reads.  The reflector scalars (norm, beta, gamma) are
// wave-uniform.
// With REC, the pivot entry u0 and gamma of every step's reflector are
// written to rec[J] and rec[NP + J] (0 and 0 for a column left as it is):
// the blocked fold builds its block reflector from them.  Rw is a packed
// triangle of row width W (the NP x NP diagonal block of a wider triangle
// when W > NP: row J of the block starts at tri_row<W>(J)).
template <int NP, int RPL, int J, bool REC = false, int W = NP>
struct FoldStep {
    __device__ static __forceinline__ void run(double (&x)[RPL][NP], double* __restrict__ Rw, double* __restrict__ Cw,
                                               const LaneOrigins<NP>& org, int lane, double* rec = nullptr) {
        if constexpr (J < NP) {
            constexpr int K = NP - J;
            double p[K];
#pragma unroll
            for (int t = 0; t < K; ++t) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) s = fma(x[i][J], x[i][J + t], s);
                p[t] = s;
            }
            const double alpha = Rw[tri_row<W>(J)];
            red_stages<K, 0>(p, lane);                  // p[0]: total of value v in this lane
            const int v = org.template get<K>();
            const double r = Rw[tri_row<W>(J) + v];
            const double s = readlane_f64(p[0], red_locate(K, 0));
            const bool apply = reflector_needed(alpha, s);
            if constexpr (REC) {
                if (!apply && lane == 0) {
                    rec[J] = 0.0;
                    rec[NP + J] = 0.0;
                }
            }
            if (apply) {
                double beta, u0, gamma;
                reflector_scalars(alpha, s, beta, u0, gamma);
                if constexpr (REC) {
                    if (lane == 0) {
                        rec[J] = u0;
                        rec[NP + J] = gamma;
                    }
                }
                const double coef = gamma * fma(u0, r, p[0]);   // gamma * (u^T column J+v)
                Rw[tri_row<W>(J) + v] = (v == 0) ? beta : fma(-coef, u0, r);
                if constexpr (K > 1) {
                    Cw[v] = coef;                        // every holder of v writes the same value
                    __builtin_amdgcn_wave_barrier();
                    double c[K];
#pragma unroll
                    for (int t = 1; t < K; ++t) c[t] = Cw[t];
#pragma unroll
                    for (int t = 1; t < K; ++t)
#pragma unroll
                        for (int i = 0; i < RPL; ++i) x[i][J + t] = fma(-c[t], x[i][J], x[i][J + t]);
                }
            }
            FoldStep<NP, RPL, J + 1, REC, W>::run(x, Rw, Cw, org, lane, rec);
        }
    }
};

// Step J of the fold (n <= 16) with the running R in registers instead of
// LDS.  Lane l keeps in rr[J] the entry R_{J, J+v} of row J for the value v
// that the transposed butterfly of step J leaves in it (every lane with the
// same v holds the same entry), so a step touches no LDS: alpha = R_JJ is
// read from a lane with v = 0, and the update coefficients of columns
// J+1.. from lanes that finished them, by v_readlane into scalar registers
// that the updates take as operands.  The arithmetic, and so the result, is
// that of FoldStep; it serves the interior panels, where the next panel may
// be streaming into LDS meanwhile.
template <int NP, int RPL, int J, int K, int T>
__device__ __forceinline__ void apply_coefs(double (&x)[RPL][NP], double coef) {
    if constexpr (T < K) {
        constexpr int src = red_locate(K, T);
        const double c = readlane_f64(coef, src);
#pragma unroll
        for (int i = 0; i < RPL; ++i) x[i][J + T] = fma(-c, x[i][J], x[i][J + T]);
        apply_coefs<NP, RPL, J, K, T + 1>(x, coef);
    }
}

template <int NP, int RPL, int J>
struct FoldStepReg {
    __device__ static __forceinline__ void run(double (&x)[RPL][NP], double (&rr)[NP], const LaneOrigins<NP>& org,
                                               int lane) {
        if constexpr (J < NP) {
            constexpr int K = NP - J;
            double p[K];
#pragma unroll
            for (int t = 0; t < K; ++t) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) s = fma(x[i][J], x[i][J + t], s);
                p[t] = s;
            }
            red_stages<K, 0>(p, lane);
            constexpr int l0 = red_locate(K, 0);
            const double s = readlane_f64(p[0], l0);
            const double alpha = readlane_f64(rr[J], l0);
            if (reflector_needed(alpha, s)) {
                double beta, u0, gamma;
                reflector_scalars(alpha, s, beta, u0, gamma);
                const int v = org.template get<K>();
                const double coef = gamma * fma(u0, rr[J], p[0]);   // gamma * (u^T column J+v)
                rr[J] = (v == 0) ? beta : fma(-coef, u0, rr[J]);
                apply_coefs<NP, RPL, J, K, 1>(x, coef);
            }
            FoldStepReg<NP, RPL, J + 1>::run(x, rr, org, lane);
        }
    }
};

// rr (the register form of FoldStepReg) from and to the packed triangle in LDS.
template <int NP, int J = 0>
__device__ __forceinline__ void load_rr(double (&rr)[NP], const double* __restrict__ Rw, const LaneOrigins<NP>& org) {
    if constexpr (J < NP) {
        rr[J] = Rw[tri_row<NP>(J) + org.template get<NP - J>()];
        load_rr<NP, J + 1>(rr, Rw, org);
    }
}

template <int NP, int J = 0>
__device__ __forceinline__ void store_rr(const double (&rr)[NP], double* __restrict__ Rw, const LaneOrigins<NP>& org) {
    if constexpr (J < NP) {
        Rw[tri_row<NP>(J) + org.template get<NP - J>()] = rr[J];   // the holders of an entry write the same value
        store_rr<NP, J + 1>(rr, Rw, org);
    } else {
        __builtin_amdgcn_wave_barrier();
    }
}

// Lane-private fold (n <= 8): lane l keeps its own running triangle Rl of
// the rows it has loaded (packed, in registers) and folds its RPL rows of a
// panel into it with no cross-lane traffic at all -- the reflector scalars
// and coefficients are per lane, so one instruction serves 64 independent
// folds.  The 64 triangles are combined once at the end (fold_lane_triangles).
// Any partition of the rows gives a valid TSQR tree (Alg. 2), so this only
// changes the order in which rows meet, not what is computed.
template <int NP, int RPL, int J>
struct LaneFoldStep {
    __device__ static __forceinline__ void run(double (&x)[RPL][NP], double (&Rl)[NP * (NP + 1) / 2]) {
        if constexpr (J < NP) {
            constexpr int K = NP - J;
            constexpr int r0 = tri_row<NP>(J);
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < RPL; ++i) s = fma(x[i][J], x[i][J], s);
            const double alpha = Rl[r0];
            double beta, u0, gamma;
            reflector_scalars(alpha, s, beta, u0, gamma);
            const bool nz = reflector_needed(alpha, s);   // a zero column is left as it is
            gamma = nz ? gamma : 0.0;
            u0 = nz ? u0 : 0.0;
            Rl[r0] = nz ? beta : alpha;
#pragma unroll
            for (int t = 1; t < K; ++t) {
                double d = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) d = fma(x[i][J], x[i][J + t], d);
                const double coef = gamma * fma(u0, Rl[r0 + t], d);   // gamma * (u^T column J+t)
                Rl[r0 + t] = fma(-coef, u0, Rl[r0 + t]);
#pragma unroll
                for (int i = 0; i < RPL; ++i) x[i][J + t] = fma(-coef, x[i][J], x[i][J + t]);
            }
            LaneFoldStep<NP, RPL, J + 1>::run(x, Rl);
        }
    }
};

template <int NP>
constexpr bool lane_private() {
    return NP <= 8;
}

// Instances for n > 16 with one row per lane are the matrix-core blocked
// fold (64-row panels, fold_rows_mfma); the column-group layout has 8 rows
// per panel and row group, so it never uses RPL = 1.
template <int NP, int RPL>
constexpr bool mf_instance() {
    return NP > 16 && RPL == 1;
}

// Instances for n = 32, 48, 64 in the 4 x 16 column-group layout
// (FoldStepG16): 4 row groups of 16 lanes, one DPP row each.
template <int NP, int RPL>
constexpr bool g16_instance() {
    return (NP == 32 && RPL == 24) || (NP == 48 && RPL == 16) || (NP == 64 && RPL == 12);
}


// Panel loads for the layout of n <= 16: lane l gets rows base + l + 64 i
// (i < RPL) into x[i][0..NP-1].
//
// Interior panel (all rows present, n == NP): buffer loads from a resource
// rebased at the panel, lane offset in a VGPR, row-stripe offset in an SGPR;
// the 16-byte chunks of one row are requested back to back, so a cache line
// is fetched once.
template <int NP, int RPL>
__device__ __forceinline__ void load_panel_1d_fast(double (&x)[RPL][NP], const double* __restrict__ X, int64_t ldx,
                                                   int64_t base, int lane) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
    const int vo = lane * (int)(ldx * 8);
    const int so = (int)(ldx * 8 * kWave);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
#pragma unroll
        for (int c = 0; c < NP; c += 2) {
            if (c + 1 < NP) {
                const f64x2 v =
                    __builtin_bit_cast(f64x2, __builtin_amdgcn_raw_buffer_load_b128(rs, vo + c * 8, so * i, 0));
                x[i][c] = v[0];
                x[i][c + 1] = v[1];
            } else {
                x[i][c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo + c * 8, so * i, 0));
            }
        }
    }
}

// Tail panel or padded width: guarded loads, zero fill.
template <int NP, int RPL>
__device__ __forceinline__ void load_panel_1d_tail(double (&x)[RPL][NP], const double* __restrict__ X, int n,
                                                   int64_t ldx, int64_t base, int64_t r_end, int lane) {
    const int64_t left = r_end - base - lane;   // rows of this lane's stripe still in range
    const double* x0 = X + (left > 0 ? base + lane : 0) * ldx;
    const int64_t step = (int64_t)kWave * ldx;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const bool ok = (int64_t)kWave * i < left;
#pragma unroll
        for (int c = 0; c < NP; ++c) x[i][c] = (ok && c < n) ? x0[step * i + c] : 0.0;
    }
}

// Interior panel of a padded width (n < NP): one 8-byte buffer load per
// column, the offset of a column c >= n clamped to column 0 (in bounds) and
// its value replaced by 0.
template <int NP, int RPL>
__device__ __forceinline__ void load_panel_1d_padded(double (&x)[RPL][NP], const double* __restrict__ X, int n,
                                                     int64_t ldx, int64_t base, int lane) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
    const int vo = lane * (int)(ldx * 8);
    const int so = (int)(ldx * 8 * kWave);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            const bool ok = c < n;
            const double v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo + (ok ? c : 0) * 8,
                                                                                             so * i, 0));
            x[i][c] = ok ? v : 0.0;
        }
    }
}

// Double buffering pays when two panels fit the registers next to the fold's
// temporaries: the next panel is then in flight while the current one is
// folded.
template <int NP, int RPL>
constexpr bool double_buffered() {
    return RPL * NP <= 40;
}

// Full panels [base, base + nfull*PANEL) with lane-private triangles; the
// 64 triangles, stacked, are then folded into the wavefront's R by one
// cross-lane pass with NP rows per lane.
template <int NP, int RPL>
__device__ __forceinline__ void fold_panels_lane_private(const double* __restrict__ X, int64_t ldx, int64_t base,
                                                         int64_t nfull, double* __restrict__ Rw,
                                                         double* __restrict__ Cw, const LaneOrigins<NP>& org,
                                                         int lane) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    double Rl[tri_size<NP>()];
#pragma unroll
    for (int e = 0; e < tri_size<NP>(); ++e) Rl[e] = 0.0;
    double xa[RPL][NP];
    if constexpr (double_buffered<NP, RPL>()) {
        double xb[RPL][NP];
        const int64_t last = base + (nfull - 1) * PANEL;
        load_panel_1d_fast<NP, RPL>(xa, X, ldx, base, lane);
        while (true) {
            load_panel_1d_fast<NP, RPL>(xb, X, ldx, base + PANEL < last ? base + PANEL : last, lane);
            LaneFoldStep<NP, RPL, 0>::run(xa, Rl);
            base += PANEL;
            if (base > last) break;
            load_panel_1d_fast<NP, RPL>(xa, X, ldx, base + PANEL < last ? base + PANEL : last, lane);
            LaneFoldStep<NP, RPL, 0>::run(xb, Rl);
            base += PANEL;
            if (base > last) break;
        }
    } else {
        for (int64_t p = 0; p < nfull; ++p, base += PANEL) {
            load_panel_1d_fast<NP, RPL>(xa, X, ldx, base, lane);
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

// Staged lane-private fold: for contiguous rows (ldx == n == NP) the panels
// stream through a wavefront-private LDS buffer with direct-to-LDS,
// nontemporal buffer loads (buffer_load_dwordx4 ... nt lds): every load
// instruction moves 1 KB of consecutive bytes, so each cache line is fetched
// by one instruction and nothing is kept in the caches.  The next panel is in
// flight while the current one, read from LDS into registers in the row
// layout, is folded.  Waits are explicit (s_waitcnt with a compiler memory
// barrier): the loads of panel p are complete before it is read from LDS,
// and the reads are complete before panel p+1 overwrites the buffer.
template <int NP, int RPL>
constexpr bool staged_instance() {
    return lane_private<NP>() && double_buffered<NP, RPL>() && (RPL * NP) % 2 == 0;
}

// The cross-lane fold of n = 10 and 16 streams its interior panels through
// LDS the same way, with FoldStepReg, which leaves LDS to the loads.  (Measured
// at m = 2^25 against the register-loaded panels: n = 10 5 % faster, n = 16
// 1.5 %; n = 12 the same and n = 14 2.5 % slower, so those stay in registers.)
template <int NP, int RPL>
constexpr bool staged_xl_instance() {
    return NP == 10 || NP == 16;
}

// Doubles of LDS staging per wavefront (one panel).
template <int NP, int RPL>
constexpr int stage_doubles() {
    return (staged_instance<NP, RPL>() || staged_xl_instance<NP, RPL>()) ? kWave * RPL * NP : 0;
}

// Wavefronts per workgroup of the fold kernel: 8 for the LDS-staged
// instances of n <= 8 (one workgroup of 8 per CU holds eight 16-18 KB
// staging buffers, and leaves half as many triangles for the tree as
// workgroups of 4 would); for the staged cross-lane instances as many (8, 4
// or 2) as fit 150 KB of LDS with their one-panel buffers; 2 where four
// packed triangles would take more than 64 KB of LDS and for the
// matrix-core instances (each wavefront also holds transposes in LDS), else
// 4.
constexpr int kStagedWpb = 8;

template <int NP, int RPL>
constexpr int waves_per_block() {
    if constexpr (staged_instance<NP, RPL>()) return kStagedWpb;
    if constexpr (staged_xl_instance<NP, RPL>()) {
        constexpr long per = (long)(stage_doubles<NP, RPL>() + tri_size<NP>() + NP) * 8;
        return 8 * per <= 150 * 1024 ? 8 : 4 * per <= 150 * 1024 ? 4 : 2;
    }
    return (mf_instance<NP, RPL>() || (tri_size<NP>() + NP) * 8 * 4 > 65536) ? 2 : 4;
}

__device__ __forceinline__ void wait_memory() {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
}

constexpr int kNontemporal = 2;   // buffer cache policy: nt

// Staging layout.  A panel is copied in 16-byte chunks; with C = NP/2
// chunks per row a power of two (n = 4, 8, 16), chunk g of the panel (row
// g / C, chunk g % C of the row) is stored at chunk position
// g ^ ((g >> 4) & (C - 1)) of the buffer: the XOR permutes chunks only within
// an aligned 256-byte group, so each direct-to-LDS load still copies one
// contiguous kilobyte of X, and it makes the 16 lanes of a 16-byte LDS read
// (each reading the same chunk of its own row) meet 16 different bank
// groups instead of 2 (n = 16) or 4 (n = 8).  Other widths keep the
// linear layout.
template <int NP>
constexpr int stage_swizzle_chunks() {
    return (NP == 4 || NP == 8 || NP == 16) ? NP / 2 : 0;
}

template <int NP, int RPL>
__device__ __forceinline__ void stage_panel(const double* __restrict__ X, int64_t base, double* stage, int lane) {
    constexpr int NCHUNK = RPL * NP / 2;   // 1 KB chunks: 64 lanes x 16 bytes
    constexpr int C = stage_swizzle_chunks<NP>();
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * NP), (short)0, 0x7FFFFFFF, 0x00020000);
    // load j, lane l fills buffer chunk 64 j + l, which holds chunk
    // 64 j + (l ^ z) of the panel, z = ((4 j + l / 16) & (C - 1)): it depends
    // on j only through j & 1 (and not at all for C <= 4)
    int vo[2] = {lane * 16, lane * 16};
    if constexpr (C > 1) {
        vo[0] = (lane ^ ((lane >> 4) & (C - 1))) * 16;
        vo[1] = (lane ^ ((4 + (lane >> 4)) & (C - 1))) * 16;
    }
#pragma unroll
    for (int j = 0; j < NCHUNK; ++j)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(stage + j * 128), 16,
                                                 vo[j & 1], j * 1024, 0, kNontemporal);
}

template <int NP, int RPL>
__device__ __forceinline__ void read_staged_panel(double (&x)[RPL][NP], const double* stage, int lane) {
    constexpr int C = stage_swizzle_chunks<NP>();
    // chunk h of row r = lane + 64 i sits at chunk h ^ zl of the row's slot,
    // zl = ((r C) >> 4) & (C - 1), the same for every i
    const int zl = C > 1 ? ((lane * C) >> 4) & (C - 1) : 0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const double* row = stage + (lane + kWave * i) * NP;
#pragma unroll
        for (int c = 0; c < NP; c += 2) {
            if constexpr (NP % 2 == 0) {
                const f64x2 v = *reinterpret_cast<const f64x2*>(row + 2 * ((c >> 1) ^ zl));
                x[i][c] = v[0];
                x[i][c + 1] = v[1];
            } else {
                x[i][c] = row[c];
                if (c + 1 < NP) x[i][c + 1] = row[c + 1];
            }
        }
    }
}

// The nfull panels start at rows base, base + step, base + 2 step, ...
// (step = one panel for a contiguous block of rows).
template <int NP, int RPL>
__device__ __forceinline__ void fold_panels_lane_private_staged(const double* __restrict__ X, int64_t base,
                                                                int64_t nfull, int64_t step, double* __restrict__ Rw,
                                                                double* __restrict__ Cw, const LaneOrigins<NP>& org,
                                                                int lane, double* stage) {
    double Rl[tri_size<NP>()];
#pragma unroll
    for (int e = 0; e < tri_size<NP>(); ++e) Rl[e] = 0.0;
    stage_panel<NP, RPL>(X, base, stage, lane);
    for (int64_t p = 0; p < nfull; ++p, base += step) {
        double x[RPL][NP];
        wait_memory();                       // panel p is in LDS
        read_staged_panel<NP, RPL>(x, stage, lane);
        wait_memory();                       // and in registers: the buffer is free
        if (p + 1 < nfull) stage_panel<NP, RPL>(X, base + step, stage, lane);
        LaneFoldStep<NP, RPL, 0>::run(x, Rl);
    }
    double xe[NP][NP];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int c = 0; c < NP; ++c) xe[i][c] = (c >= i) ? Rl[tri_row<NP>(i) + c - i] : 0.0;
    FoldStep<NP, NP, 0>::run(xe, Rw, Cw, org, lane);
}

// Staged cross-lane fold: interior panels of contiguous rows (ldx == n ==
// NP) stream through the wavefront's LDS buffer as in the lane-private
// staged fold, and are folded by FoldStepReg into rr.
template <int NP, int RPL>
__device__ __forceinline__ void fold_panels_staged_reg(const double* __restrict__ X, int64_t base, int64_t nfull,
                                                       double (&rr)[NP], const LaneOrigins<NP>& org, int lane,
                                                       double* stage) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    stage_panel<NP, RPL>(X, base, stage, lane);
    for (int64_t p = 0; p < nfull; ++p, base += PANEL) {
        double x[RPL][NP];
        wait_memory();                       // panel p is in LDS
        read_staged_panel<NP, RPL>(x, stage, lane);
        wait_memory();                       // and in registers: the buffer is free
        if (p + 1 < nfull) stage_panel<NP, RPL>(X, base + PANEL, stage, lane);
        FoldStepReg<NP, RPL, 0>::run(x, rr, org, lane);
    }
}

// Fold rows [r_begin, r_end) of a row-major X (n columns, leading dimension
// ldx) into the wavefront's R, panel by panel (layout for n <= 16).  Interior
// panels come first: for n <= 8 and at least kLanePrivateMin of them, with
// lane-private triangles; otherwise with the cross-lane fold, double-buffered
// when two panels fit (the loads of panel p+1 are issued before panel p is
// folded; the last interior panel is requested twice, so every iteration
// issues the same loads and the wait before a fold only covers the older
// panel).  The partial panel at the end, if any, follows.
constexpr int64_t kLanePrivateMin = 4;

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_1d(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                             int64_t r_end, double* __restrict__ Rw, int lane,
                                             double* stage = nullptr) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    if (r_begin >= r_end) return;
    const bool fast = (n == NP) && (PANEL * ldx * 8 < 0x7FFFFFFF);
    int64_t nfull = fast ? (r_end - r_begin) / PANEL : 0;
    LaneOrigins<NP> org;
    org.init(lane);
    double* Cw = Rw + tri_size<NP>();   // per-wavefront coefficient exchange
    double xa[RPL][NP];
    int64_t base = r_begin;
    if (n < NP && PANEL * ldx * 8 < 0x7FFFFFFF && base + PANEL <= r_end) {
        // padded width: interior panels one at a time, cross-lane fold
        double rr[NP];
        load_rr<NP>(rr, Rw, org);
        for (; base + PANEL <= r_end; base += PANEL) {
            load_panel_1d_padded<NP, RPL>(xa, X, n, ldx, base, lane);
            FoldStepReg<NP, RPL, 0>::run(xa, rr, org, lane);
        }
        store_rr<NP>(rr, Rw, org);
    }
    if constexpr (lane_private<NP>()) {
        if (nfull >= kLanePrivateMin) {
            if constexpr (staged_instance<NP, RPL>()) {
                if (stage != nullptr && ldx == NP)
                    fold_panels_lane_private_staged<NP, RPL>(X, base, nfull, PANEL, Rw, Cw, org, lane, stage);
                else
                    fold_panels_lane_private<NP, RPL>(X, ldx, base, nfull, Rw, Cw, org, lane);
            } else {
                fold_panels_lane_private<NP, RPL>(X, ldx, base, nfull, Rw, Cw, org, lane);
            }
            base += nfull * PANEL;
            nfull = 0;
        }
    }
    if (nfull > 0) {
        double rr[NP];
        load_rr<NP>(rr, Rw, org);
        if constexpr (staged_xl_instance<NP, RPL>()) {
            if (stage != nullptr && ldx == NP) {
                fold_panels_staged_reg<NP, RPL>(X, base, nfull, rr, org, lane, stage);
                base += nfull * PANEL;
                nfull = 0;
            }
        }
        if (nfull > 0) {
            if constexpr (double_buffered<NP, RPL>()) {
                double xb[RPL][NP];
                const int64_t last = base + (nfull - 1) * PANEL;
                load_panel_1d_fast<NP, RPL>(xa, X, ldx, base, lane);
                while (true) {
                    load_panel_1d_fast<NP, RPL>(xb, X, ldx, base + PANEL < last ? base + PANEL : last, lane);
                    FoldStepReg<NP, RPL, 0>::run(xa, rr, org, lane);
                    base += PANEL;
                    if (base > last) break;
                    load_panel_1d_fast<NP, RPL>(xa, X, ldx, base + PANEL < last ? base + PANEL : last, lane);
                    FoldStepReg<NP, RPL, 0>::run(xb, rr, org, lane);
                    base += PANEL;
                    if (base > last) break;
                }
            } else {
                for (int64_t p = 0; p < nfull; ++p, base += PANEL) {
                    load_panel_1d_fast<NP, RPL>(xa, X, ldx, base, lane);
                    FoldStepReg<NP, RPL, 0>::run(xa, rr, org, lane);
                }
            }
        }
        store_rr<NP>(rr, Rw, org);
    }
    for (; base < r_end; base += PANEL) {
        load_panel_1d_tail<NP, RPL>(xa, X, n, ldx, base, r_end, lane);
        FoldStep<NP, RPL, 0>::run(xa, Rw, Cw, org, lane);
    }
}

// Stage 1 of the LDS-staged lane-private instances over interleaved panels.
// With P full panels in X and W wavefronts in the launch, wavefront w folds
// panels w, w + W, w + 2W, ... and the last wavefront also the partial panel
// at the end, so at any moment the launch reads one window of about W
// consecutive panels rather than W streams far apart in memory.  On 5e7 x 8
// the fold loop alone ran 4 % faster over interleaved panels than over one
// contiguous block per wavefront (plain streaming reads gain about as much),
// and the whole stage-1 launch, combines included, 1.5-2 %.  Only the
// grouping of rows into triangles changes, and any grouping is a valid
// reduction tree (Alg. 2).  Taken when every wavefront gets at least
// kLanePrivateMin panels; a launch decides it once, for all its wavefronts.
template <int NP, int RPL>
__device__ __forceinline__ bool interleaved_stage1(int64_t m, int n, int64_t ldx, int64_t nwaves) {
    if constexpr (staged_instance<NP, RPL>())
        return n == NP && ldx == NP && m / ((int64_t)kWave * RPL) >= kLanePrivateMin * nwaves;
    else
        return false;
}

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_interleaved(const double* __restrict__ X, int64_t m, int64_t w,
                                                      int64_t nwaves, double* __restrict__ Rw, int lane,
                                                      double* stage) {
    constexpr int64_t PANEL = (int64_t)kWave * RPL;
    const int64_t P = m / PANEL;   // >= kLanePrivateMin * nwaves > w
    LaneOrigins<NP> org;
    org.init(lane);
    double* Cw = Rw + tri_size<NP>();
    fold_panels_lane_private_staged<NP, RPL>(X, w * PANEL, (P - 1 - w) / nwaves + 1, nwaves * PANEL, Rw, Cw, org,
                                             lane, stage);
    if (w == nwaves - 1 && P * PANEL < m) {
        double x[RPL][NP];
        load_panel_1d_tail<NP, RPL>(x, X, NP, NP, P * PANEL, m, lane);
        FoldStep<NP, RPL, 0>::run(x, Rw, Cw, org, lane);
    }
}

// ---------------------------------------------------------------------------
// Column-group layout for 16 < n <= 64.  Full rows no longer fit a lane's
// registers with enough rows per lane to amortise the cross-lane sums, so the
// 64 lanes form 8 row groups of 8 lanes: lane (rg, cg) holds RPL rows of its
// row group and the columns c = cg + 8u (u < NP/8).  For column J the pivot
// column is broadcast inside each row group (ds_swizzle), each lane forms the
// dot products for its own columns, and the sums run over the 8 row groups
// only (lane bits 3..5).  Cyclic column ownership keeps every lane busy as J
// advances.
constexpr int kG2 = 8;                   // column groups (lanes per row group)
constexpr int kRG2 = kWave / kG2;        // row groups

template <int CG>
__device__ __forceinline__ double bcast_in_group8(double v) {
    constexpr int off = 0x18 | (CG << 5);  // ds_swizzle bitmask mode: lane = (lane & 0x18) | CG
    int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), off);
    int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), off);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double sum_over_row_groups(double v) {
    v = v + dpp_f64<kDppRor8>(v);  // lane bit 3
    {
        int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);  // xor 16
        int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
        v = v + __hiloint2double(hi, lo);
    }
    return v + __shfl_xor(v, 32, kWave);  // lane bit 5
}

template <int NP, int RPL, int J>
struct FoldStep2D {
    static constexpr int NC = NP / kG2;
    __device__ static __forceinline__ void run(double (&x)[RPL][NP / kG2], double* __restrict__ Rw, int lane) {
        if constexpr (J < NP) {
            constexpr int cgJ = J % kG2;
            constexpr int uJ = J / kG2;
            constexpr int A = NC - uJ;  // live column slots (slot uJ only partly live)
            const int cg = lane % kG2;
            double piv[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) piv[i] = bcast_in_group8<cgJ>(x[i][uJ]);
            double p[A], r[A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) t = fma(piv[i], x[i][uJ + a], t);
                p[a] = t;
                const int c = cg + kG2 * (uJ + a);           // c < J only in finished slots: clamp
                r[a] = Rw[tri_row<NP>(J) + (c > J ? c - J : 0)];
            }
#pragma unroll
            for (int a = 0; a < A; ++a) p[a] = sum_over_row_groups(p[a]);
            const double s = readlane_f64(p[0], cgJ);   // |panel part of column J|^2
            const double alpha = Rw[tri_row<NP>(J)];
            if (reflector_needed(alpha, s)) {
                double beta, u0, gamma;
                reflector_scalars(alpha, s, beta, u0, gamma);
#pragma unroll
                for (int a = 0; a < A; ++a) {
                    const int c = cg + kG2 * (uJ + a);
                    const bool live = (a > 0) || (c > J);
                    double coef = gamma * fma(u0, r[a], p[a]);
                    coef = live ? coef : 0.0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) x[i][uJ + a] = fma(-coef, piv[i], x[i][uJ + a]);
                    if (live && lane < kG2) Rw[tri_row<NP>(J) + c - J] = fma(-coef, u0, r[a]);
                }
                if (lane == 0) Rw[tri_row<NP>(J)] = beta;
            }
            FoldStep2D<NP, RPL, J + 1>::run(x, Rw, lane);
        }
    }
};

template <int NP, int RPL>
__device__ __forceinline__ void load_panel_2d(double (&x)[RPL][NP / kG2], const double* __restrict__ X, int n,
                                              int64_t ldx, int64_t base, int64_t r_end, bool fast, int lane) {
    constexpr int NC = NP / kG2;
    constexpr int64_t PANEL = (int64_t)kRG2 * RPL;
    const int rg = lane / kG2, cg = lane % kG2;
    if (fast && base + PANEL <= r_end) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
        if (n == NP) {
            const int vo = (int)((rg * ldx + cg) * 8);
#pragma unroll
            for (int i = 0; i < RPL; ++i)
#pragma unroll
                for (int u = 0; u < NC; ++u)
                    x[i][u] = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, (int)((kRG2 * i * ldx + kG2 * u) * 8), 0));
        } else {
            // padded width: a column c >= n reads column 0 (in bounds) and is zeroed
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int c = cg + kG2 * u;
                const bool ok = c < n;
                const int vo = (int)((rg * ldx + (ok ? c : 0)) * 8);
#pragma unroll
                for (int i = 0; i < RPL; ++i) {
                    const double v = __builtin_bit_cast(
                        double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, (int)(kRG2 * i * ldx * 8), 0));
                    x[i][u] = ok ? v : 0.0;
                }
            }
        }
    } else {
        const int64_t left = r_end - base - rg;
        const double* x0 = X + (left > 0 ? base + rg : 0) * ldx;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const bool ok = (int64_t)kRG2 * i < left;
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int c = cg + kG2 * u;
                x[i][u] = (ok && c < n) ? x0[(int64_t)kRG2 * i * ldx + c] : 0.0;
            }
        }
    }
}

// Same as fold_rows_1d for the column-group layout (n > 16).
template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_2d(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                             int64_t r_end, double* __restrict__ Rw, int lane) {
    constexpr int NC = NP / kG2;
    constexpr int64_t PANEL = (int64_t)kRG2 * RPL;
    if (r_begin >= r_end) return;
    const bool fast = PANEL * ldx * 8 < 0x7FFFFFFF;   // interior panels: buffer loads (any n <= NP)
    for (int64_t base = r_begin; base < r_end; base += PANEL) {
        double x[RPL][NC];
        load_panel_2d<NP, RPL>(x, X, n, ldx, base, r_end, fast, lane);
        FoldStep2D<NP, RPL, 0>::run(x, Rw, lane);
    }
}

// ---------------------------------------------------------------------------
// 4 x 16 column-group layout for n = 32, 48, 64.  Lane (rg, cg) = (l / 16,
// l % 16) holds RPL rows (rg, rg+4, ...) of the panel and the columns
// c = cg + 16u (u < NP/16).  A row group is one 16-lane DPP row, so the pivot
// column of step J reaches the whole group with one v_mov_b64_dpp
// row_newbcast per row, and the dot products are summed over the 4 row
// groups by two v_permlane16/32_swap stages.  No LDS access in a step except
// row J of R (read by every lane for its columns, written by row group 0),
// and 64/4 = 16 rows per column slot and row group -- four times the rows
// of the 8 x 8 layout -- to amortise the per-column sums and reflector
// scalars.
constexpr int kG4 = 16;                  // column groups (lanes per row group)
constexpr int kRG4 = kWave / kG4;        // row groups

template <int CG>
__device__ __forceinline__ double bcast_row16(double v) {
    // row_newbcast:CG (DPP control 0x150 + CG): lane CG of each 16-lane row to the row
    const long r = __builtin_amdgcn_update_dpp(0L, __builtin_bit_cast(long, v), 0x150 + CG, 0xF, 0xF, true);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ double sum_over_row_groups4(double v) {
    double a, b;
    swap16_f64(v, a, b);   // lane ^ 16
    v = a + b;
    swap32_f64(v, a, b);   // lane ^ 32
    return a + b;
}

template <int NP, int RPL, int J>
struct FoldStepG16 {
    static constexpr int NC = NP / kG4;
    __device__ static __forceinline__ void run(double (&x)[RPL][NP / kG4], double* __restrict__ Rw, int lane) {
        if constexpr (J < NP) {
            constexpr int cgJ = J % kG4;
            constexpr int uJ = J / kG4;
            constexpr int A = NC - uJ;   // live column slots (slot uJ only partly live)
            const int cg = lane % kG4;
            double piv[RPL];
#pragma unroll
            for (int i = 0; i < RPL; ++i) piv[i] = bcast_row16<cgJ>(x[i][uJ]);
            double p[A], r[A];
#pragma unroll
            for (int a = 0; a < A; ++a) {
                const int c = cg + kG4 * (uJ + a);            // c <= J only in slot uJ: clamp
                r[a] = Rw[tri_row<NP>(J) + (c > J ? c - J : 0)];
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) t = fma(piv[i], x[i][uJ + a], t);
                p[a] = t;
            }
#pragma unroll
            for (int a = 0; a < A; ++a) p[a] = sum_over_row_groups4(p[a]);
            const double s = readlane_f64(p[0], cgJ);         // |panel part of column J|^2
            const double alpha = readlane_f64(r[0], cgJ);     // R_JJ
            if (reflector_needed(alpha, s)) {
                double beta, u0, gamma;
                reflector_scalars(alpha, s, beta, u0, gamma);
                double nr[A];
#pragma unroll
                for (int a = 0; a < A; ++a) {
                    const int c = cg + kG4 * (uJ + a);
                    const bool live = (a > 0) || (c > J);
                    const double coef = live ? gamma * fma(u0, r[a], p[a]) : 0.0;
#pragma unroll
                    for (int i = 0; i < RPL; ++i) x[i][uJ + a] = fma(-coef, piv[i], x[i][uJ + a]);
                    nr[a] = fma(-coef, u0, r[a]);
                }
                if (lane < kG4) {
                    // the new row J of R; a column c <= J of slot uJ writes to the lane's spare slot
#pragma unroll
                    for (int a = 0; a < A; ++a) {
                        const int c = cg + kG4 * (uJ + a);
                        const bool live = (a > 0) || (c > J);
                        Rw[live ? tri_row<NP>(J) + c - J : tri_size<NP>() + cg] = nr[a];
                    }
                    if (lane == 0) Rw[tri_row<NP>(J)] = beta;
                }
            }
            FoldStepG16<NP, RPL, J + 1>::run(x, Rw, lane);
        }
    }
};

// Panel of 4 RPL rows at `base` in the 4 x 16 layout: lane (rg, cg) gets
// rows base + rg + 4i, columns cg + 16u; rows >= r_end and columns >= n read
// as zero.  Full panels load 16 consecutive doubles of a row per group.
template <int NP, int RPL>
__device__ __forceinline__ void load_panel_g16(double (&x)[RPL][NP / kG4], const double* __restrict__ X, int n,
                                               int64_t ldx, int64_t base, int64_t r_end, bool fast, int lane) {
    constexpr int NC = NP / kG4;
    constexpr int64_t PANEL = (int64_t)kRG4 * RPL;
    const int rg = lane / kG4, cg = lane % kG4;
    if (fast && base + PANEL <= r_end) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
#pragma unroll
        for (int u = 0; u < NC; ++u) {
            const int c = cg + kG4 * u;
            const bool ok = c < n;                     // a padded column reads column 0 (in bounds), zeroed
            const int vo = (int)((rg * ldx + (ok ? c : 0)) * 8);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const double v = __builtin_bit_cast(
                    double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, (int)(kRG4 * i * ldx * 8), 0));
                x[i][u] = ok ? v : 0.0;
            }
        }
    } else {
        const int64_t left = r_end - base - rg;
        const double* x0 = X + (left > 0 ? base + rg : 0) * ldx;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const bool ok = (int64_t)kRG4 * i < left;
#pragma unroll
            for (int u = 0; u < NC; ++u) {
                const int c = cg + kG4 * u;
                x[i][u] = (ok && c < n) ? x0[(int64_t)kRG4 * i * ldx + c] : 0.0;
            }
        }
    }
}

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows_g16(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                              int64_t r_end, double* __restrict__ Rw, int lane) {
    constexpr int64_t PANEL = (int64_t)kRG4 * RPL;
    if (r_begin >= r_end) return;
    const bool fast = PANEL * ldx * 8 < 0x7FFFFFFF;
    for (int64_t base = r_begin; base < r_end; base += PANEL) {
        double x[RPL][NP / kG4];
        load_panel_g16<NP, RPL>(x, X, n, ldx, base, r_end, fast, lane);
        FoldStepG16<NP, RPL, 0>::run(x, Rw, lane);
    }
}

// ---------------------------------------------------------------------------
// Blocked fold on the FP64 matrix cores for n = 32, 48, 64 (the instances
// with one row per lane; v_mfma_f64_16x16x4f64).  A panel of 64 rows W is
// held in registers as NB = NP/16 column blocks in the matrix-core operand
// layout: register c of lane l of block K holds W[4c + l/16][16K + l%16].
// That is also the 4 x 16 column-group layout with 16 rows per lane (row
// group l/16, column l%16 of the block), so block J is folded into the
// running R column by column in place -- the reflectors of the unblocked
// fold (pivot column broadcast by DPP row_newbcast, sums over the 4 row
// groups), with their pivot entries u0_j and gamma_j recorded -- and what
// the fold leaves in its registers is V, the reflectors' part in W, already
// in the operand layout of V^T V and V^T W_K.  Its 16 reflectors
// H_j = I - gamma_j u_j u_j^T then act on the later blocks at once in
// compact WY form (forward, columnwise: H_0 H_1 ... H_15 = I - U T U^T with
// T_jj = gamma_j and T_{0:j,j} = -gamma_j T_{0:j,0:j} U_{:,0:j}^T u_j).  U
// stacks diag(u0) on the R rows of block J over V, the 64 x 16 reflector
// part in W, so U^T U = diag(u0^2) + V^T V, and only its strictly upper
// part, that of V^T V, enters T.  For a later block K, with C = [R_{J,K}; W_K]:
//   S  = U^T C = diag(u0) R_{J,K} + V^T W_K     (16 matrix-core steps)
//   S' = T^T S                                  (4)
//   R_{J,K} -= diag(u0) S',  W_K -= V S'        (16)
// which is applying the 16 reflectors in turn with the sums regrouped.
//
// V S' takes V with rows on the lane's low bits, so V goes through LDS once
// per block.  Per-wavefront LDS scratch (doubles): that 64 x 16 buffer (row
// stride 17), V^T V (16 x 16), T (stride 17), the recorded u0 and gamma.
typedef double mf64x4 __attribute__((ext_vector_type(4)));

constexpr int kMfVs = 17;                       // row stride of the transpose buffer and of T
constexpr int kMfV = 0;                         // 64 x 16 (stride 17)
constexpr int kMfY = kMfV + 64 * kMfVs;         // 16 x 16
constexpr int kMfT = kMfY + 256;                // 16 x 16 (stride 17)
constexpr int kMfRec = kMfT + 16 * kMfVs;       // u0[16], gamma[16]
constexpr int kMfScratch = kMfRec + 32;

// Block KB (columns 16KB..16KB+15) of the 64-row panel at row `base`, in
// the operand layout; rows >= r_end and columns >= n read as zero.
template <int KB>
__device__ __forceinline__ void mf_load_block(double (&gk)[16], const double* __restrict__ X, int n, int64_t ldx,
                                              int64_t base, int64_t r_end, bool fast, int lane) {
    const int lo = lane & 15, hi = lane >> 4;
    if (fast && base + 64 <= r_end) {
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + base * ldx), (short)0, 0x7FFFFFFF, 0x00020000);
        const int vo = (int)((hi * ldx + 16 * KB + lo) * 8);
#pragma unroll
        for (int c = 0; c < 16; ++c)
            gk[c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, (int)(4 * c * ldx * 8), 0));
    } else {
        const int col = 16 * KB + lo;
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            const int64_t row = base + 4 * c + hi;
            gk[c] = (row < r_end && col < n) ? X[row * ldx + col] : 0.0;
        }
    }
}

template <int NP, int KB>
__device__ __forceinline__ void mf_load_panel(double (&g)[NP / 16][16], const double* __restrict__ X, int n,
                                              int64_t ldx, int64_t base, int64_t r_end, bool fast, int lane) {
    if constexpr (KB < NP / 16) {
        mf_load_block<KB>(g[KB], X, n, ldx, base, r_end, fast, lane);
        mf_load_panel<NP, KB + 1>(g, X, n, ldx, base, r_end, fast, lane);
    }
}

// Step j of the fold of diagonal block JB (column J = 16 JB + j) in the 4 x
// 16 layout, 16 rows per lane: x[c] is row 4c + l/16 of the panel, column
// 16 JB + l%16.  Only the block's own columns are updated (R row J, columns
// 16 JB .. 16 JB + 15, and x); u0_j and gamma_j go to rec[j], rec[16 + j]
// (0 and 0 for a column left as it is).
template <int NP, int JB, int j>
struct FoldStepBlk {
    __device__ static __forceinline__ void run(double (&x)[16], double* __restrict__ Rw, double* __restrict__ rec,
                                               int lane) {
        if constexpr (j < 16) {
            constexpr int J = 16 * JB + j;
            const int cg = lane % kG4;
            const bool live = cg > j;
            double piv[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) piv[c] = bcast_row16<j>(x[c]);
            const double r = Rw[tri_row<NP>(J) + (live ? cg - j : 0)];
            double p = 0.0;
#pragma unroll
            for (int c = 0; c < 16; ++c) p = fma(piv[c], x[c], p);
            p = sum_over_row_groups4(p);
            const double s = readlane_f64(p, j);       // |panel part of column J|^2
            const double alpha = readlane_f64(r, j);   // R_JJ
            if (reflector_needed(alpha, s)) {
                double beta, u0, gamma;
                reflector_scalars(alpha, s, beta, u0, gamma);
                const double coef = live ? gamma * fma(u0, r, p) : 0.0;
#pragma unroll
                for (int c = 0; c < 16; ++c) x[c] = live ? fma(-coef, piv[c], x[c]) : x[c];
                if (lane < kG4) Rw[live ? tri_row<NP>(J) + cg - j : tri_size<NP>() + cg] = fma(-coef, u0, r);
                if (lane == 0) {
                    Rw[tri_row<NP>(J)] = beta;
                    rec[j] = u0;
                    rec[16 + j] = gamma;
                }
            } else if (lane == 0) {
                rec[j] = 0.0;
                rec[16 + j] = 0.0;
            }
            FoldStepBlk<NP, JB, j + 1>::run(x, Rw, rec, lane);
        }
    }
};

// Block JB of the panel in g: fold it into R (Rw, packed NP x NP), apply its
// reflectors to blocks JB+1.., and load block JB of the next panel (row
// `next`) into the registers it frees.
template <int NP, int JB>
__device__ __forceinline__ void mf_fold_block(double (&g)[NP / 16][16], double* __restrict__ Rw,
                                              double* __restrict__ scr, int lane, const double* __restrict__ X,
                                              int n, int64_t ldx, int64_t next, int64_t r_end, bool fast) {
    constexpr int NB = NP / 16;
    const int lo = lane & 15, hi = lane >> 4;
    double* __restrict__ rec = scr + kMfRec;
    // the x of the column fold keeps its dead columns unchanged, so what is
    // left in g[JB] is V: column j holds the panel part of reflector j
    FoldStepBlk<NP, JB, 0>::run(g[JB], Rw, rec, lane);
    if constexpr (JB + 1 < NB) {
        double* __restrict__ Vt = scr + kMfV;
#pragma unroll
        for (int c = 0; c < 16; ++c) Vt[(4 * c + hi) * kMfVs + lo] = g[JB][c];
        // Y = V^T V
        mf64x4 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 16; ++c) y = __builtin_amdgcn_mfma_f64_16x16x4f64(g[JB][c], g[JB][c], y, 0, 0, 0);
        double* __restrict__ Y = scr + kMfY;
#pragma unroll
        for (int v = 0; v < 4; ++v) Y[(4 * v + hi) * 16 + lo] = y[v];
        // T, one row per lane (row i = lane % 16): T_ii = gamma_i and, for
        // j > i, T_ij = -gamma_j sum_{i<=k<j} T_ik Y_kj
        double tr[16];
        const double gi = rec[16 + lo];
#pragma unroll
        for (int k = 0; k < 16; ++k) tr[k] = (k == lo) ? gi : 0.0;
#pragma unroll
        for (int j = 1; j < 16; ++j) {
            asm volatile("" ::: "memory");   // read each column of Y where it is used
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k) a = fma(tr[k], Y[k * 16 + j], a);
            const double gj = rec[16 + j];
            if (j > lo) tr[j] = -gj * a;
        }
        double* __restrict__ T = scr + kMfT;
        if (hi == 0) {
#pragma unroll
            for (int j = 0; j < 16; ++j) T[lo * kMfVs + j] = tr[j];
        }
        double ta[4];                        // T^T in the A layout
#pragma unroll
        for (int c = 0; c < 4; ++c) ta[c] = T[(4 * c + hi) * kMfVs + lo];
        double va[4][4];                     // -V in the A layout, row tile u
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < 4; ++c) va[u][c] = -Vt[(16 * u + lo) * kMfVs + 4 * c + hi];
        double u0r[4];                       // u0 of the R row this lane's S entries sit on
#pragma unroll
        for (int v = 0; v < 4; ++v) u0r[v] = rec[4 * v + hi];
#pragma unroll
        for (int K = JB + 1; K < NB; ++K) {
            int ri[4];
            mf64x4 s;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * JB + 4 * v + hi;
                ri[v] = tri_row<NP>(row) + 16 * K + lo - row;
                s[v] = u0r[v] * Rw[ri[v]];
            }
#pragma unroll
            for (int c = 0; c < 16; ++c) s = __builtin_amdgcn_mfma_f64_16x16x4f64(g[JB][c], g[K][c], s, 0, 0, 0);
            mf64x4 sp = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) sp = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[c], s[c], sp, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) Rw[ri[v]] = fma(-u0r[v], sp[v], Rw[ri[v]]);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mf64x4 acc = {g[K][4 * u], g[K][4 * u + 1], g[K][4 * u + 2], g[K][4 * u + 3]};
#pragma unroll
                for (int c = 0; c < 4; ++c) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u][c], sp[c], acc, 0, 0, 0);
#pragma unroll
                for (int v = 0; v < 4; ++v) g[K][4 * u + v] = acc[v];
            }
        }
    }
    if (next < r_end) mf_load_block<JB>(g[JB], X, n, ldx, next, r_end, fast, lane);
    if constexpr (JB + 1 < NB) mf_fold_block<NP, JB + 1>(g, Rw, scr, lane, X, n, ldx, next, r_end, fast);
}

// Fold rows [r_begin, r_end) of X (n <= NP columns) into Rw, 64 rows at a
// time; the loads of each panel overlap the work on the one before.
template <int NP>
__device__ __forceinline__ void fold_rows_mfma(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                               int64_t r_end, double* __restrict__ Rw, double* __restrict__ scr,
                                               int lane) {
    static_assert(NP % 16 == 0, "the matrix-core fold works on 16-column blocks");
    if (r_begin >= r_end) return;
    const bool fast = n == NP && (int64_t)64 * ldx * 8 < 0x7FFFFFFF;
    double g[NP / 16][16];
    mf_load_panel<NP, 0>(g, X, n, ldx, r_begin, r_end, fast, lane);
    for (int64_t base = r_begin; base < r_end; base += 64)
        mf_fold_block<NP, 0>(g, Rw, scr, lane, X, n, ldx, base + 64, r_end, fast);
}

template <int NP, int RPL>
__device__ __forceinline__ void fold_rows(const double* __restrict__ X, int n, int64_t ldx, int64_t r_begin,
                                          int64_t r_end, double* __restrict__ Rw, int lane,
                                          double* stage = nullptr) {
    if constexpr (mf_instance<NP, RPL>()) fold_rows_mfma<NP>(X, n, ldx, r_begin, r_end, Rw, stage, lane);
    else if constexpr (g16_instance<NP, RPL>()) fold_rows_g16<NP, RPL>(X, n, ldx, r_begin, r_end, Rw, lane);
    else if constexpr (NP <= 16) fold_rows_1d<NP, RPL>(X, n, ldx, r_begin, r_end, Rw, lane, stage);
    else fold_rows_2d<NP, RPL>(X, n, ldx, r_begin, r_end, Rw, lane);
}

// Rows of a panel for an instance (the unit rows_per_wave is rounded to).
template <int NP, int RPL>
constexpr int64_t panel_rows() {
    return (int64_t)(NP <= 16 || mf_instance<NP, RPL>() ? kWave : g16_instance<NP, RPL>() ? kRG4 : kRG2) * RPL;
}

template <int NP>
__device__ __forceinline__ void zero_r(double* __restrict__ Rw, int lane) {
    for (int e = lane; e < tri_size<NP>(); e += kWave) Rw[e] = 0.0;
    __builtin_amdgcn_wave_barrier();
}

// Load an n x n upper triangle (row-major, ld; entries below the diagonal
// ignored) into the wavefront's packed R, which zero_r has cleared.
template <int NP>
__device__ __forceinline__ void load_r(double* __restrict__ Rw, int n, const double* __restrict__ src, int64_t ld,
                                       int lane) {
    for (int J = 0; J < n; ++J)
        for (int c = J + lane; c < n; c += kWave) Rw[tri_row<NP>(J) + c - J] = src[(int64_t)J * ld + c];
    __builtin_amdgcn_wave_barrier();
}

// Write the wavefront's R (n x n, zeros below the diagonal) to out (ld).
// With normalise, rows with a negative diagonal are negated and -0.0 is
// written as +0.0.
template <int NP>
__device__ __forceinline__ void store_r(const double* __restrict__ Rw, int n, double* __restrict__ out, int64_t ld,
                                        bool normalise, int lane) {
    if (lane < n) {
        const int r = lane;
        const double sgn = (normalise && Rw[tri_row<NP>(r)] < 0.0) ? -1.0 : 1.0;
        double* o = out + (int64_t)r * ld;
        for (int c = 0; c < n; ++c) {
            const double v = (c >= r) ? Rw[tri_row<NP>(r) + c - r] : 0.0;
            o[c] = normalise ? sgn * v + 0.0 : v;
        }
    }
}

// Fold the packed triangles that wavefronts 1..count-1 of the workgroup left
// in LDS (regions Rsh0 + w*stride) into wavefront 0's (region 0, which thus
// accumulates R([R_0; R_1; ...])): their rows, stacked, form a
// (count-1)*n x n matrix, folded panel by panel in the caller's register
// layout.  The order is fixed, so the result does not depend on which
// wavefront runs it.
template <int NP, int RPL>
__device__ __forceinline__ void fold_block_triangles(double* __restrict__ Rsh0, int stride, int count, int n,
                                                     int lane) {
    double* __restrict__ Rw = Rsh0;
    const int rows = (count - 1) * n;
    auto value = [&](int r, int c) -> double {
        if (r >= rows || c >= n) return 0.0;
        const int t = r / n, i = r - t * n;
        if (c < i) return 0.0;
        return Rsh0[(t + 1) * stride + tri_row<NP>(i) + c - i];
    };
    if constexpr (NP <= 16) {
        LaneOrigins<NP> org;
        org.init(lane);
        double* Cw = Rw + tri_size<NP>();
        for (int base = 0; base < rows; base += kWave * RPL) {
            double x[RPL][NP];
#pragma unroll
            for (int i = 0; i < RPL; ++i)
#pragma unroll
                for (int c = 0; c < NP; ++c) x[i][c] = value(base + lane + kWave * i, c);
            FoldStep<NP, RPL, 0>::run(x, Rw, Cw, org, lane);
        }
    } else {
        // the matrix-core and 4 x 16 instances combine in the 8 x 8 layout with 4 rows per lane
        constexpr int CR = (mf_instance<NP, RPL>() || g16_instance<NP, RPL>()) ? 4 : RPL;
        const int rg = lane / kG2, cg = lane % kG2;
        for (int base = 0; base < rows; base += kRG2 * CR) {
            double x[CR][NP / kG2];
#pragma unroll
            for (int i = 0; i < CR; ++i)
#pragma unroll
                for (int u = 0; u < NP / kG2; ++u) x[i][u] = value(base + rg + kRG2 * i, cg + kG2 * u);
            FoldStep2D<NP, CR, 0>::run(x, Rw, lane);
        }
    }
}

// The n = 48 and 64 matrix-core instances need more than 256 registers per
// lane (one wavefront per SIMD); every other instance is built for two.  (Three
// per SIMD for the n = 16 fold with three rows per lane, at most 168
// registers, measured 3 % slower than two with four rows per lane.)
template <int NP, int RPL>
constexpr int fold_waves_per_eu() {
    return (mf_instance<NP, RPL>() && NP >= 48) ? 1 : 2;
}

// One launch of Alg. 2 (stage 1 or a tree level): wavefront w folds rows
// [w*rows_per_wave, min(m, (w+1)*rows_per_wave)) of X into a triangle (the
// LDS-staged lane-private instances take interleaved panels instead, see
// fold_rows_interleaved); the last wavefront of each workgroup to finish
// folds the triangles of wavefronts 1.. into wavefront 0's, in that order (all kept in LDS; ordering
// through a workgroup-scope atomic, which costs no cache maintenance), and
// writes the workgroup's triangle at
// Y + blockIdx.x*ystride (leading dimension ldy).  With normalise (a single
// workgroup, the final R), rows of a negative diagonal are negated.
template <int NP, int RPL>
__global__ void __launch_bounds__((64 * waves_per_block<NP, RPL>()))
__attribute__((amdgpu_waves_per_eu(fold_waves_per_eu<NP, RPL>())))
tsqr_fold_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_wave,
                 int64_t nwaves, double* __restrict__ Y, int64_t ldy, int64_t ystride, int normalise,
                 const double* Yinit) {
    constexpr int WPB = waves_per_block<NP, RPL>();
    constexpr int STRIDE = tri_size<NP>() + NP;
    constexpr int STAGE = mf_instance<NP, RPL>() ? kMfScratch : stage_doubles<NP, RPL>() > 0 ? stage_doubles<NP, RPL>() : 2;
    static_assert((size_t)WPB * (STRIDE + STAGE) * sizeof(double) + 16 <= 160 * 1024,
                  "a workgroup must fit the 160 KB of LDS of a gfx950 compute unit");
    __shared__ double Rsh[WPB][STRIDE];
    __shared__ __attribute__((aligned(16))) double stage[WPB][STAGE];
    __shared__ int arrivals;
    if (threadIdx.x == 0) arrivals = 0;
    __syncthreads();
    const int lane = lane_id();
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform (SGPR)
    const int64_t w0 = (int64_t)blockIdx.x * WPB;
    const int64_t w = w0 + wib;
    if (w >= nwaves) return;
    const int nvalid = (int)(nwaves - w0 < WPB ? nwaves - w0 : WPB);
    double* Rw = Rsh[wib];
    zero_r<NP>(Rw, lane);
    if (Yinit != nullptr && wib == 0) load_r<NP>(Rw, n, Yinit + (int64_t)blockIdx.x * ystride, ldy, lane);
    if (interleaved_stage1<NP, RPL>(m, n, ldx, nwaves)) {
        fold_rows_interleaved<NP, RPL>(X, m, w, nwaves, Rw, lane, stage[wib]);
    } else {
        const int64_t r_begin = w * rows_per_wave;
        const int64_t r_end = (r_begin + rows_per_wave < m) ? r_begin + rows_per_wave : m;
        fold_rows<NP, RPL>(X, n, ldx, r_begin, r_end, Rw, lane,
                           (mf_instance<NP, RPL>() || stage_doubles<NP, RPL>() > 0) ? stage[wib] : nullptr);
    }
    if (nvalid > 1) {
        int old = 0;
        if (lane == 0) old = __hip_atomic_fetch_add(&arrivals, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        old = __builtin_amdgcn_readfirstlane(old);
        if (old != nvalid - 1) return;   // a sibling is still folding; it will combine
        fold_block_triangles<NP, RPL>(&Rsh[0][0], STRIDE, nvalid, n, lane);
        Rw = Rsh[0];
    }
    store_r<NP>(Rw, n, Y + (int64_t)blockIdx.x * ystride, ldy, normalise != 0, lane);
}

template <int NP, int RPL>
hipError_t launch_fold(const FoldArgs& a, hipStream_t stream) {
    constexpr int WPB = waves_per_block<NP, RPL>();
    const int64_t blocks = ceil_div(a.nwaves, WPB);
    hipLaunchKernelGGL((tsqr_fold_kernel<NP, RPL>), dim3((unsigned)blocks), dim3(64 * WPB), 0, stream, a.X, a.m, a.n,
                       a.ldx, a.rows_per_wave, a.nwaves, a.Y, a.ldy, a.ystride, a.normalise, a.Yinit);
    return hipGetLastError();
}

// Last tree level of a TSQR for n <= 16 in one workgroup: wavefront w of
// kTreeWaves folds a contiguous share of the k stacked triangles into its
// triangle in LDS; after the workgroup barrier wavefront 0 folds the others'
// into its own, in wavefront order, and writes R with a non-negative
// diagonal.  Replaces the last two or three launches of a fan-in tree.
constexpr int kTreeWaves = 8;

template <int NP, int RPL>
__global__ void __launch_bounds__(64 * kTreeWaves) __attribute__((amdgpu_waves_per_eu(2)))
tsqr_tree_block_kernel(const double* __restrict__ Y, int64_t k, int n, double* __restrict__ R, int64_t ldr) {
    __shared__ double Rsh[kTreeWaves][tri_size<NP>() + NP];
    const int lane = lane_id();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double* Rw = Rsh[w];
    const int64_t per = ceil_div(k, kTreeWaves);
    const int64_t t0 = (int64_t)w * per < k ? (int64_t)w * per : k;
    const int64_t t1 = t0 + per < k ? t0 + per : k;
    zero_r<NP>(Rw, lane);
    fold_rows<NP, RPL>(Y, n, n, t0 * n, t1 * n, Rw, lane);
    __syncthreads();
    if (w == 0) {
        // the wavefronts' triangles stay in LDS: fold 1.. into 0, in order
        fold_block_triangles<NP, RPL>(&Rsh[0][0], tri_size<NP>() + NP, kTreeWaves, n, lane);
        store_r<NP>(Rsh[0], n, R, ldr, true, lane);
    }
}

template <int NP, int RPL>
hipError_t launch_tree_block(const double* Y, int64_t k, int n, double* R, int64_t ldr, hipStream_t stream) {
    hipLaunchKernelGGL((tsqr_tree_block_kernel<NP, RPL>), dim3(1), dim3(64 * kTreeWaves), 0, stream, Y, k, n, R, ldr);
    return hipGetLastError();
}

}  // namespace tsqr_detail
}  // namespace qless

// Definitions of the launch functions of one (padded width, rows per lane)
// instance, for the instance files (one file per group of widths, so that
// the instances compile in parallel).
#define QLESS_DEFINE_FOLD(NP, RPL)                                                        \
    hipError_t launch_fold_np##NP##_r##RPL(const FoldArgs& a, hipStream_t s) {             \
        return tsqr_detail::launch_fold<NP, RPL>(a, s);                                   \
    }
#define QLESS_DEFINE_TREE(NP, RPL)                                                                            \
    hipError_t launch_tree_np##NP##_r##RPL(const double* Y, int64_t k, int n, double* R, int64_t ldr,        \
                                           hipStream_t s) {                                                  \
        return tsqr_detail::launch_tree_block<NP, RPL>(Y, k, n, R, ldr, s);                                  \
    }

