// Internal declarations of the qless HIP library (not installed).
// Device helpers for wavefront-level (64-lane) data exchange on gfx950 and
// host-side launch plans shared by the C-ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/qless.h"

namespace qless {

constexpr int kWave = 64;

typedef double f64x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------ wave exchange

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Value of `v` held by lane `src` (a compile-time or wave-uniform lane index),
// broadcast to every lane through two v_readlane_b32 (result is uniform).
__device__ __forceinline__ double readlane_f64(double v, int src) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

// Partner exchange across the two 32-lane halves (lane l <-> l ^ 32):
// v_permlane32_swap moves the upper half of its first operand into the lower
// half of its second.  With both operands equal to `v`, lanes < 32 find the
// partner's value in the second result and lanes >= 32 in the first, so
// first + second is the pairwise sum in every lane.
__device__ __forceinline__ void swap32_f64(double v, double& first, double& second) {
    auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    first = __hiloint2double(hi[0], lo[0]);
    second = __hiloint2double(hi[1], lo[1]);
}

// Same for lane l <-> l ^ 16 (v_permlane16_swap pairs rows 0/1 and 2/3).
__device__ __forceinline__ void swap16_f64(double v, double& first, double& second) {
    auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    first = __hiloint2double(hi[0], lo[0]);
    second = __hiloint2double(hi[1], lo[1]);
}

// DPP move of a double: every lane receives the value of the lane selected by
// the DPP control word `ctrl` (all rows and banks enabled, every source lane
// valid for the patterns used here, so no "old" value is needed).
template <int ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), ctrl, 0xF, 0xF, true);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), ctrl, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// DPP control words (GFX9 encoding).
constexpr int kDppXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppMirror8 = 0x141;  // row_half_mirror: lane i <-> 7 - i within 8
constexpr int kDppRor8 = 0x128;     // row_ror:8: lane i <-> i ^ 8 within 16

// Sum of `v` over all 64 lanes; every lane gets the same, bitwise-identical
// value (each step adds a lane's value and its partner's, and IEEE addition
// is commutative).  Pairing order: ^32, ^16, ^8, mirror within 8, ^2, ^1 --
// six disjoint pairings whose composition covers all 64 lanes.
__device__ __forceinline__ double wave_sum_f64(double v) {
    double a, b;
    swap32_f64(v, a, b);
    v = a + b;
    swap16_f64(v, a, b);
    v = a + b;
    v = v + dpp_f64<kDppRor8>(v);
    v = v + dpp_f64<kDppMirror8>(v);
    v = v + dpp_f64<kDppXor2>(v);
    v = v + dpp_f64<kDppXor1>(v);
    return v;
}

// ---------------------------------------------- transposed multi-value sum
//
// Sum K per-lane values p[0..K-1] over the 64 lanes at the cost of about
// 1.5 exchanges per value instead of six: each of the six pairing stages
// (lane bit 5, 4, 3, 2, 1, 0 -- partners as in wave_sum_f64) halves the
// number of live slots.  For S live slots, slot t < S/2 is paired with slot
// t + S/2: the lane whose stage bit is 0 keeps slot t, its partner keeps
// slot t + S/2, and each adds the other's copy of the slot it keeps; an odd
// leftover slot is summed in both lanes.  Stages on bits 5 and 4 use one
// v_permlane32/16_swap per 32-bit half, which moves both slots at once; the
// DPP stages select what to send and keep.  After the six stages each lane
// holds the full sum of exactly one value in p[0]; which one is a
// compile-time function of the lane id (red_origin), so red_locate gives a
// lane to read value v from.

constexpr int red_next(int S) { return S >= 2 ? S / 2 + (S & 1) : 1; }

// Original value index held in p[0] by `lane` after the six stages.
constexpr int red_origin(int K, int lane) {
    int S[7] = {K, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < 6; ++s) S[s + 1] = red_next(S[s]);
    int t = 0;
    for (int s = 5; s >= 0; --s) {
        const int Ss = S[s];
        if (Ss >= 2) {
            const int P = Ss / 2;
            if (t < P) t = ((lane >> (5 - s)) & 1) ? t + P : t;
            else t = 2 * P;
        }
    }
    return t;
}

constexpr int red_locate(int K, int v) {
    for (int l = 0; l < 64; ++l)
        if (red_origin(K, l) == v) return l;
    return -1;
}

template <int STAGE>
__device__ __forceinline__ double red_pair(double a, double b, int lane) {
    if constexpr (STAGE == 0 || STAGE == 1) {
        int2 lo, hi;
        if constexpr (STAGE == 0) {
            auto l = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false, false);
            auto h = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false, false);
            lo = make_int2(l[0], l[1]);
            hi = make_int2(h[0], h[1]);
        } else {
            auto l = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false, false);
            auto h = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false, false);
            lo = make_int2(l[0], l[1]);
            hi = make_int2(h[0], h[1]);
        }
        return __hiloint2double(hi.x, lo.x) + __hiloint2double(hi.y, lo.y);
    } else {
        constexpr int bit = 5 - STAGE;
        constexpr int ctrl = STAGE == 2 ? kDppRor8 : STAGE == 3 ? kDppMirror8 : STAGE == 4 ? kDppXor2 : kDppXor1;
        const bool up = (lane >> bit) & 1;
        const double send = up ? a : b;
        const double keep = up ? b : a;
        return keep + dpp_f64<ctrl>(send);
    }
}

template <int STAGE>
__device__ __forceinline__ double red_all(double v) {
    if constexpr (STAGE == 0 || STAGE == 1) {
        double a, b;
        if constexpr (STAGE == 0) swap32_f64(v, a, b);
        else swap16_f64(v, a, b);
        return a + b;
    } else {
        constexpr int ctrl = STAGE == 2 ? kDppRor8 : STAGE == 3 ? kDppMirror8 : STAGE == 4 ? kDppXor2 : kDppXor1;
        return v + dpp_f64<ctrl>(v);
    }
}

template <int S, int STAGE>
__device__ __forceinline__ void red_stages(double* p, int lane) {
    if constexpr (STAGE < 6) {
        if constexpr (S >= 2) {
            constexpr int P = S / 2;
#pragma unroll
            for (int t = 0; t < P; ++t) p[t] = red_pair<STAGE>(p[t], p[t + P], lane);
            if constexpr (S & 1) p[P] = red_all<STAGE>(p[2 * P]);
            red_stages<P + (S & 1), STAGE + 1>(p, lane);
        } else {
            p[0] = red_all<STAGE>(p[0]);
            red_stages<1, STAGE + 1>(p, lane);
        }
    }
}

// Sum p[0..K-1] over the wavefront; on return tot[v] is the (uniform) total
// of value v in every lane.
template <int K>
__device__ __forceinline__ void wave_sum_multi(double* p, double* tot, int lane) {
    red_stages<K, 0>(p, lane);
#pragma unroll
    for (int v = 0; v < K; ++v) tot[v] = readlane_f64(p[0], red_locate(K, v));
}

// ------------------------------------------------------------- host plans

struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    size_t lds_per_block = 0;
};

// Cached properties of the current device (thread-compatible, not thread-safe
// on first use per device).
const DeviceInfo& current_device_info();

// Arguments of one launch of the TSQR fold kernel (stage 1 or a tree level):
// wavefront w folds rows [w * rows_per_wave, ...) of X (m x n, ld ldx); each
// workgroup writes one triangle at Y + block * ystride (ld ldy), with
// normalise the diagonal made non-negative.  With Yinit (may alias Y), each
// workgroup starts from its triangle there instead of zero (a running
// stage-1 state over chunks of rows).
struct FoldArgs {
    const double* X;
    int64_t m;
    int n;
    int64_t ldx, rows_per_wave, nwaves;
    double* Y;
    int64_t ldy, ystride;
    int normalise;
    const double* Yinit;
};

// Launch function of one compiled fold instance (tsqr_i*.hip).
typedef hipError_t (*FoldFn)(const FoldArgs&, hipStream_t);
// The instance of exactly this padded width and rows per lane (or null).
FoldFn find_fold(int npad, int rpl);
// Rows of one panel of an instance (the unit rows_per_wave is rounded to).
int64_t tsqr_panel_rows(int npad, int rpl);

// Plan of a TSQR call: stage-1 wave count, rows per wave, tree shape.
struct TsqrPlan {
    int npad = 0;              // padded column count of the kernel instance
    int rows_per_lane = 0;     // panel rows per lane (panel = 64 * rows_per_lane rows)
    int64_t rows_per_wave = 0; // stage-1 rows per wavefront
    int64_t k0 = 0;            // stage-1 wavefronts
    int wpb = 0;               // wavefronts per workgroup (one triangle per workgroup)
    int64_t k1 = 0;            // stage-1 triangles (workgroups)
    int fan_in = 0;            // blocks combined per tree wavefront
    int levels = 0;            // tree launches (0: stage 1 writes R directly)
    bool block_tree = false;   // the last level is one workgroup (n <= 16)
    int64_t tree_rows = 0;     // stacked rows per wavefront of that last level
    size_t ybytes_a = 0;       // stacked triangles of stage 1 (and of odd tree levels)
    size_t ybytes_b = 0;       // stacked triangles of even tree levels
    size_t work_bytes = 0;     // total workspace
};

// tuned = false ignores the qless_tune_set overrides (the default instance).
// rpl != 0 asks for the instance with that many rows per lane (it must
// exist for the padded width; callers that pair the plan with a kernel of
// their own, the two-phase fold, pass that kernel's).
TsqrPlan make_tsqr_plan(int64_t m, int64_t n, int num_cus, bool tuned = true, int rpl = 0);
// The tree of a plan over k >= 2 stacked triangles in src (dst takes the
// intermediate levels); writes R (ld ldr) with a non-negative diagonal.
hipError_t launch_tsqr_tree(const TsqrPlan& plan, double* src, double* dst, int64_t k, int64_t n, double* R,
                            int64_t ldr, hipStream_t stream);

// Per-n launch-parameter overrides (0 = default); see qless_tune_set.
int tsqr_tune_set(int64_t n, int waves_per_cu, int fan_in, int rows_per_lane);
int tsqr_tune_get(int64_t n, int* waves_per_cu, int* fan_in, int* rows_per_lane);

// Plan and launch of R <- R([R; X]) (qless_tsqr_r_update): the previous R
// joins the stacked triangles of X as one more.
TsqrPlan make_tsqr_update_plan(int64_t m, int64_t n, int num_cus);
hipError_t launch_tsqr_update(const double* X, int64_t m, int64_t n, int64_t ldx, double* R, int64_t ldr,
                              void* work, const TsqrPlan& plan, hipStream_t stream);

// Enqueue a full TSQR (stage 1 + tree + sign normalisation) into `work`.
// Arguments have been validated by the caller.
hipError_t launch_tsqr(const double* X, int64_t m, int64_t n, int64_t ldx, double* R,
                       int64_t ldr, void* work, const TsqrPlan& plan, hipStream_t stream);

// Plan of a Gram pass: wavefront count and rows per wavefront.
struct GramPlan {
    int npad = 0;              // kernel width: power of two up to 8, else a multiple of 16
    int64_t rows_per_wave = 0;
    int64_t k = 0;             // wavefronts = partial Gram matrices
    size_t part_bytes = 0;     // bytes of the k partials
};

GramPlan make_gram_plan(int64_t m, int64_t n, int num_cus);

// C = (X M)^T (X M) (M == nullptr: C = X^T X), via k wavefront partials in
// Cpart and a fixed-order sum into C (n x n, ld n).  m_upper: M is upper
// triangular with exact zeros below the diagonal, which the matrix-core
// kernel then does not multiply.
hipError_t launch_gram(const double* X, int64_t m, int64_t n, int64_t ldx, const double* M, bool m_upper,
                       double* Cpart, double* C, const GramPlan& plan, hipStream_t stream);

// Double-double Gram pass (gram_dd.hip): k workgroups of 256 threads, each
// over rows_per_block rows, writing a (hi, lo) partial of 2 n x n doubles.
struct GramDdPlan {
    int npad = 0;
    int64_t rows_per_block = 0;
    int64_t k = 0;
    size_t part_bytes = 0;
};
GramDdPlan make_gram_dd_plan(int64_t m, int64_t n, int num_cus);
// C = X^T X in double-double: hi into Chi, lo into Clo (may be null), ld ldc.
hipError_t launch_gram_dd(const double* X, int64_t m, int64_t n, int64_t ldx, double* part, double* Chi, double* Clo,
                          int64_t ldc, const GramDdPlan& plan, hipStream_t stream);
// Upper Cholesky of the double-double C (n x n, ld n): R in double-double
// (Rhi, Rlo) and R^{-1} rounded to double (Minv); *info = j on breakdown.
hipError_t launch_chol_dd(const double* Chi, const double* Clo, int n, double* Rhi, double* Rlo, double* Minv,
                          int* info, hipStream_t stream);
// out = R2 (R1hi + R1lo) (double-double products, rounded), ld ldo.
hipError_t launch_trmm_dd(const double* R2, const double* R1h, const double* R1l, int n, double* out, int64_t ldo,
                          const int* info, hipStream_t stream);

// Small n x n device steps (small.hip); every kernel runs as one workgroup.
// Upper Cholesky C = R^T R with R^{-1}; sets *info = info_base + j on a
// non-positive pivot in column j (1-based) unless *info is already non-zero.
hipError_t launch_chol_inv(const double* C, int n, double* R, double* Rinv, int* info, int info_base,
                           hipStream_t stream);
// out = R2 * R1 (upper triangular product), ld ldo; NaN everywhere if *info != 0.
hipError_t launch_trmm_out(const double* R2, const double* R1, int n, double* out, int64_t ldo, const int* info,
                           hipStream_t stream);
// Symmetric eigendecomposition (parallel cyclic Jacobi), eigenvalues decreasing.
//   first pass (first != 0): D = U L^{-1/2} (truncated), U1 and lam1 kept,
//   sigma (may be null) = sqrt(lam); second pass: Z = L2^{1/2} U2^T L1^{1/2} U1^T.
// *ntrunc accumulates the number of truncated eigenvalues (first pass resets it).
//   with Dq (second pass, D1 = the first pass's D): Dq = D1 U2 L2^{-1/2}, the
//   right factor of the explicit Q = X Dq.
hipError_t launch_svqb_eig(const double* C, int n, double trunc_tol, int first, double* U1, double* lam1,
                           double* D, double* sigma, double* Z, int64_t ldz, int* ntrunc, hipStream_t stream,
                           const double* D1 = nullptr, double* Dq = nullptr);
// Rinv = R^{-1} for upper-triangular R (ld ldr); *info (may be null) = 0, or
// the 1-based column of the first zero diagonal entry (Rinv is NaN then).
hipError_t launch_trinv(const double* R, int64_t ldr, int n, double* Rinv, int* info, hipStream_t stream);
// Q = X M (m x n, ld ldq) for an n x n M (ld n), streamed once over X; with
// m_upper, M is upper triangular and its zero blocks are not multiplied.
// A non-zero *fail (may be null) fills Q with NaN instead.
hipError_t launch_apply_right(const double* X, int64_t m, int64_t n, int64_t ldx, const double* M, bool m_upper,
                              double* Q, int64_t ldq, const int* fail, hipStream_t stream);
// x = RA^{-1} z and |rho| from Rt = R([A b]) ((n+1) x (n+1), ld ldr).
hipError_t launch_lstsq(const double* Rt, int n, int64_t ldr, double* x, double* resid, int* info,
                        hipStream_t stream);
// Copy of a device int (used to publish an internal info word).
hipError_t launch_copy_int(const int* src, int* dst, hipStream_t stream);

// Device descriptor of one matrix of a batched call (built by the host plan).
struct BatchMat {
    const double* X;
    double* R;
    int64_t m, ldx, ldr, tile_rows, slot_base;
    int n, np, accumulate, ntiles;
};

// One tree group of a batched call: fold the gsize stacked triangles at
// slots + src into one, written at slots + dst, or (dst < 0, the root) into
// the matrix's R.
struct BatchGroup {
    int64_t src, dst;
    int mat, gsize;
};

// Batched TSQR (batched.hip).
int batch_plan_create(const qless_matrix_desc* d, int32_t count, int64_t tile_bytes, int waves_per_cu,
                      qless_batch_plan** out);
int batch_plan_upload(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s);
int batch_run(const qless_batch_plan* p, void* work, size_t work_bytes, hipStream_t s);
size_t batch_plan_bytes(const qless_batch_plan* p);
int64_t batch_plan_tiles(const qless_batch_plan* p);
void batch_plan_destroy(qless_batch_plan* p);   // where the plan type is complete

// Benchmark timing hooks (api.hip).
void timing_begin(int which, hipStream_t stream);
void timing_end(int which, hipStream_t stream);
enum { kTimeTsqrStage1 = 0, kTimeGram = 1, kTimeSlots = 2 };

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Host-side checks shared by the entry points taking one m x n matrix X and
// an n x n result R (returns a qless_status).
inline int check_matrix_args(const void* X, int64_t m, int64_t n, int64_t ldx, const void* R, int64_t ldr) {
    if (n < 1 || m < 0) return QLESS_ERR_ARG;
    if (n > QLESS_MAX_N) return QLESS_ERR_UNSUPPORTED;
    if (R == nullptr || ldr < n) return QLESS_ERR_ARG;
    if (m > 0 && (X == nullptr || ldx < n)) return QLESS_ERR_ARG;
    return QLESS_OK;
}
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace qless
