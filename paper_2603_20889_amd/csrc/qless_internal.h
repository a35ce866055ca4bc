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
// the DPP control word `ctrl` (all rows and banks enabled).
template <int ctrl>
__device__ __forceinline__ double dpp_f64(double v) {
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
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

// ------------------------------------------------------------- host plans

struct DeviceInfo {
    int device = -1;
    int num_cus = 0;
    size_t lds_per_block = 0;
};

// Cached properties of the current device (thread-compatible, not thread-safe
// on first use per device).
const DeviceInfo& current_device_info();

// Plan of a TSQR call: stage-1 wave count, rows per wave, tree levels.
struct TsqrPlan {
    int npad = 0;              // padded column count of the kernel instance
    int rows_per_lane = 0;     // panel rows per lane (panel = 64 * rows_per_lane rows)
    int64_t rows_per_wave = 0; // stage-1 rows per wavefront
    int64_t k0 = 0;            // stage-1 wavefronts (= stacked R blocks)
    int fan_in = 0;            // blocks combined per tree wavefront
    int levels = 0;            // tree launches after stage 1 (0: stage 1 finalises)
    size_t ybytes_a = 0;       // bytes of the first ping-pong buffer
    size_t ybytes_b = 0;       // bytes of the second ping-pong buffer
    size_t work_bytes = 0;     // total workspace
};

TsqrPlan make_tsqr_plan(int64_t m, int64_t n, int num_cus);

// Enqueue a full TSQR (stage 1 + tree + sign normalisation) into `work`.
// Arguments have been validated by the caller.
hipError_t launch_tsqr(const double* X, int64_t m, int64_t n, int64_t ldx, double* R,
                       int64_t ldr, void* work, const TsqrPlan& plan, hipStream_t stream);

// Benchmark timing hooks (api.hip).
void timing_begin(int which, hipStream_t stream);
void timing_end(int which, hipStream_t stream);
enum { kTimeTsqrStage1 = 0, kTimeGram = 1, kTimeSlots = 2 };

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace qless
