// Gram matrix accumulated in twice the working precision, and the Cholesky-QR2
// variant built on it (the higher-precision Gramian that Sec. 2 cites as a way
// to lift Cholesky-QR's condition-number limit).
//
// C = X^T X with every entry a double-double (hi + lo): each product x_a x_b
// is split exactly into p + e (p = fl(x_a x_b), e = fma(x_a, x_b, -p)), p is
// added to the running hi with the error-free sum (s = hi + p, t = the exact
// rounding error of that sum) and t + e go to the running lo -- the Dot2
// scheme of Ogita, Rump and Oishi (2005), so each entry is about as accurate as
// if it were summed in 106-bit arithmetic and then rounded once.
//
// Layout: a workgroup of 256 threads stages a chunk of rows of X in LDS; thread
// t owns a T x T tile of C (T = n/16 rounded up for n > 16, else 1), so that
// the tiles cover the padded n x n matrix -- for n <= 16 the 256 threads form
// 256 / n^2 groups, each over every so many staged rows, whose tiles are
// added at the end; per staged row a thread reads its 2T operands from LDS
// and updates T^2 double-double accumulators.  Every
// workgroup writes its partial (hi, lo) to the workspace and a fixed-order
// double-double sum follows: no atomics, bitwise reproducible.
//
// cholqr2_dd_r: R1 from the double-double Cholesky of that Gram matrix (one
// workgroup), M = R1^{-1} rounded to double; then the plain second pass of
// Cholesky-QR2 on X M (the matrix-core Gram kernel with the fused triangular
// multiply) and R = R2 R1 with R1 still in double-double.  Because R1 is
// accurate to about u^2 kappa^2, X M has a condition number of about
// 1 + u kappa and the second pass recovers an R accurate to working
// precision for kappa(X) up to about u^{-1} (Yamazaki et al. 2015), where the
// plain Cholesky-QR2 breaks down at about u^{-1/2}.
#include "qless_internal.h"

namespace qless {
namespace {

#pragma clang fp contract(off)

// Error-free transformations (rounding to nearest; no contraction here).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
    s = a + b;
    const double t = s - a;
    e = (a - (s - t)) + (b - t);
}

__device__ __forceinline__ void quick_two_sum(double a, double b, double& s, double& e) {   // |a| >= |b|
    s = a + b;
    e = b - (s - a);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
    p = a * b;
    e = fma(a, b, -p);
}

// (hi, lo) += a * b, Dot2 style: the product's and the sum's rounding errors
// collect in lo.
__device__ __forceinline__ void dot2_acc(double& hi, double& lo, double a, double b) {
    double p, e, s, t;
    two_prod(a, b, p, e);
    two_sum(hi, p, s, t);
    hi = s;
    lo = lo + (t + e);
}

// Double-double arithmetic on (hi, lo) pairs with |lo| <= ulp(hi) / 2 after
// normalisation (the classical algorithms of Dekker, Knuth and Bailey's QD).
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd dd_norm(double hi, double lo) {
    dd r;
    two_sum(hi, lo, r.hi, r.lo);   // exact for any magnitudes (lo may exceed hi after cancellation)
    return r;
}

__device__ __forceinline__ dd dd_add(dd a, dd b) {
    double s, e, t, f;
    two_sum(a.hi, b.hi, s, e);
    two_sum(a.lo, b.lo, t, f);
    e = e + t;
    quick_two_sum(s, e, s, e);
    e = e + f;
    return dd_norm(s, e);
}

__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }

__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    double p, e;
    two_prod(a.hi, b.hi, p, e);
    e = e + (a.hi * b.lo + a.lo * b.hi);
    return dd_norm(p, e);
}

__device__ __forceinline__ dd dd_div(dd a, dd b) {
    const double q1 = a.hi / b.hi;
    dd r = dd_add(a, dd_neg(dd_mul(b, dd{q1, 0.0})));
    const double q2 = r.hi / b.hi;
    r = dd_add(r, dd_neg(dd_mul(b, dd{q2, 0.0})));
    const double q3 = r.hi / b.hi;
    return dd_add(dd_norm(q1, q2), dd{q3, 0.0});
}

__device__ __forceinline__ dd dd_sqrt(dd a) {   // a.hi > 0
    const double x = 1.0 / sqrt(a.hi);
    const double ax = a.hi * x;
    double p, e;
    two_prod(ax, ax, p, e);
    const dd diff = dd_add(a, dd_neg(dd_norm(p, e)));
    return dd_add(dd{ax, 0.0}, dd{diff.hi * (x * 0.5), 0.0});
}

// ------------------------------------------------------------ Gram kernel

constexpr int kDdThreads = 256;
constexpr int kDdStage = 2048;   // doubles of X staged per chunk (16 KB)

template <int NP>
constexpr int dd_tile() {
    return NP > 16 ? (NP + 15) / 16 : 1;
}

template <int NP>
constexpr int dd_grid() {   // tiles per dimension
    return NP > 16 ? 16 : NP;
}

template <int NP>
constexpr int dd_groups() {   // thread groups sharing the staged rows (n <= 16: 256 / tiles)
    return kDdThreads / (dd_grid<NP>() * dd_grid<NP>());
}

template <int NP>
__global__ void __launch_bounds__(kDdThreads)
gram_dd_kernel(const double* __restrict__ X, int64_t m, int n, int64_t ldx, int64_t rows_per_block,
               double* __restrict__ part) {
    constexpr int T = dd_tile<NP>();
    constexpr int G = dd_grid<NP>();
    constexpr int NG = dd_groups<NP>();              // thread groups, each over every NG-th staged row
    constexpr int LD = NP + 1;                       // odd row stride: operand reads spread over banks
    constexpr int CH = kDdStage / LD;                // rows per staged chunk
    static_assert(NG * G * G == kDdThreads && NG * 2 * T * T <= kDdStage, "thread layout of the dd Gram kernel");
    __shared__ double xs[CH * LD];
    const int tid = threadIdx.x;
    const int tile = tid % (G * G), grp = tid / (G * G);
    const int I = tile / G, J = tile % G;
    const bool active = I <= J;                      // upper tiles only (C is symmetric)
    double hi[T][T], lo[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) hi[a][b] = lo[a][b] = 0.0;
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r_end = r_begin + rows_per_block < m ? r_begin + rows_per_block : m;
    for (int64_t base = r_begin; base < r_end; base += CH) {
        const int rows = (int)(r_end - base < CH ? r_end - base : CH);
        __syncthreads();
        for (int e = tid; e < CH * NP; e += kDdThreads) {
            const int r = e / NP, c = e - r * NP;
            xs[r * LD + c] = (r < rows && c < n) ? X[(base + r) * ldx + c] : 0.0;
        }
        __syncthreads();
        if (active) {
            for (int r = grp; r < rows; r += NG) {
                double u[T], v[T];
#pragma unroll
                for (int a = 0; a < T; ++a) {
                    u[a] = xs[r * LD + I * T + a];
                    v[a] = xs[r * LD + J * T + a];
                }
#pragma unroll
                for (int a = 0; a < T; ++a)
#pragma unroll
                    for (int b = 0; b < T; ++b) dot2_acc(hi[a][b], lo[a][b], u[a], v[b]);
            }
        }
    }
    // the groups' accumulators of a tile, added in group order (double-double)
    dd acc[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) acc[a][b] = dd_norm(hi[a][b], lo[a][b]);
    if constexpr (NG > 1) {
        __syncthreads();
        xs[2 * tid] = acc[0][0].hi;
        xs[2 * tid + 1] = acc[0][0].lo;
        __syncthreads();
        if (grp != 0) return;
        for (int g = 1; g < NG; ++g) {
            const int o = 2 * (g * G * G + tile);
            acc[0][0] = dd_add(acc[0][0], dd{xs[o], xs[o + 1]});
        }
    }
    if (!active) return;
    // partial (hi, lo) of this block: 2 n x n matrices, both triangles
    double* ph = part + (int64_t)blockIdx.x * 2 * n * n;
    double* pl = ph + (int64_t)n * n;
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) {
            const int i = I * T + a, j = J * T + b;
            if (i < n && j < n) {
                ph[(int64_t)i * n + j] = acc[a][b].hi;
                pl[(int64_t)i * n + j] = acc[a][b].lo;
                ph[(int64_t)j * n + i] = acc[a][b].hi;
                pl[(int64_t)j * n + i] = acc[a][b].lo;
            }
        }
}

// C (hi, lo) = sum of the k partials in block order, in double-double.
__global__ void __launch_bounds__(256)
gram_dd_sum_kernel(const double* __restrict__ part, int64_t k, int n, double* __restrict__ Chi,
                   double* __restrict__ Clo, int64_t ldc) {
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.x * blockDim.x) {
        dd s{0.0, 0.0};
        for (int64_t w = 0; w < k; ++w) s = dd_add(s, dd{part[w * 2 * nn + e], part[w * 2 * nn + nn + e]});
        const int64_t i = e / n, j = e - i * n;
        Chi[i * ldc + j] = s.hi;
        if (Clo) Clo[i * ldc + j] = s.lo;
    }
}

// ------------------------------------------------------- n x n dd steps

constexpr int kLd = 65;

// Upper Cholesky of the double-double C = R^T R, R^{-1} rounded to double
// into Minv, and R (dd) into Rhi / Rlo (n x n, ld n, zeros below the
// diagonal).  *info = j on a non-positive pivot in column j (R and Minv NaN).
__global__ void __launch_bounds__(256)
chol_dd_kernel(const double* __restrict__ Chi, const double* __restrict__ Clo, int n, double* __restrict__ Rhi,
               double* __restrict__ Rlo, double* __restrict__ Minv, int* __restrict__ info) {
    __shared__ double Ah[64 * kLd], Al[64 * kLd];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) {
        Ah[(e / n) * kLd + e % n] = Chi[e];
        Al[(e / n) * kLd + e % n] = Clo[e];
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const dd d{Ah[j * kLd + j], Al[j * kLd + j]};
        if (!(d.hi > 0.0)) {
            if (tid == 0) bad = j + 1;
            break;
        }
        const dd rjj = dd_sqrt(d);
        __syncthreads();
        for (int c = j + 1 + tid; c < n; c += blockDim.x) {
            const dd v = dd_div(dd{Ah[j * kLd + c], Al[j * kLd + c]}, rjj);
            Ah[j * kLd + c] = v.hi;
            Al[j * kLd + c] = v.lo;
        }
        __syncthreads();
        if (tid == 0) {
            Ah[j * kLd + j] = rjj.hi;
            Al[j * kLd + j] = rjj.lo;
        }
        const int t = n - j - 1;
        for (int idx = tid; idx < t * t; idx += blockDim.x) {
            const int a = j + 1 + idx / t, b = j + 1 + idx % t;
            if (b >= a) {
                const dd v = dd_add(dd{Ah[a * kLd + b], Al[a * kLd + b]},
                                    dd_neg(dd_mul(dd{Ah[j * kLd + a], Al[j * kLd + a]}, dd{Ah[j * kLd + b], Al[j * kLd + b]})));
                Ah[a * kLd + b] = v.hi;
                Al[a * kLd + b] = v.lo;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) *info = bad;
        for (int e = tid; e < n * n; e += blockDim.x) Rhi[e] = Rlo[e] = Minv[e] = __builtin_nan("");
        return;
    }
    if (tid == 0) *info = 0;
    // R^{-1} column by column (thread c), in double-double, then rounded
    if (tid < n) {
        const int c = tid;
        dd t[64];
        t[c] = dd_div(dd{1.0, 0.0}, dd{Ah[c * kLd + c], Al[c * kLd + c]});
        for (int r = c - 1; r >= 0; --r) {
            dd s{0.0, 0.0};
            for (int k = r + 1; k <= c; ++k) s = dd_add(s, dd_mul(dd{Ah[r * kLd + k], Al[r * kLd + k]}, t[k]));
            t[r] = dd_neg(dd_div(s, dd{Ah[r * kLd + r], Al[r * kLd + r]}));
        }
        for (int r = 0; r < n; ++r) Minv[r * n + c] = r <= c ? t[r].hi : 0.0;
    }
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int a = e / n, b = e % n;
        Rhi[e] = b >= a ? Ah[a * kLd + b] : 0.0;
        Rlo[e] = b >= a ? Al[a * kLd + b] : 0.0;
    }
}

// out = R2 (R1hi + R1lo) in double-double, rounded; NaN if *info != 0.
__global__ void __launch_bounds__(256)
trmm_dd_kernel(const double* __restrict__ R2, const double* __restrict__ R1h, const double* __restrict__ R1l, int n,
               double* __restrict__ out, int64_t ldo, const int* __restrict__ info) {
    const bool failed = *info != 0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        dd s{0.0, 0.0};
        for (int k = i; k <= c; ++k) s = dd_add(s, dd_mul(dd{R2[i * n + k], 0.0}, dd{R1h[k * n + c], R1l[k * n + c]}));
        out[(int64_t)i * ldo + c] = failed ? __builtin_nan("") : (c >= i ? s.hi + 0.0 : 0.0);
    }
}

#pragma clang fp contract(on)

int gram_dd_npad(int64_t n) {
    if (n <= 8) {
        int np = 1;
        while (np < n) np <<= 1;
        return np;
    }
    return (int)ceil_div(n, 16) * 16;
}

}  // namespace

GramDdPlan make_gram_dd_plan(int64_t m, int64_t n, int num_cus) {
    GramDdPlan p;
    p.npad = gram_dd_npad(n);
    const int64_t blocks = (int64_t)(num_cus > 0 ? num_cus : 1) * 2;
    const int64_t ch = kDdStage / (p.npad + 1);
    int64_t rpb = ceil_div(m > 0 ? m : 1, blocks);
    rpb = ceil_div(rpb, ch) * ch;
    p.rows_per_block = rpb;
    p.k = m > 0 ? ceil_div(m, rpb) : 1;
    p.part_bytes = align_up((size_t)p.k * 2 * (size_t)(n * n) * sizeof(double), 256);
    return p;
}

hipError_t launch_gram_dd(const double* X, int64_t m, int64_t n, int64_t ldx, double* part, double* Chi, double* Clo,
                          int64_t ldc, const GramDdPlan& p, hipStream_t s) {
    const int ni = (int)n;
    switch (p.npad) {
#define QLESS_GDD(NP)                                                                                              \
    case NP:                                                                                                       \
        hipLaunchKernelGGL(gram_dd_kernel<NP>, dim3((unsigned)p.k), dim3(kDdThreads), 0, s, X, m, ni, ldx,         \
                           p.rows_per_block, part);                                                                \
        break;
        QLESS_GDD(1) QLESS_GDD(2) QLESS_GDD(4) QLESS_GDD(8) QLESS_GDD(16) QLESS_GDD(32) QLESS_GDD(48) QLESS_GDD(64)
#undef QLESS_GDD
        default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (m <= 0) {   // no partial was written: C = 0
        hipLaunchKernelGGL(gram_dd_sum_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)0, ni, Chi, Clo, ldc);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(gram_dd_sum_kernel, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s, part, p.k, ni, Chi,
                       Clo, ldc);
    return hipGetLastError();
}

hipError_t launch_chol_dd(const double* Chi, const double* Clo, int n, double* Rhi, double* Rlo, double* Minv,
                          int* info, hipStream_t s) {
    hipLaunchKernelGGL(chol_dd_kernel, dim3(1), dim3(256), 0, s, Chi, Clo, n, Rhi, Rlo, Minv, info);
    return hipGetLastError();
}

hipError_t launch_trmm_dd(const double* R2, const double* R1h, const double* R1l, int n, double* out, int64_t ldo,
                          const int* info, hipStream_t s) {
    hipLaunchKernelGGL(trmm_dd_kernel, dim3(1), dim3(256), 0, s, R2, R1h, R1l, n, out, ldo, info);
    return hipGetLastError();
}

}  // namespace qless
