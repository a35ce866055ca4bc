// Small n x n device steps of the Gram-based forms and the least-squares
// finish (paper Sec. 3.1, Alg. 1 steps 2, 4, 5; the SVQB2 eigendecomposition
// and truncation; Sec. 1 least squares).  The paper runs these on the host;
// here each is one workgroup on the device so that no step crosses to the
// host and a whole call can be captured in a stream or graph.  n <= 64, so
// every matrix fits in LDS.
#include "qless_internal.h"

namespace qless {
namespace {

constexpr int kLd = 65;  // LDS row stride of 64 x 64 work matrices (odd: fewer bank conflicts)

// Upper Cholesky factorisation C = R^T R (right-looking, one column per step)
// and the triangular inverse R^{-1} (column by column back substitution).
__global__ void __launch_bounds__(256)
chol_inv_kernel(const double* __restrict__ C, int n, double* __restrict__ R, double* __restrict__ Rinv,
                int* __restrict__ info, int info_base) {
    __shared__ double A[64 * kLd];
    __shared__ double T[64 * kLd];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) A[(e / n) * kLd + e % n] = C[e];
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        const double d = A[j * kLd + j];
        if (!(d > 0.0)) {            // uniform: every thread read the same pivot
            if (tid == 0) bad = j + 1;
            break;
        }
        const double rjj = sqrt(d);
        for (int c = j + 1 + tid; c < n; c += blockDim.x) A[j * kLd + c] = A[j * kLd + c] / rjj;
        __syncthreads();
        if (tid == 0) A[j * kLd + j] = rjj;
        const int t = n - j - 1;
        for (int idx = tid; idx < t * t; idx += blockDim.x) {
            const int a = j + 1 + idx / t, b = j + 1 + idx % t;
            if (b >= a) A[a * kLd + b] = fma(-A[j * kLd + a], A[j * kLd + b], A[a * kLd + b]);
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad) {
        if (tid == 0) {
            if (info_base == 0) *info = bad;
            else if (*info == 0) *info = info_base + bad;
        }
        for (int e = tid; e < n * n; e += blockDim.x) {
            R[e] = __builtin_nan("");
            Rinv[e] = __builtin_nan("");
        }
        return;
    }
    if (tid == 0 && info_base == 0) *info = 0;
    // T = R^{-1}: thread c owns column c.
    if (tid < n) {
        const int c = tid;
        T[c * kLd + c] = 1.0 / A[c * kLd + c];
        for (int r = c - 1; r >= 0; --r) {
            double s = 0.0;
            for (int k = r + 1; k <= c; ++k) s = fma(A[r * kLd + k], T[k * kLd + c], s);
            T[r * kLd + c] = -s / A[r * kLd + r];
        }
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int a = e / n, b = e % n;
        R[e] = (b >= a) ? A[a * kLd + b] : 0.0;
        Rinv[e] = (b >= a) ? T[a * kLd + b] : 0.0;
    }
}

// out = R2 R1 for upper-triangular R2, R1 (both positive diagonal).
__global__ void __launch_bounds__(256)
trmm_out_kernel(const double* __restrict__ R2, const double* __restrict__ R1, int n, double* __restrict__ out,
                int64_t ldo, const int* __restrict__ info) {
    const bool failed = (*info != 0);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        double s = 0.0;
        for (int k = i; k <= c; ++k) s = fma(R2[i * n + k], R1[k * n + c], s);
        out[(int64_t)i * ldo + c] = failed ? __builtin_nan("") : (c >= i ? s + 0.0 : 0.0);
    }
}

// Parallel cyclic Jacobi (round-robin pairing: n/2 disjoint rotations per
// round, n-1 rounds per sweep) on A = C in LDS, accumulating V.  The rotation
// and the skip threshold |a_pq| <= eps sqrt(|a_pp a_qq|) are those of the
// classical two-sided method (Golub & Van Loan Sec. 8.5).
__global__ void __launch_bounds__(256)
svqb_eig_kernel(const double* __restrict__ C, int n, double trunc_tol, int first, double* __restrict__ U1,
                double* __restrict__ lam1, double* __restrict__ D, double* __restrict__ sigma,
                double* __restrict__ Z, int64_t ldz, int* __restrict__ ntrunc, const double* __restrict__ D1,
                double* __restrict__ Dq) {
    __shared__ double A[64 * kLd];
    __shared__ double V[64 * kLd];
    __shared__ double cs_c[32], cs_s[32];
    __shared__ int pp[32], pq[32], prot[32];
    __shared__ int any_rot;
    __shared__ double lam[64];
    __shared__ int order[64];
    const int tid = threadIdx.x;
    const double eps = 1.1102230246251565e-16;  // 2^-53
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int a = e / n, b = e % n;
        A[a * kLd + b] = C[e];
        V[a * kLd + b] = (a == b) ? 1.0 : 0.0;
    }
    const int np = n + (n & 1);
    const int half = np / 2;
    __syncthreads();
    for (int sweep = 0; sweep < 40 && n > 1; ++sweep) {
        if (tid == 0) any_rot = 0;
        __syncthreads();
        for (int r = 0; r < np - 1; ++r) {
            if (tid < half) {
                const int k = tid;
                const int pa = (k == 0) ? 0 : 1 + (k - 1 + r) % (np - 1);
                const int pb = 1 + (np - 2 - k + r) % (np - 1);
                const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
                int rot = 0;
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[p * kLd + q], app = A[p * kLd + p], aqq = A[q * kLd + q];
                    if (fabs(apq) > eps * sqrt(fabs(app) * fabs(aqq))) {
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                                      : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                        rot = 1;
                    }
                }
                pp[k] = p;
                pq[k] = (q < n) ? q : -1;
                prot[k] = rot;
                cs_c[k] = c;
                cs_s[k] = s;
                if (rot) any_rot = 1;
            }
            __syncthreads();
            for (int idx = tid; idx < half * n; idx += blockDim.x) {   // columns p, q of A and V
                const int k = idx / n, i = idx % n;
                if (!prot[k]) continue;
                const int p = pp[k], q = pq[k];
                const double c = cs_c[k], s = cs_s[k];
                const double aip = A[i * kLd + p], aiq = A[i * kLd + q];
                A[i * kLd + p] = c * aip - s * aiq;
                A[i * kLd + q] = s * aip + c * aiq;
                const double vip = V[i * kLd + p], viq = V[i * kLd + q];
                V[i * kLd + p] = c * vip - s * viq;
                V[i * kLd + q] = s * vip + c * viq;
            }
            __syncthreads();
            for (int idx = tid; idx < half * n; idx += blockDim.x) {   // rows p, q of A
                const int k = idx / n, j = idx % n;
                if (!prot[k]) continue;
                const int p = pp[k], q = pq[k];
                const double c = cs_c[k], s = cs_s[k];
                const double apj = A[p * kLd + j], aqj = A[q * kLd + j];
                A[p * kLd + j] = c * apj - s * aqj;
                A[q * kLd + j] = s * apj + c * aqj;
            }
            __syncthreads();
            if (tid < half && pq[tid] >= 0) {
                A[pp[tid] * kLd + pq[tid]] = 0.0;
                A[pq[tid] * kLd + pp[tid]] = 0.0;
            }
            __syncthreads();
        }
        if (!any_rot) break;
        __syncthreads();
    }
    // eigenvalues, sorted decreasing (selection sort by one thread; n <= 64)
    if (tid == 0) {
        for (int i = 0; i < n; ++i) {
            lam[i] = A[i * kLd + i];
            order[i] = i;
        }
        for (int i = 0; i < n; ++i) {
            int best = i;
            for (int j = i + 1; j < n; ++j)
                if (lam[j] > lam[best]) best = j;
            if (best != i) {
                double tl = lam[i]; lam[i] = lam[best]; lam[best] = tl;
                int to = order[i]; order[i] = order[best]; order[best] = to;
            }
        }
        int cnt = 0;
        for (int i = 0; i < n; ++i)
            if (!(lam[i] > trunc_tol * lam[0] && lam[i] > 0.0)) ++cnt;
        if (first) *ntrunc = cnt;
        else *ntrunc += cnt;
    }
    __syncthreads();
    if (first) {
        for (int e = tid; e < n * n; e += blockDim.x) {
            const int k = e / n, t = e % n;
            const double u = V[k * kLd + order[t]];
            const bool keep = lam[t] > trunc_tol * lam[0] && lam[t] > 0.0;
            U1[e] = u;
            D[e] = keep ? u / sqrt(lam[t]) : 0.0;
        }
        if (tid < n) {
            lam1[tid] = lam[tid];
            if (sigma) sigma[tid] = lam[tid] > 0.0 ? sqrt(lam[tid]) : 0.0;
        }
        return;
    }
    // second pass: Z = L2^{1/2} U2^T (L1^{1/2} U1^T)
    for (int e = tid; e < n * n; e += blockDim.x) {   // T = L1^{1/2} U1^T into A (A is no longer needed)
        const int k = e / n, c = e % n;
        const double l1 = lam1[k];
        A[k * kLd + c] = (l1 > 0.0 ? sqrt(l1) : 0.0) * U1[c * n + k];
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        const int oi = order[i];
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(V[k * kLd + oi], A[k * kLd + c], s);
        const double l2 = lam[i];
        Z[(int64_t)i * ldz + c] = (l2 > 0.0 ? sqrt(l2) : 0.0) * s + 0.0;
    }
    if (Dq == nullptr) return;
    // Dq = D1 D2 with D2 = U2 L2^{-1/2} (truncated as in the first pass), so
    // that Q = X Dq is the explicit Q of X = Q Z
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int k = e / n, t = e % n;
        const bool keep = lam[t] > trunc_tol * lam[0] && lam[t] > 0.0;
        A[k * kLd + t] = keep ? V[k * kLd + order[t]] / sqrt(lam[t]) : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, c = e % n;
        double s = 0.0;
        for (int k = 0; k < n; ++k) s = fma(D1[i * n + k], A[k * kLd + c], s);
        Dq[e] = s;
    }
}

// Inverse of an upper-triangular R (ld ldr, any diagonal signs) into Rinv
// (n x n, ld n, zeros below the diagonal): thread c owns column c of Rinv
// and solves R t = e_c by back substitution.  A zero diagonal entry (R
// singular) sets *info to its column (1-based) and fills Rinv with NaN.
__global__ void __launch_bounds__(64)
trinv_kernel(const double* __restrict__ R, int64_t ldr, int n, double* __restrict__ Rinv, int* __restrict__ info) {
    __shared__ double A[64 * kLd];
    __shared__ int bad;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int a = e / n, b = e % n;
        A[a * kLd + b] = b >= a ? R[(int64_t)a * ldr + b] : 0.0;
    }
    if (tid == 0) {
        int j = 0;
        while (j < n && R[(int64_t)j * ldr + j] != 0.0) ++j;
        bad = j < n ? j + 1 : 0;
        if (info) *info = bad;
    }
    __syncthreads();
    if (bad) {
        for (int e = tid; e < n * n; e += blockDim.x) Rinv[e] = __builtin_nan("");
        return;
    }
    if (tid < n) {
        const int c = tid;
        double t[64];
        t[c] = 1.0 / A[c * kLd + c];
        for (int r = c - 1; r >= 0; --r) {
            double s = 0.0;
            for (int k = r + 1; k <= c; ++k) s = fma(A[r * kLd + k], t[k], s);
            t[r] = -s / A[r * kLd + r];
        }
        for (int r = 0; r < n; ++r) Rinv[r * n + c] = r <= c ? t[r] : 0.0;
    }
}

// Back substitution RA x = z from Rt = [[RA, z], [0, rho]] (one thread).
__global__ void lstsq_kernel(const double* __restrict__ Rt, int n, int64_t ldr, double* __restrict__ x,
                             double* __restrict__ resid, int* __restrict__ info) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int bad = 0;
    for (int i = n - 1; i >= 0; --i) {
        double e = Rt[(int64_t)i * ldr + n];
        for (int k = i + 1; k < n; ++k) e = fma(-Rt[(int64_t)i * ldr + k], x[k], e);
        const double d = Rt[(int64_t)i * ldr + i];
        if (d == 0.0 && !bad) bad = i + 1;
        x[i] = e / d;
    }
    if (resid) *resid = fabs(Rt[(int64_t)n * ldr + n]);
    if (info) *info = bad;
}

__global__ void copy_int_kernel(const int* __restrict__ src, int* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace

hipError_t launch_chol_inv(const double* C, int n, double* R, double* Rinv, int* info, int info_base,
                           hipStream_t s) {
    hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(256), 0, s, C, n, R, Rinv, info, info_base);
    return hipGetLastError();
}

hipError_t launch_trmm_out(const double* R2, const double* R1, int n, double* out, int64_t ldo, const int* info,
                           hipStream_t s) {
    hipLaunchKernelGGL(trmm_out_kernel, dim3(1), dim3(256), 0, s, R2, R1, n, out, ldo, info);
    return hipGetLastError();
}

hipError_t launch_svqb_eig(const double* C, int n, double trunc_tol, int first, double* U1, double* lam1,
                           double* D, double* sigma, double* Z, int64_t ldz, int* ntrunc, hipStream_t s,
                           const double* D1, double* Dq) {
    hipLaunchKernelGGL(svqb_eig_kernel, dim3(1), dim3(256), 0, s, C, n, trunc_tol, first, U1, lam1, D, sigma, Z,
                       ldz, ntrunc, D1, Dq);
    return hipGetLastError();
}

hipError_t launch_trinv(const double* R, int64_t ldr, int n, double* Rinv, int* info, hipStream_t s) {
    hipLaunchKernelGGL(trinv_kernel, dim3(1), dim3(64), 0, s, R, ldr, n, Rinv, info);
    return hipGetLastError();
}

hipError_t launch_lstsq(const double* Rt, int n, int64_t ldr, double* x, double* resid, int* info,
                        hipStream_t s) {
    hipLaunchKernelGGL(lstsq_kernel, dim3(1), dim3(64), 0, s, Rt, n, ldr, x, resid, info);
    return hipGetLastError();
}

hipError_t launch_copy_int(const int* src, int* dst, hipStream_t s) {
    hipLaunchKernelGGL(copy_int_kernel, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

}  // namespace qless
