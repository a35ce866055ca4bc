/*
 * CPU oracle for Q-less QR of tall, very skinny FP64 matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously
 * correct reference that the GPU path is checked against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never links, includes or calls it, and it shares no
 * code, header or table with the HIP sources.
 *
 * Paper: J. Thies, M. Roehrig-Zoellner, "Implementation of QR factorization
 * of tall and very skinny matrices on current GPUs" (arXiv 2603.20889).
 *
 * Contents (each function names the passage it follows):
 *   oracle_householder_r  R of X by unblocked Householder QR       (Sec. 1 problem statement; Alg. 4 per-column reflector)
 *   oracle_householder_r_chunked  the same, every length-m sum cut into fixed
 *                         64K-row chunks; OpenMP over chunks, bitwise the same
 *                         result for any thread count (for timing on host cores)
 *   oracle_cholqr2_r      Q-less Cholesky-QR2                      (Sec. 3.1, Alg. 1)
 *   oracle_shifted_cholqr3_r  Q-less shifted Cholesky-QR3          (Sec. 2 related work; shift of Fukaya et al. 2020)
 *   oracle_svqb2          Q-less SVQB applied twice, QZ form         (Sec. 1 SVQB/QZ definition; Sec. 3.1 SVQB2 paragraph)
 *   oracle_jacobi_eig     symmetric eigendecomposition (cyclic Jacobi, Golub & Van Loan Sec. 8.5) used by SVQB2
 *   oracle_lstsq_from_r   least squares from the Q-less R of [A b]   (Sec. 1, single-pass least squares)
 *   oracle_q_from_r       explicit Q = X R^{-1} rebuilt from the Q-less R (Sec. 1)
 *   oracle_two_phase_r    R of (I - Y Y^T) X and B = Y^T X         (Sec. 2, the two-phase problem)
 *   oracle_gram_dot2      X^T X accumulated in twice-working precision (Ogita-Rump-Oishi Dot2), for the error metric
 *
 * Conventions
 *   X is row-major, m x n, leading dimension ldx >= n.  R is n x n
 *   row-major with explicit zeros below the diagonal.
 *   R of an m x n X with m < n is defined as the R of X padded with zero
 *   rows to n rows (zero rows never change R).
 *   Rows of R are sign-normalised so that diag(R) >= 0, and -0.0 becomes
 *   +0.0 (the factorisation defines R only up to row signs).
 *   Every length-m sum is a pairwise (recursive halving) sum; build with
 *   -ffp-contract=off and no fast-math so that each product and each sum
 *   is one IEEE-rounded operation.
 *
 * Status codes: 0 ok, -1 bad argument, -2 out of memory, j > 0 numerical
 * breakdown (see each function).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PAIRWISE_BASE 8

/* ---------------------------------------------------------------- sums */

/* Pairwise sum of a[i*sa] * b[i*sb] for i < len.  Products are rounded,
 * then summed by recursive halving; below PAIRWISE_BASE terms a plain
 * left-to-right loop. */
static double pdot(const double *a, int64_t sa, const double *b, int64_t sb, int64_t len)
{
    if (len <= PAIRWISE_BASE) {
        double s = 0.0;
        for (int64_t i = 0; i < len; ++i) {
            double p = a[i * sa] * b[i * sb];
            s = s + p;
        }
        return s;
    }
    int64_t h = len / 2;
    double lo = pdot(a, sa, b, sb, h);
    double hi = pdot(a + h * sa, sa, b + h * sb, sb, len - h);
    return lo + hi;
}

/* ------------------------------------------------- Householder QR (O1) */

/* Sign normalisation: flip row i of the n x n upper-triangular R when
 * R_ii < 0, then add +0.0 to every entry so that no -0.0 remains. */
static void sign_normalise(double *R, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        if (R[i * n + i] < 0.0)
            for (int64_t c = 0; c < n; ++c) R[i * n + c] = -R[i * n + c];
        for (int64_t c = 0; c < n; ++c) R[i * n + c] = R[i * n + c] + 0.0;
    }
}

/* Householder QR of the column-major M x n matrix A (leading dim M, M >= n),
 * in place.  For column j the reflector H = I - tau v v^T with v_j = 1 maps
 * A(j:M, j) to (beta, 0, ..., 0); this is the textbook unblocked algorithm
 * (Golub & Van Loan Alg. 5.2.1) with LAPACK dlarfg's choice of sign:
 *   alpha = A_jj, s = sum_{i>j} A_ij^2,
 *   s == 0  ->  tau = 0, H = I (beta = alpha),
 *   else beta = -sign(alpha) sqrt(alpha^2 + s), v_i = A_ij / (alpha - beta),
 *        tau = (beta - alpha) / beta,
 * and H is applied to every later column c: w = A_jc + sum_{i>j} v_i A_ic,
 * A_ic -= tau w v_i.  This is the per-column step of the paper's trapezoidal
 * kernel (Alg. 4) without the column pairing, which only reorders work. */
static void householder_colmajor(double *A, int64_t M, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        double *a = A + j * M;           /* column j */
        double alpha = a[j];
        int64_t below = M - j - 1;
        double s = pdot(a + j + 1, 1, a + j + 1, 1, below);
        if (s == 0.0)
            continue;                    /* tau = 0: identity reflector */
        double norm = sqrt(alpha * alpha + s);
        double beta = (alpha >= 0.0) ? -norm : norm;   /* sign(+0) = + */
        double scale = 1.0 / (alpha - beta);
        for (int64_t i = j + 1; i < M; ++i) a[i] = a[i] * scale;   /* v_i */
        double tau = (beta - alpha) / beta;
        a[j] = beta;
        for (int64_t c = j + 1; c < n; ++c) {
            double *ac = A + c * M;
            double w = ac[j] + pdot(a + j + 1, 1, ac + j + 1, 1, below);
            double tw = tau * w;
            ac[j] = ac[j] - tw;
            for (int64_t i = j + 1; i < M; ++i) ac[i] = ac[i] - tw * a[i];
        }
    }
}

/* R of X (row-major m x n, ldx >= n) by O1; R is n x n row-major.
 * Returns 0, -1 on bad arguments, -2 if the working copy cannot be allocated. */
int oracle_householder_r(const double *X, int64_t m, int64_t n, int64_t ldx, double *R)
{
    if (n < 1 || m < 0 || (m > 0 && (X == NULL || ldx < n)) || R == NULL)
        return -1;
    int64_t M = m > n ? m : n;           /* zero-pad to at least n rows */
    double *A = (double *)calloc((size_t)(M * n), sizeof(double));
    if (!A) return -2;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) A[j * M + i] = X[i * ldx + j];
    householder_colmajor(A, M, n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < n; ++c) R[i * n + c] = (c >= i) ? A[c * M + i] : 0.0;
    free(A);
    sign_normalise(R, n);
    return 0;
}

/* ------------------------------------- chunked Householder QR (O7) */

/* The same factorisation as oracle_householder_r, with every length-M sum
 * taken in fixed chunks of CHUNK_ROWS terms: each chunk is summed pairwise
 * (pdot), then the chunk totals are summed pairwise.  The chunk boundaries
 * depend only on the length, never on the thread count, so OpenMP over the
 * chunks (and over rows for the element-wise updates) gives bitwise the same
 * R for any number of threads.  Exists so that the oracle can be timed on
 * all host cores; the arithmetic per column is that of householder_colmajor. */
#define CHUNK_ROWS 65536

static double pairwise_array(const double *p, int64_t len)
{
    if (len <= 0) return 0.0;
    if (len == 1) return p[0];
    int64_t h = len / 2;
    return pairwise_array(p, h) + pairwise_array(p + h, len - h);
}

/* sum_{i < len} a[i] b[i], chunked; part has room for ceil(len/CHUNK_ROWS). */
static double chunked_dot(const double *a, const double *b, int64_t len, double *part)
{
    int64_t nc = (len + CHUNK_ROWS - 1) / CHUNK_ROWS;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t lo = c * CHUNK_ROWS;
        int64_t cl = (len - lo < CHUNK_ROWS) ? len - lo : CHUNK_ROWS;
        part[c] = pdot(a + lo, 1, b + lo, 1, cl);
    }
    return pairwise_array(part, nc);
}

int oracle_householder_r_chunked(const double *X, int64_t m, int64_t n, int64_t ldx, double *R, int nthreads)
{
    if (n < 1 || m < 0 || (m > 0 && (X == NULL || ldx < n)) || R == NULL || nthreads < 1)
        return -1;
    int64_t M = m > n ? m : n;
    double *A = (double *)calloc((size_t)(M * n), sizeof(double));
    double *part = (double *)malloc((size_t)((M + CHUNK_ROWS - 1) / CHUNK_ROWS + 1) * sizeof(double));
    if (!A || !part) { free(A); free(part); return -2; }
    int saved = omp_get_max_threads();
    omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j) A[j * M + i] = X[i * ldx + j];
    for (int64_t j = 0; j < n; ++j) {
        double *a = A + j * M;
        double alpha = a[j];
        int64_t below = M - j - 1;
        double s = chunked_dot(a + j + 1, a + j + 1, below, part);
        if (s == 0.0)
            continue;
        double norm = sqrt(alpha * alpha + s);
        double beta = (alpha >= 0.0) ? -norm : norm;
        double scale = 1.0 / (alpha - beta);
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < M; ++i) a[i] = a[i] * scale;
        double tau = (beta - alpha) / beta;
        a[j] = beta;
        for (int64_t c = j + 1; c < n; ++c) {
            double *ac = A + c * M;
            double w = ac[j] + chunked_dot(a + j + 1, ac + j + 1, below, part);
            double tw = tau * w;
            ac[j] = ac[j] - tw;
#pragma omp parallel for schedule(static)
            for (int64_t i = j + 1; i < M; ++i) ac[i] = ac[i] - tw * a[i];
        }
    }
    omp_set_num_threads(saved);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < n; ++c) R[i * n + c] = (c >= i) ? A[c * M + i] : 0.0;
    free(A);
    free(part);
    sign_normalise(R, n);
    return 0;
}

/* ------------------------------------------------------------ CholQR2 */

/* C = X^T X (n x n, row-major, symmetric), each entry a pairwise sum over
 * the m rows.  Paper Alg. 1 step 1 (tsmttsm). */
static void gram(const double *X, int64_t m, int64_t n, int64_t ldx, double *C)
{
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = a; b < n; ++b) {
            double s = (m > 0) ? pdot(X + a, ldx, X + b, ldx, m) : 0.0;
            C[a * n + b] = s;
            C[b * n + a] = s;
        }
}

/* Upper Cholesky factor U (U^T U = C, positive diagonal), row-major n x n.
 * Returns 0, or j+1 if the pivot of column j is not positive (U is then
 * incomplete).  Textbook column-by-column Cholesky. */
static int cholesky_upper(const double *C, int64_t n, double *U)
{
    memset(U, 0, (size_t)(n * n) * sizeof(double));
    for (int64_t j = 0; j < n; ++j) {
        double d = C[j * n + j];
        for (int64_t k = 0; k < j; ++k) d = d - U[k * n + j] * U[k * n + j];
        if (!(d > 0.0)) return (int)(j + 1);
        double ujj = sqrt(d);
        U[j * n + j] = ujj;
        for (int64_t c = j + 1; c < n; ++c) {
            double e = C[j * n + c];
            for (int64_t k = 0; k < j; ++k) e = e - U[k * n + j] * U[k * n + c];
            U[j * n + c] = e / ujj;
        }
    }
    return 0;
}

/* Q-less Cholesky-QR2, paper Alg. 1:
 *   C = X^T X;  R1 = chol(C);  C = (X R1^{-1})^T (X R1^{-1});  R2 = chol(C);
 *   R = R2 R1.
 * X R1^{-1} is formed row by row by forward substitution (the paper's X/R1)
 * in a temporary copy.  Returns 0; j (1..n) if the first Cholesky breaks
 * down at column j, n + j for the second; -1 bad args, -2 no memory.  On
 * breakdown R is filled with NaN. */
int oracle_cholqr2_r(const double *X, int64_t m, int64_t n, int64_t ldx, double *R)
{
    if (n < 1 || m < 0 || (m > 0 && (X == NULL || ldx < n)) || R == NULL)
        return -1;
    double *C = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *R1 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *R2 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *Y = (double *)malloc((size_t)((m > 0 ? m : 1) * n) * sizeof(double));
    int rc = 0;
    if (!C || !R1 || !R2 || !Y) { rc = -2; goto done; }

    gram(X, m, n, ldx, C);
    rc = cholesky_upper(C, n, R1);
    if (rc != 0) goto breakdown;

    for (int64_t i = 0; i < m; ++i) {
        const double *x = X + i * ldx;
        double *y = Y + i * n;
        for (int64_t c = 0; c < n; ++c) {
            double e = x[c];
            for (int64_t k = 0; k < c; ++k) e = e - y[k] * R1[k * n + c];
            y[c] = e / R1[c * n + c];
        }
    }
    gram(Y, m, n, n, C);
    rc = cholesky_upper(C, n, R2);
    if (rc != 0) { rc += (int)n; goto breakdown; }

    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < n; ++c) {
            double s = 0.0;
            for (int64_t k = i; k <= c; ++k) s = s + R2[i * n + k] * R1[k * n + c];
            R[i * n + c] = (c >= i) ? s : 0.0;
        }
    goto done;
breakdown:
    for (int64_t i = 0; i < n * n; ++i) R[i] = NAN;
done:
    free(C); free(R1); free(R2); free(Y);
    return rc;
}

/* Q-less shifted Cholesky-QR3 -- the robust Gram variant for ill-conditioned
 * X that Sec. 2 names; the shift is the one of Fukaya, Kannan, Nakatsukasa,
 * Zhang and Yamamoto (SIAM J. Sci. Comput. 42, 2020):
 *   C = X^T X;  s = 11 (m n + n (n + 1)) u ||X||^2 with u = 2^-53 and
 *   ||X||^2 taken as ||X||_F^2 = trace C (an upper bound of ||X||_2^2, so the
 *   shift is never smaller than the published one);
 *   R1 = chol(C + s I);  Y = X R1^{-1} (forward substitution, row by row);
 *   R23 = Q-less CholQR2 of Y;  R = R23 R1.
 * Returns 0; j (1..n) if chol(C + s I) breaks down at column j, n + j or
 * 2n + j for the two CholQR2 passes; -1 bad args, -2 no memory.  On
 * breakdown R is filled with NaN. */
int oracle_shifted_cholqr3_r(const double *X, int64_t m, int64_t n, int64_t ldx, double *R)
{
    if (n < 1 || m < 0 || (m > 0 && (X == NULL || ldx < n)) || R == NULL)
        return -1;
    double *C = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *R1 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *R23 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *Y = (double *)malloc((size_t)((m > 0 ? m : 1) * n) * sizeof(double));
    int rc = 0;
    if (!C || !R1 || !R23 || !Y) { rc = -2; goto done; }

    gram(X, m, n, ldx, C);
    double tr = 0.0;
    for (int64_t j = 0; j < n; ++j) tr = tr + C[j * n + j];
    const double shift = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * 0x1p-53 * tr;
    for (int64_t j = 0; j < n; ++j) C[j * n + j] = C[j * n + j] + shift;
    rc = cholesky_upper(C, n, R1);
    if (rc != 0) goto breakdown;

    for (int64_t i = 0; i < m; ++i) {
        const double *x = X + i * ldx;
        double *y = Y + i * n;
        for (int64_t c = 0; c < n; ++c) {
            double e = x[c];
            for (int64_t k = 0; k < c; ++k) e = e - y[k] * R1[k * n + c];
            y[c] = e / R1[c * n + c];
        }
    }
    rc = oracle_cholqr2_r(Y, m, n, n, R23);
    if (rc < 0) goto done;
    if (rc > 0) { rc += (int)n; goto breakdown; }

    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t k = i; k <= c; ++k) acc = acc + R23[i * n + k] * R1[k * n + c];
            R[i * n + c] = (c >= i) ? acc : 0.0;
        }
    goto done;
breakdown:
    for (int64_t i = 0; i < n * n; ++i) R[i] = NAN;
done:
    free(C); free(R1); free(R23); free(Y);
    return rc;
}

/* ------------------------------------------------------- Jacobi eigen */

/* Symmetric eigendecomposition A = V diag(w) V^T of the n x n row-major
 * symmetric matrix A by the cyclic Jacobi method (Golub & Van Loan,
 * Alg. 8.5.2 "symmetric Schur" rotation inside Alg. 8.5.3 row-cyclic
 * sweeps).  V is row-major with eigenvectors as columns.  An off-diagonal
 * entry is treated as zero (and set to zero) when
 * |a_pq| <= eps * sqrt(|a_pp| |a_qq|), eps = 2^-53, the usual threshold of
 * one-sided/two-sided Jacobi; sweeps stop when a whole sweep rotates
 * nothing, or after 60 sweeps.  Eigenpairs are returned sorted by
 * decreasing eigenvalue.  Returns the number of sweeps, or -2 when out of
 * memory. */
int oracle_jacobi_eig(const double *A_in, int64_t n, double *w, double *V)
{
    double *A = (double *)malloc((size_t)(n * n) * sizeof(double));
    if (!A) return -2;
    memcpy(A, A_in, (size_t)(n * n) * sizeof(double));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;

    const double eps = ldexp(1.0, -53);
    int sweep = 0;
    for (; sweep < 60; ++sweep) {
        int64_t rotated = 0;
        for (int64_t p = 0; p < n - 1; ++p)
            for (int64_t q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                double app = A[p * n + p], aqq = A[q * n + q];
                if (fabs(apq) <= eps * sqrt(fabs(app) * fabs(aqq))) {
                    A[p * n + q] = 0.0;
                    A[q * n + p] = 0.0;
                    continue;
                }
                ++rotated;
                /* symmetric 2x2 Schur decomposition: c, s with
                 * [c s; -s c]^T [app apq; apq aqq] [c s; -s c] diagonal */
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                        : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = t * c;
                /* A <- J^T A J, J = I except J_pp = J_qq = c, J_pq = s, J_qp = -s */
                for (int64_t k = 0; k < n; ++k) {          /* columns p, q */
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) {          /* rows p, q */
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                A[p * n + q] = 0.0;                        /* zeroed by construction */
                A[q * n + p] = 0.0;
                for (int64_t k = 0; k < n; ++k) {          /* V <- V J */
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        if (rotated == 0) break;
    }
    for (int64_t i = 0; i < n; ++i) w[i] = A[i * n + i];
    /* selection sort, decreasing */
    for (int64_t i = 0; i < n; ++i) {
        int64_t best = i;
        for (int64_t j = i + 1; j < n; ++j) if (w[j] > w[best]) best = j;
        if (best != i) {
            double tw = w[i]; w[i] = w[best]; w[best] = tw;
            for (int64_t k = 0; k < n; ++k) {
                double tv = V[k * n + i]; V[k * n + i] = V[k * n + best]; V[k * n + best] = tv;
            }
        }
    }
    free(A);
    return sweep;
}

/* --------------------------------------------------------------- SVQB2 */

/* Q-less SVQB applied twice (paper Sec. 1 and the SVQB2 paragraph of
 * Sec. 3.1): C1 = X^T X = U1 L1 U1^T; D1 = U1 L1^{-1/2}, with the entries of
 * L1^{-1/2} set to 0 where lambda <= trunc_tol * lambda_max (truncation);
 * C2 = (X D1)^T (X D1) = U2 L2 U2^T; D2 likewise; then
 *   Q = X D1 D2 (never formed),  X = Q Z  with  Z = L2^{1/2} U2^T L1^{1/2} U1^T.
 * Outputs Z (n x n row-major), sigma (n, the square roots of the first-pass
 * eigenvalues, decreasing; may be NULL) and, if R is not NULL, R = qr_R(Z)
 * sign-normalised.  Returns the number of truncated eigenvalues over both
 * passes (>= 0), -1 bad args, -2 no memory. */
int oracle_svqb2(const double *X, int64_t m, int64_t n, int64_t ldx, double trunc_tol,
                 double *Z, double *sigma, double *R)
{
    if (n < 1 || m < 0 || (m > 0 && (X == NULL || ldx < n)) || Z == NULL)
        return -1;
    double *C = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *U1 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *U2 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *l1 = (double *)malloc((size_t)n * sizeof(double));
    double *l2 = (double *)malloc((size_t)n * sizeof(double));
    double *D1 = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *T = (double *)malloc((size_t)(n * n) * sizeof(double));
    double *Y = (double *)malloc((size_t)((m > 0 ? m : 1) * n) * sizeof(double));
    int ntrunc = 0, rc = 0;
    if (!C || !U1 || !U2 || !l1 || !l2 || !D1 || !T || !Y) { rc = -2; goto done; }

    gram(X, m, n, ldx, C);
    if (oracle_jacobi_eig(C, n, l1, U1) < 0) { rc = -2; goto done; }
    for (int64_t j = 0; j < n; ++j) {
        int keep = l1[j] > trunc_tol * l1[0] && l1[j] > 0.0;
        if (!keep) ++ntrunc;
        double d = keep ? 1.0 / sqrt(l1[j]) : 0.0;
        for (int64_t i = 0; i < n; ++i) D1[i * n + j] = U1[i * n + j] * d;
    }
    for (int64_t i = 0; i < m; ++i)                     /* Y = X D1 */
        for (int64_t c = 0; c < n; ++c) {
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k) s = s + X[i * ldx + k] * D1[k * n + c];
            Y[i * n + c] = s;
        }
    gram(Y, m, n, n, C);
    if (oracle_jacobi_eig(C, n, l2, U2) < 0) { rc = -2; goto done; }
    for (int64_t j = 0; j < n; ++j)
        if (!(l2[j] > trunc_tol * l2[0] && l2[j] > 0.0)) ++ntrunc;

    /* T = L1^{1/2} U1^T */
    for (int64_t i = 0; i < n; ++i) {
        double s1 = l1[i] > 0.0 ? sqrt(l1[i]) : 0.0;
        for (int64_t c = 0; c < n; ++c) T[i * n + c] = s1 * U1[c * n + i];
    }
    /* Z = L2^{1/2} U2^T T */
    for (int64_t i = 0; i < n; ++i) {
        double s2 = l2[i] > 0.0 ? sqrt(l2[i]) : 0.0;
        for (int64_t c = 0; c < n; ++c) {
            double s = 0.0;
            for (int64_t k = 0; k < n; ++k) s = s + U2[k * n + i] * T[k * n + c];
            Z[i * n + c] = s2 * s;
        }
    }
    if (sigma)
        for (int64_t j = 0; j < n; ++j) sigma[j] = l1[j] > 0.0 ? sqrt(l1[j]) : 0.0;
    if (R)
        rc = oracle_householder_r(Z, n, n, n, R);
    if (rc == 0) rc = ntrunc;
done:
    free(C); free(U1); free(U2); free(l1); free(l2); free(D1); free(T); free(Y);
    return rc;
}

/* --------------------------------------------------- explicit Q from R */

/* Q = X R^{-1}: Sec. 1 notes that for well-conditioned X the Q of the
 * Q-less factorisation can be rebuilt afterwards from X and R.  Row i of Q
 * solves q R = x_i by forward substitution (R upper triangular, row-major
 * n x n, ldr >= n; Q row-major m x n, ldq >= n).  Returns 0; j + 1 if
 * R_jj == 0 (Q is then not defined and left unwritten); -1 bad args. */
int oracle_q_from_r(const double *X, int64_t m, int64_t n, int64_t ldx, const double *R, int64_t ldr,
                    double *Q, int64_t ldq)
{
    if (n < 1 || m < 0 || R == NULL || ldr < n || (m > 0 && (X == NULL || Q == NULL || ldx < n || ldq < n)))
        return -1;
    for (int64_t j = 0; j < n; ++j)
        if (R[j * ldr + j] == 0.0) return (int)(j + 1);
    for (int64_t i = 0; i < m; ++i) {
        const double *x = X + i * ldx;
        double *q = Q + i * ldq;
        for (int64_t c = 0; c < n; ++c) {
            double e = x[c];
            for (int64_t k = 0; k < c; ++k) e = e - q[k] * R[k * ldr + c];
            q[c] = e / R[c * ldr + c];
        }
    }
    return 0;
}

/* ------------------------------------------- two-phase orthogonalisation */

/* The "two-phase" problem named in Sec. 2: orthogonalise X (m x n) against
 * an m x p Y with orthonormal columns and factor what is left,
 * Q R = (I - Y Y^T) X.  B = Y^T X (p x n, pairwise sums over the m rows),
 * Z = X - Y B row by row, R = R(Z) by oracle_householder_r.  B is row-major
 * p x n (may be NULL when p == 0).  Returns what oracle_householder_r
 * returns; -1 bad args, -2 no memory. */
int oracle_two_phase_r(const double *Y, int64_t p, int64_t ldy, const double *X, int64_t m, int64_t n,
                       int64_t ldx, double *B, double *R)
{
    if (n < 1 || m < 0 || p < 0 || R == NULL || (m > 0 && (X == NULL || ldx < n)) ||
        (p > 0 && (B == NULL || (m > 0 && (Y == NULL || ldy < p)))))
        return -1;
    double *Z = (double *)malloc((size_t)((m > 0 ? m : 1) * n) * sizeof(double));
    if (!Z) return -2;
    for (int64_t a = 0; a < p; ++a)
        for (int64_t c = 0; c < n; ++c)
            B[a * n + c] = (m > 0) ? pdot(Y + a, ldy, X + c, ldx, m) : 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c) {
            double z = X[i * ldx + c];
            for (int64_t a = 0; a < p; ++a) z = z - Y[i * ldy + a] * B[a * n + c];
            Z[i * n + c] = z;
        }
    int rc = oracle_householder_r(Z, m, n, n, R);
    free(Z);
    return rc;
}

/* ------------------------------------------------------ least squares */

/* Least squares from the Q-less R of [A b] (paper Sec. 1): with
 * Rt = R([A b]) = [[RA, z], [0, rho]] ((n+1) x (n+1) row-major, ldr >= n+1),
 * x solves RA x = z by back substitution and |rho| = ||A x - b||_2.
 * Returns 0, j+1 if RA_jj == 0 (x is then not defined), -1 bad args. */
int oracle_lstsq_from_r(const double *Rt, int64_t n, int64_t ldr, double *x, double *resid)
{
    if (n < 1 || ldr < n + 1 || Rt == NULL || x == NULL) return -1;
    for (int64_t i = n - 1; i >= 0; --i) {
        double e = Rt[i * ldr + n];
        for (int64_t k = i + 1; k < n; ++k) e = e - Rt[i * ldr + k] * x[k];
        double d = Rt[i * ldr + i];
        if (d == 0.0) return (int)(i + 1);
        x[i] = e / d;
    }
    if (resid) resid[0] = fabs(Rt[n * ldr + n]);
    return 0;
}

/* ------------------------------------------- extended-precision Gram */

/* Error-free transformations (Knuth TwoSum; TwoProduct via fma). */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

/* C = X^T X with every entry from Dot2 (Ogita, Rump & Oishi 2005,
 * Alg. 5.3): the result is as accurate as if computed in twice the working
 * precision and then rounded.  Used for the Gram-residual metric only. */
void oracle_gram_dot2(const double *X, int64_t m, int64_t n, int64_t ldx, double *C)
{
    for (int64_t a = 0; a < n; ++a)
        for (int64_t b = a; b < n; ++b) {
            double p = 0.0, s = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                double xa = X[i * ldx + a], xb = X[i * ldx + b];
                double h = xa * xb;
                double r = fma(xa, xb, -h);
                double q;
                two_sum(p, h, &p, &q);
                s = s + (q + r);
            }
            double v = p + s;
            C[a * n + b] = v;
            C[b * n + a] = v;
        }
}

/* Stacked R: R([R_1; ...; R_k]) where the k blocks are given row-major and
 * contiguous (k*n x n).  Convenience for the stacking-identity checks of
 * Alg. 2; it is exactly oracle_householder_r on the stacked matrix. */
int oracle_stacked_r(const double *Y, int64_t k, int64_t n, double *R)
{
    return oracle_householder_r(Y, k * n, n, n, R);
}
