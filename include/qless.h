/*
 * qless.h -- Q-less QR of tall, very skinny FP64 matrices on AMD MI355X (gfx950).
 *
 * Method: J. Thies, M. Roehrig-Zoellner, "Implementation of QR factorization
 * of tall and very skinny matrices on current GPUs", arXiv 2603.20889.
 *
 * Problem (Sec. 1): for a real dense X (m x n, m >> n) find R (n x n, upper
 * triangular) with X = QR and Q^T Q = I, returning only R ("Q-less": neither
 * Q nor the Householder reflectors are ever written).
 *
 * Conventions shared by every entry point
 *   - FP64 only.  X is ROW-MAJOR with leading dimension ldx >= n (element
 *     (i, j) at X[i * ldx + j]); 64-bit indexing throughout.
 *   - R (and Z) are n x n ROW-MAJOR with leading dimension ldr >= n.  Every
 *     entry is written: zeros below the diagonal, diag(R) >= 0 (R is unique
 *     only up to row signs; the sign of each row is fixed so its diagonal
 *     entry is non-negative, and -0.0 is written as +0.0).
 *   - m may be smaller than n (including m = 0): the result is then the R of
 *     X padded with zero rows to n rows.  1 <= n <= QLESS_MAX_N.
 *   - X, R, Z, sigma, info and work are DEVICE pointers owned by the caller.
 *     The library never allocates, frees or synchronises in these calls;
 *     every call only enqueues kernels on `stream` and returns.
 *   - work/work_bytes: caller-provided device scratch of at least
 *     qless_workspace_bytes(method, m, n) bytes, 256-byte aligned.  Two calls
 *     that are in flight at the same time must not share a workspace.
 *   - Errors found on the host (bad arguments, too-small workspace, launch
 *     failure) are returned synchronously as a negative qless_status before
 *     (or instead of) any launch.  Numerical conditions found on the device
 *     are reported through `info` (see each function).
 *   - Non-finite input propagates into the result; it is not checked.
 *   - Results are deterministic: the same inputs, sizes and device give
 *     bitwise-identical outputs (no atomics in any reduction).
 */
#ifndef QLESS_H
#define QLESS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QLESS_MAX_N 64

typedef enum {
    QLESS_OK = 0,
    QLESS_ERR_ARG = -1,          /* null pointer, n < 1, m < 0, ldx < n, ldr < n, ... */
    QLESS_ERR_UNSUPPORTED = -2,  /* n > QLESS_MAX_N */
    QLESS_ERR_WORKSPACE = -3,    /* work is NULL, misaligned or smaller than required */
    QLESS_ERR_HIP = -4           /* a HIP runtime call or kernel launch failed */
} qless_status;

typedef enum {
    QLESS_METHOD_TSQR = 0,       /* qless_tsqr_r */
    QLESS_METHOD_CHOLQR2 = 1,    /* cholqr2_r */
    QLESS_METHOD_SVQB = 2,       /* svqb */
    QLESS_METHOD_TSQR_UPDATE = 3, /* qless_tsqr_r_update */
    QLESS_METHOD_SHIFTED_CHOLQR3 = 4, /* shifted_cholqr3_r */
    QLESS_METHOD_Q_FROM_R = 5,    /* qless_q_from_r */
    QLESS_METHOD_GRAM = 6,        /* qless_gram */
    QLESS_METHOD_CHOLQR2_DD = 7   /* cholqr2_dd_r */
} qless_method;

typedef enum {
    QLESS_SVQB_R = 0,            /* write R = qr_R(Z) (sign-normalised) */
    QLESS_SVQB_QZ = 1            /* write Z of X = QZ */
} qless_svqb_out;

/* Human-readable name of a qless_status value. */
const char *qless_status_string(int status);

/* Library version string, e.g. "qless 0.1 gfx950". */
const char *qless_version(void);

/* Workspace size in bytes that `method` needs for an m x n problem on the
 * current device (the size depends on the device's compute-unit count).
 * Returns 0 for invalid arguments. */
size_t qless_workspace_bytes(int method, int64_t m, int64_t n);

/*
 * qless_tsqr_r -- Q-less Householder TSQR (Alg. 2 with the per-block
 * streaming kernel of Alg. 3 and the trapezoidal Householder step of Alg. 4).
 *
 * Stage 1: k row blocks, each factored by one wavefront that streams
 * coalesced row panels and keeps its running R_i on chip; stage 2: a tree of
 * stacked-R reductions R = R([R_1; ...; R_k]).  X is read exactly once; only
 * the k small R_i (in `work`) and the final R are written.
 *
 * Arguments: X (m x n, ldx), R (n x n, ldr) as above.  X and R must not
 * overlap.  Returns QLESS_OK or a negative qless_status.  Rank-deficient X
 * is not an error: R then has (near-)zero diagonal entries (Sec. 1).
 */
int qless_tsqr_r(const double *X, int64_t m, int64_t n, int64_t ldx,
                 double *R, int64_t ldr, void *work, size_t work_bytes,
                 hipStream_t stream);

/*
 * qless_tsqr_r_noalloc -- qless_tsqr_r for callers that cannot allocate
 * device memory or pass a workspace (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The same launches and
 * results as qless_tsqr_r; the stacked triangles live in a library-owned
 * device array of qless_noalloc_scratch_bytes() bytes (64 MiB: the largest
 * plan on a 256-CU device, n = 64), one copy per GPU the library runs on,
 * held until the process ends; its device address is looked up on the
 * first call made with a device current.  Allocates nothing; a plan larger
 * than the array returns QLESS_ERR_WORKSPACE.  Every call on one GPU shares
 * that GPU's array, so calls that overlap on one GPU (different streams or
 * host threads) race and must be ordered by the caller; nothing in the
 * array needs clearing between calls.  Other arguments and errors as for
 * qless_tsqr_r.
 */
size_t qless_noalloc_scratch_bytes(void);
int qless_tsqr_r_noalloc(const double *X, int64_t m, int64_t n, int64_t ldx,
                         double *R, int64_t ldr, hipStream_t stream);

/*
 * qless_tsqr_r_update -- running R over chunks of rows: R <- R([R; X]), the
 * Q-less R of the previous rows stacked on the new ones (Alg. 2 applied to
 * the stack, Sec. 1: the R of all rows seen so far).  R (n x n, ldr, upper
 * triangular, any signs; entries below the diagonal are ignored) is read and
 * overwritten with the new R, diagonal >= 0.  m may be 0 (then R only gets
 * its row signs fixed).  Same launches as qless_tsqr_r plus one n x n copy;
 * workspace from qless_workspace_bytes(QLESS_METHOD_TSQR_UPDATE, m, n).
 * Arguments and errors as for qless_tsqr_r; X and R must not overlap.
 */
int qless_tsqr_r_update(const double *X, int64_t m, int64_t n, int64_t ldx,
                        double *R, int64_t ldr, void *work, size_t work_bytes,
                        hipStream_t stream);

/*
 * cholqr2_r -- Q-less Cholesky-QR2 (Alg. 1): C = X^T X; R1 = chol(C);
 * C = (X R1^{-1})^T (X R1^{-1}); R2 = chol(C); R = R2 R1.  Two passes over X;
 * the n x n steps run on the device.  Suitable only for kappa(X) below about
 * eps^{-1/2} (Sec. 3.1).
 *
 * info (device int32, may be NULL): 0 on success; j (1..n) if the first
 * Cholesky meets a non-positive pivot in column j, n + j for the second
 * Cholesky.  On breakdown every entry of R is NaN.
 */
int cholqr2_r(const double *X, int64_t m, int64_t n, int64_t ldx,
              double *R, int64_t ldr, int32_t *info, void *work,
              size_t work_bytes, hipStream_t stream);

/*
 * qless_gram -- the Gram matrix C = X^T X (tsmttsm, Alg. 1 step 1) on its
 * own.  C_lo == NULL: FP64, as the first pass of cholqr2_r (matrix cores
 * for n > 8).  C_lo != NULL: accumulated in twice the working precision
 * (Dot2: error-free products and sums, the errors collected in a second
 * word), C = C_hi + C_lo with each entry about as accurate as a 106-bit sum
 * rounded once -- the higher-precision Gramian of the robust Gram variants
 * (Sec. 2).  C and C_lo: device, n x n, ldc >= n (both triangles written).
 * Workspace from qless_workspace_bytes(QLESS_METHOD_GRAM, m, n).
 */
int qless_gram(const double *X, int64_t m, int64_t n, int64_t ldx, double *C, int64_t ldc,
               double *C_lo, void *work, size_t work_bytes, hipStream_t stream);

/*
 * cholqr2_dd_r -- Cholesky-QR2 with its first Gram matrix accumulated and
 * factored in twice the working precision (the higher-precision Gramian
 * that Sec. 2 cites, after Yamazaki et al. 2015): C1 = X^T X in
 * double-double, R1 = chol(C1) and R1^{-1} in double-double, M = R1^{-1}
 * rounded; then the plain second pass C2 = (X M)^T (X M), R2 = chol(C2) and
 * R = R2 R1 (R1 in double-double).  Two passes over X like cholqr2_r, the
 * first one FP64-compute bound; completes with a backward-stable R for
 * kappa(X) up to about u^{-1}, where cholqr2_r breaks down at about
 * u^{-1/2}.  Arguments, errors and info as for cholqr2_r (workspace
 * QLESS_METHOD_CHOLQR2_DD).
 */
int cholqr2_dd_r(const double *X, int64_t m, int64_t n, int64_t ldx, double *R, int64_t ldr,
                 int32_t *info, void *work, size_t work_bytes, hipStream_t stream);

/*
 * shifted_cholqr3_r -- Q-less shifted Cholesky-QR3, the robust Gram variant
 * for ill-conditioned X that the related work (Sec. 2) names; the shift is
 * that of Fukaya et al. (SIAM J. Sci. Comput. 42, 2020):
 * C = X^T X; s = 11 (m n + n (n + 1)) u trace(C) with u = 2^-53 (trace C =
 * ||X||_F^2 bounds ||X||_2^2); R1 = chol(C + s I); then Cholesky-QR twice on
 * X R1^{-1}: R2 = chol((X R1^{-1})^T (X R1^{-1})), R3 = chol of the Gram
 * matrix of X R1^{-1} R2^{-1}; R = R3 R2 R1.  Three passes over X (the
 * triangular multiplies fused into the Gram passes); the n x n steps run on
 * the device.  Completes for kappa(X) up to about u^{-1} where CholQR2 breaks
 * down above about u^{-1/2}.
 *
 * Arguments, layout, workspace (QLESS_METHOD_SHIFTED_CHOLQR3) and errors as
 * for cholqr2_r.  info: 0; j (1..n) if the shifted Cholesky meets a
 * non-positive pivot in column j, n + j or 2n + j for the second or third.
 * On breakdown every entry of R is NaN.
 */
int shifted_cholqr3_r(const double *X, int64_t m, int64_t n, int64_t ldx,
                      double *R, int64_t ldr, int32_t *info, void *work,
                      size_t work_bytes, hipStream_t stream);

/*
 * svqb -- Q-less SVQB applied twice (Sec. 1 and Sec. 3.1, SVQB2):
 * C1 = X^T X = U1 L1 U1^T, D1 = U1 L1^{-1/2}; C2 = (X D1)^T (X D1) =
 * U2 L2 U2^T; X = Q Z with Q = X D1 D2 (never formed) and
 * Z = L2^{1/2} U2^T L1^{1/2} U1^T.  Entries of L^{-1/2} whose eigenvalue is
 * <= trunc_tol * lambda_max are replaced by 0 (truncation); trunc_tol <= 0
 * selects n * 2^-52.
 *
 * out = QLESS_SVQB_QZ writes Z (n x n, ldz); QLESS_SVQB_R writes
 * R = qr_R(Z) with diag >= 0 (then R equals the R of X up to rounding).
 * sigma (device, n doubles, may be NULL): square roots of the first-pass
 * eigenvalues, decreasing.  info (device int32, may be NULL): number of
 * truncated eigenvalues over both passes (informational, not an error).
 */
int svqb(const double *X, int64_t m, int64_t n, int64_t ldx, int out,
         double *Z_or_R, int64_t ldz, double *sigma, double trunc_tol,
         int32_t *info, void *work, size_t work_bytes, hipStream_t stream);

/*
 * svqb_q -- SVQB2 with the explicit Q (the variant that stores Q, compared
 * with the Q-less one in Sec. 4.6, Fig. 3): the two Gram passes of svqb,
 * then one more streaming pass Q = X D1 D2 with D2 = U2 L2^{-1/2}, so that
 * X = Q Z with Q^T Q = I up to rounding (for truncated eigenvalues the
 * corresponding columns of Q are zero).  Q: device, m x n row-major, ldq >= n,
 * must not overlap X.  Z, sigma, trunc_tol and info as for svqb with
 * out = QLESS_SVQB_QZ; workspace from qless_workspace_bytes(QLESS_METHOD_SVQB,
 * m, n).  Three passes over X, one over Q (8mn bytes written).
 */
int svqb_q(const double *X, int64_t m, int64_t n, int64_t ldx, double *Q, int64_t ldq,
           double *Z, int64_t ldz, double *sigma, double trunc_tol, int32_t *info,
           void *work, size_t work_bytes, hipStream_t stream);

/*
 * qless_q_from_r -- the explicit Q = X R^{-1} rebuilt from X and its Q-less R
 * (Sec. 1: Q is not stored, and can be recovered from X and R afterwards
 * when X is well conditioned).  R^{-1} is formed once on the device (one
 * workgroup), then X is streamed once: Q = X R^{-1} row by row (8mn bytes
 * read, 8mn written; the zero blocks of the triangular R^{-1} are skipped).
 *
 * R: device, n x n upper triangular (ldr >= n; entries below the diagonal
 * are ignored; any diagonal signs).  Q: device, m x n row-major, ldq >= n,
 * must not overlap X.  info (device int32, may be NULL): 0, or j (1..n) if
 * R_jj == 0 -- then every entry of Q is NaN.  Workspace from
 * qless_workspace_bytes(QLESS_METHOD_Q_FROM_R, m, n).  Orthonormality of Q
 * degrades with the condition number of X (about kappa^2 u for the R of a
 * Householder TSQR).
 */
int qless_q_from_r(const double *X, int64_t m, int64_t n, int64_t ldx, const double *R, int64_t ldr,
                   double *Q, int64_t ldq, int32_t *info, void *work, size_t work_bytes,
                   hipStream_t stream);

/*
 * qless_two_phase_r -- the two-phase problem of Sec. 2 in one streaming pass:
 * for Y (m x p, orthonormal columns) and X (m x n), B = Y^T X and the Q-less
 * R of the projected block, Q R = (I - Y Y^T) X.  One Q-less TSQR of the
 * concatenation [Y X] (read from the two pointers; never formed) gives
 * R([Y X]) = [[I, B], [0, R]] up to rounding, because Y's own R is the
 * identity; Y and X are each read once.  Y must have orthonormal columns to
 * working precision (else B is Q1^T X for the Q1 of Y = Q1 R11).
 *
 * Y: device, m x p row-major, ldy >= p (may be NULL when p == 0 or m == 0);
 * p >= 0, n >= 1, p + n <= QLESS_MAX_N (else QLESS_ERR_UNSUPPORTED).
 * X: device, m x n row-major, ldx >= n.  B: device, p x n row-major,
 * ldb >= n (may be NULL when p == 0).  R: device, n x n, ldr >= n, diagonal
 * >= 0.  B and R must not overlap Y or X.  The kernel addresses one panel of
 * rows (at most 2048) of Y and X with 32-bit byte offsets: a leading
 * dimension ldy or ldx for which a panel would span 2^31 bytes or more
 * (never below 131072) gives QLESS_ERR_UNSUPPORTED.  Workspace of
 * qless_two_phase_workspace_bytes(m, p, n) bytes (0 for invalid sizes).
 */
size_t qless_two_phase_workspace_bytes(int64_t m, int64_t p, int64_t n);
int qless_two_phase_r(const double *Y, int64_t p, int64_t ldy, const double *X, int64_t m, int64_t n,
                      int64_t ldx, double *B, int64_t ldb, double *R, int64_t ldr, void *work,
                      size_t work_bytes, hipStream_t stream);

/*
 * qless_lstsq_finish -- least squares from the Q-less R of [A b] (Sec. 1):
 * Rt = R([A b]) = [[RA, z], [0, rho]] ((n+1) x (n+1) row-major, ldr >= n+1)
 * gives x = RA^{-1} z by back substitution and |rho| = ||A x - b||_2.
 * x: device, n doubles.  resid: device, 1 double (may be NULL).
 * info (device int32, may be NULL): 0, or j (1..n) if RA_jj == 0.
 */
int qless_lstsq_finish(const double *Rt, int64_t n, int64_t ldr, double *x,
                       double *resid, int32_t *info, hipStream_t stream);

/* ------------------------------------------------------------ autotuning */

/*
 * Launch parameters of qless_tsqr_r for column count n, as chosen by an
 * autotuner: waves_per_cu = stage-1 wavefronts per compute unit (row blocks
 * k = CUs * waves_per_cu; 0 = default 8, at most 32), fan_in = blocks combined
 * per tree wavefront (0 = default: one panel of stacked rows for n <= 16,
 * else 4; explicit values 2..256), rows_per_lane = panel rows
 * per lane, one of the compiled variants for that n (0 = default;
 * QLESS_ERR_UNSUPPORTED if no such variant).  For n padding to 32, 48 or 64
 * columns, rows_per_lane = 1 selects the blocked fold on the FP64 matrix
 * cores (64-row panels, 16-column blocks in compact WY form; the same
 * reflectors, sums regrouped).  Process-wide, not thread-safe;
 * query qless_workspace_bytes after changing it (a call given a workspace
 * sized under other parameters that is now too small returns
 * QLESS_ERR_WORKSPACE before any launch).  qless_tune_get returns the
 * values in effect (defaults resolved).
 */
int qless_tune_set(int64_t n, int32_t waves_per_cu, int32_t fan_in, int32_t rows_per_lane);
int qless_tune_get(int64_t n, int32_t *waves_per_cu, int32_t *fan_in, int32_t *rows_per_lane);

/* ------------------------------------------------------------- batched */

/*
 * Batched Q-less TSQR: many independent matrices of uneven m and n in one
 * persistent stage-1 launch plus one launch per tree level (Alg. 2 applied
 * to each).  Descriptor fields follow
 * qless_tsqr_r: X (device, m x n row-major, ldx >= n; may be NULL when
 * m == 0), R (device, n x n, ldr >= n), 1 <= n <= QLESS_MAX_N.  With
 * accumulate != 0 the matrix's current R (any upper-triangular n x n, e.g.
 * the R of rows seen earlier) is stacked in: the result is R([R_old; X]),
 * which lets a caller keep a running R over chunks of rows.
 */
typedef struct {
    const double *X;
    int64_t m, n, ldx;
    double *R;
    int64_t ldr;
    int32_t accumulate;
} qless_matrix_desc;

/* Opaque host-side plan: tiles every matrix into row ranges of about
 * tile_bytes (<= 0: 4 MiB) and orders them longest first; waves_per_cu
 * (<= 0: 8) sets the persistent grid (wavefronts per compute unit).  The descriptors are copied; their
 * device pointers must stay valid while the plan is used.  Returns
 * QLESS_ERR_ARG / QLESS_ERR_UNSUPPORTED for an invalid descriptor. */
typedef struct qless_batch_plan qless_batch_plan;
int qless_batch_plan_create(const qless_matrix_desc *descs, int32_t count, int64_t tile_bytes,
                            int32_t waves_per_cu, qless_batch_plan **plan);
void qless_batch_plan_destroy(qless_batch_plan *plan);
/* Device workspace the plan needs (bytes, 256-byte aligned buffer). */
size_t qless_batch_plan_workspace_bytes(const qless_batch_plan *plan);
/* Number of row tiles in the plan. */
int64_t qless_batch_plan_tiles(const qless_batch_plan *plan);
/* Copy the plan's tables (matrices, tiles, tree groups) into `work`;
 * synchronises `stream`.  Call once per workspace before the first
 * qless_tsqr_r_batched. */
int qless_batch_plan_upload(const qless_batch_plan *plan, void *work, size_t work_bytes, hipStream_t stream);
/* Enqueue the launches computing every matrix's R (1 + tree levels, all on
 * `stream`).  Allocates nothing, copies nothing from the host, issues no
 * memset and keeps no state between calls, so the sequence can be captured
 * in a hipGraph and replayed.  Calls sharing a workspace must not overlap. */
int qless_tsqr_r_batched(const qless_batch_plan *plan, void *work, size_t work_bytes, hipStream_t stream);

/* ------------------------------------------------------- more than 64 columns */

/*
 * qless_wide_r -- R (and the explicit Q) of an m x n X with n beyond one
 * TSQR panel: block classical Gram-Schmidt with reorthogonalisation (BCGS2)
 * over column panels of `panel` (<= QLESS_MAX_N) columns, the variant that
 * stores Q which Sec. 4.6 names for more than 64 columns.  Each panel is
 * orthogonalised twice against the Q of the earlier ones (library GEMMs),
 * factored by the Q-less TSQR (R_jj, diagonal >= 0) and its Q rebuilt by
 * the streaming Q = V R_jj^{-1} pass; R's block above R_jj is the sum of
 * the two projections.  Needs m >= n and, for an accurate R, kappa(X) well
 * below u^{-1/2} (BCGS2's range).
 *
 * X: device, m x n row-major, ldx >= n.  R: device, n x n, ldr >= n, zeros
 * below the diagonal.  Q: device, m x n, ldq >= n (written: orthonormal
 * columns, X = Q R).  info (device int32, may be NULL): 0, or the first
 * column j (1-based) whose R_jj is zero -- Q is then NaN from that panel on.
 * Workspace of qless_wide_workspace_bytes(m, n, panel) bytes.  Uses a
 * rocBLAS handle per device, created on the first call (this entry point
 * allocates on its first call on a device).
 */
size_t qless_wide_workspace_bytes(int64_t m, int64_t n, int64_t panel);
int qless_wide_r(const double *X, int64_t m, int64_t n, int64_t ldx, double *R, int64_t ldr, double *Q,
                 int64_t ldq, int64_t panel, int32_t *info, void *work, size_t work_bytes,
                 hipStream_t stream);

/* -------------------------------------------------- running factorisation */

/*
 * Running Q-less TSQR with the partial tree state on the device: the rows of
 * one matrix arrive in chunks (any sizes, any number), each chunk is folded
 * into a device state by one stage-1 launch, and a finishing call runs the
 * stacked-R tree once (Alg. 2 with its first stage spread over several
 * calls; the R of all rows seen, Sec. 1).  m_total is the planned total row
 * count; it sizes the state and fixes the stage-1 split (one triangle per
 * stage-1 workgroup of the qless_tsqr_r plan for m_total rows, without tuning
 * overrides) and must be the same in every call on one state.  Folding
 * chunks this way costs one launch per chunk and one tree in all, and gives
 * R([X_1; X_2; ...]) for any chunking.
 *
 * state: device, qless_tsqr_state_bytes(m_total, n) bytes (0 for invalid
 * sizes), 256-byte aligned, owned by the caller; it holds n x n triangles
 * between the calls.  qless_tsqr_state_init clears it (a fill kernel, no
 * memset, so the sequence can be captured).  qless_tsqr_state_fold folds X
 * (m x n row-major, ldx >= n; m may be 0).  qless_tsqr_state_finish writes R
 * (n x n, ldr >= n, diagonal >= 0) and consumes the state (init it again
 * before reuse).  Calls on one state must be ordered on one stream (or by
 * events).  Errors as for qless_tsqr_r; a state smaller than required is
 * QLESS_ERR_WORKSPACE.
 */
size_t qless_tsqr_state_bytes(int64_t m_total, int64_t n);
int qless_tsqr_state_init(void *state, size_t state_bytes, int64_t m_total, int64_t n, hipStream_t stream);
int qless_tsqr_state_fold(const double *X, int64_t m, int64_t ldx, void *state, size_t state_bytes,
                          int64_t m_total, int64_t n, hipStream_t stream);
int qless_tsqr_state_finish(void *state, size_t state_bytes, int64_t m_total, int64_t n, double *R,
                            int64_t ldr, hipStream_t stream);

/* ---------------------------------------------------------- timing hooks */

/*
 * Optional per-kernel event timing for benchmarks.  While enabled, the
 * library records a hipEvent pair around every launch of its stage-1 TSQR
 * kernel ("tsqr_stage1") and Gram kernels ("gram") on the launch stream.
 * qless_timing_read synchronises those events and returns the summed
 * duration in milliseconds and the launch count since the last reset.
 * Not thread-safe; intended for single-threaded benchmark drivers.
 */
int qless_timing_enable(int on);
int qless_timing_reset(void);
int qless_timing_read(const char *kernel, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif

#endif /* QLESS_H */
