"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names what fixes the expected value: exact rational arithmetic,
a closed form, an invariant of the factorisation, a construction with a
known answer, or an independent library routine (LAPACK through scipy/numpy).
Paper: Thies & Roehrig-Zoellner, arXiv 2603.20889.  The factorisation being
pinned is X = QR, Q^T Q = I, R upper triangular (Sec. 1); R is unique once
its diagonal is made non-negative, which the oracle does.
"""
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as wl
from tolerances import e_row

EPS = 2.0 ** -52


# ------------------------------------------------------------- helpers

def exact_r_via_gram(X: np.ndarray, digits: int = 60):
    """R with positive diagonal and R^T R = X^T X, from the exact rational
    Gram matrix and a Cholesky factorisation in `digits`-digit decimals.
    Independent of Householder: only the definition R^T R = X^T X."""
    getcontext().prec = digits
    m, n = X.shape
    F = [[Fraction(float(v)) for v in row] for row in X]
    G = [[sum((F[i][a] * F[i][b] for i in range(m)), Fraction(0)) for b in range(n)] for a in range(n)]
    Gd = [[Decimal(g.numerator) / Decimal(g.denominator) for g in row] for row in G]
    R = [[Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        d = Gd[j][j] - sum((R[k][j] * R[k][j] for k in range(j)), Decimal(0))
        if d <= 0:
            return None
        R[j][j] = d.sqrt()
        for c in range(j + 1, n):
            R[j][c] = (Gd[j][c] - sum((R[k][j] * R[k][c] for k in range(j)), Decimal(0))) / R[j][j]
    return R


def lapack_r(X: np.ndarray) -> np.ndarray:
    """R from LAPACK dgeqrf (scipy), padded to n x n, rows sign-normalised."""
    m, n = X.shape
    Xp = X if m >= n else np.vstack([X, np.zeros((n - m, n))])
    R = sla.qr(Xp, mode="r")[0][:n]
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return d[:, None] * R


# ------------------------------------------------ exact / closed forms

@pytest.mark.parametrize("seed", range(12))
def test_householder_matches_exact_rational_r(seed):
    """P1: tiny dyadic matrices; R from exact Gram + 60-digit Cholesky."""
    g = wl.rng(100 + seed)
    n = int(g.integers(1, 5))
    m = int(g.integers(n, 13))
    X = wl.dyadic(m, n, seed=200 + seed)
    Rx = exact_r_via_gram(X)
    if Rx is None:
        pytest.skip("rank-deficient draw")
    R = oracle.householder_r(X)
    Rf = np.array([[float(v) for v in row] for row in Rx])
    kappa = np.linalg.cond(Rf)
    err = max(abs(Decimal(float(R[i, j])) - Rx[i][j]) for i in range(n) for j in range(n))
    assert float(err) <= 64 * EPS * kappa * float(np.abs(Rf).max())
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0.0)


@pytest.mark.parametrize("m", [1, 2, 7, 1000, 100_003])
def test_single_column_is_the_two_norm(m):
    """P2: n = 1, R = ||x||_2, exact sum of squares then a 60-digit sqrt."""
    x = wl.gaussian(m, 1, seed=7 + m)
    getcontext().prec = 60
    s = sum((Fraction(float(v)) ** 2 for v in x[:, 0]), Fraction(0))
    exact = (Decimal(s.numerator) / Decimal(s.denominator)).sqrt()
    R = oracle.householder_r(x)
    assert R.shape == (1, 1)
    rel = abs(Decimal(float(R[0, 0])) - exact) / exact
    assert float(rel) <= (np.ceil(np.log2(m)) + 4) * EPS


def test_empty_matrix_gives_zero_r():
    R = oracle.householder_r(np.zeros((0, 5)))
    assert np.array_equal(R, np.zeros((5, 5)))
    assert not np.signbit(R).any()


# ----------------------------------------------- known-answer constructions

@pytest.mark.parametrize("n,k", [(1, 0), (2, 4), (4, 4), (8, 0), (8, 4), (16, 4), (16, 8), (32, 4), (64, 4)])
def test_known_r0_recovered(n, k):
    """P3: X = Q0 R0 with R0 upper triangular, diag >= 0 => R(X) = R0.
    Tolerances: e_R <= 1e-12 at kappa <= 1e4 (the project's bar); the
    construction's own rounding is about kappa * eps."""
    X, R0 = wl.known_r(4000 + n, n, wl.logspace_sigma(n, k), seed=31 * n + k)
    R = oracle.householder_r(X)
    tol = 1e-13 if k <= 4 else 1e-12
    assert oracle.rel_err_r(R, R0) <= tol
    assert oracle.gram_residual(X, R) <= 1e-14


@pytest.mark.parametrize("m,n", [(50, 1), (64, 3), (200, 5), (1000, 8), (333, 17), (4096, 32), (700, 64), (64, 64), (5, 9)])
def test_householder_matches_lapack(m, n):
    """Independent library routine: LAPACK dgeqrf via scipy, signs fixed."""
    X = wl.gaussian(m, n, seed=m * 131 + n)
    R = oracle.householder_r(X)
    assert oracle.rel_err_r(R, lapack_r(X)) <= 1e-13


def test_gram_invariant_holds_with_extended_gram():
    """P4: R^T R = X^T X (Dot2 Gram), the backward-error pin."""
    X = wl.gaussian(20000, 12, seed=5)
    X[:, 3] *= 1e-6
    R = oracle.householder_r(X)
    assert oracle.gram_residual(X, R) <= 1e-14


def exact_gram(X: np.ndarray):
    """X^T X in exact rational arithmetic (every double is a dyadic rational,
    so every product and sum is exact as a Fraction)."""
    m, n = X.shape
    F = [[Fraction(float(v)) for v in row] for row in X]
    return [[sum((F[i][a] * F[i][b] for i in range(m)), Fraction(0)) for b in range(n)] for a in range(n)]


def dot2_violations(C: np.ndarray, X: np.ndarray) -> list:
    """Entries of C that break the Dot2 error bound of Ogita, Rump and Oishi
    (2005, Prop. 5.5): |res - x^T y| <= u |x^T y| + gamma_{m}^2 |x|^T |y| with
    u = 2^-53 and gamma_m = m u / (1 - m u) -- the bound of a dot product
    computed in twice the working precision and rounded once."""
    m, n = X.shape
    u = 2.0 ** -53
    gam = m * u / (1.0 - m * u)
    Cx = exact_gram(X)
    A = np.abs(X).T @ np.abs(X)
    bad = []
    for a in range(n):
        for b in range(n):
            err = abs(Fraction(float(C[a, b])) - Cx[a][b])
            bound = Fraction(u) * abs(Cx[a][b]) + Fraction(gam * gam * 1.01 * float(A[a, b]))
            if err > bound:
                bad.append((a, b, float(err), float(bound)))
    return bad


def dot2_pin_inputs():
    """Inputs for the Dot2 pin: (1) iid N(0,1) entries with full 53-bit
    mantissas; (2) rows in pairs (a, b), (-a, b + t) with t ~ 1e-9, so the
    off-diagonal sum cancels to about 1e-9 of its terms -- a sum of rounded
    products then carries an error many orders above the Dot2 bound."""
    g = wl.rng(4242)
    X1 = g.standard_normal((1500, 3))
    a = g.standard_normal(1000)
    b = g.standard_normal(1000)
    t = 1e-9 * g.standard_normal(1000)
    X2 = np.empty((2000, 2))
    X2[0::2, 0], X2[0::2, 1] = a, b
    X2[1::2, 0], X2[1::2, 1] = -a, b + t
    return [X1, X2]


def test_gram_dot2_is_twice_working_precision():
    """The Gram matrix behind the e_G metric: every entry of the oracle's
    Dot2 X^T X is within the Dot2 bound of the exact rational X^T X, on
    generic data and on data whose off-diagonal sum cancels almost fully."""
    for X in dot2_pin_inputs():
        C = oracle.gram_dot2(X)
        assert dot2_violations(C, X) == []
    # the cancelling case is one that plain float64 accumulation gets wrong
    X = dot2_pin_inputs()[1]
    assert dot2_violations(X.T @ X, X) != []


# ------------------------------------------------ chunked variant (O7)

@pytest.mark.parametrize("m,n", [(1, 3), (5, 8), (65536, 2), (65537, 3), (300_001, 5), (200_000, 16)])
def test_chunked_is_independent_of_threads_and_matches(m, n):
    """The chunked oracle gives bitwise the same R on 1, 3 and 8 threads, and
    agrees with the plain oracle and LAPACK (only the summation order of the
    length-m sums differs)."""
    X = wl.gaussian(m, n, seed=m + 17 * n)
    R1 = oracle.householder_r_chunked(X, threads=1)
    for t in (3, 8):
        assert np.array_equal(oracle.householder_r_chunked(X, threads=t), R1)
    assert oracle.rel_err_r(R1, oracle.householder_r(X)) <= 1e-14
    assert oracle.rel_err_r(R1, lapack_r(X)) <= 1e-13


def test_chunked_known_r_and_exact():
    Xk, R0 = wl.known_r(150_000, 6, wl.logspace_sigma(6, 4), seed=71)
    assert oracle.rel_err_r(oracle.householder_r_chunked(Xk, threads=4), R0) <= 1e-12
    X = wl.dyadic(9, 3, seed=5)
    Rf = np.array([[float(v) for v in row] for row in exact_r_via_gram(X)])
    assert oracle.rel_err_r(oracle.householder_r_chunked(X, threads=2), Rf) <= 1e-13


# --------------------------------------------------- special structure

@pytest.mark.parametrize("n,extra", [(4, 0), (8, 5), (16, 100), (33, 1)])
def test_stacked_triangle_over_zeros_is_bitwise_r0(n, extra):
    """P5: [R0; 0] -> R0 bitwise (every reflector is the identity, tau = 0)."""
    R0 = wl.triangular_with_singular_values(wl.logspace_sigma(n, 3), wl.rng(n))
    X = np.vstack([R0, np.zeros((extra, n))])
    R = oracle.householder_r(X)
    assert np.array_equal(R, R0)


@pytest.mark.parametrize("s", [-200, -7, 5, 200])
def test_power_of_two_scaling_is_exact(s):
    """P5: R(2^s X) = 2^s R(X) bitwise (every operation commutes with exact
    power-of-two scaling when nothing over- or underflows)."""
    X = wl.gaussian(3001, 7, seed=9)
    R1 = oracle.householder_r(X)
    R2 = oracle.householder_r(np.ldexp(X, s))
    assert np.array_equal(R2, np.ldexp(R1, s))


def test_row_permutation_and_duplication():
    """P5: R(PX) = R(X); R([X; X]) = sqrt(2) R(X)."""
    X = wl.gaussian(5000, 9, seed=11)
    R = oracle.householder_r(X)
    P = wl.rng(3).permutation(5000)
    assert oracle.rel_err_r(oracle.householder_r(X[P]), R) <= 1e-14
    assert oracle.rel_err_r(oracle.householder_r(np.vstack([X, X])), np.sqrt(2.0) * R) <= 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 7, 16])
def test_stacking_identity(k):
    """O2 (Alg. 2): R(X) = R([R(X_1); ...; R(X_k)]) for any row partition,
    including empty and shorter-than-n blocks."""
    X = wl.gaussian(3000, 6, seed=k)
    g = wl.rng(40 + k)
    cuts = np.sort(g.integers(0, 3001, size=k - 1))
    if k >= 3:
        cuts[0] = cuts[1]          # force an empty block
    parts = np.split(X, cuts)
    Rs = [oracle.householder_r(p) for p in parts]
    assert oracle.rel_err_r(oracle.stacked_r(Rs), oracle.householder_r(X)) <= 1e-14


def test_zero_column_gives_exact_zero_column():
    """Rank deficiency (Sec. 1): an exactly zero column yields an exactly
    zero column of R, including a zero diagonal entry."""
    X = wl.gaussian(1000, 6, seed=4)
    X[:, 2] = 0.0
    R = oracle.householder_r(X)
    assert np.all(R[:, 2] == 0.0)
    assert oracle.gram_residual(X, R) <= 1e-14


def test_repeated_column_rank_deficient():
    X = wl.gaussian(1000, 5, seed=8)
    X[:, 3] = X[:, 1]
    R = oracle.householder_r(X)
    assert abs(R[3, 3]) <= 1e-13 * np.abs(R).max()
    assert oracle.gram_residual(X, R) <= 1e-14


@pytest.mark.parametrize("m,n", [(1, 4), (3, 8), (7, 8)])
def test_fewer_rows_than_columns(m, n):
    """m < n: R of X padded with zero rows; compare with LAPACK."""
    X = wl.gaussian(m, n, seed=m + n)
    R = oracle.householder_r(X)
    assert np.all(R[m:] == 0.0)
    assert oracle.rel_err_r(R, lapack_r(X)) <= 1e-13


# ----------------------------------------------------------- CholQR2 (Alg. 1)

@pytest.mark.parametrize("seed", range(6))
def test_cholqr2_matches_exact_rational_r(seed):
    g = wl.rng(300 + seed)
    n = int(g.integers(1, 5))
    m = int(g.integers(n, 13))
    X = wl.dyadic(m, n, seed=400 + seed)
    Rx = exact_r_via_gram(X)
    if Rx is None:
        pytest.skip("rank-deficient draw")
    R, info = oracle.cholqr2_r(X)
    assert info == 0
    Rf = np.array([[float(v) for v in row] for row in Rx])
    kappa = np.linalg.cond(Rf)
    assert oracle.rel_err_r(R, Rf) <= 64 * EPS * kappa ** 2


@pytest.mark.parametrize("n,k", [(4, 0), (8, 4), (16, 4), (32, 2)])
def test_cholqr2_postcondition_and_agreement(n, k):
    """Alg. 1 ENSURE: (X R^{-1})^T (X R^{-1}) = I; R equals the Householder R
    for kappa <= 1e4."""
    X, R0 = wl.known_r(5000, n, wl.logspace_sigma(n, k), seed=77 + n)
    R, info = oracle.cholqr2_r(X)
    assert info == 0
    Q = sla.solve_triangular(R, X.T, trans="T", lower=False).T   # X R^{-1} by LAPACK
    orth = np.linalg.norm(oracle.gram_dot2(Q) - np.eye(n))
    assert orth <= 1e-13
    assert oracle.rel_err_r(R, R0) <= 1e-12


def test_cholqr2_breakdown_reports_column():
    """Sec. 3.1: Gram methods break down on (numerically) singular X; a zero
    column j gives a zero pivot at j, info = j (1-based), R = NaN."""
    X = wl.gaussian(500, 5, seed=2)
    X[:, 3] = 0.0
    R, info = oracle.cholqr2_r(X)
    assert info == 4
    assert np.isnan(R).all()


# ------------------------------------------ shifted CholQR3 (robust variant)

@pytest.mark.parametrize("n,k", [(4, 0), (8, 4), (16, 4), (32, 2)])
def test_shifted_cholqr3_postcondition_and_agreement(n, k):
    """Well-conditioned X: (X R^{-1})^T (X R^{-1}) = I and R equals the
    known R0 (and so the Householder R) to the CholQR2 bar."""
    X, R0 = wl.known_r(5000, n, wl.logspace_sigma(n, k), seed=79 + n)
    R, info = oracle.shifted_cholqr3_r(X)
    assert info == 0
    Q = sla.solve_triangular(R, X.T, trans="T", lower=False).T
    assert np.linalg.norm(oracle.gram_dot2(Q) - np.eye(n)) <= 1e-13
    assert oracle.rel_err_r(R, R0) <= 1e-12
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= 1e-12


@pytest.mark.parametrize("n,k", [(8, 10), (16, 12), (5, 12)])
def test_shifted_cholqr3_beyond_cholqr2(n, k):
    """kappa = 10^k far above eps^{-1/2}, spread over all columns
    (X = U diag(sigma) V^T): CholQR2's Gram matrix is numerically singular
    and a Cholesky fails; the shifted variant completes, its R is backward
    stable (Gram residual against the extended-precision X^T X at the level
    of u) and agrees with the Householder R normwise."""
    X = wl.svd_form(4000, n, wl.logspace_sigma(n, k), seed=83 + n + k)
    _, info2 = oracle.cholqr2_r(X)
    assert info2 != 0
    R, info = oracle.shifted_cholqr3_r(X)
    assert info == 0
    assert np.all(np.diag(R) > 0.0) and np.all(np.tril(R, -1) == 0.0)
    assert oracle.gram_residual(X, R) <= 1e-14
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= 1e-12


def test_shifted_cholqr3_scaled_orthogonal_columns():
    """Orthogonal columns of lengths 2^a: R = diag(2^a) up to rounding,
    whatever the (tiny) shift did to the first factor."""
    n = 6
    Q = wl.orthonormal_columns(3000, n, wl.rng(5))
    d = 2.0 ** np.array([0, 3, -2, 7, 1, -5])
    R, info = oracle.shifted_cholqr3_r(Q * d)
    assert info == 0
    assert oracle.rel_err_r(R, np.diag(d)) <= 1e-14


def test_shifted_cholqr3_zero_column_still_breaks_down():
    """An exactly zero column stays singular after the shift only if the
    shift is zero; with X = 0 the trace, and so the shift, is zero and the
    first Cholesky reports column 1."""
    R, info = oracle.shifted_cholqr3_r(np.zeros((100, 3)))
    assert info == 1
    assert np.isnan(R).all()


# --------------------------------------------------------------- SVQB2

def test_jacobi_matches_lapack_eigh():
    A = wl.gaussian(40, 40, seed=12)
    A = A + A.T
    w, V, sweeps = oracle.jacobi_eig(A)
    wl_ = np.linalg.eigvalsh(A)[::-1]
    assert np.max(np.abs(w - wl_)) <= 1e-13 * np.abs(wl_).max()
    assert np.linalg.norm(A @ V - V * w) <= 1e-13 * np.linalg.norm(A)
    assert np.linalg.norm(V.T @ V - np.eye(40)) <= 1e-13
    assert sweeps < 20


@pytest.mark.parametrize("n,k", [(1, 0), (4, 0), (8, 4), (16, 4), (24, 3)])
def test_svqb2_qz_form(n, k):
    """SVQB (Sec. 1): X B = Q, X = Q Z.  Pins: Z^T Z = X^T X, qr_R(Z) = R(X),
    sigma = singular values of X (LAPACK SVD)."""
    X, R0 = wl.known_r(6000, n, wl.logspace_sigma(n, k), seed=5 * n + k)
    Z, sig, Rz, ntr = oracle.svqb2(X)
    assert ntr == 0
    G = oracle.gram_dot2(X)
    assert np.linalg.norm(Z.T @ Z - G) <= 1e-14 * np.linalg.norm(G) * max(1.0, 10.0 ** k / 1e2)
    assert oracle.rel_err_r(Rz, R0) <= 1e-12
    s_ref = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(sig - s_ref) / s_ref) <= 1e-8 * 10.0 ** (k / 2)


def test_svqb2_orthonormal_input_gives_identity():
    """k = 0 style: X with orthonormal columns => qr_R(Z) = I."""
    Q0 = wl.orthonormal_columns(3000, 6, wl.rng(1))
    Z, sig, Rz, ntr = oracle.svqb2(Q0)
    assert np.linalg.norm(Rz - np.eye(6)) <= 1e-14


def test_svqb2_truncates_zero_direction():
    X = wl.gaussian(800, 5, seed=21)
    X[:, 1] = 0.0
    Z, sig, Rz, ntr = oracle.svqb2(X)
    assert ntr >= 1
    assert sig[-1] == 0.0 or sig[-1] <= 1e-6 * sig[0]


# -------------------------------------------------------- least squares

@pytest.mark.parametrize("n", [1, 3, 10, 47])
def test_lstsq_from_r_matches_lapack(n):
    """Sec. 1: Q-less R of [A b] gives x and the residual in one pass."""
    Ab, x0 = wl.ls_request_data(3000, n, seed=n)
    A, b = Ab[:, :n], Ab[:, n]
    Rt = oracle.householder_r(Ab)
    x, res = oracle.lstsq_from_r(Rt)
    x_ref, *_ = np.linalg.lstsq(A, b, rcond=None)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    assert abs(res - np.linalg.norm(A @ x_ref - b)) <= 1e-10 * max(res, 1e-300)
    assert np.linalg.norm(x - x0) <= 1e-5 * np.linalg.norm(x0)


# ------------------------------------------- explicit Q = X R^{-1} (Sec. 1)

def test_q_from_r_identity_and_exact_scaling():
    """R = I gives Q = X exactly; R = diag(2^a) divides column j by 2^a_j
    exactly; an upper bidiagonal R with power-of-two entries on dyadic data
    gives the exact rational solution of q R = x."""
    X = wl.dyadic(50, 4, seed=3)
    assert np.array_equal(oracle.q_from_r(X, np.eye(4)), X)
    d = 2.0 ** np.array([3, -1, 0, 5])
    assert np.array_equal(oracle.q_from_r(X, np.diag(d)), X / d)
    R = np.diag(d) + np.diag([0.5, 0.25, 2.0], 1)
    Q = oracle.q_from_r(X, R)
    for i in range(X.shape[0]):
        q = [Fraction(0)] * 4
        for c in range(4):
            e = Fraction(X[i, c]) - sum((q[k] * Fraction(R[k, c]) for k in range(c)), Fraction(0))
            q[c] = e / Fraction(R[c, c])
        assert all(Fraction(Q[i, c]) == q[c] for c in range(4))


@pytest.mark.parametrize("n,k", [(4, 0), (8, 4), (16, 4)])
def test_q_from_r_rebuilds_an_orthonormal_q(n, k):
    """With the Householder R of a well-conditioned X, X R^{-1} has
    orthonormal columns (to about kappa u) and Q R reproduces X."""
    X = wl.svd_form(3000, n, wl.logspace_sigma(n, k), seed=60 + n)
    R = oracle.householder_r(X)
    Q = oracle.q_from_r(X, R)
    assert np.linalg.norm(oracle.gram_dot2(Q) - np.eye(n)) <= 100 * EPS * 10.0 ** k
    assert np.linalg.norm(Q @ R - X) <= 100 * EPS * np.linalg.norm(X)


def test_q_from_r_rejects_singular_r():
    R = np.triu(np.ones((3, 3)))
    R[1, 1] = 0.0
    with pytest.raises(RuntimeError):
        oracle.q_from_r(np.ones((5, 3)), R)


# ------------------------------------- two-phase orthogonalisation (Sec. 2)

def test_two_phase_with_coordinate_basis_is_exact():
    """Y = [e_1, e_2]: the projection zeroes the first two rows exactly, so
    B is those rows and R is the Householder R of the rest, bit for bit."""
    X = wl.dyadic(40, 5, seed=8)
    Y = np.zeros((40, 2))
    Y[0, 0] = Y[1, 1] = 1.0
    B, R = oracle.two_phase_r(Y, X)
    assert np.array_equal(B, X[:2])
    Z = X.copy()
    Z[:2] = 0.0
    assert np.array_equal(R, oracle.householder_r(Z))


def test_two_phase_without_basis_is_plain_r():
    X = wl.gaussian(300, 6, seed=4)
    B, R = oracle.two_phase_r(np.zeros((300, 0)), X)
    assert B.shape == (0, 6)
    assert np.array_equal(R, oracle.householder_r(X))


@pytest.mark.parametrize("p,n,k", [(3, 4, 0), (8, 8, 4), (16, 5, 2)])
def test_two_phase_recovers_known_parts(p, n, k):
    """X = Y B0 + W R0 with [Y W] orthonormal: B = B0 and R = R0."""
    g = wl.rng(90 + p + n)
    U = wl.orthonormal_columns(2000, p + n, g)
    Y, W = U[:, :p], U[:, p:]
    B0 = g.standard_normal((p, n))
    R0 = wl.triangular_with_singular_values(wl.logspace_sigma(n, k), g)
    B, R = oracle.two_phase_r(Y, Y @ B0 + W @ R0)
    assert np.linalg.norm(B - B0) <= 1e-13 * np.linalg.norm(B0)
    assert oracle.rel_err_r(R, R0) <= 100 * EPS * max(1.0, 10.0 ** k)   # about kappa u


def test_two_phase_of_a_vector_in_the_span_leaves_nothing():
    g = wl.rng(7)
    Y = wl.orthonormal_columns(1000, 4, g)
    X = Y @ g.standard_normal((4, 3))
    _, R = oracle.two_phase_r(Y, X)
    assert np.linalg.norm(R) <= 1e-14 * np.linalg.norm(X)


def test_row_scaled_metric_sees_a_wrong_trailing_row():
    """The row-wise metric of the parity tests flags an error in the smallest
    row that the normwise e_R cannot see: X = Q0 diag(sigma) with sigma from
    1 down to 1e-4 has R = diag(sigma), and a 1e-9 relative error in R_nn
    moves e_R by only 1e-13."""
    sig = wl.logspace_sigma(8, 4)
    X = wl.orthonormal_columns(20000, 8, wl.rng(5)) * sig
    Ro = oracle.householder_r(X)
    assert np.allclose(np.abs(np.diag(Ro)), sig, rtol=1e-12)
    bad = Ro.copy()
    bad[-1, -1] *= 1.0 + 1e-9
    floor = 1e-4 * oracle.col_norm_max(X)
    assert oracle.rel_err_r(bad, Ro) <= 1e-12
    assert oracle.row_scaled_err(bad, Ro, floor) > e_row(8)
    assert oracle.row_scaled_err(oracle.cholqr2_r(X)[0], Ro, floor) <= e_row(8)
