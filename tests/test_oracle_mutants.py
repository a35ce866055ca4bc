"""The oracle's pins catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle's C source
(on the CPU only: a dropped term, a wrong sign or index, a transposed
output, a lost summand), builds it, and checks that at least one pin of
``test_oracle_pins`` style rejects it.  The real oracle is untouched.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as wl

from test_oracle_pins import exact_r_via_gram, lapack_r

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "drop_alpha_in_norm": ("sqrt(alpha * alpha + s)", "sqrt(s)"),
    "drop_pivot_term_in_w": ("double w = ac[j] + pdot(", "double w = pdot("),
    "shifted_index_in_w": ("pdot(a + j + 1, 1, ac + j + 1, 1, below)", "pdot(a + j + 1, 1, ac + j, 1, below)"),
    "tau_over_alpha": ("double tau = (beta - alpha) / beta;", "double tau = (beta - alpha) / alpha;"),
    "transposed_output": ("(c >= i) ? A[c * M + i] : 0.0", "(c >= i) ? A[i * M + c] : 0.0"),
    "update_sign": ("ac[i] = ac[i] - tw * a[i]", "ac[i] = ac[i] + tw * a[i]"),
    "pairwise_drops_last": ("b + h * sb, sb, len - h)", "b + h * sb, sb, len - h - 1)"),
    "no_sign_normalisation": ("if (R[i * n + i] < 0.0)", "if (0)"),
    "skip_pivot_update": ("ac[j] = ac[j] - tw;", ";"),
    "scale_not_applied": ("a[i] = a[i] * scale;", "a[i] = a[i];"),
}


def build_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new, 1)
    c = tmp_path / ("%s.c" % name)
    so = tmp_path / ("%s.so" % name)
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-w", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_householder_r.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, dp]
    lib.oracle_householder_r.restype = ctypes.c_int
    return lib


def mutant_r(lib, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    R = np.empty((n, n))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_householder_r(X.ctypes.data_as(dp), m, n, n, R.ctypes.data_as(dp))
    return R


def pins_pass(r_of) -> bool:
    """A compact battery of the independent pins."""
    # exact rational R (tiny)
    X = wl.dyadic(9, 3, seed=5)
    Rx = exact_r_via_gram(X)
    Rf = np.array([[float(v) for v in row] for row in Rx])
    if not np.all(np.isfinite(r_of(X))) or oracle.rel_err_r(r_of(X), Rf) > 1e-13:
        return False
    # closed form n = 1
    x = wl.gaussian(1000, 1, seed=3)
    if abs(r_of(x)[0, 0] - np.sqrt(np.sum(x * x))) > 1e-13 * np.sqrt(np.sum(x * x)):
        return False
    # known R0 and LAPACK
    Xk, R0 = wl.known_r(777, 6, wl.logspace_sigma(6, 3), seed=1)
    Rk = r_of(Xk)
    if not np.all(np.isfinite(Rk)) or oracle.rel_err_r(Rk, R0) > 1e-12:
        return False
    Xg = wl.gaussian(300, 5, seed=2)
    if oracle.rel_err_r(r_of(Xg), lapack_r(Xg)) > 1e-13:
        return False
    return True


def test_battery_accepts_real_oracle():
    assert pins_pass(oracle.householder_r)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_battery_rejects_mutant(tmp_path, name):
    lib = build_mutant(tmp_path, name)
    with np.errstate(all="ignore"):
        assert not pins_pass(lambda X: mutant_r(lib, X)), name


# Shifted CholQR3: mistakes planted inside oracle_shifted_cholqr3_r only.
MUTANTS_SHIFTED = {
    "no_shift": ("C[j * n + j] = C[j * n + j] + shift;", "C[j * n + j] = C[j * n + j];"),
    "negative_shift": ("C[j * n + j] = C[j * n + j] + shift;", "C[j * n + j] = C[j * n + j] - shift;"),
    "first_factor_dropped": ("acc = acc + R23[i * n + k] * R1[k * n + c];",
                             "acc = acc + R23[i * n + k] * (k == c ? 1.0 : 0.0);"),
    "factors_reversed": ("acc = acc + R23[i * n + k] * R1[k * n + c];",
                         "acc = acc + R1[i * n + k] * R23[k * n + c];"),
    "substitution_sign": ("for (int64_t k = 0; k < c; ++k) e = e - y[k] * R1[k * n + c];",
                          "for (int64_t k = 0; k < c; ++k) e = e + y[k] * R1[k * n + c];"),
}


def build_shifted_mutant(tmp_path, name):
    old, new = MUTANTS_SHIFTED[name]
    src = open(SRC).read()
    start = src.index("int oracle_shifted_cholqr3_r(")
    body = src[start:]
    assert body.count(old) >= 1, name
    src = src[:start] + body.replace(old, new, 1)
    c = tmp_path / ("%s.c" % name)
    so = tmp_path / ("%s.so" % name)
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-w", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_shifted_cholqr3_r.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, dp]
    lib.oracle_shifted_cholqr3_r.restype = ctypes.c_int
    return lib


def shifted_mutant_r(lib, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    R = np.empty((n, n))
    dp = ctypes.POINTER(ctypes.c_double)
    info = lib.oracle_shifted_cholqr3_r(X.ctypes.data_as(dp), m, n, n, R.ctypes.data_as(dp))
    return R, info


def shifted_pins_pass(r_of) -> bool:
    # well conditioned: the known R0
    Xk, R0 = wl.known_r(2000, 6, wl.logspace_sigma(6, 3), seed=1)
    R, info = r_of(Xk)
    if info != 0 or not np.all(np.isfinite(R)) or oracle.rel_err_r(R, R0) > 1e-12:
        return False
    # kappa = 1e12 spread over the columns: completes, backward stable
    Xs = wl.svd_form(2000, 8, wl.logspace_sigma(8, 12), seed=9)
    R, info = r_of(Xs)
    if info != 0 or not np.all(np.isfinite(R)) or oracle.gram_residual(Xs, R) > 1e-14:
        return False
    return oracle.rel_err_r(R, oracle.householder_r(Xs)) <= 1e-12


def test_shifted_battery_accepts_real_oracle():
    assert shifted_pins_pass(oracle.shifted_cholqr3_r)


@pytest.mark.parametrize("name", sorted(MUTANTS_SHIFTED))
def test_shifted_battery_rejects_mutant(tmp_path, name):
    lib = build_shifted_mutant(tmp_path, name)
    with np.errstate(all="ignore"):
        assert not shifted_pins_pass(lambda X: shifted_mutant_r(lib, X)), name


# Dot2 Gram (the reference X^T X of the Gram-residual metric): mistakes
# planted inside oracle_gram_dot2 only; the pin is the Dot2 error bound
# against the exact rational X^T X.
MUTANTS_DOT2 = {
    "drop_two_product_error": ("s = s + (q + r);", "s = s + q;"),
    "drop_two_sum_error": ("s = s + (q + r);", "s = s + r;"),
    "plain_product_sum": ("two_sum(p, h, &p, &q);", "p = p + h; q = 0.0;"),
}


def build_dot2_mutant(tmp_path, name):
    old, new = MUTANTS_DOT2[name]
    src = open(SRC).read()
    start = src.index("void oracle_gram_dot2(")
    body = src[start:]
    assert body.count(old) >= 1, name
    src = src[:start] + body.replace(old, new, 1)
    c = tmp_path / ("%s.c" % name)
    so = tmp_path / ("%s.so" % name)
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-w", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_gram_dot2.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, dp]
    lib.oracle_gram_dot2.restype = None
    return lib


def dot2_mutant_gram(lib, X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    C = np.empty((n, n))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_gram_dot2(X.ctypes.data_as(dp), m, n, n, C.ctypes.data_as(dp))
    return C


def dot2_pins_pass(gram_of) -> bool:
    from test_oracle_pins import dot2_pin_inputs, dot2_violations
    return all(dot2_violations(gram_of(X), X) == [] for X in dot2_pin_inputs())


def test_dot2_battery_accepts_real_oracle():
    assert dot2_pins_pass(oracle.gram_dot2)


@pytest.mark.parametrize("name", sorted(MUTANTS_DOT2))
def test_dot2_battery_rejects_mutant(tmp_path, name):
    lib = build_dot2_mutant(tmp_path, name)
    assert not dot2_pins_pass(lambda X: dot2_mutant_gram(lib, X)), name


# Chunked Householder variant: mistakes planted inside its own code.
MUTANTS_CHUNKED = {
    "chunk_tail_dropped": ("int64_t cl = (len - lo < CHUNK_ROWS) ? len - lo : CHUNK_ROWS;",
                           "int64_t cl = CHUNK_ROWS < len - lo ? CHUNK_ROWS : 0;"),
    "chunk_totals_lose_last": ("return pairwise_array(part, nc);", "return pairwise_array(part, nc - 1);"),
    "chunked_pivot_term_dropped": ("double w = ac[j] + chunked_dot(", "double w = chunked_dot("),
}


def build_chunked_mutant(tmp_path, name):
    old, new = MUTANTS_CHUNKED[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    src = src.replace(old, new, 1)
    c = tmp_path / ("%s.c" % name)
    so = tmp_path / ("%s.so" % name)
    c.write_text(src)
    subprocess.check_call(["gcc", *oracle.GCC_FLAGS, "-w", str(c), "-o", str(so), "-lm"])
    lib = ctypes.CDLL(str(so))
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_householder_r_chunked.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, dp,
                                                 ctypes.c_int]
    lib.oracle_householder_r_chunked.restype = ctypes.c_int
    return lib


def chunked_pins_pass(r_of) -> bool:
    Xk, R0 = wl.known_r(150_000, 5, wl.logspace_sigma(5, 3), seed=3)
    Rk = r_of(Xk)
    if not np.all(np.isfinite(Rk)) or oracle.rel_err_r(Rk, R0) > 1e-12:
        return False
    Xg = wl.gaussian(70_001, 4, seed=8)
    return oracle.rel_err_r(r_of(Xg), lapack_r(Xg)) <= 1e-13


def test_chunked_battery_accepts_real_oracle():
    assert chunked_pins_pass(lambda X: oracle.householder_r_chunked(X, threads=2))


@pytest.mark.parametrize("name", sorted(MUTANTS_CHUNKED))
def test_chunked_battery_rejects_mutant(tmp_path, name):
    lib = build_chunked_mutant(tmp_path, name)

    def r_of(X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        m, n = X.shape
        R = np.empty((n, n))
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_householder_r_chunked(X.ctypes.data_as(dp), m, n, n, R.ctypes.data_as(dp), 2)
        return R
    with np.errstate(all="ignore"):
        assert not chunked_pins_pass(r_of), name
