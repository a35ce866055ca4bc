"""CPU oracle for Q-less QR of tall, very skinny FP64 matrices.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this package.  It wraps the plain
C implementation in ``oracle.c`` (built with ``-ffp-contract=off``, no
fast-math) through ctypes and shares no code with the HIP library.

Every function takes and returns numpy float64 arrays; X is row-major
(m x n), R is n x n with zeros below a non-negative diagonal.

Paper: Thies & Roehrig-Zoellner, arXiv 2603.20889.
  householder_r : R of X, Sec. 1 (X = QR, R upper triangular), per-column
                  Householder reflector of Alg. 4 without the column pairing
  householder_r_chunked : the same with every length-m sum in fixed
                  64K-row chunks, OpenMP over chunks; bitwise independent
                  of the thread count (for timing on all host cores)
  cholqr2_r     : Q-less Cholesky-QR2, Alg. 1
  shifted_cholqr3_r : Q-less shifted Cholesky-QR3, the robust variant Sec. 2
                  names (shift of Fukaya et al. 2020)
  svqb2         : Q-less SVQB applied twice; QZ form of Sec. 1, SVQB2
                  paragraph of Sec. 3.1
  lstsq_from_r  : least squares via the Q-less R of [A b], Sec. 1
  q_from_r      : explicit Q = X R^{-1} rebuilt from X and the Q-less R, Sec. 1
  two_phase_r   : R of (I - Y Y^T) X and B = Y^T X, the two-phase problem of Sec. 2
  gram_dot2     : X^T X in twice-working precision (the Gram-residual metric and
                  the reference of the GPU's double-double Gram)
Metrics: rel_err_r (normwise e_R), row_scaled_err (row-wise, floored at a
given scale), col_norm_max, gram_residual (e_G).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
             "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so next to it (gcc, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_householder_r.argtypes = [dp, i64, i64, i64, dp]
        lib.oracle_householder_r.restype = ctypes.c_int
        lib.oracle_householder_r_chunked.argtypes = [dp, i64, i64, i64, dp, ctypes.c_int]
        lib.oracle_householder_r_chunked.restype = ctypes.c_int
        lib.oracle_cholqr2_r.argtypes = [dp, i64, i64, i64, dp]
        lib.oracle_cholqr2_r.restype = ctypes.c_int
        lib.oracle_shifted_cholqr3_r.argtypes = [dp, i64, i64, i64, dp]
        lib.oracle_shifted_cholqr3_r.restype = ctypes.c_int
        lib.oracle_svqb2.argtypes = [dp, i64, i64, i64, ctypes.c_double, dp, dp, dp]
        lib.oracle_svqb2.restype = ctypes.c_int
        lib.oracle_jacobi_eig.argtypes = [dp, i64, dp, dp]
        lib.oracle_jacobi_eig.restype = ctypes.c_int
        lib.oracle_lstsq_from_r.argtypes = [dp, i64, i64, dp, dp]
        lib.oracle_lstsq_from_r.restype = ctypes.c_int
        lib.oracle_q_from_r.argtypes = [dp, i64, i64, i64, dp, i64, dp, i64]
        lib.oracle_q_from_r.restype = ctypes.c_int
        lib.oracle_two_phase_r.argtypes = [dp, i64, i64, dp, i64, i64, i64, dp, dp]
        lib.oracle_two_phase_r.restype = ctypes.c_int
        lib.oracle_gram_dot2.argtypes = [dp, i64, i64, i64, dp]
        lib.oracle_gram_dot2.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _as_rowmajor(X) -> tuple[np.ndarray, int, int, int]:
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2:
        raise ValueError("X must be 2-D")
    m, n = X.shape
    if X.strides[1] != 8 or (m > 1 and X.strides[0] % 8) or (m > 1 and X.strides[0] < 8 * n):
        X = np.ascontiguousarray(X)
    ldx = X.strides[0] // 8 if m > 1 else n
    return X, m, n, ldx


def householder_r(X) -> np.ndarray:
    """Sign-normalised R of X by unblocked Householder QR (pairwise sums)."""
    X, m, n, ldx = _as_rowmajor(X)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_householder_r(_ptr(X), m, n, ldx, _ptr(R))
    if rc != 0:
        raise RuntimeError("oracle_householder_r failed: %d" % rc)
    return R


def householder_r_chunked(X, threads: int = 1) -> np.ndarray:
    """householder_r with chunked sums, on `threads` OpenMP threads; the
    result does not depend on the thread count."""
    X, m, n, ldx = _as_rowmajor(X)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_householder_r_chunked(_ptr(X), m, n, ldx, _ptr(R), int(threads))
    if rc != 0:
        raise RuntimeError("oracle_householder_r_chunked failed: %d" % rc)
    return R


def stacked_r(blocks) -> np.ndarray:
    """R([R_1; ...; R_k]) -- the second stage of Alg. 2 on given blocks."""
    return householder_r(np.vstack([np.asarray(b, dtype=np.float64) for b in blocks]))


def cholqr2_r(X) -> tuple[np.ndarray, int]:
    """Q-less CholQR2 (Alg. 1).  Returns (R, info); info = j or n+j on a
    non-positive pivot in the first or second Cholesky (R is NaN then)."""
    X, m, n, ldx = _as_rowmajor(X)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_cholqr2_r(_ptr(X), m, n, ldx, _ptr(R))
    if rc < 0:
        raise RuntimeError("oracle_cholqr2_r failed: %d" % rc)
    return R, rc


def shifted_cholqr3_r(X) -> tuple[np.ndarray, int]:
    """Q-less shifted CholQR3.  Returns (R, info); info = j, n+j or 2n+j on a
    non-positive pivot in the shifted or one of the two later Choleskys."""
    X, m, n, ldx = _as_rowmajor(X)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_shifted_cholqr3_r(_ptr(X), m, n, ldx, _ptr(R))
    if rc < 0:
        raise RuntimeError("oracle_shifted_cholqr3_r failed: %d" % rc)
    return R, rc


def svqb2(X, trunc_tol: float | None = None) -> tuple[np.ndarray, np.ndarray, np.ndarray, int]:
    """Q-less SVQB2.  Returns (Z, sigma, R, ntrunc) with X = Q Z, Q^T Q = I,
    sigma the first-pass singular-value estimates and R = qr_R(Z)."""
    X, m, n, ldx = _as_rowmajor(X)
    if trunc_tol is None:
        trunc_tol = n * 2.0 ** -52
    Z = np.empty((n, n), dtype=np.float64)
    sig = np.empty(n, dtype=np.float64)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_svqb2(_ptr(X), m, n, ldx, float(trunc_tol), _ptr(Z), _ptr(sig), _ptr(R))
    if rc < 0:
        raise RuntimeError("oracle_svqb2 failed: %d" % rc)
    return Z, sig, R, rc


def jacobi_eig(A) -> tuple[np.ndarray, np.ndarray, int]:
    """Cyclic-Jacobi eigendecomposition of a symmetric matrix:
    returns (w decreasing, V with eigenvectors as columns, sweeps)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.empty(n, dtype=np.float64)
    V = np.empty((n, n), dtype=np.float64)
    sweeps = _load().oracle_jacobi_eig(_ptr(A), n, _ptr(w), _ptr(V))
    if sweeps < 0:
        raise RuntimeError("oracle_jacobi_eig failed")
    return w, V, sweeps


def lstsq_from_r(Rt) -> tuple[np.ndarray, float]:
    """x and |rho| from R([A b]) ((n+1) x (n+1))."""
    Rt = np.ascontiguousarray(Rt, dtype=np.float64)
    n = Rt.shape[0] - 1
    x = np.empty(n, dtype=np.float64)
    res = np.empty(1, dtype=np.float64)
    rc = _load().oracle_lstsq_from_r(_ptr(Rt), n, n + 1, _ptr(x), _ptr(res))
    if rc != 0:
        raise RuntimeError("oracle_lstsq_from_r: singular R_A at %d" % rc)
    return x, float(res[0])


def q_from_r(X, R) -> np.ndarray:
    """Q = X R^{-1} (forward substitution per row); raises if R is singular."""
    X, m, n, ldx = _as_rowmajor(X)
    R = np.ascontiguousarray(R, dtype=np.float64)
    Q = np.empty((m, n), dtype=np.float64)
    rc = _load().oracle_q_from_r(_ptr(X), m, n, ldx, _ptr(R), n, _ptr(Q), n)
    if rc != 0:
        raise RuntimeError("oracle_q_from_r failed: %d" % rc)
    return Q


def two_phase_r(Y, X) -> tuple[np.ndarray, np.ndarray]:
    """(B, R): B = Y^T X and R = R((I - Y Y^T) X) for Y (m x p) with
    orthonormal columns."""
    X, m, n, ldx = _as_rowmajor(X)
    Y = np.ascontiguousarray(Y, dtype=np.float64).reshape(m, -1)
    p = Y.shape[1]
    B = np.empty((max(p, 1), n), dtype=np.float64)
    R = np.empty((n, n), dtype=np.float64)
    rc = _load().oracle_two_phase_r(_ptr(Y), p, max(p, 1), _ptr(X), m, n, ldx, _ptr(B), _ptr(R))
    if rc != 0:
        raise RuntimeError("oracle_two_phase_r failed: %d" % rc)
    return B[:p], R


def gram_dot2(X) -> np.ndarray:
    """X^T X with each entry accurate to about twice working precision."""
    X, m, n, ldx = _as_rowmajor(X)
    C = np.empty((n, n), dtype=np.float64)
    _load().oracle_gram_dot2(_ptr(X), m, n, ldx, _ptr(C))
    return C


# ----------------------------------------------------------- error metrics

def rel_err_r(R, R_ref) -> float:
    """e_R = ||R - R_ref||_F / ||R_ref||_F (0 when both are zero)."""
    R = np.asarray(R, dtype=np.float64)
    R_ref = np.asarray(R_ref, dtype=np.float64)
    d = np.linalg.norm(R - R_ref)
    nr = np.linalg.norm(R_ref)
    return float(d / nr) if nr > 0 else float(d)


def row_scaled_err(R, R_ref, floor: float = 0.0) -> float:
    """max over i, j of |R - R_ref|_ij / max(|R_ref|_ii, floor): each row's
    error against that row's own scale, so a wrong small trailing row is seen
    even where the normwise e_R is dominated by the large leading rows.  The
    floor bounds the scale from below where a row is small only because the
    input is ill-conditioned relative to its largest column (a backward
    stable R has errors of about u times the largest column norm in every
    row); with floor = 1e-4 * max_j ||x_j||, rows are judged as if kappa were
    at most 1e4.  Rows whose scale is zero are left out (rank-deficient
    inputs)."""
    R = np.asarray(R, dtype=np.float64)
    R_ref = np.asarray(R_ref, dtype=np.float64)
    d = np.maximum(np.abs(np.diag(R_ref)), float(floor))
    ok = d > 0
    if not ok.any():
        return 0.0
    return float(np.max(np.abs(R - R_ref)[ok] / d[ok, None]))


def col_norm_max(X) -> float:
    """Largest column 2-norm of X (the scale of the backward error of R)."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.sqrt(np.max(np.einsum("ij,ij->j", X, X)))) if X.size else 0.0


def gram_residual(X, R, G=None) -> float:
    """e_G = ||X^T X - R^T R||_F / ||X||_2^2, with X^T X from Dot2 (pass G to
    reuse it) and ||X||_2^2 = largest eigenvalue of that Gram matrix."""
    if G is None:
        G = gram_dot2(X)
    R = np.asarray(R, dtype=np.float64)
    w = np.linalg.eigvalsh(G)
    scale = float(w[-1]) if w.size and w[-1] > 0 else 1.0
    return float(np.linalg.norm(G - R.T @ R) / scale)
