"""Writes the stored expected values under tests/golden/ (run from the
repository root: python tests/golden/make_golden.py).  Nothing here uses the
HIP library.

tiny_exact_r.txt -- a 9 x 3 matrix with small dyadic entries and its R by
    the definition of Sec. 1 (X = QR, R upper triangular with a positive
    diagonal, so R^T R = X^T X): the exact rational Gram matrix and a
    Cholesky factorisation in 60-digit decimals, rounded to FP64.
config1_r.txt -- the R of the 100000 x 4 iid N(0,1) workload (seed 1) by
    the CPU oracle's Householder QR (diag >= 0).
"""
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle          # noqa: E402
import workloads as wl  # noqa: E402

TINY = [[3, -1, 2], [0.5, 4, -2], [-1, 0.25, 1], [2, 2, -0.5], [0, -3, 1.5],
        [1, 0, 0], [-0.75, 1, 2], [4, -2, 0.125], [1, 1, 1]]


def exact_r(X, digits=60):
    getcontext().prec = digits
    m, n = len(X), len(X[0])
    F = [[Fraction(v) for v in row] for row in X]
    G = [[sum((F[i][a] * F[i][b] for i in range(m)), Fraction(0)) for b in range(n)] for a in range(n)]
    Gd = [[Decimal(g.numerator) / Decimal(g.denominator) for g in row] for row in G]
    R = [[Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        R[j][j] = (Gd[j][j] - sum((R[k][j] * R[k][j] for k in range(j)), Decimal(0))).sqrt()
        for c in range(j + 1, n):
            R[j][c] = (Gd[j][c] - sum((R[k][j] * R[k][c] for k in range(j)), Decimal(0))) / R[j][j]
    return [[float(v) for v in row] for row in R]


def write(path, header, arrays):
    with open(path, "w") as f:
        for line in header.strip().splitlines():
            f.write("# " + line + "\n")
        for name, A in arrays:
            A = np.atleast_2d(np.asarray(A, dtype=np.float64))
            f.write("%s %d %d\n" % (name, A.shape[0], A.shape[1]))
            for row in A:
                f.write(" ".join("%.17g" % v for v in row) + "\n")


def main():
    write(os.path.join(HERE, "tiny_exact_r.txt"),
          "R of X by the definition of Sec. 1 (R^T R = X^T X, upper triangular, positive diagonal),\n"
          "exact rational Gram + 60-digit Cholesky, rounded to FP64.  Made by tests/golden/make_golden.py.",
          [("X", TINY), ("R", exact_r(TINY))])
    write(os.path.join(HERE, "config1_r.txt"),
          "R of the 100000 x 4 iid N(0,1) workload (seed 1) by the CPU oracle's Householder QR\n"
          "(Sec. 1, diag >= 0).  Made by tests/golden/make_golden.py.",
          [("R", oracle.householder_r(wl.config1()))])


if __name__ == "__main__":
    main()
