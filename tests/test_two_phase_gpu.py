"""GPU parity of the one-pass two-phase orthogonalisation (Sec. 2: Q R =
(I - Y Y^T) X against an orthonormal Y, with B = Y^T X) against the CPU
oracle, which forms B by pairwise sums, Z = X - Y B row by row and R(Z) by
plain Householder.  The GPU runs one Q-less TSQR over [Y X] read from the two
pointers.

Bar: e_R(R, R_oracle) <= 1e-12 and the row-scaled error <= e_row(p + n) (as for
qless_tsqr_r, rows judged at kappa <= 1e4 relative to X's largest column,
whose part in span(Y) makes it larger than R's) at kappa(R0) <= 1e4 on inputs X = Y B0 + W R0 with [Y W]
orthonormal, where the projected part is not small against X; B within
1e-13 of the oracle's relative to ||X||_F (both are Y^T X up to rounding;
the GPU's B is Q1^T X with Q1 = Y R11^{-1} and R11 = I + O(u))."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl
from tolerances import e_row

pytestmark = pytest.mark.gpu

E_R = 1e-12
E_B = 1e-13


def run(Y, X, dev):
    B, R = q.qless_two_phase_r(torch.from_numpy(np.ascontiguousarray(Y)).to(dev),
                               torch.from_numpy(np.ascontiguousarray(X)).to(dev))
    torch.cuda.synchronize(dev)
    return B.cpu().numpy(), R.cpu().numpy()


def check(Y, X, B, R):
    Bo, Ro = oracle.two_phase_r(Y, X)
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
    assert oracle.rel_err_r(R, Ro) <= E_R, oracle.rel_err_r(R, Ro)
    assert oracle.row_scaled_err(R, Ro, 1e-4 * oracle.col_norm_max(X)) <= e_row(Y.shape[1] + X.shape[1])
    if Y.shape[1]:
        assert np.linalg.norm(B - Bo) <= E_B * np.linalg.norm(X), np.linalg.norm(B - Bo) / np.linalg.norm(X)
    return Bo, Ro


# (m, p, n, kappa exponent): total widths p + n across every kernel layout
# (cross-lane fold for p + n <= 16, column groups above), ragged row counts
CASES = [(3000, 1, 1, 0), (20000, 3, 4, 2), (50000, 4, 4, 4), (777, 2, 6, 1), (40000, 8, 8, 4), (65537, 5, 11, 3),
         (30000, 16, 8, 3), (20000, 8, 24, 4), (12345, 32, 16, 3), (9000, 16, 47, 2), (10000, 48, 16, 4),
         (70000, 1, 63, 2), (5000, 63, 1, 0), (20000, 20, 28, 3), (300_001, 10, 35, 2)]


@pytest.mark.parametrize("m,p,n,k", CASES)
def test_two_phase_matches_oracle(gpu, m, p, n, k):
    print("case two-phase m=%d p=%d n=%d k=%d" % (m, p, n, k), flush=True)
    Y, X, B0, R0 = wl.two_phase_data(m, p, n, k, seed=m + 10 * p + n)
    B, R = run(Y, X, gpu)
    check(Y, X, B, R)
    assert np.linalg.norm(B - B0) <= 1e-12 * np.linalg.norm(B0)
    assert oracle.rel_err_r(R, R0) <= E_R


def test_two_phase_full_size_multi_level(gpu):
    """Every wavefront of the stage-1 grid folds several panels and the tree
    has levels (the path large inputs take)."""
    m, p, n = 3_000_000, 8, 8
    print("case two-phase full size m=%d p=%d n=%d" % (m, p, n), flush=True)
    Y, X, B0, R0 = wl.two_phase_data(m, p, n, 4, seed=11)
    B, R = run(Y, X, gpu)
    check(Y, X, B, R)


def test_two_phase_empty_basis_is_plain_tsqr(gpu):
    X = wl.gaussian(40000, 9, seed=3)
    B, R = q.qless_two_phase_r(torch.zeros((40000, 0), dtype=torch.float64, device=gpu),
                               torch.from_numpy(X).to(gpu))
    torch.cuda.synchronize(gpu)
    assert B.shape == (0, 9)
    assert oracle.rel_err_r(R.cpu().numpy(), oracle.householder_r(X)) <= E_R


def test_two_phase_coordinate_basis(gpu):
    """Y = [e_1 e_2]: B is the first two rows of X, R the R of the rest."""
    X = wl.gaussian(5000, 5, seed=8)
    Y = np.zeros((5000, 2))
    Y[0, 0] = Y[1, 1] = 1.0
    B, R = run(Y, X, gpu)
    Bo, Ro = check(Y, X, B, R)
    assert np.allclose(B, X[:2], rtol=0, atol=1e-15 * np.abs(X).max())


def test_two_phase_x_in_span_of_y(gpu):
    g = wl.rng(7)
    Y = wl.orthonormal_columns(20000, 4, g)
    X = Y @ g.standard_normal((4, 3))
    B, R = run(Y, X, gpu)
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(X)


def test_two_phase_argument_errors(gpu):
    Y = torch.zeros((100, 40), dtype=torch.float64, device=gpu)
    X = torch.zeros((100, 30), dtype=torch.float64, device=gpu)
    with pytest.raises(q.QlessError):
        q.qless_two_phase_r(Y, X)           # p + n = 70 > 64
    with pytest.raises(ValueError):
        q.qless_two_phase_r(Y[:50], X)      # row counts differ


# Enough rows that every stage-1 wavefront folds at least four full panels,
# so the lane-private fold of the narrow widths (p + n <= 8) runs, with its
# partial last panel; Y orthonormal, X iid N(0, 1), checked against the oracle.
@pytest.mark.parametrize("m,p,n", [(2_100_000, 4, 4), (4_300_000, 1, 3), (3_300_000, 2, 5)])
def test_two_phase_lane_private(gpu, m, p, n):
    print("case two-phase lane-private m=%d p=%d n=%d" % (m, p, n), flush=True)
    Y = wl.orthonormal_columns(m, p, wl.rng(m + p))
    X = wl.gaussian(m, n, seed=m + n)
    B, R = run(Y, X, gpu)
    check(Y, X, B, R)
