"""GPU parity of the Gram matrix accumulated in twice the working precision
(qless_gram with C_lo) and of Cholesky-QR2 on it (cholqr2_dd_r), the
higher-precision Gramian Sec. 2 cites as the way past Cholesky-QR's
condition-number limit.

The Gram matrix is compared with the oracle's Dot2 Gram (pinned to the exact
rational X^T X): both are accurate to about u |G| plus m u^2 |X|^T |X|, so
they must agree to 4 u |G| + 4 m u^2 (|X|^T |X|) entrywise; inputs are chosen
so that many entries cancel (|G_ij| much smaller than (|X|^T |X|)_ij), where
a plain FP64 sum would miss this bar by orders of magnitude (checked on the
same data).  cholqr2_dd_r is compared with the Householder oracle: e_R <=
1e-12 (row-scaled <= e_row(n)) at kappa <= 1e4, and at kappa = 1e10 .. 1e13 it
completes where cholqr2_r breaks down, with a Gram residual <= 1e-13 and
e_R <= 1e-12 against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl
from tolerances import e_row

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def cancelling(m, n, seed):
    """Columns nearly orthogonal to each other: off-diagonal Gram entries
    are small sums of large terms."""
    X = wl.orthonormal_columns(m, n, wl.rng(seed)) * np.sqrt(m)
    X[:, 0] += 1e-3 * wl.gaussian(m, 1, seed + 1)[:, 0]
    return X


@pytest.mark.parametrize("m,n", [(50_000, 1), (40_000, 3), (100_000, 8), (30_000, 13), (70_000, 16), (20_000, 32),
                                 (9_000, 47), (12_000, 64), (3_000_000, 8), (0, 5)])
def test_dd_gram_matches_dot2_oracle(gpu, m, n):
    print("case dd gram m=%d n=%d" % (m, n), flush=True)
    X = cancelling(m, n, seed=m + n) if m >= n else np.zeros((m, n))
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(gpu)
    Ch, Cl = q.qless_gram(Xd, double_double=True)
    Cp, _ = q.qless_gram(Xd)
    torch.cuda.synchronize(gpu)
    Ch, Cl, Cp = Ch.cpu().numpy(), Cl.cpu().numpy(), Cp.cpu().numpy()
    Go = oracle.gram_dot2(X)
    A = np.abs(X).T @ np.abs(X)
    bound = 4 * U * np.abs(Go) + 4 * max(m, 1) * U * U * A
    assert np.all(np.abs(Ch - Go) <= bound)
    assert np.all(np.abs(Cl) <= 2 * U * np.abs(Ch) + 1e-300)        # normalised (hi, lo) pairs
    assert np.array_equal(Ch, Ch.T) and np.array_equal(Cl, Cl.T)
    if m >= 1000 and n > 1:
        assert not np.all(np.abs(Cp - Go) <= bound)                   # the FP64 sum misses this bar


@pytest.mark.parametrize("m,n", [(20000, 4), (100_000, 8), (30000, 16), (20000, 32), (9000, 47), (12000, 64)])
def test_cholqr2_dd_matches_oracle(gpu, m, n):
    print("case cholqr2_dd m=%d n=%d" % (m, n), flush=True)
    X, R0 = wl.known_r(m, n, wl.logspace_sigma(n, 4), seed=m + 11 * n)
    R, info = q.cholqr2_dd_r(torch.from_numpy(X).to(gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    R = R.cpu().numpy()
    Ro = oracle.householder_r(X)
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0.0)
    assert oracle.rel_err_r(R, Ro) <= 1e-12
    assert oracle.row_scaled_err(R, Ro, 1e-4 * oracle.col_norm_max(X)) <= e_row(X.shape[1])
    assert oracle.gram_residual(X, R) <= 1e-13


@pytest.mark.parametrize("m,n,k", [(20000, 8, 10), (30000, 16, 12), (12000, 48, 11), (9000, 64, 10),
                                   (50000, 8, 13)])
def test_cholqr2_dd_beyond_cholqr2(gpu, m, n, k):
    print("case cholqr2_dd kappa=1e%d m=%d n=%d" % (k, m, n), flush=True)
    X = wl.svd_form(m, n, wl.logspace_sigma(n, k), seed=800 + n + k)
    Xd = torch.from_numpy(X).to(gpu)
    _, info2 = q.cholqr2_r(Xd)
    R, info = q.cholqr2_dd_r(Xd)
    torch.cuda.synchronize(gpu)
    assert int(info2.item()) != 0
    assert int(info.item()) == 0
    R = R.cpu().numpy()
    assert oracle.gram_residual(X, R) <= 1e-13
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= 1e-12


def test_cholqr2_dd_breakdown(gpu):
    X = wl.gaussian(4000, 6, seed=2)
    X[:, 3] = 0.0
    R, info = q.cholqr2_dd_r(torch.from_numpy(X).to(gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 4
    assert torch.isnan(R).all()
