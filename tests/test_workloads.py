"""The seeded input generators (no GPU): shapes, determinism and the
structure the tests rely on -- prescribed singular values, orthonormal
factors, a known R, the Poisson request stream and the batched shapes."""
import numpy as np
import pytest

import workloads as wl


@pytest.mark.parametrize("n,k", [(1, 0), (6, 4), (16, 8), (32, 12)])
def test_svd_form_has_the_prescribed_singular_values(n, k):
    sig = wl.logspace_sigma(n, k)
    X = wl.svd_form(500, n, sig, seed=3)
    s = np.linalg.svd(X, compute_uv=False)
    assert np.max(np.abs(s - sig) / sig) <= 1e-12 * max(1.0, 10.0 ** (k - 4))
    assert np.array_equal(X, wl.svd_form(500, n, sig, seed=3))          # seeded


def test_svd_form_spreads_ill_conditioning_over_columns():
    """Column-scaled condition stays near kappa (unlike a graded R0)."""
    n, k = 8, 8
    X = wl.svd_form(2000, n, wl.logspace_sigma(n, k), seed=5)
    D = np.linalg.norm(X, axis=0)
    assert np.linalg.cond(X / D) >= 1e-2 * 10.0 ** k


@pytest.mark.parametrize("n,k", [(4, 0), (8, 4), (12, 8)])
def test_known_r_structure(n, k):
    X, R0 = wl.known_r(700, n, wl.logspace_sigma(n, k), seed=11)
    assert np.all(np.tril(R0, -1) == 0.0) and np.all(np.diag(R0) >= 0.0)
    s = np.linalg.svd(R0, compute_uv=False)
    assert np.max(np.abs(s - wl.logspace_sigma(n, k)) / wl.logspace_sigma(n, k)) <= 1e-10
    Q = np.linalg.solve(R0.T, X.T).T
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 1e-12 * max(1.0, 10.0 ** k)


def test_orthonormal_columns():
    Q = wl.orthonormal_columns(300, 7, wl.rng(1))
    assert np.linalg.norm(Q.T @ Q - np.eye(7)) <= 1e-14


def test_server_requests_stream():
    reqs = wl.server_requests(200, rate_per_s=50.0, seed=5)
    t = np.array([r["arrival_s"] for r in reqs])
    assert np.all(np.diff(t) > 0)
    assert 0.5 * 200 / 50.0 < t[-1] < 2.0 * 200 / 50.0                   # Poisson at 50 / s
    ms = np.array([r["m"] for r in reqs])
    ns = np.array([r["n"] for r in reqs])
    assert ms.min() >= 1e4 and ms.max() <= 5e7 and ns.min() >= 3 and ns.max() <= 47
    assert len({r["seed"] for r in reqs}) == len(reqs)


def test_batched_shapes():
    sh = wl.batched_shapes(512, seed=4)
    assert len(sh) == 512
    assert {n for _, n in sh} <= {4, 8, 16, 32}
    assert min(m for m, _ in sh) >= 1e4 and max(m for m, _ in sh) <= 1e7
    assert sh == wl.batched_shapes(512, seed=4)
