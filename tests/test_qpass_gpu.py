"""GPU parity of the explicit-Q passes against the CPU oracle.

qless_q_from_r: Q = X R^{-1} rebuilt from X and its Q-less R (Sec. 1).  The
GPU gets the oracle's own R, so both sides compute Q from identical inputs;
the oracle solves q R = x row by row (forward substitution), the GPU
multiplies by R^{-1} formed once.  Bar: every column of Q within 1e-11 of
the oracle's, relative to the column's norm, at kappa <= 1e4 (u * kappa * n
* 15 at n = 64; the two methods on the CPU differ by up to 1.5e-13 there),
and Q^T Q = I as far as the oracle's own Q is orthonormal.

svqb_q: X = Q Z with Q = X D1 D2 (the variant of Sec. 4.6 that stores Q).
Q is unique only up to a right orthogonal factor (as Z is up to a left
one), so it is checked through Q Z = X, Q^T Q = I and Q_oracle^T Q being
orthogonal.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl

pytestmark = pytest.mark.gpu

E_Q = 1e-11

SHAPES = [(1000, 1), (5000, 2), (777, 3), (20000, 4), (3333, 5), (100_000, 8), (40000, 13), (65537, 16),
          (30000, 17), (20000, 32), (9000, 47), (12000, 64), (70, 64)]


def col_err(Q, Qo):
    return float(np.max(np.linalg.norm(Q - Qo, axis=0) / np.linalg.norm(Qo, axis=0)))


def check_q_from_r(X, dev):
    m, n = X.shape
    Ro = oracle.householder_r(X)
    Qo = oracle.q_from_r(X, Ro)
    Q, info = q.qless_q_from_r(torch.from_numpy(np.ascontiguousarray(X)).to(dev), torch.from_numpy(Ro).to(dev))
    torch.cuda.synchronize(dev)
    assert int(info.item()) == 0
    Q = Q.cpu().numpy()
    assert col_err(Q, Qo) <= E_Q, col_err(Q, Qo)
    if m >= n:
        e_orth_o = np.linalg.norm(oracle.gram_dot2(Qo) - np.eye(n))
        assert np.linalg.norm(oracle.gram_dot2(Q) - np.eye(n)) <= 2 * e_orth_o + 1e-14
    return Q


@pytest.mark.parametrize("m,n", SHAPES)
def test_q_from_r_matches_oracle(gpu, m, n):
    print("case q_from_r m=%d n=%d" % (m, n), flush=True)
    X, _ = wl.known_r(m, n, wl.logspace_sigma(n, 4), seed=m + 7 * n) if m >= n else (wl.gaussian(m, n, 3), None)
    check_q_from_r(X, gpu)


# The streaming pass's full-size path: every wavefront of the 8-per-CU grid
# streams several full stages (see the Gram tests), with a ragged last one.
@pytest.mark.parametrize("n,rpw", [(8, 2048), (4, 4096), (16, 448), (13, 448), (32, 256), (48, 192), (64, 128),
                                   (61, 128)])
def test_q_from_r_full_size_path(gpu, n, rpw):
    cus = torch.cuda.get_device_properties(gpu).multi_processor_count
    m = cus * 8 * rpw - 40
    print("case q_from_r full path m=%d n=%d" % (m, n), flush=True)
    X, _ = wl.known_r(m, n, wl.logspace_sigma(n, 4), seed=500 + n)
    check_q_from_r(X, gpu)


def test_q_from_r_padded_layouts(gpu):
    """ldx > n and ldq > n (views into wider buffers); the padding of Q is
    left untouched."""
    X = wl.gaussian(30000, 6, seed=7)
    Ro = oracle.householder_r(X)
    Xb = torch.zeros((30000, 9), dtype=torch.float64, device=gpu)
    Xb[:, :6] = torch.from_numpy(X).to(gpu)
    Qb = torch.full((30000, 10), 5.0, dtype=torch.float64, device=gpu)
    Q, info = q.qless_q_from_r(Xb[:, :6], torch.from_numpy(Ro).to(gpu), Q=Qb[:, :6])
    torch.cuda.synchronize(gpu)
    assert col_err(Qb[:, :6].cpu().numpy(), oracle.q_from_r(X, Ro)) <= E_Q
    assert torch.all(Qb[:, 6:] == 5.0)


def test_q_from_r_end_to_end_with_gpu_r(gpu):
    """The whole use of Sec. 1: Q-less TSQR on the GPU, then Q from its R:
    Q R = X and Q^T Q = I."""
    X, _ = wl.known_r(200_000, 12, wl.logspace_sigma(12, 2), seed=12)
    Xd = torch.from_numpy(X).to(gpu)
    R = q.qless_tsqr_r(Xd)
    Q, info = q.qless_q_from_r(Xd, R)
    torch.cuda.synchronize(gpu)
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    assert np.linalg.norm(Q @ R - X) <= 1e-14 * np.linalg.norm(X)
    assert np.linalg.norm(oracle.gram_dot2(Q) - np.eye(12)) <= 1e-13


def test_q_from_r_singular(gpu):
    X = wl.gaussian(5000, 5, seed=1)
    R = np.triu(wl.gaussian(5, 5, seed=2))
    R[3, 3] = 0.0
    Q, info = q.qless_q_from_r(torch.from_numpy(X).to(gpu), torch.from_numpy(R).to(gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 4
    assert torch.isnan(Q).all()


@pytest.mark.parametrize("m,n", [(20000, 4), (100_000, 8), (30000, 16), (9000, 33), (12000, 64), (500, 7)])
def test_svqb_q(gpu, m, n):
    print("case svqb_q m=%d n=%d" % (m, n), flush=True)
    X, _ = wl.known_r(m, n, wl.logspace_sigma(n, 3), seed=3 * m + n)
    Q, Z, sig, info = q.svqb_q(torch.from_numpy(X).to(gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    Q, Z = Q.cpu().numpy(), Z.cpu().numpy()
    assert np.linalg.norm(Q @ Z - X) <= 1e-13 * np.linalg.norm(X)
    assert np.linalg.norm(oracle.gram_dot2(Q) - np.eye(n)) <= 1e-13
    Zo, sig_o, _, nt = oracle.svqb2(X)
    assert nt == 0
    Qo = X @ np.linalg.inv(Zo)
    W = Qo.T @ Q                     # orthogonal when Q = Qo W
    assert np.linalg.norm(W.T @ W - np.eye(n)) <= 1e-10
    assert np.linalg.norm(Qo @ W - Q) <= 1e-10 * np.linalg.norm(Q)
    assert np.max(np.abs(sig.cpu().numpy() - sig_o) / sig_o.max()) <= 1e-12
