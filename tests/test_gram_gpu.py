"""GPU parity of the Gram-based comparison forms and the least-squares finish.

cholqr2_r (Alg. 1) and svqb (SVQB2, Sec. 1 / Sec. 3.1) are compared with the
CPU oracle's CholQR2 / SVQB2 and with its Householder R on identical seeded
inputs: e_R <= 1e-12 at kappa <= 1e4, Gram residual <= 1e-13.  Z of the QZ
form is unique only up to a left orthogonal factor, so it is checked through
Z^T Z = X^T X and qr_R(Z) = R(X).
"""
import numpy as np
import pytest
import scipy.linalg as sla
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl
from tolerances import e_row

pytestmark = pytest.mark.gpu

E_R = 1e-12
E_G = 1e-13

SHAPES = [(1000, 1), (5000, 2), (777, 3), (20000, 4), (3333, 5), (100_000, 8), (40000, 13), (65537, 16),
          (30000, 17), (20000, 32), (9000, 47), (12000, 64)]


def dev_tensor(X, dev):
    return torch.from_numpy(np.ascontiguousarray(X)).to(dev)


@pytest.mark.parametrize("m,n", SHAPES)
def test_cholqr2_matches_oracle(gpu, m, n):
    print("case cholqr2 m=%d n=%d" % (m, n), flush=True)
    X, R0 = wl.known_r(m, n, wl.logspace_sigma(n, 3), seed=m + 3 * n)
    R, info = q.cholqr2_r(dev_tensor(X, gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    R = R.cpu().numpy()
    Ro, info_o = oracle.cholqr2_r(X)
    assert info_o == 0
    assert oracle.rel_err_r(R, Ro) <= E_R
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= E_R
    assert oracle.gram_residual(X, R) <= E_G
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0.0)


def test_cholqr2_postcondition(gpu):
    """Alg. 1 ENSURE: (X R^{-1})^T (X R^{-1}) = I."""
    X, _ = wl.known_r(50_000, 12, wl.logspace_sigma(12, 4), seed=4)
    R, info = q.cholqr2_r(dev_tensor(X, gpu))
    R = R.cpu().numpy()
    Qm = sla.solve_triangular(R, X.T, trans="T", lower=False).T
    assert np.linalg.norm(oracle.gram_dot2(Qm) - np.eye(12)) <= 1e-13


def test_cholqr2_breakdown(gpu):
    X = wl.gaussian(4000, 6, seed=2)
    X[:, 3] = 0.0
    R, info = q.cholqr2_r(dev_tensor(X, gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 4
    assert torch.isnan(R).all()


def test_cholqr2_empty_breaks_down(gpu):
    R, info = q.cholqr2_r(torch.zeros((0, 3), dtype=torch.float64, device=gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 1


@pytest.mark.parametrize("m,n", SHAPES)
def test_shifted_cholqr3_matches_oracle(gpu, m, n):
    print("case shifted cholqr3 m=%d n=%d" % (m, n), flush=True)
    X, R0 = wl.known_r(m, n, wl.logspace_sigma(n, 3), seed=m + 5 * n)
    R, info = q.shifted_cholqr3_r(dev_tensor(X, gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    R = R.cpu().numpy()
    Ro, info_o = oracle.shifted_cholqr3_r(X)
    assert info_o == 0
    assert oracle.rel_err_r(R, Ro) <= E_R
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= E_R
    assert oracle.gram_residual(X, R) <= E_G
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) > 0.0)


@pytest.mark.parametrize("m,n,k", [(20000, 8, 10), (30000, 16, 12), (12000, 48, 10), (9000, 64, 11)])
def test_shifted_cholqr3_beyond_cholqr2(gpu, m, n, k):
    """kappa = 10^k spread over all columns: CholQR2 breaks down on the
    device, the shifted variant completes with a backward-stable R."""
    print("case shifted cholqr3 kappa=1e%d m=%d n=%d" % (k, m, n), flush=True)
    X = wl.svd_form(m, n, wl.logspace_sigma(n, k), seed=700 + n + k)
    Xd = dev_tensor(X, gpu)
    _, info2 = q.cholqr2_r(Xd)
    R, info = q.shifted_cholqr3_r(Xd)
    torch.cuda.synchronize(gpu)
    assert int(info2.item()) != 0
    assert int(info.item()) == 0
    R = R.cpu().numpy()
    assert oracle.gram_residual(X, R) <= E_G
    assert oracle.rel_err_r(R, oracle.householder_r(X)) <= E_R


def test_shifted_cholqr3_zero_matrix_breaks_down(gpu):
    R, info = q.shifted_cholqr3_r(torch.zeros((500, 3), dtype=torch.float64, device=gpu))
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 1
    assert torch.isnan(R).all()


@pytest.mark.parametrize("m,n", SHAPES)
def test_svqb_r_mode_matches_oracle(gpu, m, n):
    print("case svqb-R m=%d n=%d" % (m, n), flush=True)
    X, R0 = wl.known_r(m, n, wl.logspace_sigma(n, 3), seed=2 * m + n)
    Rg, sig, info = q.svqb(dev_tensor(X, gpu), out=q.QLESS_SVQB_R)
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    Rg = Rg.cpu().numpy()
    Zo, sig_o, Ro, nt = oracle.svqb2(X)
    assert nt == 0
    assert oracle.rel_err_r(Rg, Ro) <= E_R
    assert oracle.rel_err_r(Rg, oracle.householder_r(X)) <= E_R
    assert oracle.gram_residual(X, Rg) <= E_G
    assert np.max(np.abs(sig.cpu().numpy() - sig_o) / sig_o.max()) <= 1e-12


@pytest.mark.parametrize("m,n", [(20000, 4), (100_000, 8), (30000, 16), (9000, 33), (12000, 64)])
def test_svqb_qz_mode(gpu, m, n):
    X, _ = wl.known_r(m, n, wl.logspace_sigma(n, 2), seed=m + n)
    Z, sig, info = q.svqb(dev_tensor(X, gpu), out=q.QLESS_SVQB_QZ)
    torch.cuda.synchronize(gpu)
    Z = Z.cpu().numpy()
    G = oracle.gram_dot2(X)
    assert np.linalg.norm(Z.T @ Z - G) <= 1e-13 * np.linalg.norm(G)
    assert oracle.rel_err_r(oracle.householder_r(Z), oracle.householder_r(X)) <= E_R
    # Z is unique only up to a left orthogonal factor (the second-pass Gram
    # matrix is close to I, so its eigenvectors are arbitrary): Z = W Zo with
    # W orthogonal.
    Zo, _, _, _ = oracle.svqb2(X)
    W = Z @ np.linalg.inv(Zo)
    assert np.linalg.norm(W.T @ W - np.eye(n)) <= 1e-10


def test_svqb_truncation_counts(gpu):
    X = wl.gaussian(8000, 5, seed=21)
    X[:, 1] = 0.0
    Z, sig, info = q.svqb(dev_tensor(X, gpu), out=q.QLESS_SVQB_QZ)
    torch.cuda.synchronize(gpu)
    _, _, _, nt = oracle.svqb2(X)
    assert int(info.item()) == nt >= 1


@pytest.mark.parametrize("n", [1, 3, 10, 47])
def test_lstsq_finish_matches_oracle(gpu, n):
    """Sec. 1: Q-less TSQR of [A b], then back substitution on the device."""
    Ab, x0 = wl.ls_request_data(30000, n, seed=n)
    Rt = q.qless_tsqr_r(dev_tensor(Ab, gpu))
    x, res, info = q.qless_lstsq_finish(Rt)
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0
    Rt_h = Rt.cpu().numpy()
    xo, reso = oracle.lstsq_from_r(Rt_h)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-13 * np.linalg.norm(xo)
    assert abs(float(res.item()) - reso) <= 1e-14 * reso
    xl, *_ = np.linalg.lstsq(Ab[:, :n], Ab[:, n], rcond=None)
    assert np.linalg.norm(x.cpu().numpy() - xl) <= 1e-10 * np.linalg.norm(xl)


@pytest.mark.slow
def test_config2_full_size_gram_forms(gpu):
    print("case config2 full size cholqr2/svqb", flush=True)
    X, R0 = wl.config2(device=gpu)
    R1, info = q.cholqr2_r(X)
    R2, sig, info2 = q.svqb(X, out=q.QLESS_SVQB_R)
    torch.cuda.synchronize(gpu)
    assert int(info.item()) == 0 and int(info2.item()) == 0
    assert oracle.rel_err_r(R1.cpu().numpy(), R0) <= E_R
    assert oracle.rel_err_r(R2.cpu().numpy(), R0) <= E_R


# Full-size code path of the Gram kernels.  The plan gives each of the
# 8 * CUs wavefronts a contiguous range of rows, rounded to whole slabs; at
# the sizes above every wavefront holds a single stage, so only the guarded
# tail loader runs.  Here m is chosen per kernel width so that every
# wavefront streams several full stages through the unguarded,
# double-buffered loop (the path the benchmark sizes take), and the last
# wavefront also ends in a partial stage.  Stage heights: 16 * (8, 4, 2, 1)
# rows for 1..4 blocks of 16 columns; the row kernel for n <= 8 uses panels
# of 64 * 64 / n rows (64 * 32 / n with the fused multiply).
FULL_PATH = [
    # (n, rows per wavefront): 16-column blocks NB = ceil(n / 16)
    (16, 448), (13, 448),          # NB = 1: three 128-row stages + a 64-row tail
    (32, 256), (30, 256),          # NB = 2: four 64-row stages
    (48, 192), (47, 192),          # NB = 3: six 32-row stages
    (64, 128), (61, 128),          # NB = 4: eight 16-row stages
    (8, 2048), (3, 4096), (2, 4096), (1, 8192),   # row kernel: four full panels of pass 1
]


def full_path_matrix(gpu, n, rpw, seed):
    cus = torch.cuda.get_device_properties(gpu).multi_processor_count
    m = cus * 8 * rpw - 40
    X, R0 = wl.known_r(m, n, wl.logspace_sigma(n, 3), seed=seed)
    return X, R0, m


def check_gram_r(X, R, Ro):
    assert oracle.rel_err_r(R, Ro) <= E_R
    assert oracle.row_scaled_err(R, Ro, 1e-4 * oracle.col_norm_max(X)) <= e_row(X.shape[1])
    assert oracle.gram_residual(X, R) <= E_G


@pytest.mark.parametrize("n,rpw", FULL_PATH)
def test_gram_forms_full_size_path(gpu, n, rpw):
    X, R0, m = full_path_matrix(gpu, n, rpw, seed=31 * n + rpw)
    print("case gram full path m=%d n=%d" % (m, n), flush=True)
    Xd = dev_tensor(X, gpu)
    Rc, ic = q.cholqr2_r(Xd)
    Rs, ss, is_ = q.svqb(Xd, out=q.QLESS_SVQB_R)
    R3, i3 = q.shifted_cholqr3_r(Xd)
    torch.cuda.synchronize(gpu)
    del Xd
    assert int(ic.item()) == 0 and int(is_.item()) == 0 and int(i3.item()) == 0
    Rh = oracle.householder_r(X)
    Ro, info_o = oracle.cholqr2_r(X)
    assert info_o == 0
    check_gram_r(X, Rc.cpu().numpy(), Ro)
    R3o, info3 = oracle.shifted_cholqr3_r(X)
    assert info3 == 0
    check_gram_r(X, R3.cpu().numpy(), R3o)
    Zo, sig_o, Rso, nt = oracle.svqb2(X)
    assert nt == 0
    check_gram_r(X, Rs.cpu().numpy(), Rso)
    for R in (Rc, Rs, R3):
        assert oracle.rel_err_r(R.cpu().numpy(), Rh) <= E_R
