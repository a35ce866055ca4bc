"""GPU parity of the batched Q-less TSQR (one persistent stage-1 launch plus
one launch per tree level for many matrices of uneven m and n) against the CPU
oracle, plus its replay, graph capture and running-R (accumulate) behaviour."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl

pytestmark = pytest.mark.gpu

SHAPES = [(0, 3), (1, 4), (5, 8), (100, 1), (3000, 3), (20000, 4), (77777, 5), (4096, 8), (250_000, 8),
          (9000, 13), (100_000, 16), (12345, 17), (60000, 32), (2000, 33), (30000, 64), (1_000_003, 4),
          (50000, 45), (40000, 61)]


def make(shapes, seed0=0):
    Xh = [wl.gaussian(m, n, seed=seed0 + i) for i, (m, n) in enumerate(shapes)]
    return Xh


def test_batched_matches_oracle(gpu):
    Xh = make(SHAPES)
    Xs = [torch.from_numpy(X).to(gpu) for X in Xh]
    plan = q.BatchPlan(Xs, tile_bytes=1 << 20)
    print("case batched tiles=%d" % plan.tiles, flush=True)
    Rs = plan.run()
    torch.cuda.synchronize(gpu)
    for X, R in zip(Xh, Rs):
        R = R.cpu().numpy()
        Ro = oracle.householder_r(X)
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
        assert oracle.rel_err_r(R, Ro) <= 1e-12, X.shape
        assert oracle.gram_residual(X, R) <= 1e-13, X.shape
    # replay: no state survives a call -> bitwise identical
    first = [R.clone() for R in Rs]
    plan.run()
    torch.cuda.synchronize(gpu)
    for a, b in zip(first, plan.Rs):
        assert torch.equal(a, b)


def test_batched_equals_single_matrix_calls(gpu):
    shapes = [(50_000, 4), (200_000, 8), (80_000, 16), (40_000, 32)]
    Xs = [torch.from_numpy(X).to(gpu) for X in make(shapes, 50)]
    Rb = q.qless_tsqr_r_batched(Xs, tile_bytes=256 << 10)
    for X, R in zip(Xs, Rb):
        R1 = q.qless_tsqr_r(X)
        torch.cuda.synchronize(gpu)
        assert oracle.rel_err_r(R.cpu().numpy(), R1.cpu().numpy()) <= 1e-12


def test_batched_accumulate_running_r(gpu):
    """R([R_old; X2]) = R([X1; X2]) (the sufficient-statistic property of R)."""
    X1 = wl.gaussian(30_000, 9, seed=1)
    X2 = wl.gaussian(45_000, 9, seed=2)
    R = q.qless_tsqr_r(torch.from_numpy(X1).to(gpu))
    plan = q.BatchPlan([torch.from_numpy(X2).to(gpu)], Rs=[R], accumulate=[True], tile_bytes=1 << 20)
    plan.run()
    torch.cuda.synchronize(gpu)
    Ro = oracle.householder_r(np.vstack([X1, X2]))
    assert oracle.rel_err_r(R.cpu().numpy(), Ro) <= 1e-12


def test_batched_graph_replay(gpu):
    """Capture the batched launch in a graph; every replay matches eager."""
    shapes = [(100_000, 4), (30_000, 8), (60_000, 16), (20_000, 32)]
    Xs = [torch.from_numpy(X).to(gpu) for X in make(shapes, 70)]
    plan = q.BatchPlan(Xs, tile_bytes=512 << 10)
    s = torch.cuda.Stream(device=gpu)
    s.wait_stream(torch.cuda.current_stream(gpu))
    with torch.cuda.stream(s):
        plan.run()                       # eager reference on the capture stream
    torch.cuda.current_stream(gpu).wait_stream(s)
    torch.cuda.synchronize(gpu)
    ref = [R.clone() for R in plan.Rs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.run()
    for rep in range(3):
        for R in plan.Rs:
            R.fill_(-1.0)
        torch.cuda.synchronize(gpu)
        g.replay()
        torch.cuda.synchronize(gpu)
        _ = torch.ones(10, device=gpu).sum().item()   # eager work between replays
        for a, b in zip(ref, plan.Rs):
            assert torch.equal(a, b), "replay %d" % rep


def test_batched_rejects_bad_descriptor(gpu):
    with pytest.raises(q.QlessError):
        q.BatchPlan([torch.zeros((10, 70), dtype=torch.float64, device=gpu)])
