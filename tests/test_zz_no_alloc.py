"""qless_tsqr_r_noalloc (the TSQR entry point for callers that cannot
allocate) against qless_tsqr_r through the C-ABI: two calls in a row, the
second on a smaller input, each equal to the workspace entry point's R (the
same launches, so bit for bit) and within the oracle's tolerance; plus its
host-side argument errors."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl

pytestmark = pytest.mark.gpu


def noalloc(X, R):
    lib = q.load()
    m, n = X.shape
    st = lib.qless_tsqr_r_noalloc(ctypes.c_void_p(X.data_ptr()), m, n, X.stride(0), ctypes.c_void_p(R.data_ptr()),
                                  R.stride(0), ctypes.c_void_p(torch.cuda.current_stream(X.device).cuda_stream))
    return st


@pytest.mark.parametrize("shapes", [[(3_000_000, 8), (100_000, 8)], [(1_000_000, 64), (20_000, 33)],
                                    [(2_000_000, 16), (5_000, 3)]])
def test_noalloc_matches_workspace_entry_point(gpu, shapes):
    outs = []
    for i, (m, n) in enumerate(shapes):
        print("case noalloc call %d m=%d n=%d" % (i, m, n), flush=True)
        X = wl.gaussian(m, n, seed=60 + i + n)
        Xd = torch.from_numpy(X).to(gpu)
        R = torch.full((n, n), np.nan, dtype=torch.float64, device=gpu)
        assert noalloc(Xd, R) == q.QLESS_OK
        Rw = q.qless_tsqr_r(Xd)
        torch.cuda.synchronize(gpu)
        outs.append((X, R.cpu().numpy(), Rw.cpu().numpy()))
    for X, R, Rw in outs:
        assert np.array_equal(R, Rw)
        assert oracle.rel_err_r(R, oracle.householder_r(X)) <= 1e-12
        assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)


def test_noalloc_argument_errors(gpu):
    lib = q.load()
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    assert lib.qless_tsqr_r_noalloc(fake, 100, 0, 8, fake, 8, null) == q.QLESS_ERR_ARG
    assert lib.qless_tsqr_r_noalloc(fake, 100, 65, 65, fake, 65, null) == q.QLESS_ERR_UNSUPPORTED
    assert lib.qless_tsqr_r_noalloc(null, 100, 4, 4, fake, 4, null) == q.QLESS_ERR_ARG
    assert lib.qless_noalloc_scratch_bytes() >= q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, 1 << 30, 64)
