"""Served form on the GPU: every request's result is the same alone and in
the mix (within the stated tolerance), and matches the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl
from paper_2603_20889_amd.server import FifoServer, GpuExecutor, LstsqServer, make_requests

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["batched", "update"])
def test_served_equals_alone(gpu, mode):
    reqs = make_requests(24, rate_per_s=1e6, seed=17, mlo=1e4, mhi=4e5, nlo=3, nhi=20)
    srv = LstsqServer(GpuExecutor(gpu, mode=mode), hbm_budget_bytes=200 << 20, step_bytes=64 << 20, max_active=8)
    st = srv.run(reqs, realtime=False)
    print("case served %s: %s" % (mode, st), flush=True)
    assert st["completed"] == len(reqs)
    assert srv.ex.steps > 1
    for r in reqs:
        assert r.info == 0
        Ab, x0 = wl.ls_request_data(r.m, r.n, r.seed, device=gpu)
        Rt = q.qless_tsqr_r(Ab)                      # the same request alone, one call
        x, res, info = q.qless_lstsq_finish(Rt)
        torch.cuda.synchronize(gpu)
        x = x.cpu().numpy()
        assert np.linalg.norm(r.x - x) <= 1e-10 * np.linalg.norm(x)
        assert abs(r.resid - float(res.item())) <= 1e-10 * float(res.item())
        xo, reso = oracle.lstsq_from_r(oracle.householder_r(Ab.cpu().numpy()))
        assert np.linalg.norm(r.x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert np.linalg.norm(r.x - x0) <= 1e-4 * np.linalg.norm(x0)


def test_fifo_baseline_on_gpu(gpu):
    reqs = make_requests(6, rate_per_s=1e6, seed=3, mlo=1e4, mhi=1e5, nlo=3, nhi=10)
    st = FifoServer(GpuExecutor(gpu)).run(reqs, realtime=False)
    assert st["completed"] == 6
    for r in reqs:
        assert r.info == 0
