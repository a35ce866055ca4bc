"""Served form on the GPU: every request's R([A b]) is the same alone and in
the mix (e_R <= 1e-12 between the two, and against the CPU oracle), and so
are its least-squares solution and residual (Sec. 1: least squares through
the Q-less R of [A b]).  The mix holds requests of the served workload's
shapes: n from 3 to 47 (48 columns with b) and several m >= 1e6, next to
many short ones, so the long ones are folded over many steps while short
ones come and go."""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2603_20889_amd as q
import workloads as wl
from tolerances import e_row
from paper_2603_20889_amd.server import FifoServer, GpuExecutor, LstsqServer, Request, make_requests

pytestmark = pytest.mark.gpu

E_R = 1e-12
LONG = [(1_200_000, 47), (3_000_000, 21), (1_000_000, 40), (2_000_000, 33), (1_500_000, 3)]


def mixed_requests():
    reqs = make_requests(40, rate_per_s=1e6, seed=17, mlo=1e4, mhi=4e5, nlo=3, nhi=47)
    nid = len(reqs)
    for i, (m, n) in enumerate(LONG):
        # the long requests arrive among the short ones
        reqs.append(Request(id=nid + i, arrival_s=reqs[5 * i].arrival_s, m=m, n=n, seed=9000 + i))
    return reqs


def oracle_r(Ab):
    if Ab.shape[0] > 200_000:
        return oracle.householder_r_chunked(Ab, threads=min(16, os.cpu_count() or 1))
    return oracle.householder_r(Ab)


@pytest.mark.parametrize("mode", ["state", "update", "batched"])
def test_served_equals_alone(gpu, mode):
    reqs = mixed_requests()
    srv = LstsqServer(GpuExecutor(gpu, mode=mode, keep_r=True), hbm_budget_bytes=2 << 30,
                      step_bytes=64 << 20, max_active=16)
    st = srv.run(reqs, realtime=False)
    print("case served %s: %s" % (mode, st), flush=True)
    assert st["completed"] == len(reqs)
    assert srv.ex.steps > 20
    for r in reqs:
        assert r.info == 0
        Ab, x0 = wl.ls_request_data(r.m, r.n, r.seed, device=gpu)
        Rt = q.qless_tsqr_r(Ab)                      # the same request alone, one call
        x, res, info = q.qless_lstsq_finish(Rt)
        torch.cuda.synchronize(gpu)
        R_mix = r.R.cpu().numpy()
        R_alone = Rt.cpu().numpy()
        # rows judged at kappa <= 1e4 relative to the largest column (b: the
        # last row, |rho|, is small by construction)
        floor = 1e-4 * float(torch.linalg.norm(Ab, dim=0).max())
        assert oracle.rel_err_r(R_mix, R_alone) <= E_R, (r.m, r.n)
        assert oracle.row_scaled_err(R_mix, R_alone, floor) <= e_row(r.n + 1), (r.m, r.n)
        Ro = oracle_r(Ab.cpu().numpy())
        del Ab
        assert oracle.rel_err_r(R_mix, Ro) <= E_R, (r.m, r.n)
        assert oracle.row_scaled_err(R_mix, Ro, floor) <= e_row(r.n + 1), (r.m, r.n)
        x = x.cpu().numpy()
        assert np.linalg.norm(r.x - x) <= 1e-10 * np.linalg.norm(x)
        # |rho| is the trailing diagonal entry: the row-wise bar with its floor
        assert abs(r.resid - float(res.item())) <= e_row(r.n + 1) * max(float(res.item()), floor)
        xo, reso = oracle.lstsq_from_r(Ro)
        assert np.linalg.norm(r.x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert np.linalg.norm(r.x - x0) <= 1e-4 * np.linalg.norm(x0)


def test_fifo_baseline_on_gpu(gpu):
    reqs = make_requests(6, rate_per_s=1e6, seed=3, mlo=1e4, mhi=1e5, nlo=3, nhi=10)
    st = FifoServer(GpuExecutor(gpu)).run(reqs, realtime=False)
    assert st["completed"] == 6
    for r in reqs:
        assert r.info == 0
