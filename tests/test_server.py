"""Scheduling logic of the continuous-batching least-squares server, driven
on the CPU by a stand-in executor that uses the oracle (no GPU)."""
import numpy as np

import oracle
import workloads as wl
from paper_2603_20889_amd.server import FifoServer, LstsqServer, Request, make_requests


class OracleExecutor:
    """Executes each step with the CPU oracle: R <- R([R; chunk])."""

    def __init__(self):
        self.steps = 0
        self.chunks_per_step = []

    def admit(self, r):
        r.state = {"Ab": wl.ls_request_data(r.m, r.n, r.seed)[0], "R": np.zeros((r.n + 1, r.n + 1))}

    def step(self, chunks):
        self.steps += 1
        self.chunks_per_step.append([(r.id, lo, hi) for r, lo, hi in chunks])
        for r, lo, hi in chunks:
            r.state["R"] = oracle.householder_r(np.vstack([r.state["R"], r.state["Ab"][lo:hi]]))

    def finish(self, r):
        r.x, r.resid = oracle.lstsq_from_r(r.state["R"])
        r.info = 0
        r.state = None


class BudgetCheckingServer(LstsqServer):
    def step(self):
        ok = super().step()
        assert self.in_use <= self.budget
        assert sum(r.footprint for r in self.active) + sum(r.footprint for r, _ in self.finishing) == self.in_use
        return ok


def small_requests(count=12, seed=9):
    return make_requests(count, rate_per_s=1e6, seed=seed, mlo=2e3, mhi=6e4, nlo=2, nhi=9)


def test_all_complete_and_match_alone():
    reqs = small_requests()
    srv = BudgetCheckingServer(OracleExecutor(), hbm_budget_bytes=6_000_000, step_bytes=1_500_000)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    for r in reqs:
        Ab, x0 = wl.ls_request_data(r.m, r.n, r.seed)
        xo, reso = oracle.lstsq_from_r(oracle.householder_r(Ab))   # the request alone, in one piece
        assert np.linalg.norm(r.x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert abs(r.resid - reso) <= 1e-10 * reso
        assert np.linalg.norm(r.x - x0) <= 1e-4 * np.linalg.norm(x0)


def test_admission_respects_budget_and_queues():
    reqs = small_requests(16, seed=3)
    budget = max(r.footprint for r in reqs) + 10
    srv = BudgetCheckingServer(OracleExecutor(), hbm_budget_bytes=budget, step_bytes=1 << 20)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == 16
    assert st["max_queue"] >= 2            # the budget forced waiting


def test_oversized_request_rejected():
    big = Request(id=0, arrival_s=0.0, m=100_000, n=10, seed=1)
    ok = Request(id=1, arrival_s=0.0, m=1000, n=3, seed=2)
    srv = LstsqServer(OracleExecutor(), hbm_budget_bytes=1_000_000)
    st = srv.run([big, ok], realtime=False)
    assert st["completed"] == 1 and st["rejected"] == 1
    assert srv.rejected[0].id == 0


def test_requests_overlap_in_steps():
    """Continuous batching: a short request admitted while a long one is in
    flight shares steps with it and finishes first."""
    long_r = Request(id=0, arrival_s=0.0, m=200_000, n=4, seed=11)
    short_r = Request(id=1, arrival_s=0.0, m=5_000, n=4, seed=12)
    ex = OracleExecutor()
    srv = LstsqServer(ex, hbm_budget_bytes=1 << 30, step_bytes=400_000)
    srv.run([long_r, short_r], realtime=False)
    assert ex.steps > 1
    assert ex.chunks_per_step[0] and {c[0] for c in ex.chunks_per_step[0]} == {0, 1}
    assert short_r.done_s <= long_r.done_s
    covered = [c for s in ex.chunks_per_step for c in s if c[0] == 0]
    assert covered[0][1] == 0 and covered[-1][2] == long_r.m
    assert all(a[2] == b[1] for a, b in zip(covered, covered[1:]))   # contiguous, no row twice


def test_fifo_baseline_runs():
    reqs = small_requests(5, seed=4)
    st = FifoServer(OracleExecutor()).run(reqs, realtime=False)
    assert st["completed"] == 5


def test_short_requests_bypass_and_long_ones_keep_order():
    """Step budget policy: a short request finishes in the first step even
    behind long ones, alongside the oldest long one; the long ones complete
    in arrival order."""
    a = Request(id=0, arrival_s=0.0, m=120_000, n=4, seed=21)
    b = Request(id=1, arrival_s=0.001, m=120_000, n=4, seed=22)
    c = Request(id=2, arrival_s=0.002, m=6_000, n=4, seed=23)
    ex = OracleExecutor()
    srv = LstsqServer(ex, hbm_budget_bytes=1 << 30, step_bytes=1_000_000)
    srv.run([a, b, c], realtime=False)
    first = {ch[0]: ch[2] - ch[1] for ch in ex.chunks_per_step[0]}
    assert first[2] == c.m                     # the short one, whole
    assert first[0] > 0 and 1 not in first     # the oldest long one takes the rest
    assert a.done_s <= b.done_s
    assert all(c.done_s <= r.done_s for r in (a, b))


class AsyncOracleExecutor(OracleExecutor):
    """Completes a finished request only after its handle has been polled a
    few times, as the GPU executor's event-driven finish does."""

    def __init__(self, delay=3):
        super().__init__()
        self.delay = delay

    def finish_async(self, r):
        return {"left": self.delay}

    def poll(self, h):
        h["left"] -= 1
        return h["left"] < 0

    def collect(self, r, h):
        self.finish(r)


def test_async_finish_keeps_serving_and_accounts_memory():
    reqs = small_requests(14, seed=21)
    budget = 3 * max(r.footprint for r in reqs)
    srv = BudgetCheckingServer(AsyncOracleExecutor(), hbm_budget_bytes=budget, step_bytes=400_000)
    st = srv.run(reqs, realtime=False)
    assert st["completed"] == len(reqs) and srv.in_use == 0 and not srv.finishing
    for r in reqs:
        xo, reso = oracle.lstsq_from_r(oracle.householder_r(wl.ls_request_data(r.m, r.n, r.seed)[0]))
        assert np.linalg.norm(r.x - xo) <= 1e-10 * np.linalg.norm(xo)
        assert r.done_s >= r.admit_s >= r.arrival_s
