"""Continuous-batching server for least-squares requests via Q-less TSQR.

A request carries [A b] (m x (n+1), FP64) and is answered with
x = argmin ||A x - b||_2 and |rho| = ||A x - b||_2, read off R([A b]) =
[[R_A, z], [0, rho]] (paper Sec. 1: least squares in a single pass over
the data through the Q-less QR of the extended matrix).

Serving loop (continuous batching, not a queue alone):
  * requests wait in an admission queue until their HBM footprint
    (8 m (n+1) bytes of data plus the running state) fits the budget and an
    active slot is free;
  * every step gives rows to the active requests within the step's byte
    budget: requests with little work left get all of it (smallest first)
    and the rest of the budget goes to the others oldest first, so short
    requests do not wait behind long ones and long ones keep their arrival
    order; each chunk is folded into its request's state on the device
    (by default a running Q-less TSQR whose stage-1 triangles stay in HBM
    between steps, the tree running once when the rows are exhausted --
    R([X_1; X_2; ...]) does not depend on the chunking), and the chunks of
    different requests run on different streams, so their work overlaps on
    the device;
  * a request whose rows are exhausted gets its tree and back substitution
    on the device and an asynchronous copy of its result to the host; the
    loop keeps serving while the copy is on its way, and completes the
    request (latency, memory back to the budget, admission of the next
    waiting requests) when its event has fired.

The executor does the device work (``GpuExecutor``, through libqless); the
scheduling logic only calls its admit / step / finish methods, so tests can
drive it with a stand-in executor on the CPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Optional


@dataclasses.dataclass
class Request:
    id: int
    arrival_s: float
    m: int
    n: int
    seed: int
    # filled in by the server
    admit_s: float = math.nan
    done_s: float = math.nan
    rows_done: int = 0
    x: object = None
    R: object = None          # final R([A b]) on the device, when the executor keeps it
    resid: float = math.nan
    info: int = 0
    state: object = None      # executor-owned per-request state (data, running R)

    @property
    def footprint(self) -> int:
        return 8 * self.m * (self.n + 1) + 8 * (self.n + 1) ** 2

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuExecutor:
    """Device executor: request data and per-request state live in HBM.

    mode "state" (default): each request keeps a running Q-less TSQR state on
    the device (the stage-1 triangles of its plan, ``TsqrState``); a step
    enqueues one stage-1 launch per request that got rows, and a finishing
    request gets the tree, the back substitution and an asynchronous copy of
    (x, |rho|) to pinned host memory, completed when its event has fired.
    Requests are spread round-robin over ``streams`` HIP streams, so the
    launches of different requests overlap on the device (one stream's
    draining launch leaves compute units to the next one's); at most
    ``inflight`` steps are enqueued ahead of the device.
    mode "update": each step runs, per request, the single-matrix kernels on
    its chunk with the previous R stacked in (``qless_tsqr_r_update``: a
    full tree per chunk), on one stream, waiting for each finished request.
    mode "batched": each step is one persistent batched launch (plus tree
    levels) over all chunks (``BatchPlan`` with accumulate), built per step."""

    def __init__(self, device, tile_bytes: int = 1 << 20, data_fn: Optional[Callable] = None,
                 mode: str = "state", keep_r: bool = False, streams: int = 4, inflight: int = 2):
        import torch

        import paper_2603_20889_amd as q
        import workloads
        if mode not in ("state", "batched", "update"):
            raise ValueError("mode must be 'state', 'batched' or 'update'")
        self.q = q
        self.torch = torch
        self.device = device
        self.tile_bytes = tile_bytes
        self.mode = mode
        self._data = data_fn or (lambda r: workloads.ls_request_data(r.m, r.n, r.seed, device=device)[0])
        self.stream = torch.cuda.current_stream(device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, streams))] if mode == "state" else []
        self.inflight = max(1, inflight)
        self._step_events = collections.deque()
        self.steps = 0
        self.keep_r = keep_r
        self._work = None

    def _workspace(self, nbytes: int):
        if self._work is None or self._work.numel() < nbytes:
            self._work = self.torch.empty(max(nbytes, 1 << 20), dtype=self.torch.uint8, device=self.device)
        return self._work

    def admit(self, r: Request):
        torch = self.torch
        Ab = self._data(r)
        if self.mode == "state":
            s = self.streams[r.id % len(self.streams)]
            s.wait_stream(self.stream)           # the data is made on the default stream
            Ab.record_stream(s)                   # and read on s: keep it until s is done with it
            r.state = {"Ab": Ab, "stream": s, "st": self.q.TsqrState(r.m, r.n + 1, self.device, stream=s)}
            return
        R = torch.zeros((r.n + 1, r.n + 1), dtype=torch.float64, device=self.device)
        r.state = {"Ab": Ab, "R": R}

    def step(self, chunks):
        if self.mode == "state":
            while len(self._step_events) >= self.inflight:     # bounded run-ahead of the host
                for ev in self._step_events.popleft():
                    ev.synchronize()
            used = {}
            for r, lo, hi in chunks:
                r.state["st"].fold(r.state["Ab"][lo:hi])
                used[id(r.state["stream"])] = r.state["stream"]
            evs = []
            for s in used.values():
                ev = self.torch.cuda.Event()
                ev.record(s)
                evs.append(ev)
            self._step_events.append(evs)
        elif self.mode == "update":
            for r, lo, hi in chunks:
                need = self.q.qless_workspace_bytes(self.q.QLESS_METHOD_TSQR_UPDATE, hi - lo, r.n + 1)
                self.q.qless_tsqr_r_update(r.state["Ab"][lo:hi], r.state["R"], work=self._workspace(need))
        else:
            Xs = [r.state["Ab"][lo:hi] for r, lo, hi in chunks]
            Rs = [r.state["R"] for r, _, _ in chunks]
            plan = self.q.BatchPlan(Xs, Rs=Rs, accumulate=[True] * len(chunks), tile_bytes=self.tile_bytes)
            plan.run()
            self.torch.cuda.current_stream(self.device).synchronize()
            plan.close()
        self.steps += 1

    def solve(self, r: Request):
        """One request alone with the plain single-matrix call (the baseline):
        R([A b]) by qless_tsqr_r in one call, then the back substitution."""
        Ab = self._data(r)
        R = self.q.qless_tsqr_r(Ab)
        r.state = {"Ab": Ab, "R": R}
        self.steps += 1
        self._read(r, *self.q.qless_lstsq_finish(R), R)

    def finish_async(self, r: Request):
        """Enqueue a finished request's tree and back substitution on its
        stream with an asynchronous copy of the results to pinned memory;
        returns a handle for poll / collect.  Modes other than "state"
        finish at once (the handle is ready)."""
        torch = self.torch
        if self.mode != "state":
            self.finish(r)
            return None
        s = r.state["stream"]
        with torch.cuda.stream(s):
            R = r.state["st"].finish()
            x, res, info = self.q.qless_lstsq_finish(R)
            hx = torch.empty(r.n, dtype=torch.float64, pin_memory=True)
            hres = torch.empty(1, dtype=torch.float64, pin_memory=True)
            hinfo = torch.empty(1, dtype=torch.int32, pin_memory=True)
            hx.copy_(x, non_blocking=True)
            hres.copy_(res, non_blocking=True)
            hinfo.copy_(info, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"ev": ev, "x": hx, "res": hres, "info": hinfo, "R": R, "dev": (x, res, info)}

    def poll(self, handle) -> bool:
        return handle is None or handle["ev"].query()

    def collect(self, r: Request, handle):
        if handle is None:
            return
        handle["ev"].synchronize()
        r.x = handle["x"].numpy().copy()
        r.resid = float(handle["res"][0])
        r.info = int(handle["info"][0])
        if self.keep_r:
            r.R = handle["R"]
        r.state = None

    def finish(self, r: Request):
        if self.mode == "state":
            self.collect(r, self.finish_async(r))
            return
        self._read(r, *self.q.qless_lstsq_finish(r.state["R"]), r.state["R"])

    def _read(self, r: Request, x, res, info, R):
        self.torch.cuda.current_stream(self.device).synchronize()
        r.x = x.cpu().numpy()
        r.resid = float(res.item())
        r.info = int(info.item())
        if self.keep_r:
            r.R = R
        r.state = None


class LstsqServer:
    """Admission by HBM footprint, continuous batching of row chunks."""

    def __init__(self, executor, hbm_budget_bytes: int, step_bytes: int = 1 << 30, max_active: int = 256,
                 clock: Callable[[], float] = time.perf_counter, short_bytes: Optional[int] = None):
        self.ex = executor
        self.budget = int(hbm_budget_bytes)
        self.step_bytes = int(step_bytes)
        self.short_bytes = int(short_bytes if short_bytes is not None else step_bytes // 2)
        self.max_active = int(max_active)
        self.clock = clock
        self.queue: collections.deque[Request] = collections.deque()
        self.active: list[Request] = []
        self.done: list[Request] = []
        self.rejected: list[Request] = []
        self.in_use = 0
        self.finishing: list = []           # (request, executor handle) whose results are on their way
        self.max_queue = 0
        self.max_active_seen = 0
        self.t0 = 0.0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, r: Request):
        if r.footprint > self.budget:        # can never fit: reject at once
            self.rejected.append(r)
            return
        self.queue.append(r)
        self.max_queue = max(self.max_queue, len(self.queue))

    def _admit(self):
        while self.queue and len(self.active) < self.max_active and self.in_use + self.queue[0].footprint <= self.budget:
            r = self.queue.popleft()
            self.ex.admit(r)
            r.admit_s = self.now()
            self.in_use += r.footprint
            self.active.append(r)
        self.max_active_seen = max(self.max_active_seen, len(self.active))

    def _chunks(self):
        """Next row ranges, within the step's byte budget: (1) requests whose
        remaining work is at most short_bytes get all of it (smallest first),
        so short requests finish at once instead of queueing behind long
        ones; (2) what is left goes to the other requests oldest first, so
        long requests keep their arrival order.  A request may get no rows in
        a step; each step is one batch over the requests that got some."""
        if not self.active:
            return []
        rows = {r.id: 0 for r in self.active}
        left = lambda r: (r.m - r.rows_done - rows[r.id]) * 8 * (r.n + 1)
        budget = self.step_bytes
        for r in sorted(self.active, key=left):
            if budget <= 0 or left(r) > self.short_bytes:
                break
            take = min(left(r), budget) // (8 * (r.n + 1))
            rows[r.id] += take
            budget -= take * 8 * (r.n + 1)
        for r in sorted(self.active, key=lambda r: (r.arrival_s, r.id)):
            if budget <= 0:
                break
            take = min(left(r), budget) // (8 * (r.n + 1))
            rows[r.id] += take
            budget -= take * 8 * (r.n + 1)
        if all(v == 0 for v in rows.values()):           # budget below one row: still progress
            r = min(self.active, key=lambda r: (r.arrival_s, r.id))
            rows[r.id] = 1
        return [(r, r.rows_done, r.rows_done + rows[r.id]) for r in self.active if rows[r.id] > 0]

    def _poll(self):
        """Complete the finishing requests whose results have arrived; their
        memory then goes back to the budget."""
        still = []
        for r, h in self.finishing:
            if self.ex.poll(h):
                self.ex.collect(r, h)
                r.done_s = self.now()
                self.in_use -= r.footprint
                self.done.append(r)
            else:
                still.append((r, h))
        self.finishing = still

    def step(self):
        self._poll()
        self._admit()
        chunks = self._chunks()
        if not chunks:
            return False
        self.ex.step(chunks)
        for r, lo, hi in chunks:
            r.rows_done = hi
        still = []
        for r in self.active:                   # requests without rows this step stay active
            if r.rows_done >= r.m:
                if hasattr(self.ex, "finish_async"):
                    self.finishing.append((r, self.ex.finish_async(r)))
                else:
                    self.ex.finish(r)
                    r.done_s = self.now()
                    self.in_use -= r.footprint
                    self.done.append(r)
            else:
                still.append(r)
        self.active = still
        self._poll()
        return True

    def run(self, requests, realtime: bool = True):
        """Serve `requests` (sorted by arrival).  With realtime, arrivals are
        released by the wall clock; otherwise all arrive at t = 0."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        self.t0 = self.clock()
        while pending or self.queue or self.active or self.finishing:
            t = self.now()
            while pending and (not realtime or pending[0].arrival_s <= t):
                self.submit(pending.popleft())
            if not self.step():
                if self.finishing:
                    time.sleep(20e-6)             # results on their way: poll again soon
                elif pending:
                    wait = pending[0].arrival_s - self.now()
                    if wait > 0:
                        time.sleep(min(wait, 0.001))
                elif self.queue and not self.active:
                    raise RuntimeError("request does not fit the HBM budget")
        return self.stats()

    def stats(self) -> dict:
        lat = sorted(r.latency_s for r in self.done)
        span = (max(r.done_s for r in self.done) - min(r.arrival_s for r in self.done)) if self.done else 0.0

        def pct(p):
            if not lat:
                return math.nan
            k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
            return lat[k]
        return {"completed": len(self.done), "rejected": len(self.rejected),
                "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "mean_ms": 1e3 * (sum(lat) / len(lat)) if lat else math.nan,
                "solves_per_s": len(self.done) / span if span > 0 else math.nan,
                "steps": getattr(self.ex, "steps", 0), "max_queue": self.max_queue,
                "max_active": self.max_active_seen}


class FifoServer:
    """Baseline: one request at a time in arrival order, each solved by the
    plain single-matrix call (no batching), its result read back before the
    next one starts."""

    def __init__(self, executor, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.clock = clock
        self.done: list[Request] = []
        self.t0 = 0.0

    def run(self, requests, realtime: bool = True):
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        self.t0 = self.clock()
        while pending:
            r = pending.popleft()
            now = self.clock() - self.t0
            if realtime and r.arrival_s > now:
                time.sleep(r.arrival_s - now)
            r.admit_s = self.clock() - self.t0
            if hasattr(self.ex, "solve"):
                self.ex.solve(r)
            else:
                self.ex.admit(r)
                self.ex.step([(r, 0, r.m)])
                self.ex.finish(r)
            r.done_s = self.clock() - self.t0
            self.done.append(r)
        lat = sorted(r.latency_s for r in self.done)
        span = max(r.done_s for r in self.done) - min(r.arrival_s for r in self.done)
        k50 = max(0, int(math.ceil(0.5 * len(lat))) - 1)
        k99 = max(0, int(math.ceil(0.99 * len(lat))) - 1)
        return {"completed": len(lat), "p50_ms": 1e3 * lat[k50], "p99_ms": 1e3 * lat[k99],
                "mean_ms": 1e3 * sum(lat) / len(lat), "solves_per_s": len(lat) / span if span > 0 else math.nan}


def make_requests(count: int, rate_per_s: float, seed: int = 5, mlo: float = 1e4, mhi: float = 5e7,
                  nlo: int = 3, nhi: int = 47) -> list[Request]:
    import workloads
    return [Request(id=d["id"], arrival_s=d["arrival_s"], m=d["m"], n=d["n"], seed=d["seed"])
            for d in workloads.server_requests(count, rate_per_s, seed, mlo, mhi, nlo, nhi)]
