#!/usr/bin/env python3
"""Benchmark: Q-less TSQR HBM throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-cpu]

A step is one complete ``qless_tsqr_r`` call (stage-1 streaming kernel, the
stacked-R tree and the sign normalisation) on the 5e7 x 8 FP64 workload
X = Q0 R0 with kappa = 1e4, resident in HBM.  ``value`` is algorithmic GB/s =
8 m n bytes per step / step time.  The JSON line adds
  roofline     : the stage-1 kernel's algorithmic bytes per launch over its
                 average launch duration (HIP events around each launch on
                 the launch stream), against the 8 TB/s HBM peak;
  cpu_baseline : the CPU oracle (plain Householder, one thread) timed on this
                 host on the same matrix;
  sweep        : m = 2^25, n in {1, 2, 4, 8, 16, 32, 64} (kappa = 1e4):
                 GB/s, fraction of HBM peak and FP64 TF/s per n;
  compare      : CholQR2 and SVQB2 on the same 5e7 x 8 matrix when built.
Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, published
TUNE_TABLE = os.path.join(ROOT, "paper_2603_20889_amd", "tuning_gfx950.json")
FP64_PEAK_TFS = 78.6        # MI355X FP64 vector, published


def tsqr_bytes(m: int, n: int) -> int:
    """Algorithmic bytes of Q-less TSQR: X read once (Sec. 3.2 model)."""
    return 8 * m * n


def tsqr_flops(m: int, n: int) -> int:
    """Lower bound of the FP64 flop count: 2 m n^2 (Sec. 3.2 model)."""
    return 2 * m * n * n


def gram2_bytes(m: int, n: int) -> int:
    """CholQR2 / SVQB2: two passes over X (Sec. 3.1 model)."""
    return 16 * m * n


# Sources that define, instantiate or plan the profiled launches: the TSQR
# fold and tree kernels with their launch plan, the Gram kernels, and the
# shared device helpers.  Entry-point glue, the small n x n kernels and the
# batched form do not change those launches.
PROFILED_SOURCES = ("qless_internal.h", "tsqr_kernels.h", "gram.hip")


def kernel_source_hash() -> str:
    """Hash of the profiled kernels' HIP sources (PROFILED_SOURCES and every
    tsqr*.hip) with comments and blank space removed, so that a change of
    wording does not retire counter data taken on the same code."""
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_20889_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn in PROFILED_SOURCES or (fn.startswith("tsqr") and fn.endswith(".hip")):
            text = open(os.path.join(csrc, fn)).read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            h.update(fn.encode())
            h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per stage-1 launch from committed rocprofv3 counter runs,
    if they were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "tsqr_stage1_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_source_hash() or d.get("workload") != workload:
        return None
    return d.get("traffic_bytes_per_launch")


def host_threads():
    """(threads the CPU oracle runs on, cores this process may use): the
    cores in this process's affinity mask, capped by OMP_NUM_THREADS when it
    is set (the host's CPU share for this GPU)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    use = min(avail, int(cap)) if cap.isdigit() and int(cap) > 0 else avail
    return max(1, use), avail


def timed(fn):
    t0 = time.perf_counter()
    r = fn()
    return r, time.perf_counter() - t0


def time_calls(fn, steps: int, warmup: int):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--m", type=int, default=50_000_000)
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--ns", type=str, default="1,2,4,8,16,32,64",
                    help="column counts of the m = 2^25 sweep")
    ap.add_argument("--sweep-ks", type=str, default="0,4,8",
                    help="condition exponents k of the sweep (sigma down to 10^-k); timing runs at k = 4")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=2000)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (torch) for HBM-counter calibration")
    ap.add_argument("--tune", type=str, default="",
                    help="launch-parameter overrides n:rows_per_lane[:waves_per_cu[:fan_in]],... "
                         "(qless_tune_set) applied before any timing, e.g. 32:1,64:1 for the "
                         "matrix-core fold")
    ap.add_argument("--tune-table", type=str, default=TUNE_TABLE,
                    help="autotuner table (JSON written by --autotune) applied before any timing; "
                         "'' for the library defaults")
    ap.add_argument("--autotune", type=str, default="",
                    help="run the autotuner for these n (comma list) first and write its table to this "
                         "path (--autotune-out), then apply it")
    ap.add_argument("--autotune-out", type=str, default="gpurun_out/tuning_gfx950.json")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(rows would shard across GPUs, each GPU folding its rows to one n x n "
              "triangle, with one gather of the triangles and a last fold).",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2603_20889_amd as q
    import workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    q.load()
    m, n = args.m, args.n
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)
    tuned = {}       # the launch parameters in effect per n (defaults resolved)
    tuned_raw = {}   # what was passed to qless_tune_set (0 = library default)
    tune_src = None
    if args.autotune:
        from paper_2603_20889_amd import autotune
        ns_t = [int(v) for v in args.autotune.split(",") if v]
        log("autotuning n = %s" % ns_t)
        table = autotune.tune_tsqr(ns_t, device=dev, log=log)
        os.makedirs(os.path.dirname(os.path.abspath(args.autotune_out)), exist_ok=True)
        with open(args.autotune_out, "w") as f:
            json.dump({"arch": "gfx950", "kernel_hash": kernel_source_hash(),
                       "table": {str(k): v for k, v in table.items()}}, f, indent=1, sort_keys=True)
        tune_src = args.autotune_out
    elif args.tune_table and os.path.exists(args.tune_table):
        tune_src = args.tune_table
    if tune_src:
        data = json.load(open(tune_src))
        for k, v in data["table"].items():
            tuned_raw[int(k)] = (int(v["waves_per_cu"]), int(v["fan_in"]), int(v["rows_per_lane"]))
            q.qless_tune_set(int(k), *tuned_raw[int(k)])
            tuned[int(k)] = q.qless_tune_get(int(k))
        log("tuning table %s applied (taken on kernel sources %s, now %s)" %
            (tune_src, data.get("kernel_hash"), kernel_source_hash()))
    for item in filter(None, args.tune.split(",")):
        f = [int(v) for v in item.split(":")] + [0, 0]
        tuned_raw[f[0]] = (f[2], f[3], f[1])
        q.qless_tune_set(f[0], *tuned_raw[f[0]])
        tuned[f[0]] = q.qless_tune_get(f[0])
    if tuned:
        log("tuning overrides: %s" % tuned)

    log("generating X = Q0 R0 (%d x %d, kappa 1e4) on the GPU" % (m, n))
    X, R0 = wl.config2(m=m, n=n, device=dev)
    torch.cuda.synchronize()
    R = torch.empty((n, n), dtype=torch.float64, device=dev)
    work, wb = q._workspace(q.QLESS_METHOD_TSQR, m, n, dev)

    def step():
        q.qless_tsqr_r(X, R=R, work=work)

    log("timing %d steps after %d warm-up" % (args.steps, args.warmup))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    q.timing_reset()
    q.timing_enable(True)
    ms, wall = time_calls(step, args.steps, 0)
    q.timing_enable(False)
    st_ms, st_cnt = q.timing_read("tsqr_stage1")
    q.timing_reset()
    e_r = float(np.linalg.norm(R.cpu().numpy() - R0) / np.linalg.norm(R0))
    log("step %.4f ms, stage-1 %.4f ms x %d, e_R vs R0 %.2e" % (ms, st_ms / max(st_cnt, 1), st_cnt, e_r))

    nbytes = tsqr_bytes(m, n)
    value = nbytes / (ms * 1e-3) / 1e9
    st_avg = st_ms / max(st_cnt, 1)
    achieved = nbytes / (st_avg * 1e-3) / 1e9
    workload = "tsqr_config2_%dx%d" % (m, n)
    traffic = load_traffic(workload)

    out = {
        "metric": "Q-less TSQR HBM GB/s (% of peak), n=1..64; batched solves/s + p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "qless_tsqr_r on X = Q0*R0, m=%d, n=%d, kappa=1e4, FP64 row-major, "
                               "resident in HBM" % (m, n), "m": m, "n": n},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "tsqr_stage1", "kernel_ms": round(st_avg, 5),
                     "algorithmic_bytes_per_launch": nbytes},
        "accuracy": {"e_R_vs_R0": e_r},
        "kernel_hash": kernel_source_hash(),
        "tuning_overrides": {str(k): v for k, v in tuned.items()} or None,
        "tuning_table": os.path.relpath(tune_src, ROOT) if tune_src else None,
        "pct_hbm_peak_step": round(100.0 * value / HBM_PEAK_GBS, 2),
    }

    # context: a plain library read of the same bytes (torch.sum over X), timed
    # the same way -- what a generic streaming kernel reaches on this GPU
    rd_ms, _ = time_calls(lambda: torch.sum(X), 5, 2)
    out["plain_read_reference"] = {"kernel": "torch.sum over X", "ms": round(rd_ms, 5),
                                   "GBps": round(nbytes / (rd_ms * 1e-3) / 1e9, 1)}

    # the per-call distribution (outside the timed region): each call between
    # its own pair of events, mean / median / p99
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in evs:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    calls = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    out["step_ms_distribution"] = {"calls": len(calls), "mean": round(sum(calls) / len(calls), 5),
                                   "median": round(calls[len(calls) // 2], 5),
                                   "p99": round(calls[min(len(calls) - 1, int(0.99 * len(calls)))], 5)}

    # one GPU's share of the headline at its real shape were it split over 8
    # GPUs by rows (m / 8 x n), the cache flushed between calls
    ms8 = m // 8
    X8 = X[:ms8]
    R8 = torch.empty((n, n), dtype=torch.float64, device=dev)
    w8, _ = q._workspace(q.QLESS_METHOD_TSQR, ms8, n, dev)
    flush8 = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
    for e0, e1 in evs:
        torch.sum(flush8)
        e0.record()
        q.qless_tsqr_r(X8, R=R8, work=w8)
        e1.record()
    torch.cuda.synchronize()
    t8 = sorted(e0.elapsed_time(e1) for e0, e1 in evs)[len(evs) // 2]
    out["shard_of_8"] = {"m": ms8, "n": n, "ms_median": round(t8, 5),
                         "GBps": round(tsqr_bytes(ms8, n) / (t8 * 1e-3) / 1e9, 1),
                         "note": "rows [0, m/8) of the headline matrix: one GPU's share under an 8-way row split"}
    del X8, R8, w8, flush8

    cpu_threads = None
    if not args.no_cpu:
        import oracle
        cpu_threads, cpu_avail = host_threads()
        log("CPU oracle on the same matrix (host copy), 1 and %d threads" % cpu_threads)
        Xh = X.cpu().numpy()
        R1, t1 = timed(lambda: oracle.householder_r_chunked(Xh, 1))
        RN, tN = timed(lambda: oracle.householder_r_chunked(Xh, cpu_threads))
        c1 = wl.config1()
        c1_1 = min(timed(lambda: oracle.householder_r_chunked(c1, 1))[1] for _ in range(3))
        c1_N = min(timed(lambda: oracle.householder_r_chunked(c1, cpu_threads))[1] for _ in range(3))
        out["cpu_baseline"] = {
            "value": round(nbytes / tN / 1e9, 4), "unit": "GB/s", "cores": cpu_threads,
            "cores_available": cpu_avail, "kind": "oracle", "seconds": round(tN, 3),
            "sample": "the full %d x %d benchmark matrix, one call of the oracle with its length-m sums in "
                      "fixed 64K-row chunks (OpenMP over chunks, result bitwise independent of the thread "
                      "count), on %d host threads" % (m, n, cpu_threads),
            "single_thread": {"value": round(nbytes / t1 / 1e9, 4), "unit": "GB/s", "seconds": round(t1, 3)},
            "bitwise_equal_1_vs_all_threads": bool(np.array_equal(R1, RN)),
            "config1_100000x4": {"seconds_1_thread": round(c1_1, 5), "seconds_all_threads": round(c1_N, 5),
                                 "GBps_1_thread": round(c1.nbytes / c1_1 / 1e9, 4),
                                 "GBps_all_threads": round(c1.nbytes / c1_N / 1e9, 4)},
        }
        out["accuracy"]["e_R_vs_oracle"] = float(np.linalg.norm(R.cpu().numpy() - RN) / np.linalg.norm(RN))
        log("cpu: %s" % json.dumps(out["cpu_baseline"]))
        del Xh

    if not args.no_compare:
        comp = {}
        forms = (("cholqr2", lambda: q.cholqr2_r(X), 2), ("svqb2", lambda: q.svqb(X, out=q.QLESS_SVQB_R), 2),
                 ("shifted_cholqr3", lambda: q.shifted_cholqr3_r(X), 3))
        for name, fn, passes in forms:
            log("compare %s" % name)
            c_ms, _ = time_calls(fn, max(5, args.steps // 3), 2)
            res = fn()
            torch.cuda.synchronize()
            Rc = res[0].cpu().numpy()
            comp[name] = {"ms": round(c_ms, 5), "passes_over_X": passes,
                          "GBps": round(passes * tsqr_bytes(m, n) / (c_ms * 1e-3) / 1e9, 1),
                          "e_R_vs_R0": float(np.linalg.norm(Rc - R0) / np.linalg.norm(R0)),
                          "info": int(res[-1].item())}
            log(json.dumps(comp[name]))
        # the explicit Q of Sec. 1 from X and the Q-less R (one pass: read X, write Q),
        # next to a plain device copy of the same bytes (the read + write ceiling)
        log("compare q_from_r")
        Q = torch.empty_like(X)
        qinfo = torch.empty(1, dtype=torch.int32, device=dev)
        qwork, _ = q._workspace(q.QLESS_METHOD_Q_FROM_R, m, n, dev)
        qf_ms, _ = time_calls(lambda: q.qless_q_from_r(X, R, Q=Q, info=qinfo, work=qwork), max(5, args.steps // 3), 2)
        cp_ms, _ = time_calls(lambda: Q.copy_(X), max(5, args.steps // 3), 2)
        q.qless_q_from_r(X, R, Q=Q, info=qinfo, work=qwork)
        Qs = Q[:200_000].cpu().numpy()
        Xs_ = X[:200_000].cpu().numpy()
        comp["q_from_r"] = {"ms": round(qf_ms, 5), "bytes": 2 * nbytes,
                            "GBps": round(2 * nbytes / (qf_ms * 1e-3) / 1e9, 1),
                            "frac_hbm": round(2 * nbytes / (qf_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "copy_ms": round(cp_ms, 5), "copy_GBps": round(2 * nbytes / (cp_ms * 1e-3) / 1e9, 1),
                            "frac_of_copy": round(cp_ms / qf_ms, 4), "info": int(qinfo.item()),
                            "QR_minus_X_rel_sample": float(np.linalg.norm(Qs @ R.cpu().numpy() - Xs_) /
                                                           np.linalg.norm(Xs_))}
        log(json.dumps(comp["q_from_r"]))
        del Q, Qs, Xs_, qwork
        log("compare cholqr2_dd")
        dd_ms, _ = time_calls(lambda: q.cholqr2_dd_r(X), max(5, args.steps // 3), 2)
        Rd, dinfo = q.cholqr2_dd_r(X)
        torch.cuda.synchronize()
        comp["cholqr2_dd"] = {"ms": round(dd_ms, 5), "passes_over_X": 2,
                              "e_R_vs_R0": float(np.linalg.norm(Rd.cpu().numpy() - R0) / np.linalg.norm(R0)),
                              "info": int(dinfo.item())}
        log(json.dumps(comp["cholqr2_dd"]))
        comp["tsqr_speedup_vs_svqb2"] = round(comp["svqb2"]["ms"] / ms, 3)
        comp["tsqr_speedup_vs_cholqr2"] = round(comp["cholqr2"]["ms"] / ms, 3)
        out["compare"] = comp

    if args.calib_copy:
        # a plain streaming kernel of known traffic for HBM-counter calibration:
        # torch.neg reads 1 GiB and writes 1 GiB (kernel name contains "neg")
        src = torch.empty(2 ** 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = src.numel() * 8
        del src, dst

    del X, work
    torch.cuda.empty_cache()

    if not args.no_sweep:
        out["sweep"] = bench_sweep(q, wl, dev, log, [int(v) for v in args.ns.split(",") if v],
                                   ks=tuple(int(v) for v in args.sweep_ks.split(",") if v),
                                   cpu_threads=cpu_threads, tuned=tuned, tuned_raw=tuned_raw)

    if not args.no_batched:
        out["batched"] = bench_batched(q, wl, dev, log)
    if not args.no_served:
        out["served"] = bench_served(q, dev, log, args.served_requests)

    print(json.dumps(out), flush=True)
    return 0


# CPU oracle timing in the sweep (k = 4): all host threads up to this n, one
# thread up to the smaller one -- together about 15 s of host work at 16 threads.
CPU_SWEEP_MAX_N_ALL = 32
CPU_SWEEP_MAX_N_ONE = 8


def bench_sweep(q, wl, dev, log, ns, m: int = 2 ** 25, ks=(0, 4, 8), cpu_threads=None, tuned=None,
                tuned_raw=None):
    """Column sweep m = 2^25, n in ns, sigma log-spaced to 10^-k, k in ks
    (default {0, 4, 8}): accuracy of TSQR and CholQR2 for every (n, k); timing
    (k = 4) of the TSQR launch (HIP events around it) and of the whole
    CholQR2 call; with cpu_threads, the CPU oracle (chunked sums) on the same
    matrix for the smaller n."""
    import numpy as np
    import torch
    sweep = []
    for ns in ns:
        rec = {"n": ns, "m": m, "rows_per_lane": q.qless_tune_get(ns)["rows_per_lane"]}
        tuned_n = q.qless_tune_get(ns) if tuned and ns in tuned else None
        if tuned_n is not None:
            rec["tuned"] = tuned_n
        for k in ks:
            log("sweep m=2^25 n=%d k=%d" % (ns, k))
            Xs, R0s = wl.config3(ns, k, m=m, device=dev)
            Rs = torch.empty((ns, ns), dtype=torch.float64, device=dev)
            ws, _ = q._workspace(q.QLESS_METHOD_TSQR, m, ns, dev)
            q.qless_tsqr_r(Xs, R=Rs, work=ws)
            Rc, info = q.cholqr2_r(Xs)
            torch.cuda.synchronize()
            nR0 = np.linalg.norm(R0s)
            rec["tsqr_e_R_k%d" % k] = float(np.linalg.norm(Rs.cpu().numpy() - R0s) / nR0)
            rec["cholqr2_e_R_k%d" % k] = float(np.linalg.norm(Rc.cpu().numpy() - R0s) / nR0)
            rec["cholqr2_info_k%d" % k] = int(info.item())
            if k == max(ks):
                # the robust Gram variants at the worst conditioning of the sweep
                for name, fn in (("shifted_cholqr3", q.shifted_cholqr3_r), ("cholqr2_dd", q.cholqr2_dd_r)):
                    Rv, iv = fn(Xs)
                    torch.cuda.synchronize()
                    rec["%s_e_R_k%d" % (name, k)] = float(np.linalg.norm(Rv.cpu().numpy() - R0s) / nR0)
                    rec["%s_info_k%d" % (name, k)] = int(iv.item())
                    del Rv, iv
            if k == 4:
                steps = 20 if ns <= 16 else 5
                flush = torch.ones(2 ** 27, dtype=torch.float64, device=dev) if ns <= 4 else None

                def f():
                    if flush is not None:      # evict the 256 MB MALL between calls: read 1 GiB
                        torch.sum(flush)       # (a read leaves no dirty lines to write back)
                    q.qless_tsqr_r(Xs, R=Rs, work=ws)

                def measure(fn):
                    """(stage-1 kernel ms, whole-call ms) averaged over `steps` calls"""
                    q.timing_reset()
                    q.timing_enable(True)
                    call_ms, _ = time_calls(fn, steps, 2)
                    q.timing_enable(False)
                    tot, cnt = q.timing_read("tsqr_stage1")
                    q.timing_reset()
                    return tot / max(cnt, 1), call_ms

                # tuned and default timed in interleaved rounds (median of 3), so
                # that a drift of the box over time weighs on both alike
                wd = None
                if tuned_n is not None:
                    q.qless_tune_set(ns, 0, 0, 0)
                    wd, _ = q._workspace(q.QLESS_METHOD_TSQR, m, ns, dev)
                    q.qless_tune_set(ns, *tuned_raw[ns])

                def fd():
                    if flush is not None:
                        torch.sum(flush)
                    q.qless_tsqr_r(Xs, R=Rs, work=wd)

                runs, druns = [], []
                for _ in range(3):
                    runs.append(measure(f))
                    if tuned_n is not None:
                        # the same calls with the library defaults, for tuned against default
                        # (stage-1 kernel time; the whole call where no flush is interleaved)
                        q.qless_tune_set(ns, 0, 0, 0)
                        druns.append(measure(fd))
                        q.qless_tune_set(ns, *tuned_raw[ns])
                med = lambda v: sorted(v)[len(v) // 2]
                k_avg, t_ms = med([r[0] for r in runs]), med([r[1] for r in runs])
                if druns:
                    rec["tsqr_ms_default"] = round(med([r[0] for r in druns]), 5)
                    if flush is None:
                        rec["tsqr_step_ms_default"] = round(med([r[1] for r in druns]), 5)
                del wd
                gbs = tsqr_bytes(m, ns) / (k_avg * 1e-3) / 1e9
                rec.update({"tsqr_ms": round(k_avg, 5), "tsqr_GBps": round(gbs, 1),
                            "tsqr_frac_hbm": round(gbs / HBM_PEAK_GBS, 4),
                            "tsqr_TFps": round(tsqr_flops(m, ns) / (k_avg * 1e-3) / 1e12, 2),
                            "tsqr_frac_fp64": round(tsqr_flops(m, ns) / (k_avg * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)})
                if flush is None:
                    rec["tsqr_step_ms"] = round(t_ms, 5)
                cw, _ = q._workspace(q.QLESS_METHOD_CHOLQR2, m, ns, dev)
                q.timing_reset()
                q.timing_enable(True)
                c_ms, _ = time_calls(lambda: q.cholqr2_r(Xs, work=cw), max(3, steps // 4), 1)
                q.timing_enable(False)
                g_ms, g_cnt = q.timing_read("gram")
                q.timing_reset()
                rec.update({"cholqr2_ms": round(c_ms, 5),
                            "cholqr2_gram_ms_per_pass": round(g_ms / max(g_cnt, 1), 5),
                            "cholqr2_GBps": round(gram2_bytes(m, ns) / (c_ms * 1e-3) / 1e9, 1),
                            "cholqr2_TFps": round(5.0 * m * ns * ns / (c_ms * 1e-3) / 1e12, 2)})
                del flush
                if cpu_threads and ns <= CPU_SWEEP_MAX_N_ALL:
                    import oracle
                    Xh = Xs.cpu().numpy()
                    _, tN = timed(lambda: oracle.householder_r_chunked(Xh, cpu_threads))
                    rec["cpu_oracle_GBps_all_threads"] = round(tsqr_bytes(m, ns) / tN / 1e9, 4)
                    rec["cpu_oracle_threads"] = cpu_threads
                    if ns <= CPU_SWEEP_MAX_N_ONE:
                        _, t1 = timed(lambda: oracle.householder_r_chunked(Xh, 1))
                        rec["cpu_oracle_GBps_1_thread"] = round(tsqr_bytes(m, ns) / t1 / 1e9, 4)
                    del Xh
            del Xs, ws
            torch.cuda.empty_cache()
        sweep.append(rec)
        log(json.dumps(rec))
    return sweep


def bench_batched(q, wl, dev, log, count: int = 512, seed: int = 4):
    """512 independent matrices (m log-uniform [1e4, 1e7], n in {4, 8, 16,
    32}, iid N(0,1), each its own device allocation) in one persistent
    stage-1 launch per width class plus the tree levels (eager and replayed
    from a captured graph) vs one qless_tsqr_r launch sequence per matrix."""
    import torch
    shapes = wl.batched_shapes(count, seed)
    Xs = [wl.gaussian_torch(m, n, seed=seed * 100_000 + i, device=dev) for i, (m, n) in enumerate(shapes)]
    torch.cuda.synchronize()
    total_bytes = sum(8 * m * n for m, n in shapes)
    log("batched: %d independent matrices, %.1f GB" % (count, total_bytes / 1e9))
    from paper_2603_20889_amd import autotune
    tuned = autotune.tune_batched(Xs, dev, log=log)
    plan = q.BatchPlan(Xs, tile_bytes=tuned["tile_bytes"], waves_per_cu=tuned["waves_per_cu"])
    plan.run()
    torch.cuda.synchronize()
    t_eager, _ = time_calls(plan.run, 5, 1)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        plan.run()
    torch.cuda.synchronize()
    t_graph, _ = time_calls(graph.replay, 5, 1)
    Rb = [R.clone() for R in plan.Rs]
    # one launch per matrix, same stream, workspace sized for the largest
    wmax = max(q.qless_workspace_bytes(q.QLESS_METHOD_TSQR, m, n) for m, n in shapes)
    work = torch.empty(wmax, dtype=torch.uint8, device=dev)
    Rs1 = [torch.empty((n, n), dtype=torch.float64, device=dev) for _, n in shapes]

    def singles():
        for X, R in zip(Xs, Rs1):
            q.qless_tsqr_r(X, R=R, work=work)
    t_single, _ = time_calls(singles, 3, 1)
    err = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(Rb, Rs1))
    by_width = {}
    for m, n in shapes:
        by_width[n] = by_width.get(n, 0) + 8 * m * n
    res = {"matrices": count, "independent_allocations": True, "total_GB": round(total_bytes / 1e9, 2),
           "GB_by_n": {str(k): round(v / 1e9, 2) for k, v in sorted(by_width.items())}, "tiles": plan.tiles,
           "tuned_plan": tuned,
           "batched_ms": round(t_eager, 3), "batched_graph_ms": round(t_graph, 3),
           "single_launches_ms": round(t_single, 3),
           "solves_per_s": round(count / (t_graph * 1e-3), 1),
           "solves_per_s_single": round(count / (t_single * 1e-3), 1),
           "GBps": round(total_bytes / (t_graph * 1e-3) / 1e9, 1),
           "max_rel_diff_vs_single": err}
    plan.close()
    log("batched: %s" % json.dumps(res))
    del Xs, work
    torch.cuda.empty_cache()
    return res


def bench_served(q, dev, log, count: int, loads=(0.5, 0.8, 0.95), pool_gb: float = 40.0, sample: int = 40):
    """Poisson least-squares requests [A b] (m log-uniform [1e4, 5e7], n in
    3..47): the continuous-batching server (running TSQR state per request,
    chunks of different requests on different streams, asynchronous
    completion) vs one request per launch (FIFO), at 0.5x, 0.8x and 0.95x of
    the measured one-at-a-time capacity.  Every request's [A b] is its own
    window of a device-resident N(0,1) pool (a random offset per request), so
    the data of all requests differ and none is generated inside the timed
    serving loop.  Accuracy: the served R([A b]) of a sample of requests
    against the same request solved alone."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2603_20889_amd.server import FifoServer, GpuExecutor, LstsqServer, make_requests

    pool_len = int(pool_gb * 1e9 / 8)
    pool = wl.gaussian_torch(pool_len, 1, seed=55, device=dev).view(-1)
    shapes = [(r.m, r.n) for r in make_requests(count, rate_per_s=1.0, seed=5)]
    g = wl.rng(56)
    offs = [int(g.integers(0, pool_len - m * (n + 1) + 1)) for m, n in shapes]
    data_fn = lambda r: pool[offs[r.id]:offs[r.id] + r.m * (r.n + 1)].view(r.m, r.n + 1)
    total_gb = sum(8 * m * (n + 1) for m, n in shapes) / 1e9
    log("served: %d requests, %.1f GB of [A b] in all, windows of a %.0f GB device pool" % (count, total_gb, pool_gb))
    reqs_at = lambda rate: make_requests(count, rate_per_s=rate, seed=5)
    warm = reqs_at(1e9)[:8]
    FifoServer(GpuExecutor(dev, data_fn=data_fn)).run(warm, realtime=False)
    torch.cuda.synchronize()
    probe = reqs_at(1e9)[:200]
    t0 = time.perf_counter()
    FifoServer(GpuExecutor(dev, data_fn=data_fn)).run(probe, realtime=False)
    torch.cuda.synchronize()
    capacity = len(probe) / (time.perf_counter() - t0)
    log("served: one-at-a-time capacity %.1f req/s" % capacity)
    fmt = lambda st: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}
    res = {"requests": count, "distinct_requests": count, "total_GB": round(total_gb, 1),
           "capacity_one_at_a_time_per_s": round(capacity, 1), "loads": []}
    bad = 0
    for load in loads:
        rate = load * capacity
        reqs = reqs_at(rate)
        srv = LstsqServer(GpuExecutor(dev, data_fn=data_fn, mode="state", keep_r=True),
                          hbm_budget_bytes=96 << 30, step_bytes=4 << 30, max_active=64)
        st_srv = fmt(srv.run(reqs, realtime=True))
        bad += sum(1 for r in reqs if r.info != 0)
        st_fifo = fmt(FifoServer(GpuExecutor(dev, data_fn=data_fn)).run(reqs_at(rate), realtime=True))
        # the served R of a sample against the same requests alone
        ids = sorted(set(int(i) for i in wl.rng(57).integers(0, count, sample)))
        err = 0.0
        for i in ids:
            r = reqs[i]
            Ra = q.qless_tsqr_r(data_fn(r))
            err = max(err, float(torch.linalg.norm(r.R - Ra) / torch.linalg.norm(Ra)))
        rec = {"load": load, "offered_rate_per_s": round(rate, 1), "server": st_srv, "fifo_one_per_launch": st_fifo,
               "sampled_requests": len(ids), "max_e_R_served_vs_alone": err}
        res["loads"].append(rec)
        log("served: %s" % json.dumps(rec))
        del reqs, srv
    res["failed"] = bad
    del pool
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    sys.exit(main())
