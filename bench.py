#!/usr/bin/env python3
"""Benchmark of the NNFFT (Algorithm 2.2) and the fast sinc transform
(Algorithm 6.1) on one MI355X.

Headline workload: N = 4096, M1 = M2 = 2^20, v_k, x_j iid uniform in
[-1/2, 1/2), f_k complex Gaussian, sigma1 = sigma2 = 2, m1 = m2 = 6 (seeded
synthetic inputs).  One step = one nnfft_exec (spreading, merge +
deconvolution + FFT, interpolation + correction) with the plan and all inputs
resident in HBM.

Reported (one JSON line):
  value          (M1 + M2) points/s of the FP32 compensated path over the timed steps
  step_ms        mean (wall clock), median and p99 (device span of each exec)
  fp64_plain     the same for the FP64 plain path (the comparator)
  rel_err_inf    E_inf of both results against the FP64 CPU oracle (all outputs)
  latency_ms     p50 / p99 of exec latency (submit to completion, one at a time)
  roofline       the dominant kernel's algorithmic bytes per launch / its
                 average duration; durations come from HIP events attached to
                 each kernel's dispatch during the timed steps (on the stream
                 the kernels run on); kernels: every FP32 kernel's fraction
  cpu_baseline   the FP64 CPU oracle NNFFT on the same workload
  sinc           the fast sinc transform: N = 1024, L1 = L2 = 2^18
                 Chebyshev-distributed nodes, 2048 Gauss-Legendre nodes,
                 (L1 + L2) points/s and E_inf against the direct sum (6.2)
  clustered      N = 16384, M1 = M2 = 2^24 nodes in 32 Gaussian clusters, m = 8:
                 pts/s (FP32, FP64), spreading GB/s, E_inf against the direct sum
  batched        the served request mix (N log-uniform in [64, 8192], M1, M2
                 log-uniform in [2^10, 2^20]) as resident plans run by
                 nnfft_exec_batch: FP32 (m=6) against FP64 plain (m=12) pts/s
  served         the same mix through the serving layer (plans built per
                 request, admitted by HBM footprint, continuous batching), all
                 10,000 requests: closed-loop capacity, then Poisson arrivals at
                 0.5, 0.8 and 1.0 times that rate with p50 / p99 latency
                 measured from each request's scheduled arrival
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NNFFT (M1+M2) pts/s at ≤1e-5 rel err, FP32 vs FP64 plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


# the sources of the exec kernels whose traffic the counter runs measured
KERNEL_SOURCES = ["kernels.hip", "internal.h"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2107_02671_amd", "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of each kernel from the rocprofv3 counter runs, if
    they were taken on the current kernel sources (else {})."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    if t.get("source_sha256") != kernel_source_hash():
        return {}
    return {k: float(v["bytes_per_launch"]) for k, v in t.get("kernels", {}).items()}


PROFILE_STATS = os.path.join(ROOT, "profiles", "nnfft_large_kernel_stats.txt")


def profiled_kernel_avg_ms():
    """Average kernel durations (ms) of the FP32 headline kernels in the
    committed rocprofv3 kernel-trace summary, if it was taken on the current
    kernel sources (else {})."""
    import csv
    import re
    try:
        with open(PROFILE_STATS) as fh:
            text = fh.read()
    except OSError:
        return {}
    if kernel_source_hash()[:16] not in text:
        return {}
    out = {}
    rows = [ln for ln in text.splitlines() if ln and not ln.startswith("#")]
    for r in csv.DictReader(rows):
        name = r["Name"]
        mt = re.search(r"nnfft::(k_\w+)", name)
        if not mt or "double" in name or "64" in mt.group(1):
            continue
        out.setdefault(mt.group(1), float(r["AverageNs"]) * 1e-6)
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def time_steps(fn, steps, warmup, torch, before=None):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if before is not None:
        before()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def pct(a, q):
    import numpy as np
    return float(np.percentile(np.asarray(a), q)) if len(a) else None


def kernel_bytes(name, M1, M2, info, b):
    """Algorithmic bytes per launch of one kernel (b: bytes per complex value).
    Spreading reads f and an 8-byte node record per point and writes the grid
    (G1 values); stage A reads the grid and writes the N2-point intermediate;
    stage B (or the one-workgroup FFT) writes the 2S + 1 consumed outputs;
    interpolation reads them and a record per point and writes y."""
    import math
    G1, N2 = info["G1"], info["N2"]
    # outputs |s| <= S of the FFT are consumed by the interpolation
    S = min(N2 // 2, math.ceil(N2 * info["N_star"] / (2 * info["N1"])) + info["m2"])
    rec = 8 if b == 8 else 12
    if name.startswith("k_spread"):
        return M1 * (b + rec) + G1 * b
    if name == "k_fft_stageA":
        return G1 * b + N2 * b
    if name == "k_fft_stageB":
        return N2 * b + (2 * S + 1) * b
    if name == "k_fft_single":
        return G1 * b + (2 * S + 1) * b
    if name.startswith("k_interp"):
        return M2 * (rec + b) + (2 * S + 1) * b
    return None


def profiled_steps(P, torch, plan, step, steps, warmup):
    """Three passes of `steps` execs: (1) the timed region, host clock around
    the whole pass, nothing else recorded; (2) a HIP event pair recorded on
    the stream around each exec, for the spread of the step time; (3) kernel
    events attached to every kernel dispatch (nnfft_profile_start), for each
    kernel's own duration.  The events of (2) and (3) add marker packets and
    host work between kernels, so (1) alone gives the throughput."""
    s = time_steps(step, steps, warmup, torch)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    spans = [a.elapsed_time(b) for a, b in ev]
    P.nnfft_profile_start(plan.handle, steps)
    for _ in range(steps):
        step()
    kern, _ = P.nnfft_profile_kernels(plan.handle, steps)
    return s, spans, kern


def roofline_table(kern, M1, M2, info, b, traffic):
    out = {}
    for k in kern:
        ab = kernel_bytes(k["name"], M1, M2, info, b)
        if ab is None:
            continue
        gbs = ab / (k["avg_ms"] * 1e-3) / 1e9
        out[k["name"]] = {"avg_ms": k["avg_ms"], "min_ms": k["min_ms"], "max_ms": k["max_ms"],
                          "algorithmic_bytes": ab, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                          "traffic": traffic.get(k["name"])}
    return out


def request_inputs(torch, req, fp32, dev):
    """Seeded device inputs of one served request: uniform nodes, complex Gaussian f."""
    g = torch.Generator(device=dev)
    g.manual_seed(4_000_000 + req["id"])
    v = torch.rand(req["M1"], dtype=torch.float64, device=dev, generator=g) - 0.5
    x = torch.rand(req["M2"], dtype=torch.float64, device=dev, generator=g) - 0.5
    cdt = torch.complex64 if fp32 else torch.complex128
    f = torch.randn(req["M1"], dtype=cdt, device=dev, generator=g)
    y = torch.empty(req["M2"], dtype=cdt, device=dev)
    return v, x, f, y


def sinc_benchmark(P, W, torch, steps, warmup, accuracy):
    """Fast sinc transform, N = 1024, L1 = L2 = 2^18 Chebyshev nodes, 2N
    Gauss-Legendre nodes, sigma = 2, m = 6."""
    import numpy as np
    dev = torch.device("cuda:0")
    N, a, b, c, w = W.nnfft_inputs("sinc")
    nq, sig, m = w["n_quad"], w["sigma"], w["m"]
    ta, tb = torch.tensor(a, device=dev), torch.tensor(b, device=dev)
    out = {"workload": "sinc_chebyshev_N1024_L2^18_GL2048_m6_sigma2", "N": N, "L1": len(a), "L2": len(b),
           "n_quad": nq, "quadrature": "Gauss-Legendre"}
    res = {}
    for name, prec, cdt in [("fp32", P.NNFFT_FP32_COMP, torch.complex64),
                            ("fp64", P.NNFFT_FP64_PLAIN, torch.complex128)]:
        t0 = time.perf_counter()
        sp = P.SincPlan(N, ta, tb, nq, P.SINC_QUAD_GAUSS_LEGENDRE, sig, sig, m, m, prec)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        mid = P.sinc_middle(sp.handle)
        tc = torch.tensor(c, dtype=cdt, device=dev)
        h = torch.empty(len(b), dtype=cdt, device=dev)
        st = torch.cuda.current_stream()
        fn = lambda: P.binding.lib().sinc_exec(sp.handle, P.binding._ptr(tc), P.binding._ptr(h),  # noqa: E731
                                               P.binding._stream(st))
        t = time_steps(fn, steps, warmup, torch)
        fn()
        torch.cuda.synchronize()
        res[name] = {"ms_per_step": t * 1e3, "value": (len(a) + len(b)) / t, "unit": "pts/s",
                     "plan_s": plan_s, "middle_operator": bool(mid["active"]), "h": h.cpu().numpy()}
        if mid["active"]:
            # the two-kernel form of the same plan, for reference
            P.sinc_middle(sp.handle, 0)
            res[name]["two_kernel_ms_per_step"] = time_steps(fn, steps, warmup, torch) * 1e3
            P.sinc_middle(sp.handle, 1)
        sp.close()
    for name in res:
        out[name] = {k: v for k, v in res[name].items() if k != "h"}
    if accuracy:
        import oracle
        idx = np.linspace(0, len(b) - 1, 1024).astype(np.int64)
        ho = oracle.sinc_direct(N, a, c + 0j, b[idx])
        den = np.abs(ho).max()
        out["rel_err_inf"] = {name: float(np.abs(res[name]["h"][idx] - ho).max() / den) for name in res}
        out["rel_err_inf"]["reference"] = "direct sum (6.2) in FP64 on 1024 evenly spaced outputs"
    return out


def clustered_benchmark(P, W, torch, steps, warmup, accuracy, traffic):
    """N = 16384, M1 = M2 = 2^24 nodes in 32 Gaussian clusters, m = 8."""
    import numpy as np
    dev = torch.device("cuda:0")
    N, v, x, f, w = W.nnfft_inputs("clustered")
    M1, M2, m, sig = len(v), len(x), w["m"], w["sigma"]
    tv, tx = torch.tensor(v, device=dev), torch.tensor(x, device=dev)
    out = {"workload": "nnfft_clustered32_N16384_M2^24_m8_sigma2", "N": N, "M1": M1, "M2": M2, "m": m,
           "nodes": "32 Gaussian clusters, std 1e-3, centres uniform in [-0.45, 0.45]"}
    ys = {}
    for name, prec, cdt, b in [("fp32", P.NNFFT_FP32_COMP, torch.complex64, 8),
                               ("fp64", P.NNFFT_FP64_PLAIN, torch.complex128, 16)]:
        t0 = time.perf_counter()
        p = P.Plan(N, tv, tx, sig, sig, m, m, prec)
        plan_s = time.perf_counter() - t0
        tf = torch.tensor(f, dtype=cdt, device=dev)
        y = torch.empty(M2, dtype=cdt, device=dev)
        st = torch.cuda.current_stream()
        fn = lambda: P.binding.lib().nnfft_exec(p.handle, P.binding._ptr(tf), P.binding._ptr(y),  # noqa: E731
                                                P.binding._stream(st))
        t, spans, kern = profiled_steps(P, torch, p, fn, steps, warmup)
        info = P.nnfft_info(p.handle)
        out[name] = {"ms_per_step": t * 1e3, "value": (M1 + M2) / t, "unit": "pts/s",
                     "step_ms_median": pct(spans, 50), "plan_s": plan_s,
                     "kernels": roofline_table(kern, M1, M2, info, b, traffic if name == "fp32" else {})}
        fn()
        torch.cuda.synchronize()
        ys[name] = y.cpu().numpy()
        p.close()
        del tf, y
    out["speedup_fp32_over_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    if accuracy:
        import oracle
        g = W.rng(55)
        idx = np.sort(g.choice(M2, 64, replace=False))
        yo = oracle.direct(N, v, f, x[idx])
        den = np.abs(yo).max()
        out["rel_err_inf"] = {name: float(np.abs(ys[name][idx] - yo).max() / den) for name in ys}
        out["rel_err_inf"]["reference"] = "direct sum (1.2) in FP64 on 64 random outputs"
    return out


def batched_benchmark(P, W, torch, nplans, reps=20):
    """Resident plans of the served mix, one nnfft_exec_batch per step."""
    dev = torch.device("cuda:0")
    reqs = W.served_requests(nplans * 4, seed=4)
    out = {}
    for name, fp32, prec, m in [("fp32", True, P.NNFFT_FP32_COMP, 6), ("fp64", False, P.NNFFT_FP64_PLAIN, 12)]:
        sel = [r for r in reqs if r["fp32"] == fp32][:nplans]
        plans, fs, ys, pts = [], [], [], 0
        for r in sel:
            v, x, f, y = request_inputs(torch, r, fp32, dev)
            plans.append(P.Plan(r["N"], v, x, 2.0, 2.0, m, m, prec))
            fs.append(f)
            ys.append(y)
            pts += r["M1"] + r["M2"]
        handles = [p.handle for p in plans]
        t = time_steps(lambda: P.nnfft_exec_batch(handles, fs, ys), reps, 3, torch)
        out[name] = {"plans": len(plans), "points_per_step": pts, "ms_per_step": t * 1e3,
                     "value": pts / t, "unit": "pts/s", "m": m}
        for p in plans:
            p.close()
    out["speedup_fp32_over_fp64"] = out["fp32"]["value"] / out["fp64"]["value"]
    return out


def served_benchmark(P, W, torch, n_req, planners=12, budget=16 << 30):
    """The served request stream: closed loop for capacity, then Poisson
    arrivals.  Under Poisson arrivals a request's latency runs from its
    scheduled arrival (not from its submit call) to its completion, so time
    the generator spends behind schedule counts against the server.

    Request inputs are windows of seeded device pools (2^21 uniform nodes per
    side, complex Gaussian coefficients in both precisions) at seeded random
    offsets, so that submitting a request costs no generation work (the
    server handle keeps each request's arrays referenced until it is
    waited for)."""
    import threading

    import numpy as np
    dev = torch.device("cuda:0")
    reqs = W.served_requests(10000, seed=4)[:n_req]
    pool = 1 << 21
    g = torch.Generator(device=dev)
    g.manual_seed(4_000_000)
    v_pool = torch.rand(pool, dtype=torch.float64, device=dev, generator=g) - 0.5
    x_pool = torch.rand(pool, dtype=torch.float64, device=dev, generator=g) - 0.5
    f_pool = {True: torch.randn(pool, dtype=torch.complex64, device=dev, generator=g),
              False: torch.randn(pool, dtype=torch.complex128, device=dev, generator=g)}
    offs = W.rng(44).integers(0, pool - (1 << 20), (len(reqs), 2))
    torch.cuda.synchronize()

    def run(rate):
        srv = P.Server(hbm_budget_bytes=budget, planner_threads=planners, streams=2)
        results = [None] * len(reqs)
        tickets = [None] * len(reqs)
        t_sub = np.zeros(len(reqs))      # perf_counter just before each submit call
        t_sched = np.zeros(len(reqs))    # scheduled arrival (perf_counter clock)
        ready = threading.Semaphore(0)
        window = threading.Semaphore(256)      # at most 256 outstanding (input memory)

        def collect():
            for i in range(len(reqs)):
                ready.acquire()
                results[i] = srv.wait(tickets[i])
                window.release()

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        arrival = 0.0
        for i, r in enumerate(reqs):
            if rate is not None:
                arrival += r["gap"] / rate
                t_sched[i] = t0 + arrival
                while time.perf_counter() < t_sched[i]:
                    time.sleep(min(1e-3, max(0.0, t_sched[i] - time.perf_counter())))
            window.acquire()
            o1, o2 = int(offs[i, 0]), int(offs[i, 1])
            v, x = v_pool[o1:o1 + r["M1"]], x_pool[o2:o2 + r["M2"]]
            f = f_pool[r["fp32"]][o1:o1 + r["M1"]]
            y = torch.empty(r["M2"], dtype=f.dtype, device=dev)
            prec = P.NNFFT_FP32_COMP if r["fp32"] else P.NNFFT_FP64_PLAIN
            t_sub[i] = time.perf_counter()
            tickets[i] = srv.submit(r["N"], v, x, f, y, sigma1=2.0, sigma2=2.0, m1=r["m"], m2=r["m"], prec=prec)
            if rate is None:
                t_sched[i] = t_sub[i]
            ready.release()
        th.join()
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        sub_ms = np.array([res["submit_ms"] for res in results])
        done_ms = np.array([res["done_ms"] for res in results])
        built = [res for res in results if res["status"] == 0 and not res["plan_reused"]]
        plan_ms = np.array([res["admit_ms"] - res["plan_ms"] for res in built]) if built else np.zeros(1)
        queue_ms = np.array([res["plan_ms"] - res["submit_ms"] for res in results])
        # server clock (ms since its creation, steady clock) -> perf_counter
        # seconds (both CLOCK_MONOTONIC): the submit stamp is taken inside the
        # submit call, after t_sub, so every t_sub - submit stamp is at most
        # the offset and the largest one is the closest
        off = float(np.max(t_sub - sub_ms * 1e-3))
        done = done_ms * 1e-3 + off
        lat = (done - t_sched) * 1e3
        lag = (t_sub - t_sched) * 1e3
        ok = sum(res["status"] == 0 for res in results)
        pts = sum(r["M1"] + r["M2"] for r in reqs)
        return {"requests": len(reqs), "ok": ok, "wall_s": wall, "req_per_s": len(reqs) / wall,
                "value": pts / wall, "unit": "pts/s", "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "latency_from": "submit" if rate is None else "scheduled arrival",
                "server_p50_ms": pct(done_ms - sub_ms, 50), "server_p99_ms": pct(done_ms - sub_ms, 99),
                "generator_lag_ms": {"p50": pct(lag, 50), "p99": pct(lag, 99), "max": float(lag.max())},
                "planning_ms": {"mean": float(plan_ms.mean()), "p50": pct(plan_ms, 50), "p99": pct(plan_ms, 99),
                                "kind": "planner took the request up -> plan admitted into the arena"},
                "queue_ms": {"p50": pct(queue_ms, 50), "p99": pct(queue_ms, 99),
                             "kind": "submitted -> a planner took it up"},
                "mean_group": float(np.mean([res["group_size"] for res in results])),
                "admission_waits": st["admission_waits"], "arena_peak_bytes": st["arena_peak"]}

    closed = run(None)
    out = {"closed_loop": closed, "planner_threads": planners, "hbm_budget_bytes": budget,
           "mix": "N logU[64,8192], M1,M2 logU[2^10,2^20], FP32 m=6 / FP64 m=12 (1:1), uniform nodes"}
    cap = closed["req_per_s"]
    for frac in (0.5, 0.8, 1.0):
        print(f"[bench] served, Poisson arrivals at {frac} x {cap:.0f} req/s", file=sys.stderr, flush=True)
        out[f"poisson_{frac}"] = run(frac * cap)
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="skip the FP64 plain comparator")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 256 MiB device copy (counter calibration runs)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per served run (the request stream has 10000; 0 skips)")
    ap.add_argument("--batch-plans", type=int, default=48,
                    help="resident plans per precision in the batched measurement (0 skips)")
    ap.add_argument("--no-sinc", action="store_true", help="skip the fast sinc transform leg")
    ap.add_argument("--no-clustered", action="store_true", help="skip the clustered 2^24-node leg")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): this implementation "
              f"targets a single MI355X; see DESIGN.md for how the transform would shard.", flush=True)
        return 2

    import numpy as np
    import torch

    import paper_2107_02671_amd as P
    from paper_2107_02671_amd import workloads as W

    dev = torch.device("cuda:0")
    traffic = measured_traffic()
    N, v, x, f, w = W.nnfft_inputs("large")
    M1, M2, m, sig = len(v), len(x), w["m"], w["sigma"]
    tv = torch.tensor(v, device=dev)
    tx = torch.tensor(x, device=dev)
    f32 = torch.tensor(f, dtype=torch.complex64, device=dev)
    f64 = torch.tensor(f, dtype=torch.complex128, device=dev)
    print(f"[bench] plans N={N} M1={M1} M2={M2} m={m}", file=sys.stderr, flush=True)
    t_plan = time.perf_counter()
    p32 = P.Plan(N, tv, tx, sig, sig, m, m, P.NNFFT_FP32_COMP)
    t_plan32 = time.perf_counter() - t_plan
    t_plan = time.perf_counter()
    p64 = P.Plan(N, tv, tx, sig, sig, m, m, P.NNFFT_FP64_PLAIN)
    t_plan64 = time.perf_counter() - t_plan
    y32 = torch.empty(M2, dtype=torch.complex64, device=dev)
    y64 = torch.empty(M2, dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def step32():
        P.binding.lib().nnfft_exec(p32.handle, P.binding._ptr(f32), P.binding._ptr(y32),
                                   P.binding._stream(stream))

    def step64():
        P.binding.lib().nnfft_exec(p64.handle, P.binding._ptr(f64), P.binding._ptr(y64),
                                   P.binding._stream(stream))

    # timed region: exactly `steps` FP32 execs, synchronized on both sides;
    # then the same steps again with events (step spread, kernel durations)
    print(f"[bench] timing FP32 ({args.steps} steps)", file=sys.stderr, flush=True)
    s32, spans32, kern32 = profiled_steps(P, torch, p32, step32, args.steps, args.warmup)
    if not args.fp32_only:
        print(f"[bench] timing FP64 plain ({args.steps} steps)", file=sys.stderr, flush=True)
        s64, spans64, kern64 = profiled_steps(P, torch, p64, step64, args.steps, args.warmup)
    else:
        s64, spans64, kern64 = float("nan"), [], []

    # exec latency, one call at a time
    lat = []
    for _ in range(100):
        t0 = time.perf_counter()
        step32()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)

    info32 = P.nnfft_info(p32.handle)
    info64 = P.nnfft_info(p64.handle)
    out = {
        "metric": METRIC,
        "value": (M1 + M2) / s32,
        "unit": "pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": s32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "nnfft_uniform_N4096_M2^20_m6_sigma2", "N": N, "M1": M1, "M2": M2,
                   "sigma1": sig, "sigma2": sig, "m1": m, "m2": m,
                   "nodes": "iid uniform [-1/2,1/2)", "coefficients": "complex Gaussian",
                   "precision": "FP32 data path, two-sum compensated grid cells, FP64 phi_hat"},
        "step_ms": {"mean": s32 * 1e3, "median": pct(spans32, 50), "p99": pct(spans32, 99),
                    "min": float(min(spans32)),
                    "kind": "mean: host clock over the timed steps; median/p99/min: HIP event pair "
                            "recorded on the stream around each of the same number of execs"},
        "fp64_plain": {"value": (M1 + M2) / s64, "unit": "pts/s", "ms_per_step": s64 * 1e3,
                       "step_ms_median": pct(spans64, 50), "step_ms_p99": pct(spans64, 99),
                       "speedup_fp32_over_fp64": s64 / s32,
                       "kernels": roofline_table(kern64, M1, M2, info64, 16, {})},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                       "kind": "single exec, submit to completion"},
        "plan_s": {"fp32": t_plan32, "fp64": t_plan64},
    }
    out["plan_info"] = {k: info32[k] for k in ["N_star", "N1", "G1", "N2", "fft_n1", "fft_n2",
                                               "spread_workgroups", "interp_workgroups",
                                               "items_points", "block_points", "window_degree",
                                               "window_fit_err", "corr_degree"]}

    # roofline: every FP32 kernel's algorithmic bytes per launch over its
    # average dispatch duration in the timed steps; the dominant kernel (the
    # longest) is the headline figure
    kt = roofline_table(kern32, M1, M2, info32, 8, traffic)
    dom = max(kt, key=lambda k: kt[k]["avg_ms"])
    d = kt[dom]
    prof = profiled_kernel_avg_ms()
    for kname, rec in kt.items():
        if kname in prof:
            rec["profile_avg_ms"] = prof[kname]
            rec["frac_from_profile"] = rec["algorithmic_bytes"] / (prof[kname] * 1e-3) / 1e9 / HBM_PEAK_GBS
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": d["frac"], "traffic": d["traffic"],
                       "algorithmic_bytes_per_launch": d["algorithmic_bytes"], "avg_launch_ms": d["avg_ms"],
                       "launches_timed": args.steps,
                       "profile_avg_ms": d.get("profile_avg_ms"), "frac_from_profile": d.get("frac_from_profile"),
                       "timing": "HIP events attached to each kernel dispatch (hipExtLaunchKernel) over "
                                 "as many execs as the timed steps, on the exec stream",
                       "kernels": kt}

    if not args.no_accuracy or not args.no_cpu_baseline:
        import oracle
    if not args.no_accuracy:
        print("[bench] accuracy vs FP64 oracle", file=sys.stderr, flush=True)
        step32()
        if not args.fp32_only:
            step64()
        torch.cuda.synchronize()
        yo = oracle.nnfft(N, v, f, x, sig, sig, m, m)
        den = np.abs(yo).max()
        out["rel_err_inf"] = {
            "fp32": float(np.abs(y32.cpu().numpy() - yo).max() / den),
            "fp64": float(np.abs(y64.cpu().numpy() - yo).max() / den),
            "reference": "FP64 CPU oracle NNFFT, all M2 outputs"}
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        reps, tot = 0, 0.0
        while reps < 200 and tot < 12.0:
            t0 = time.perf_counter()
            oracle.nnfft(N, v, f, x, sig, sig, m, m)
            tot += time.perf_counter() - t0
            reps += 1
        out["cpu_baseline"] = {"value": (M1 + M2) * reps / tot, "unit": "pts/s",
                               "cores": oracle.num_threads(), "kind": "oracle",
                               "cpu_model": cpu_model(), "nproc": os.cpu_count(),
                               "affinity_cpus": len(os.sched_getaffinity(0)),
                               "sample": f"full workload (M1=M2=2^20, N=4096, m=6), {reps} runs of "
                                         f"the FP64 oracle NNFFT (plan + all steps), {tot:.1f} s"}
    p32.close()
    p64.close()
    del f32, f64, y32, y64, tv, tx
    if not args.no_sinc:
        print("[bench] fast sinc transform", file=sys.stderr, flush=True)
        out["sinc"] = sinc_benchmark(P, W, torch, max(20, args.steps // 4), 5, not args.no_accuracy)
    if not args.no_clustered:
        print("[bench] clustered 2^24-node transform", file=sys.stderr, flush=True)
        out["clustered"] = clustered_benchmark(P, W, torch, 20, 3, not args.no_accuracy, traffic)
    if args.batch_plans > 0:
        print("[bench] batched resident plans", file=sys.stderr, flush=True)
        out["batched"] = batched_benchmark(P, W, torch, args.batch_plans)
    if args.serve_requests > 0:
        print("[bench] served request stream", file=sys.stderr, flush=True)
        out["served"] = served_benchmark(P, W, torch, args.serve_requests)
    if args.calibrate_copy:
        a = torch.empty(1 << 26, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = {"read": a.numel() * 4, "write": b.numel() * 4}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
