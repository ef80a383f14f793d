#!/usr/bin/env python3
"""Benchmark: pairs/s of the fused log-likelihood + gradient of the spatiotemporal Hawkes model
(arXiv 2005.10123, Section 2.1) at N = 85,000 events on one MI355X, FP32-compensated path, with the
FP64 path beside it, the pairwise kernel's VALU roofline, the FP64 oracle on the host as a CPU
baseline, and p50/p99 latency of batched requests from many concurrent chains.

One step = one blocking hawkes_grad call on the resident dataset (pairwise pass, per-event
epilogue, fixed-order reduction, 56-byte readback).  pairs/s = N^2 / seconds per step.  Before the
warm-up steps, 0.25 s of untimed evaluations bring the device to its steady clock.
Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Roofline of the pairwise pass (per ordered pair, averaged over the N^2 pairs of which about half
# are causal): 13.5 FP32 lane operations (FMA = 1) and 1.5 exponentials for log-likelihood +
# gradient; 10.5 and 1.5 for the log-likelihood alone.
WORK = {True: (13.5, 1.5), False: (10.5, 1.5)}
# The symmetric enumeration (the default pass) evaluates each unordered pair once: 3 differences,
# 2 for r^2, 1 for dt^2, 1 background and 2 trigger exponent arguments, the background term and its
# two moments added to both events (6) and the trigger term and its two moments to the later one
# (3), i.e. 18 lane operations and 2 exponentials per unordered pair = 9 and 1 per ordered pair.
# Without the gradient: 7 + 2 + 1 + 1 + 2 (background term to both events) + 2 + 1 = 16 and 2 per
# unordered pair = 8 and 1 per ordered pair.
WORK_SYM = {True: (9.0, 1.0), False: (8.0, 1.0)}
CUS, CLOCK = 256, 2.4e9
P_OPS32 = 157.3e12 / 2          # FP32 vector: 157.3 TFLOP/s with FMA = 2 FLOP
P_OPS64 = 78.6e12 / 2           # FP64 vector
P_EXP32 = CUS * 32 * CLOCK      # v_exp_f32 lanes per second (32 per CU per clock, measured)
FP64_EXP_OPS = 15               # FP64 lane operations of one exp2 (range reduction + degree-10 poly)


KERNEL_SOURCES = ("hawkes_kernels.hip", "hawkes_device.h", "hawkes_internal.h")


def leg(name, fn, *args, **kwargs):
    """Run one part of the bench and note on stderr that it ended (the JSON line stays on stdout)."""
    a = time.perf_counter()
    r = fn(*args, **kwargs)
    print(json.dumps({"done": name, "seconds": round(time.perf_counter() - a, 2)}), file=sys.stderr, flush=True)
    return r


def kernel_source_sha256() -> str:
    """sha256 over the code (comments and blank lines dropped) of the sources compiled into the
    pairwise kernels, in KERNEL_SOURCES order."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_2005_10123_amd", "csrc", name)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(line.rstrip() for line in text.splitlines() if line.strip()).encode())
    return h.hexdigest()


def measured_traffic(record: str):
    """HBM bytes per launch of the pairwise kernel from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    recorded in profiles/ (copy-calibrated), or None when the kernel sources changed since."""
    try:
        rec = json.load(open(record))
        sha = kernel_source_sha256()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def roofline_pairs(grad: bool, fp64: bool = False, executed: bool = False) -> float:
    """Ordered pairs per second at the chip's peak rates for the method's work per ordered pair
    (the direct enumeration's), or with ``executed`` for the work the symmetric pass executes."""
    ops, exps = WORK_SYM[grad] if executed else WORK[grad]
    if fp64:
        return 1.0 / ((ops + exps * FP64_EXP_OPS) / P_OPS64)
    return 1.0 / (ops / P_OPS32 + exps / P_EXP32)


def oracle_errors(ell, g, ref, theta):
    """Errors of one GPU result against the oracle's whole evaluation: relative error of ell and,
    per gradient component, the plain relative error, the error over the l1 norm of the per-event
    terms (sum_i |g_i,p|) and the cancellation factor kappa_p = sum_i |g_i,p| / |g_p|."""
    out = {"ell_rel": abs(ell - ref["ell"]) / abs(ref["ell"])}
    if g is not None:
        g = np.asarray(g, float)
        l1 = np.abs(ref["row_grad"]).sum(axis=0)
        out["grad_plain_rel"] = (np.abs(g - ref["grad"]) / np.maximum(np.abs(ref["grad"]), 1e-300)).tolist()
        out["grad_l1_normalised"] = (np.abs(g - ref["grad"]) / np.maximum(l1, 1e-300)).tolist()
        out["kappa"] = (l1 / np.maximum(np.abs(ref["grad"]), 1e-300)).tolist()
    return out


def time_steps(ctx, ds, theta, precision, grad, steps, warmup, spin_up_s=0.0):
    """Time `steps` blocking evaluations after `warmup` untimed ones.  spin_up_s: seconds of
    further untimed evaluations before the warm-up, so the timed steps run at the device's steady
    clock (it ramps up over the first ~25 ms of back-to-back passes)."""
    import torch

    call = (lambda: ctx.grad(ds, theta, precision)) if grad else (lambda: ctx.loglik(ds, theta, precision))
    t_spin = time.perf_counter()
    while time.perf_counter() - t_spin < spin_up_s:
        call()
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ctx.kernel_time(reset=True)
    ctx.profile(True)
    per = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        out = call()
        per.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.profile(False)
    kms, launches = ctx.kernel_time(reset=True)
    return out, wall, np.array(per), kms / max(launches, 1)


def cpu_baseline(x, y, t, theta, budget_s=12.0):
    """The FP64 oracle (single thread) on a bounded sample: evenly spaced rows against all N columns."""
    import oracle

    n = x.size
    probe = np.linspace(0, n - 1, 8).astype(np.int64)
    a = time.perf_counter()
    oracle.rows(x, y, t, theta, probe)
    per_row = (time.perf_counter() - a) / probe.size
    m = int(max(8, min(n, budget_s / max(per_row, 1e-9))))
    idx = np.linspace(0, n - 1, m).astype(np.int64)
    a = time.perf_counter()
    oracle.rows(x, y, t, theta, idx)
    sec = time.perf_counter() - a
    return {"value": m * n / sec, "unit": "pairs/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{m} evenly spaced events (rows) of the {n}-event workload, each against all {n} "
                      f"events, log-likelihood + gradient terms, single-threaded FP64 C; {sec:.1f} s",
            "per_row_s": sec / m}


def cpu_all_cores_run(x, y, t, theta):
    """The same FP64 oracle over the whole workload, its rows split into contiguous ranges run on
    the host's cores (one thread each, at most 16): the multi-core host context, and the oracle's
    whole result that every GPU result of this workload is compared with."""
    import oracle

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    n = x.size
    a = time.perf_counter()
    ref = oracle.evaluate_parallel(x, y, t, theta, threads=threads)
    sec = time.perf_counter() - a
    return {"value": float(n) * n / sec, "unit": "pairs/s", "cores": threads, "kind": "oracle", "seconds": sec,
            "sample": f"all {n} events of the workload against all {n}, split into {threads} contiguous row "
                      f"ranges run concurrently"}, ref


def host_simd_run(x, y, t, theta, ref):
    """The library's host evaluation (hawkes_host_eval: the paper's multi-core CPU design with SIMD
    loops, binary64, every ordered pair) on the whole workload over the host's cores (at most 16),
    against the oracle's whole evaluation."""
    from paper_2005_10123_amd import binding

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    n = x.size
    binding.host_eval(x[:2000], y[:2000], t[:2000], theta, threads=threads)  # warm-up
    a = time.perf_counter()
    ell, g = binding.host_eval(x, y, t, theta, threads=threads)
    sec = time.perf_counter() - a
    return {"value": float(n) * n / sec, "unit": "pairs/s", "cores": threads, "seconds": sec,
            "kind": "hawkes_host_eval (multi-core SIMD, binary64)",
            "sample": f"all {n} events of the workload against all {n}",
            "vs_oracle": oracle_errors(ell, g, ref, theta)}


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gfx_clocks_ghz():
    """Graphics clocks (GHz) that amd-smi reports now, per GPU it lists: {gpu: [one per XCD]}, or None."""
    import re
    import subprocess
    try:
        r = subprocess.run(["amd-smi", "metric", "-c", "--json"], capture_output=True, text=True, timeout=30)
        data = json.loads(r.stdout)
    except (OSError, ValueError, subprocess.SubprocessError):
        return None
    clocks = {}

    def walk(o, path):
        if isinstance(o, dict):
            for k, v in o.items():
                walk(v, path + [str(k)])
        elif isinstance(o, list):
            for i, v in enumerate(o):
                walk(v, path + [str(i)])
        elif isinstance(o, (int, float)):
            m = re.search(r"(^|/)(\d+)/clock/gfx_\d+/clk/value$", "/".join(path))
            if m:
                clocks.setdefault(int(m.group(2)), []).append(o / 1e3)

    walk(data, [])
    return clocks or None


def engine_clock(ctx, ds, theta, nsamples=2):
    """The graphics clock while the FP32C gradient runs back to back: amd-smi sampled under that
    load, after a second of it (its reading lags a change of load by a fraction of a second); of
    the GPUs it lists, the one with the highest mean clock (the loaded one).  None where amd-smi
    is unavailable."""
    import threading
    stop = threading.Event()
    done = [0]

    def load():
        while not stop.is_set():
            ctx.grad(ds, theta, "fp32c")
            done[0] += 1

    worker = threading.Thread(target=load)
    worker.start()
    samples = []
    try:
        time.sleep(1.0)
        for _ in range(nsamples):
            c = gfx_clocks_ghz()
            if c is None:
                break
            gpu = max(c, key=lambda k: sum(c[k]) / len(c[k]))
            samples.append(c[gpu])
            time.sleep(0.25)
    finally:
        stop.set()
        worker.join()
    if not samples:
        return None
    per_xcd = [sum(v) / len(v) for v in zip(*samples)]
    return {"measured_ghz": sum(per_xcd) / len(per_xcd), "per_xcd_ghz": per_xcd, "samples": len(samples),
            "evaluations_meanwhile": done[0]}


def cpu_full_run():
    """One-off: the FP64 oracle over whole workloads on the host (not part of the default run):
    the 2,000-event workload, a seeded 20,000-event subsample of the 10^6-event one, and the full
    85,000-event gradient workload single-threaded and over all host cores (row partitions).
    Minutes of CPU work."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_2005_10123_amd import synth

    out = {"cpu_model": cpu_model(), "host_threads": len(os.sched_getaffinity(0)), "runs": []}
    (x, y, t), th = synth.config_events("small_2k")
    a = time.perf_counter()
    oracle.evaluate(x, y, t, th)
    sec = time.perf_counter() - a
    out["runs"].append({"workload": "small_2k", "n_events": x.size, "threads": 1, "seconds": sec,
                        "pairs_per_s": float(x.size) ** 2 / sec})
    (x, y, t), th = synth.config_events("stress_1m")
    xs, ys, ts = synth.subsample(x, y, t, 20000)
    a = time.perf_counter()
    oracle.evaluate(xs, ys, ts, th)
    sec = time.perf_counter() - a
    out["runs"].append({"workload": "stress_1m subsample", "n_events": xs.size, "threads": 1, "seconds": sec,
                        "pairs_per_s": float(xs.size) ** 2 / sec})
    (x, y, t), th = synth.config_events("city_85k_10km")
    n = x.size
    print(json.dumps({"progress": "city_85k_10km single thread: starting"}), flush=True)
    a = time.perf_counter()
    ell, _ = oracle.evaluate(x, y, t, th)
    sec = time.perf_counter() - a
    print(json.dumps({"progress": "city_85k_10km single thread", "seconds": sec}), flush=True)
    out["runs"].append({"workload": "city_85k_10km", "n_events": n, "threads": 1, "seconds": sec,
                        "pairs_per_s": float(n) ** 2 / sec, "loglik": ell})
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    parts = np.array_split(np.arange(n), threads)
    with ThreadPoolExecutor(threads) as pool:
        a = time.perf_counter()
        list(pool.map(lambda r: oracle.rows(x, y, t, th, r), parts))
        sec = time.perf_counter() - a
    out["runs"].append({"workload": "city_85k_10km", "n_events": n, "threads": threads, "seconds": sec,
                        "pairs_per_s": float(n) ** 2 / sec})
    return out


THETA_POSTERIOR = (1.0, 1.6, 14.0, 0.153, 1440.0, 0.0695)


def posterior_regime(ctx):
    """FP32C against FP64 (both on the GPU) at the paper's posterior regime, on the 85,000-event
    15 km / 5,000-day workload: tau_x = 1.6 km and tau_t = 14 days as fixed in Section 2.1, and the
    Section 3.2 posterior means h = 69.5 m, omega = 1440 per day (1 / omega = one minute),
    theta = 0.153 (mu0 = 1, not reported).  A stress of binary32 time resolution: reported, not gated."""
    from paper_2005_10123_amd import synth

    (x, y, t), _ = synth.config_events("city_85k_15km")
    ds = ctx.dataset(x, y, t)
    ell32, g32 = ctx.grad(ds, THETA_POSTERIOR, "fp32c")
    ell64, g64 = ctx.grad(ds, THETA_POSTERIOR, "fp64")
    rows = ctx.rows(ds, THETA_POSTERIOR, "fp64")
    ds.close()
    l1 = np.abs(rows["grad"]).sum(axis=0)
    floor = abs(ell64) / np.maximum(np.abs(np.asarray(THETA_POSTERIOR)), 1.0)
    return {"workload": "city_85k_15km", "theta": list(THETA_POSTERIOR), "loglik_fp64": ell64,
            "ell_rel": abs(ell32 - ell64) / abs(ell64),
            "grad_l1_normalised": (np.abs(g32 - g64) / np.maximum(l1, floor)).tolist(),
            "grad_plain_rel": (np.abs(g32 - g64) / np.abs(g64)).tolist()}


def loglik_workload(ctx, steps=20):
    """The log-likelihood-only workload (85,000 events on 15 x 15 km over 5,000 days): both
    precisions, kernel and call times (after a spin-up to the steady clock, as for the timed
    steps), FP32C against FP64."""
    from paper_2005_10123_amd import synth

    (x, y, t), theta = synth.config_events("city_85k_15km")
    n = x.size
    ds = ctx.dataset(x, y, t)
    out = {"workload": "city_85k_15km", "n_events": n, "theta": list(theta)}
    ell = {}
    for prec in ("fp32c", "fp64"):
        ell[prec], wall, _, kms = time_steps(ctx, ds, theta, prec, False, steps, 2,
                                             spin_up_s=0.25 if prec == "fp32c" else 0.1)
        achieved = float(n) * n / (kms * 1e-3)
        out[prec] = {"ms_per_call": wall / steps * 1e3, "kernel_ms": kms, "pairs_per_s": float(n) * n * steps / wall,
                     # the pairwise kernel against the roofline of the work it executes
                     "roofline_frac": achieved / roofline_pairs(False, prec == "fp64", executed=True)}
        if prec == "fp32c":
            # and against the roofline of the method's work (the direct enumeration's)
            out[prec]["method_work_frac"] = achieved / roofline_pairs(False)
    ds.close()
    out["ell_rel_fp32c_vs_fp64"] = abs(ell["fp32c"] - ell["fp64"]) / abs(ell["fp64"])
    out["ell"] = ell
    out["events"] = (x, y, t)
    return out


def small_workload(ctx, steps=20):
    """The 2,000-event workload (10 x 10 km, 1,000 days): one log-likelihood per call, FP64 (its
    stated precision) and FP32C beside it, call and pairwise-kernel times.  The oracle's whole
    evaluation of it is compared with both in the CPU leg."""
    from paper_2005_10123_amd import synth

    (x, y, t), theta = synth.config_events("small_2k")
    n = x.size
    ds = ctx.dataset(x, y, t)
    out = {"workload": "small_2k", "n_events": n, "theta": list(theta)}
    for prec in ("fp64", "fp32c"):
        ell, wall, _, kms = time_steps(ctx, ds, theta, prec, False, steps, 3)
        out[prec] = {"ms_per_call": wall / steps * 1e3, "kernel_ms": kms, "pairs_per_s": float(n) * n * steps / wall,
                     "ell": ell}
    ds.close()
    return out, (x, y, t, theta)


def stress_workload(ctx):
    """The 1,000,000-event workload (40 x 40 km, 20,000 days): FP32C and FP64 log-likelihood +
    gradient at full size, compared with each other, and a seeded 20,000-event subsample evaluated
    as its own dataset by both precisions (compared with the oracle in the CPU leg)."""
    from paper_2005_10123_amd import synth

    (x, y, t), theta = synth.config_events("stress_1m")
    n = x.size
    ds = ctx.dataset(x, y, t)
    out = {"workload": "stress_1m", "n_events": n, "theta": list(theta)}
    res = {}
    for prec in ("fp32c", "fp64"):
        res[prec], wall, _, kms = time_steps(ctx, ds, theta, prec, True, 1, 1)
        out[prec] = {"ms_per_call": wall * 1e3, "kernel_ms": kms, "pairs_per_s": float(n) * n / wall}
    rows64 = ctx.rows(ds, theta, "fp64")
    ds.close()
    (e32, g32), (e64, g64) = res["fp32c"], res["fp64"]
    l1 = np.abs(rows64["grad"]).sum(axis=0)
    out["fp32c_vs_fp64"] = {"ell_rel": abs(e32 - e64) / abs(e64),
                            "grad_plain_rel": (np.abs(g32 - g64) / np.abs(g64)).tolist(),
                            "grad_l1_normalised": (np.abs(g32 - g64) / l1).tolist()}
    xs, ys, ts = synth.subsample(x, y, t, 20000)
    ds = ctx.dataset(xs, ys, ts)
    sub = {prec: ctx.grad(ds, theta, prec) for prec in ("fp32c", "fp64")}
    ds.close()
    return out, (xs, ys, ts, theta, sub)


def zero_skip_run(ctx, steps=10):
    """Zero-tile skipping (off by default; hawkes_set_zero_tile_skipping): the same evaluations
    with column tiles whose pair terms are all exactly zero left out.  Reported beside the headline,
    which always evaluates every pair: the 10 x 10 km / 1,000-day gradient workload, the 15 x 15 km /
    5,000-day log-likelihood workload, the paper's posterior parameters on the latter, and the
    1,000,000-event / 20,000-day gradient workload with both enumerations (the direct one being the
    memory-linear fallback for data whose triangle does not fit)."""
    from paper_2005_10123_amd import synth

    cases = [("city_85k_10km", None, True, "symmetric", "fp32c"), ("city_85k_15km", None, False, "symmetric", "fp32c"),
             ("city_85k_15km", THETA_POSTERIOR, True, "symmetric", "fp32c"),
             ("city_85k_15km", THETA_POSTERIOR, True, "symmetric", "fp64"),
             ("stress_1m", None, True, "symmetric", "fp32c"), ("stress_1m", None, True, "direct", "fp32c")]
    out = []
    for workload, theta_override, grad, scheme, prec in cases:
        n_steps = 3 if workload == "stress_1m" else steps
        (x, y, t), theta = synth.config_events(workload)
        if theta_override is not None:
            theta = theta_override
        n = x.size
        ds = ctx.dataset(x, y, t)
        rec = {"workload": workload, "theta": list(theta), "gradient": grad, "precision": prec,
               "enumeration": scheme}
        ctx.set_pair_scheme(scheme)
        res = {}
        for skip in (False, True):
            ctx.set_zero_tile_skipping(skip)
            r, wall, _, kms = time_steps(ctx, ds, theta, prec, grad, n_steps, 1)
            res[skip] = r
            rec["skip" if skip else "all_pairs"] = {"ms_per_call": wall / n_steps * 1e3, "kernel_ms": kms,
                                                    "pairs_per_s": float(n) * n * n_steps / wall}
        ctx.set_zero_tile_skipping(False)
        ctx.set_pair_scheme("symmetric")
        ds.close()
        ell0, ell1 = (res[False][0], res[True][0]) if grad else (res[False], res[True])
        rec["speedup"] = rec["all_pairs"]["ms_per_call"] / rec["skip"]["ms_per_call"]
        rec["ell_rel_skip_vs_all_pairs"] = abs(ell1 - ell0) / abs(ell0)
        if grad:
            g0, g1 = np.asarray(res[False][1]), np.asarray(res[True][1])
            rec["grad_rel_skip_vs_all_pairs"] = (np.abs(g1 - g0) / np.maximum(np.abs(g0), 1e-300)).tolist()
        out.append(rec)
    return out


def shard_run(ctx, nshards=8, workload="stress_1m"):
    """One GPU's share of an evaluation split over `nshards` devices, at its real shape: the
    pairwise-kernel time of each shard of the 1,000,000-event workload (FP32C, log-likelihood +
    gradient) next to the whole evaluation's.  The shards run one after another on this GPU; the
    per-event sums they return (6 doubles per event) are what the devices would add in an
    all-reduce before hawkes_finish."""
    from paper_2005_10123_amd import synth

    (x, y, t), theta = synth.config_events(workload)
    n = x.size
    ds = ctx.dataset(x, y, t)
    ctx.grad(ds, theta, "fp32c")
    ctx.kernel_time(reset=True)
    ctx.profile(True)
    ell_whole, _ = ctx.grad(ds, theta, "fp32c")
    whole_ms, _ = ctx.kernel_time(reset=True)
    shard_ms, total = [], np.zeros((n, 6))
    for k in range(nshards):
        total += ctx.shard_sums(ds, theta, k, nshards, "fp32c")
        ms, _ = ctx.kernel_time(reset=True)
        shard_ms.append(ms)
    ctx.profile(False)
    ell_sharded, _ = ctx.finish(ds, theta, total)
    ds.close()
    return {"workload": workload, "n_events": n, "shards": nshards, "kernel_ms_whole": whole_ms,
            "kernel_ms_per_shard": shard_ms, "max_shard_share_of_whole": max(shard_ms) / whole_ms,
            "ell_rel_sharded_vs_whole": abs(ell_sharded - ell_whole) / abs(ell_whole),
            "exchange_bytes_per_device": n * 6 * 8}


def serving_run(ctx, seconds=8.0, chains=256, datasets=16, utilisation=0.8, seed=4, warmup=1.0,
                min_requests=10000, max_seconds=20.0, grad=True):
    """Closed-loop chains with Poisson think times over 16 resident datasets of log-uniform size,
    FP32C requests with the gradient (grad) or log-likelihood only.
    Latencies count from the requests submitted after `warmup` seconds; submission goes on for at
    least `seconds` and until `min_requests` have been measured (at most `max_seconds`)."""
    from paper_2005_10123_amd import binding, synth

    sizes = synth.loguniform_sizes(datasets, 5e3, 1.2e5)
    dss = []
    for d, n in enumerate(sizes):
        spec = synth.SimSpec(n, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 4, d))
        dss.append(ctx.dataset(*synth.simulate(spec)))
    theta0 = np.array(synth.THETA_CFG1)
    rng = np.random.default_rng(seed)
    # Capacity estimate from one blocking evaluation per dataset.
    cost = []
    evaluate = ctx.grad if grad else ctx.loglik
    for ds in dss:
        evaluate(ds, theta0, "fp32c")
        a = time.perf_counter()
        evaluate(ds, theta0, "fp32c")
        cost.append(time.perf_counter() - a)
    mean_service = float(np.mean([cost[k % datasets] for k in range(chains)]))
    # Offered load: chains / (think + service) requests per second = utilisation / mean_service.
    think = max(chains * mean_service / utilisation - mean_service, 0.0)
    next_t = time.perf_counter() + rng.exponential(think, chains)
    waiting = np.ones(chains, dtype=bool)
    lat, lat_ds, pairs, tag_chain = [], [], 0.0, {}
    tag = 0
    t_start = time.perf_counter()
    t_measure = t_start + warmup
    issuing = True
    t_last = t_measure
    while issuing or tag_chain:
        now = time.perf_counter()
        if issuing and (now - t_start >= max_seconds or (now - t_measure >= seconds and len(lat) >= min_requests)):
            issuing = False
        due = np.nonzero(waiting & (next_t <= now))[0] if issuing else []
        if len(due):
            reqs = []
            for k in due:
                th = theta0 * np.exp(0.1 * rng.standard_normal(6))
                reqs.append(binding.request(dss[k % datasets], th, "fp32c", grad, tag))
                tag_chain[tag] = (k, now >= t_measure)
                tag += 1
                waiting[k] = False
            ctx.submit(reqs)
        for r in ctx.poll(cap=512, timeout_us=200):
            k, measured = tag_chain.pop(r.tag)
            if r.status != 0:
                raise RuntimeError(f"request failed with status {r.status}")
            if measured:
                lat.append((r.t_done_ns - r.t_submit_ns) * 1e-9)
                lat_ds.append(k % datasets)
                pairs += float(sizes[k % datasets]) ** 2
                t_last = time.perf_counter()
            waiting[k] = True
            next_t[k] = time.perf_counter() + rng.exponential(think)
    wall = t_last - t_measure
    for ds in dss:
        ds.close()
    lat, lat_ds = np.array(lat), np.array(lat_ds)
    by_size = []
    for d in np.argsort(sizes):
        ld = lat[lat_ds == d]
        if ld.size:
            by_size.append({"n": int(sizes[d]), "solo_ms": cost[d] * 1e3, "requests": int(ld.size),
                            "p50_ms": float(np.percentile(ld, 50) * 1e3), "p99_ms": float(np.percentile(ld, 99) * 1e3)})
    return {"requests": int(lat.size), "chains": chains, "datasets": datasets, "offered_utilisation": utilisation,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p90_ms": float(np.percentile(lat, 90) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "pairs_per_s": pairs / wall, "seconds": wall, "warmup_seconds": warmup,
            "sizes": [int(s) for s in sizes], "largest_solo_ms": max(cost) * 1e3, "by_dataset": by_size}


def pi_batch_run(ctx, n=55000, samples=64, seed=7):
    """Self-excitation probabilities for many posterior-like parameter vectors (the paper evaluates
    pi_n for 1,000 posterior samples over 55,000 events spanning about 5,000 days): the
    multi-parameter pass against one single-parameter evaluation per vector, and the same pass with
    zero-tile skipping.  Data: 55,000 events of the 15 x 15 km / 5,000-day workload; vectors
    scattered around the paper's posterior parameters."""
    from paper_2005_10123_amd import synth
    import torch

    (x, y, t), _ = synth.config_events("city_85k_15km", n=n)
    ds = ctx.dataset(x, y, t)
    rng = np.random.default_rng(seed)
    th = np.array(THETA_POSTERIOR) * np.exp(0.05 * rng.standard_normal((samples, 6)))
    res = {}
    for skip in (False, True):
        ctx.set_zero_tile_skipping(skip)
        ctx.loglik_multi(ds, th[:4], "fp32c")  # warm-up
        torch.cuda.synchronize()
        a = time.perf_counter()
        res[skip] = (ctx.loglik_multi(ds, th, "fp32c"), time.perf_counter() - a)
    ctx.set_zero_tile_skipping(False)
    (ll, pi), multi_s = res[False]
    (ll_z, pi_z), multi_z = res[True]
    k = 8
    a = time.perf_counter()
    for s in range(k):
        ctx.rows(ds, th[s], "fp32c")
    single_s = (time.perf_counter() - a) / k * samples
    ds.close()
    pairs = float(n) * n * samples
    return {"workload": "city_85k_15km", "n_events": n, "samples": samples, "seconds": multi_s,
            "theta_pairs_per_s": pairs / multi_s, "seconds_per_1000_samples": multi_s / samples * 1000,
            "one_vector_at_a_time_seconds": single_s, "speedup_vs_one_at_a_time": single_s / multi_s,
            "zero_tile_skip": {"seconds": multi_z, "seconds_per_1000_samples": multi_z / samples * 1000,
                               "speedup": multi_s / multi_z,
                               "max_abs_pi_diff": float(np.max(np.abs(pi_z - pi))),
                               "max_rel_ell_diff": float(np.max(np.abs(ll_z - ll) / np.abs(ll)))},
            "mean_pi": float(pi.mean())}


PARAM_NAMES = ("mu0", "tau_x", "tau_t", "theta", "omega", "h")


def mcmc_run(ctx, chains=4, steps=2000, hmc_iterations=300, hmc_warmup=100, seed=11):
    """The paper's sampler at its scale (Section 3.2: 4 chains of Algorithm 1 over the 85,000-event
    data) for `steps` states per chain, and 4 HMC chains (leapfrog on log Theta with the fused
    gradient) for `hmc_iterations` (the first `hmc_warmup` tune the step size and are not kept), both
    through the serving API, with and without zero-tile skipping: evaluations/s, acceptance, and
    per free parameter the effective sample size summed over chains (second half of each MH chain,
    all kept HMC draws) and ESS/s.  Data: the 15 x 15 km / 5,000-day workload; chains start at its
    generating parameters (tau_x, tau_t held fixed)."""
    from paper_2005_10123_amd import mcmc, synth

    (x, y, t), theta0 = synth.config_events("city_85k_15km")
    ds = ctx.dataset(x, y, t)
    out = {"workload": "city_85k_15km", "chains": chains, "mh_states_per_chain": steps,
           "hmc_iterations": hmc_iterations, "hmc_warmup": hmc_warmup, "theta_start": list(theta0)}

    def ess_report(ess, sec):
        return {PARAM_NAMES[d]: {"ess": v, "ess_per_s": v / sec} for d, v in ess.items()}

    for skip in (False, True):
        ctx.set_zero_tile_skipping(skip)
        chs = [mcmc.ChainState(np.array(theta0, float), np.random.default_rng(seed + k)) for k in range(chains)]
        a = time.perf_counter()
        served = mcmc.run_served(ctx, chs, [ds] * chains, steps)
        sec = time.perf_counter() - a
        mh = {"seconds": sec, "evaluations": served, "evaluations_per_s": served / sec,
              "hours_per_10000_states_per_chain": sec / steps * 10000 / 3600,
              "acceptance": float(np.mean([c.accepted / max(c.steps, 1) for c in chs])),
              "ess": ess_report(mcmc.chain_ess(chs), sec)}
        hch = [mcmc.HMCChain(np.array(theta0, float), np.random.default_rng(seed + 100 + k), warmup=hmc_warmup)
               for k in range(chains)]
        a = time.perf_counter()
        served = mcmc.run_hmc_served(ctx, hch, [ds] * chains, hmc_iterations)
        sec = time.perf_counter() - a
        hmc = {"seconds": sec, "gradient_evaluations": served, "evaluations_per_s": served / sec,
               "acceptance": float(np.mean([c.accepted / max(c.iters, 1) for c in hch])),
               "step_size": [c.eps for c in hch], "ess": ess_report(mcmc.chain_ess(hch, 0.0), sec)}
        out["zero_tile_skip" if skip else "all_pairs"] = {"mh": mh, "hmc": hmc}
    ctx.set_zero_tile_skipping(False)
    # The MH chains' log-likelihood requests in shared multi-parameter passes (off by default).
    ctx.set_shared_passes(True)
    chs = [mcmc.ChainState(np.array(theta0, float), np.random.default_rng(seed + k)) for k in range(chains)]
    a = time.perf_counter()
    served = mcmc.run_served(ctx, chs, [ds] * chains, steps)
    sec = time.perf_counter() - a
    ctx.set_shared_passes(False)
    out["all_pairs_shared_passes"] = {"mh": {"seconds": sec, "evaluations": served, "evaluations_per_s": served / sec,
                                             "acceptance": float(np.mean([c.accepted / max(c.steps, 1) for c in chs]))}}
    out["shared_pass_speedup_mh"] = (served / sec) / out["all_pairs"]["mh"]["evaluations_per_s"]
    ds.close()
    return out


def chain_serving_run(ctx, chains=256, datasets=16, iterations=5, seed=21):
    """The serving workload driven by real samplers instead of synthetic arrivals: 256 HMC chains
    (8 leapfrog steps, so 8 log-likelihood + gradient requests per iteration) over 16 resident
    datasets of log-uniform size in [5,000, 120,000], chain k on dataset k mod 16, each keeping one
    request in flight and submitting its next one as soon as its result is polled (closed loop, no
    think time): p50/p99 latency and aggregate pairs/s."""
    from paper_2005_10123_amd import mcmc, synth

    sizes = synth.loguniform_sizes(datasets, 5e3, 1.2e5)
    dss = [ctx.dataset(*synth.simulate(synth.SimSpec(n, 10.0, 1000.0, 3, 0.5, 0.1, 0.3, (10123, 4, d))))
           for d, n in enumerate(sizes)]
    rng = np.random.default_rng(seed)
    theta0 = np.array(synth.THETA_CFG1)
    chs = [mcmc.HMCChain(theta0 * np.exp(0.1 * rng.standard_normal(6)), np.random.default_rng(seed + k),
                         warmup=iterations) for k in range(chains)]
    lat, pairs = [], [0.0]

    def record(k, r):
        lat.append((r.t_done_ns - r.t_submit_ns) * 1e-9)
        pairs[0] += float(sizes[k % datasets]) ** 2

    a = time.perf_counter()
    served = mcmc.run_hmc_served(ctx, chs, [dss[k % datasets] for k in range(chains)], iterations, on_result=record)
    sec = time.perf_counter() - a
    for d in dss:
        d.close()
    lat = np.array(lat)
    return {"chains": chains, "datasets": datasets, "hmc_iterations": iterations, "requests": served,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p90_ms": float(np.percentile(lat, 90) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "pairs_per_s": pairs[0] / sec, "seconds": sec}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="city_85k_10km")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-shards", action="store_true",
                    help="skip the one-GPU-share run of the 1,000,000-event workload cut into 8 shards")
    ap.add_argument("--timing-only", action="store_true",
                    help="only the timed steps and the FP64 comparison (for profiler runs): implies "
                         "--no-serving --no-cpu-baseline --no-shards and skips the posterior-regime report")
    ap.add_argument("--serving-seconds", type=float, default=8.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB mebibytes (5 times), the reference "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters, then exit")
    ap.add_argument("--loglik-only", action="store_true",
                    help="only the log-likelihood-only workload (both precisions), for profiler runs")
    ap.add_argument("--cpu-full", action="store_true",
                    help="only time the FP64 oracle over whole workloads on the host (minutes), then exit")
    args = ap.parse_args()
    if args.cpu_full:
        print(json.dumps(cpu_full_run()), flush=True)
        return
    if args.timing_only:
        args.no_serving = args.no_cpu_baseline = args.no_shards = True
    if args.copy_calibration:
        import torch

        src = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "copies": 5}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (one evaluation would "
              "split the symmetric pass's work units over the devices and add their per-event sums with one "
              "all-reduce; see hawkes_shard_sums / hawkes_finish, not driven across devices here)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.loglik_only:
        from paper_2005_10123_amd import binding

        with binding.Context(0) as ctx:
            lw = loglik_workload(ctx)
            lw.pop("events", None)  # the events kept for the oracle comparison of the full run
            print(json.dumps({"loglik_workload": lw}), flush=True)
        return

    from paper_2005_10123_amd import binding, synth

    (x, y, t), theta = synth.config_events(args.workload)
    spec = synth.CONFIGS[args.workload][0]
    n = x.size
    ctx = binding.Context(0)
    ds = ctx.dataset(x, y, t)

    (ell, g), wall, per, kms = leg("timed steps", time_steps, ctx, ds, theta, "fp32c", True, args.steps, args.warmup,
                                  spin_up_s=0.25)
    steps64 = max(3, args.steps // 3)
    (ell64, g64), wall64, per64, kms64 = leg("fp64 steps", time_steps, ctx, ds, theta, "fp64", True, steps64, 1,
                                              spin_up_s=0.1)
    rows64 = ctx.rows(ds, theta, "fp64")
    l1 = np.abs(rows64["grad"]).sum(axis=0)
    pairs = float(n) * n
    value = pairs * args.steps / wall
    roof = roofline_pairs(True)
    achieved = pairs / (kms * 1e-3)

    result = {
        "metric": "pairs/s for loglik+grad at N=85k (FP32-comp vs FP64); p50/p99 under chain load",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",  # pair terms in binary32 with compensated sums; epilogue and reductions in binary64
        "data": "synthetic: seeded branching (Hawkes cluster) simulation, 3-component Gaussian-mixture background",
        "config": {"workload": f"{args.workload}: N={n} events, {spec.L:g}x{spec.L:g} km, {spec.T_end:g} days; "
                               f"theta=(mu0, tau_x, tau_t, theta, omega, h)={tuple(theta)}; fused log-likelihood + "
                               f"gradient, FP32-compensated",
                   "n_events": n, "pairs_per_step": pairs, "zero_tile_skipping": False},
        "roofline": {"bound": "alu", "achieved": achieved / 1e9, "peak": roof / 1e9, "unit": "Gpair/s",
                     "frac": achieved / roof,
                     "traffic": measured_traffic(os.path.join(ROOT, "profiles", "pair_sym_fp32c_grad_city85k.json")),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, copy-calibrated)",
                     "kernel": "pair_sym_fp32c<grad>", "kernel_ms": kms,
                     "model": "algorithmic work of the method per ordered pair (13.5 FP32 lane ops + 1.5 exp, as "
                              "the direct enumeration evaluates it): 1/(13.5 / 78.65e12 ops/s + 1.5 / 19.66e12 exp/s); "
                              "FP32 vector 157.3 TFLOP/s (FMA=2) and v_exp_f32 at 32 lanes/CU/clk x 256 CU x 2.4 GHz",
                     "executed_work_peak": roofline_pairs(True, executed=True) / 1e9,
                     "executed_work_frac": achieved / roofline_pairs(True, executed=True),
                     "executed_work_model": "the work the symmetric pass executes per ordered pair (9 FP32 lane ops "
                                            "+ 1 exp): 1/(9 / 78.65e12 + 1 / 19.66e12)",
                     "method_tflops": achieved * 19.0 / 1e12},
        "p10_ms_step": float(np.percentile(per, 10) * 1e3),
        "p50_ms_step": float(np.percentile(per, 50) * 1e3),
        "p90_ms_step": float(np.percentile(per, 90) * 1e3),
        "p99_ms_step": float(np.percentile(per, 99) * 1e3),
        "fp64": {"pairs_per_s": pairs * steps64 / wall64, "ms_per_step": wall64 / steps64 * 1e3, "kernel_ms": kms64,
                 # against the roofline of the work the symmetric FP64 pass executes (9 FP64 ops + one
                 # 16-op exp2 per ordered pair at 78.6 TFLOP/s)
                 "roofline_frac": (pairs / (kms64 * 1e-3)) / roofline_pairs(True, True, executed=True),
                 "roofline_pairs_per_s": roofline_pairs(True, True, executed=True),
                 "direct_enumeration_roofline_pairs_per_s": roofline_pairs(True, True)},
        "fp32c_vs_fp64": {"ell_rel": abs(ell - ell64) / abs(ell64),
                          "grad_l1_normalised": (np.abs(g - g64) / l1).tolist(),
                          "grad_plain_rel": (np.abs(g - g64) / np.abs(g64)).tolist()},
        "loglik": ell,
    }
    if not args.timing_only:
        clk = engine_clock(ctx, ds, theta)
        if clk is not None:
            # Both rates of R32 scale with the clock.
            clk["spec_ghz"] = CLOCK / 1e9
            clk["frac_at_measured_clock"] = achieved / (roof * clk["measured_ghz"] / clk["spec_ghz"])
            clk["source"] = ("amd-smi metric -c: per-XCD graphics clocks sampled twice while the gradient "
                             "pass ran back to back after the timed steps")
        result["roofline"]["clock"] = clk
    ds.close()
    lw = sw = stw = None
    if not args.timing_only:
        result["posterior_regime"] = leg("posterior_regime", posterior_regime, ctx)
        result["loglik_workload"] = lw = leg("loglik_workload", loglik_workload, ctx)
        result["small_workload"], sw = leg("small_workload", small_workload, ctx)
        result["stress_workload"], stw = leg("stress_workload", stress_workload, ctx)
        result["zero_tile_skip"] = leg("zero_tile_skip", zero_skip_run, ctx)
    if not args.no_shards:
        result["shard_share"] = leg("shard_share", shard_run, ctx)
    if not args.no_serving:
        result["serving"] = leg("serving", serving_run, ctx, seconds=args.serving_seconds)
        result["serving_sweep"] = []
        for u in (0.5, 1.0, 2.0):
            r = leg(f"serving_sweep {u}", serving_run, ctx, seconds=3.0, utilisation=u, min_requests=0)
            result["serving_sweep"].append({k: r[k] for k in ("offered_utilisation", "requests", "p50_ms", "p99_ms",
                                                              "pairs_per_s")})
        # The same closed loop with zero-tile skipping on (capacity re-estimated with it on).
        ctx.set_zero_tile_skipping(True)
        r = leg("serving_zero_tile_skip", serving_run, ctx, seconds=4.0, min_requests=5000)
        ctx.set_zero_tile_skipping(False)
        result["serving_zero_tile_skip"] = {k: r[k] for k in ("offered_utilisation", "requests", "p50_ms", "p90_ms",
                                                               "p99_ms", "pairs_per_s")}
        result["serving_chains"] = leg("serving_chains", chain_serving_run, ctx)
        # Log-likelihood-only load (the requests of Algorithm 1's chains) with the scheduler's shared
        # multi-parameter passes and without them, saturated (offered load 2.0) and at 0.8.
        result["serving_loglik"] = {}
        for shared in (True, False):
            ctx.set_shared_passes(shared)
            for u in (0.8, 2.0):
                r = leg(f"serving_loglik shared={shared} {u}", serving_run, ctx, seconds=3.0, utilisation=u,
                        min_requests=0, grad=False)
                result["serving_loglik"][f"{'shared' if shared else 'unshared'}_{u}"] = {
                    k: r[k] for k in ("offered_utilisation", "requests", "p50_ms", "p99_ms", "pairs_per_s")}
        ctx.set_shared_passes(False)
        result["pi_batch"] = leg("pi_batch", pi_batch_run, ctx)
        result["mcmc"] = leg("mcmc", mcmc_run, ctx)
    ctx.close()
    if not args.no_cpu_baseline:
        import oracle

        result["cpu_baseline"] = leg("cpu_baseline", cpu_baseline, x, y, t, theta)
        result["cpu_baseline"].pop("per_row_s")
        result["cpu_baseline"]["gpu_speedup"] = value / result["cpu_baseline"]["value"]
        result["cpu_all_cores"], ref = leg("cpu_all_cores", cpu_all_cores_run, x, y, t, theta)
        result["cpu_all_cores"]["gpu_speedup"] = value / result["cpu_all_cores"]["value"]
        # Every GPU result against the oracle's whole evaluation of its workload.
        result["fp32c_vs_oracle"] = oracle_errors(ell, g, ref, theta)
        result["fp64_vs_oracle"] = oracle_errors(ell64, g64, ref, theta)
        result["cpu_host_simd"] = leg("cpu_host_simd", host_simd_run, x, y, t, theta, ref)
        if lw is not None:
            ref2 = leg("oracle loglik_workload", oracle.evaluate_parallel, *lw.pop("events"), lw["theta"])
            for prec in ("fp32c", "fp64"):
                lw[prec]["vs_oracle"] = oracle_errors(lw["ell"][prec], None, ref2, lw["theta"])
        if sw is not None:
            xs, ys, ts, ths = sw
            ref1 = oracle.evaluate_parallel(xs, ys, ts, ths)
            for prec in ("fp64", "fp32c"):
                result["small_workload"][prec]["vs_oracle"] = oracle_errors(result["small_workload"][prec].pop("ell"),
                                                                            None, ref1, ths)
        if stw is not None:
            xs, ys, ts, ths, sub = stw
            ref5 = leg("oracle stress subsample", oracle.evaluate_parallel, xs, ys, ts, ths)
            result["stress_workload"]["subsample_20k_vs_oracle"] = {
                prec: oracle_errors(sub[prec][0], sub[prec][1], ref5, ths) for prec in ("fp32c", "fp64")}
    if lw is not None:
        lw.pop("events", None)
        lw.pop("ell", None)
    torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
