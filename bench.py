#!/usr/bin/env python3
"""Benchmark: replica-exchange Wang-Landau on one MI355X.

One step = one complete REWL run of the workload (default: 2D Ising 32x32,
16 windows x 4 walkers): start-up on the device, rounds until every window has
reached ln f_final, stitching of ln g on the host; fresh seed per step.

Reported on one JSON line:
  value         sweep attempts per second (every attempt, accepted or not,
                start-up excluded) over the timed plain steps, wall clock;
  time_to_dos_s p50 / p99 seconds from creation to the stitched ln g on the
                host, plain form;
  batched       the same workload, `--batch` seeds at once in one batch
                (walkers per wave chosen by the autotuner): aggregate
                attempts/s and per-run time-to-DOS p50 / p99;
  max_abs_dlng_vs_exact  per step, max |ln g - ln g_exact| over the bins
                (Ising sizes with a stored exact DOS);
  batched_glasses  256 independent 24x24 +-J glasses, 8 windows x 4 walkers
                each, in one batch, walkers per wave and attempts between
                exchanges autotuned: attempts/s over a fixed number of attempts
                and the sweep kernel's roofline (same definition as below);
  roofline      the sweep kernel's VALU work per attempt times its attempts,
                over its own time measured with HIP events recorded on the run's
                stream around each sweep launch, against the MI355X vector-ALU
                peak;
  cpu_baseline  the CPU oracle on the same workload, all host cores, on a
                bounded sample of rounds; its time-to-DOS is extrapolated
                exactly: the oracle is bit-identical to the GPU run, so it makes
                the same rounds with the same windows active, and its OpenMP
                static schedule gives each round's time from the per-thread
                rate.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ising32]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-slots one sweep attempt needs (Ising; quarter-rate 32-bit
# multiplies count 4): Philox4x32-10 100, site draw 4, ln u 50, neighbours 20,
# the accept/update chain 20; the glasses add the coupling terms, the 3D one
# two more neighbours.  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_ATTEMPT = {"ising": 194, "ea": 200, "potts": 204, "ea3": 212}
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

WORKLOAD_TEXT = {
    "ising32": "2D Ising L=32 periodic J=1, E in [-2048,2048] step 4, 16 windows x 4 walkers, "
               "overlap 0.75, flatness 0.8, ln f 1 -> 1e-8 halving, 1e4 attempts/walker/round",
    "ising8": "2D Ising L=8 periodic J=1, 4 windows x 2 walkers, overlap 0.75, flatness 0.8, "
              "ln f 1 -> 1e-6 halving, 1e4 attempts/walker/round",
    "potts64": "2D q=10 Potts L=64 periodic, 32 windows x 8 walkers, overlap 0.75, flatness 0.8, "
               "ln f 1 -> 1e-8, 1e4 attempts/walker/round",
    "ea24": "2D +-J EA glass L=24 periodic, 8 windows x 4 walkers, overlap 0.75, flatness 0.8, "
            "ln f 1 -> 1e-6, 1e4 attempts/walker/round",
    "ea3d12": "3D +-J EA glass 12x12x12 periodic, 8 windows x 4 walkers, overlap 0.75, "
              "flatness 0.8, ln f 1 -> 1e-6, 1e4 attempts/walker/round",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("rewl_kernels.hip", "rewl_device.h", "rewl_internal.h")


def kernel_sources_hash():
    """sha256 over the device sources; a stored counter profile applies to the
    kernels only while this hash is unchanged."""
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1305_5615_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(tag):
    """HBM bytes per sweep launch from profiles/sweep_<tag>.md (FETCH_SIZE and
    WRITE_SIZE scaled by a device copy of known size), or None when the file is
    missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"sweep_{tag}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch",
                                                      "kernel_sources_sha256"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if vals.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    return float(vals["traffic_bytes_per_launch"])


def sweep_kernel_name(P, waves):
    """The sweep instantiation a launch of `waves` waves runs: the per-step bin
    records sit in registers when waves outnumber the compute units."""
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return f"sweep_kernel<{P}, {'true' if waves > cus else 'false'}>"


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def run_kwargs(p):
    keys = ("model", "L", "q", "couplings", "e_min", "e_max", "n_windows", "overlap",
            "walkers_per_window", "flatness", "lnf_init", "lnf_final", "S", "seed", "schedule",
            "windows")
    return {k: p[k] for k in keys if k in p}


def gpu_full_run(rewl, p, max_rounds):
    """One complete plain run.  Returns a dict with seconds, attempts, rounds,
    sweep time and launches, convergence, and each window's finishing round."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = rewl.Run(**run_kwargs(p))
    r.set_timing(True)
    ok, issued, rounds = False, 0, 0
    while not ok and issued < max_rounds:
        chunk = min(2000, max_rounds - issued)
        ok, rounds = r.run(chunk)
        issued += chunk
        if not ok:
            log(f"  ... {r.info()['rounds']} rounds issued")
    lng = r.lng()
    t1 = time.perf_counter()
    ms, n = r.timing()
    info = r.info()
    finish = [w["finish_round"] for w in r.windows()]
    r.close()
    assert lng.shape[0] == info["n_bins"]
    return dict(seconds=t1 - t0, attempts=info["attempts"], rounds=rounds, sweep_ms=ms,
                launches=n, converged=ok, finish=finish, lng=lng)


def exact_error(p, lng):
    """max |ln g - ln g_exact| over the bins of an Ising run whose exact DOS is
    stored under tests/golden (None for other models and sizes)."""
    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"ising_exact_L{p['L']}.txt")
    if p["model"] != "ising" or not os.path.exists(path):
        return None
    ref = []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            v = line.split()[1]
            if p["L"] <= 16:
                n = int(v)
                ref.append(math.log(n) if n > 0 else -math.inf)
            else:
                ref.append(float(v))
    ref = np.array(ref)
    fin = np.isfinite(ref)
    if not np.array_equal(np.isfinite(lng), fin):
        return float("inf")
    return float(np.abs(lng[fin] - ref[fin]).max())


def gpu_glasses(rewl, n_runs, rounds, candidates=(4, 8), s_candidates=(1000, 10_000, 100_000)):
    """The batched glass workload: n_runs independent 24x24 +-J instances in one
    batch.  The autotuner picks walkers per wave from `candidates` and attempts
    per walker between exchanges from `s_candidates` by attempts/s over the same
    number of attempts (4e4 per walker) each; then `rounds` x 1e4 attempts per
    walker are timed at the chosen setting.  Returns throughput, the setting and
    the sweep kernel's own time."""
    import torch

    from workloads import run_params

    def make(P, S):
        runs = [dict(run_kwargs(run_params("ea24", seed=1 + i)), S=S) for i in range(n_runs)]
        return rewl.Batch(runs, walkers_per_wave=P, graph_rounds=0)

    def measure(b, S, attempts_per_walker):
        b.step(1)
        torch.cuda.synchronize()
        a0 = sum(b[i].info()["attempts"] for i in range(n_runs))
        t0 = time.perf_counter()
        b.step(max(1, attempts_per_walker // S))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return (sum(b[i].info()["attempts"] for i in range(n_runs)) - a0) / dt

    best, best_rate = None, -1.0
    for S in s_candidates:
        for P in candidates:
            b = make(P, S)
            rate = measure(b, S, 40_000)
            b.close()
            log(f"autotune: glasses P={P} S={S}: {rate / 1e9:.2f} G attempts/s")
            if rate > best_rate:
                best, best_rate = (P, S), rate
    P, S = best
    b = make(P, S)
    b.set_timing(True)
    b.step(1)
    torch.cuda.synchronize()
    a0 = sum(b[i].info()["attempts"] for i in range(n_runs))
    ms0, n0 = b.timing()
    t0 = time.perf_counter()
    b.step(max(1, rounds * 10_000 // S))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = b.timing()
    att = sum(b[i].info()["attempts"] for i in range(n_runs)) - a0
    b.close()
    return dict(P=P, S=S, attempts=att, wall=wall, sweep_ms=ms - ms0, launches=n - n0)


def gpu_batched(rewl, params, walkers_per_wave, graph_rounds, max_rounds):
    """All runs in one batch; a run's time-to-DOS is the wall clock once the
    first poll that sees it done has its stitched ln g on the host."""
    import numpy as np
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = rewl.Batch([run_kwargs(p) for p in params], walkers_per_wave=walkers_per_wave,
                   graph_rounds=graph_rounds)
    done_at = [None] * len(params)
    lngs = [None] * len(params)
    issued, chunk = 0, 64
    while issued < max_rounds:
        b.step(chunk)
        issued += chunk
        d = b.done()
        for i in np.nonzero(d)[0]:
            if done_at[i] is None:
                lngs[i] = b[int(i)].lng()
                done_at[i] = time.perf_counter() - t0
        if d.all():
            break
        if issued % 8192 == 0:
            log(f"  ... batched: {issued} rounds, {int(d.sum())}/{len(params)} runs done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    attempts = sum(b[i].info()["attempts"] for i in range(len(params)))
    b.close()
    return dict(wall=wall, attempts=attempts, done_at=done_at, lng=lngs)


def autotune(rewl, params, candidates=(1, 2, 4, 8), rounds=6):
    """Walkers per wave with the highest attempts/s over a few rounds of this
    batch (results do not depend on the choice)."""
    import torch

    best, best_rate = 1, -1.0
    b = rewl.Batch([run_kwargs(p) for p in params], walkers_per_wave=1)
    for P in candidates:
        try:
            b.set_walkers_per_wave(P)
        except rewl.RewlError:
            continue
        b.step(1)
        torch.cuda.synchronize()
        a0 = sum(b[i].info()["attempts"] for i in range(len(params)))
        t0 = time.perf_counter()
        b.step(rounds)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rate = (sum(b[i].info()["attempts"] for i in range(len(params))) - a0) / dt
        log(f"autotune: walkers per wave {P}: {rate / 1e9:.3f} G attempts/s")
        if rate > best_rate:
            best, best_rate = P, rate
    b.close()
    return best


def cpu_baseline(p, seconds, finish, threads):
    """The oracle on the same workload with `threads` OpenMP threads over its
    first rounds (all windows active); the time-to-DOS follows from its
    per-walker round time and the static schedule over the GPU run's rounds."""
    from oracle import core

    o = core.Run(**run_kwargs(p), n_threads=threads)
    a0 = o.stats()["attempts"]
    t0 = time.perf_counter()
    rounds = 0
    while True:
        o.step(1)
        rounds += 1
        el = time.perf_counter() - t0
        if el >= seconds or o.info()["done"]:
            break
    att = o.stats()["attempts"] - a0
    nw = p["n_windows"] * p["walkers_per_window"]
    m = p["walkers_per_window"]
    chunk = math.ceil(nw / threads)                   # walkers per thread, static schedule
    per_walker_round = el / rounds / chunk            # one walker's S attempts on one thread
    total = 0.0
    edges = sorted(set([0] + [f + 1 for f in finish]))
    for r0, r1 in zip(edges, edges[1:]):
        per_thread = [0] * threads
        for w in range(nw):
            if finish[w // m] >= r0:
                per_thread[w // chunk] += 1
        total += (r1 - r0) * max(per_thread) * per_walker_round
    return {"value": att / el, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"{p['name']} seed {p['seed']}: first {rounds} rounds after start-up "
                      f"({att} sweep attempts in {el:.1f} s, OpenMP static over {nw} walkers)",
            "time_to_dos_s_extrapolated": total}


def profile(rewl, args, run_params):
    """Fixed rounds of one run (or of a batch) after start-up, for profilers."""
    import torch

    over = {"S": args.attempts_per_round} if args.attempts_per_round else {}
    if args.batch > 1 and args.walkers_per_wave > 0:
        runs = [run_kwargs(run_params(args.workload, seed=1 + i, **over))
                for i in range(args.batch)]
        P = args.walkers_per_wave
        r = rewl.Batch(runs, walkers_per_wave=P, graph_rounds=0)
        label = f"{len(runs)} x {args.workload}, P={P}"
        views = [r[i] for i in range(len(runs))]
    else:
        r = rewl.Run(**run_kwargs(run_params(args.workload, seed=1, **over)))
        label = args.workload
        views = [r]
    r.set_timing(True)
    r.step(1)
    torch.cuda.synchronize()
    a0 = sum(v.info()["attempts"] for v in views)
    ms0, n0 = r.timing()
    t0 = time.perf_counter()
    r.step(args.rounds)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = r.timing()
    att = sum(v.info()["attempts"] for v in views) - a0
    log(f"profile: {label}, {args.rounds} rounds, {att} attempts, {dt:.3f} s, "
        f"{att / dt / 1e9:.3f} G attempts/s, sweep avg {1e3 * (ms - ms0) / max(n - n0, 1):.1f} us")
    r.close()


def served(rewl, args):
    """The served workload: Poisson arrivals of mixed REWL requests, once through
    the continuous-batching server and once as plain runs in arrival order (FIFO,
    one run on the device at a time).  Latency = finish - arrival."""
    import numpy as np
    import torch

    from workloads import served_stream

    reqs = served_stream(args.served, args.rate, seed=7, lnf_choices=(1e-3, 1e-4),
                         sizes=args.served_sizes)
    kinds = [r["params"] for r in reqs]

    # continuous batching
    # one walker per wave measured best for this stream (p99 8.1 s vs 9.2 s at 2)
    srv = rewl.Server(device_budget_bytes=args.budget_mb << 20,
                      walkers_per_wave=args.walkers_per_wave or 1, rounds_per_tick=8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pending = list(range(len(reqs)))
    ids, lat = {}, {}
    ticks = 0
    failed = []
    while len(lat) < len(reqs):
        now = time.perf_counter() - t0
        while pending and reqs[pending[0]]["arrival"] <= now:
            i = pending.pop(0)
            ids[srv.submit(**run_kwargs(reqs[i]["params"]))] = i
        running, queued = srv.tick()
        ticks += 1
        if ticks % 5000 == 0:
            log(f"served: {ticks} ticks, {running} running, {queued} queued, {len(lat)} done")
        while True:
            d = srv.next_done()
            if d is None:
                break
            i = ids[d[0]]
            try:
                srv.result(d[0])
            except rewl.RewlError as e:
                failed.append(i)
                log(f"served: request {i} failed: {e}")
            srv.release(d[0])
            lat[i] = time.perf_counter() - t0 - reqs[i]["arrival"]
            log(f"served: request {i} done, latency {lat[i]:.2f} s ({len(lat)}/{len(reqs)})")
        if running == 0 and queued == 0 and pending:
            time.sleep(max(0.0, reqs[pending[0]]["arrival"] - (time.perf_counter() - t0)))
    srv_wall = time.perf_counter() - t0
    srv.close()
    ok_lat = [v for k, v in lat.items() if k not in failed]
    log(f"served: server {len(reqs)} runs in {srv_wall:.1f} s ({len(failed)} failed at start-up), "
        f"p50 {percentile(ok_lat, 50):.2f} s, p99 {percentile(ok_lat, 99):.2f} s")

    # plain FIFO
    t0 = time.perf_counter()
    fifo_lat, fifo_att = [], 0
    for r in ([] if args.no_fifo else reqs):
        now = time.perf_counter() - t0
        if now < r["arrival"]:
            time.sleep(r["arrival"] - now)
        try:
            run = rewl.Run(**run_kwargs(r["params"]))
        except rewl.RewlError as e:
            fifo_lat.append(time.perf_counter() - t0 - r["arrival"])
            log(f"served: FIFO request {len(fifo_lat) - 1} failed: {e}")
            continue
        while not run.run(50_000)[0]:
            log(f"served: FIFO request {len(fifo_lat)}: {run.info()['rounds']} rounds")
        run.lng()
        fifo_att += run.info()["attempts"]
        run.close()
        fifo_lat.append(time.perf_counter() - t0 - r["arrival"])
        log(f"served: FIFO request {len(fifo_lat) - 1} done, latency {fifo_lat[-1]:.2f} s")
    fifo_wall = time.perf_counter() - t0
    log(f"served: FIFO {len(reqs)} runs in {fifo_wall:.1f} s")

    att = fifo_att  # the served runs are bit-identical to the plain ones: same attempts
    if args.no_fifo:
        att = None  # attempts are counted on the plain runs
    out = {
        "metric": "served REWL stream: p50/p99 latency, continuous batching vs plain FIFO",
        "requests": len(reqs), "rate_per_s": args.rate, "sizes": args.served_sizes,
        "lnf_final": [1e-3, 1e-4],
        "mix": {m: sum(1 for k in kinds if k["model"] == m) for m in ("ising", "potts", "ea")},
        "failed_at_start_up": sorted(failed),
        "served": {"p50_s": percentile(ok_lat, 50), "p99_s": percentile(ok_lat, 99),
                   "wall_s": srv_wall, "attempts_per_s": att / srv_wall if att else None},
        "fifo": None if args.no_fifo else {
            "p50_s": percentile([v for k, v in enumerate(fifo_lat) if k not in failed], 50),
            "p99_s": percentile([v for k, v in enumerate(fifo_lat) if k not in failed], 99),
            "wall_s": fifo_wall, "attempts_per_s": att / fifo_wall},
        "walkers_per_wave": args.walkers_per_wave or 1,
    }
    print(json.dumps(out), flush=True)


def balanced(rewl, args):
    """Time-to-DOS with run-time balanced windows (a pre-run on the equal
    partition to every window's first merge, then the run on the derived
    windows) against the plain run on the equal partition, same seeds."""
    import torch

    from workloads import run_params

    out = {"metric": "time-to-converged ln g, run-time balanced vs equal windows",
           "workload": WORKLOAD_TEXT[args.workload], "unit": "s", "runs": []}
    for i in range(args.steps):
        p = run_params(args.workload, seed=1 + i)
        eq = gpu_full_run(rewl, p, args.max_rounds)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo, hi, pre_rounds = rewl.balanced_windows(chunk=16, **run_kwargs(p))
        torch.cuda.synchronize()
        t_pre = time.perf_counter() - t0
        bal = gpu_full_run(rewl, dict(p, windows=(lo, hi)), args.max_rounds)
        rec = {"seed": p["seed"],
               "equal": {"seconds": eq["seconds"], "rounds": eq["rounds"],
                         "finish_rounds": eq["finish"],
                         "max_abs_dlng_vs_exact": exact_error(p, eq["lng"])},
               "balanced": {"pre_run_seconds": t_pre, "pre_run_rounds": pre_rounds,
                            "run_seconds": bal["seconds"], "seconds": t_pre + bal["seconds"],
                            "rounds": bal["rounds"], "finish_rounds": bal["finish"],
                            "windows": [[int(a), int(b)] for a, b in zip(lo, hi)],
                            "max_abs_dlng_vs_exact": exact_error(p, bal["lng"])}}
        out["runs"].append(rec)
        log(f"seed {p['seed']}: equal {eq['seconds']:.1f} s ({eq['rounds']} rounds), balanced "
            f"{t_pre:.1f} + {bal['seconds']:.1f} s ({bal['rounds']} rounds)")
    print(json.dumps(out), flush=True)


def errors(rewl, args):
    """Independent-run error bars and their dependence on the walkers per
    window m (and a weaker flatness with larger m): for each setting, R seeds
    of the workload in one batch to convergence, the jackknife mean and error
    of ln g per bin, compared with the exact DOS where one is stored."""
    import numpy as np
    import torch

    from workloads import run_params

    R = args.errors
    settings = [(1, 0.8), (2, 0.8), (4, 0.8), (8, 0.8), (8, 0.6)]
    out = {"metric": "jackknife error of ln g over independent runs vs walkers per window",
           "workload": WORKLOAD_TEXT[args.workload], "runs_per_setting": R, "settings": []}
    for m, flat in settings:
        params = [dict(run_params(args.workload, seed=101 + i), walkers_per_window=m,
                       flatness=flat) for i in range(R)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = rewl.Batch([run_kwargs(p) for p in params], walkers_per_wave=1, graph_rounds=16)
        issued = 0
        while not b.done().all() and issued < args.max_rounds:
            b.step(256)
            issued += 256
        lngs = np.array([b[i].lng() for i in range(R)])
        rounds = [max(w["finish_round"] for w in b[i].windows()) + 1 for i in range(R)]
        wall = time.perf_counter() - t0
        b.close()
        mean, err = rewl.jackknife(lngs)
        fin = np.isfinite(mean)
        rec = {"walkers_per_window": m, "flatness": flat, "wall_s": wall,
               "rounds_mean": float(np.mean(rounds)),
               "jackknife_err_mean": float(np.nanmean(err[fin])),
               "jackknife_err_max": float(np.nanmax(err[fin]))}
        exact = [exact_error(params[0], lg) for lg in lngs]
        if exact[0] is not None:
            rec["max_abs_dlng_vs_exact_per_run_mean"] = float(np.mean(exact))
            rec["max_abs_dlng_vs_exact_of_mean"] = exact_error(params[0], mean)
        out["settings"].append(rec)
        log(f"m={m} p={flat}: {wall:.1f} s, rounds {np.mean(rounds):.0f}, "
            f"jackknife err mean {rec['jackknife_err_mean']:.4f}")
    print(json.dumps(out), flush=True)


def calibrate_copy(mb):
    """One device-to-device copy of `mb` MiB (read mb, write mb) for scaling
    the FETCH_SIZE / WRITE_SIZE counters."""
    import torch

    src = torch.ones(mb << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy: {mb} MiB read, {mb} MiB written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="ising32", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--max-rounds", type=int, default=400000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch", type=int, default=16,
                    help="runs in the batched comparison (0: skip); in profile mode with "
                         "--walkers-per-wave, the batch size")
    ap.add_argument("--walkers-per-wave", type=int, default=0,
                    help="batched form: walkers per wave (0: autotune)")
    ap.add_argument("--graph", type=int, default=16, help="batched form: rounds per graph")
    ap.add_argument("--glasses", type=int, default=256,
                    help="batched glass leg: independent 24x24 +-J runs in one batch (0: skip)")
    ap.add_argument("--glass-rounds", type=int, default=100,
                    help="batched glass leg: rounds timed after start-up")
    ap.add_argument("--rounds", type=int, default=0,
                    help="profile mode: run this many rounds after start-up, then exit")
    ap.add_argument("--attempts-per-round", type=int, default=0,
                    help="profile mode: attempts per walker between exchanges (0: the workload's)")
    ap.add_argument("--served", type=int, default=0,
                    help="served mode: this many Poisson-arriving requests")
    ap.add_argument("--rate", type=float, default=2.0, help="served mode: arrivals per second")
    ap.add_argument("--served-sizes", default="small", choices=("small", "full"),
                    help="served mode: lattice sizes of the request mix")
    ap.add_argument("--no-fifo", action="store_true",
                    help="served mode: skip the plain FIFO comparison")
    ap.add_argument("--budget-mb", type=int, default=4096, help="served mode: device budget")
    ap.add_argument("--balanced", action="store_true",
                    help="time-to-DOS with run-time balanced windows vs equal windows "
                         "(--steps seeds)")
    ap.add_argument("--errors", type=int, default=0,
                    help="error-bar mode: this many independent runs per walkers-per-window "
                         "setting")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="counter calibration: one device copy of this many MiB")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: each REWL run lives on one device and "
              "the library has no multi-GPU path (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    import paper_1305_5615_amd as rewl
    from workloads import run_params

    if args.rounds > 0:
        profile(rewl, args, run_params)
        return
    if args.served > 0:
        served(rewl, args)
        return
    if args.copy_mb > 0:
        calibrate_copy(args.copy_mb)
        return
    if args.balanced:
        balanced(rewl, args)
        return
    if args.errors > 1:
        errors(rewl, args)
        return

    base = dict(run_params(args.workload, seed=1))
    model = base["model"]
    for i in range(args.warmup):
        res = gpu_full_run(rewl, run_params(args.workload, seed=900 + i), args.max_rounds)
        log(f"warmup {i}: {res['seconds']:.2f} s, {res['rounds']} rounds")

    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = gpu_full_run(rewl, run_params(args.workload, seed=1 + i), args.max_rounds)
        if not res["converged"]:
            log(f"step {i}: not converged within {args.max_rounds} rounds")
        runs.append(res)
        log(f"step {i}: {res['seconds']:.2f} s, {res['rounds']} rounds, "
            f"{res['attempts'] / res['seconds'] / 1e9:.3f} G attempts/s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    attempts = sum(r["attempts"] for r in runs)
    sweep_ms = sum(r["sweep_ms"] for r in runs)
    launches = sum(r["launches"] for r in runs)
    times = [r["seconds"] for r in runs]

    slots = VALU_SLOTS_PER_ATTEMPT[model]
    achieved = slots * attempts / (sweep_ms * 1e-3) / 1e12 if sweep_ms > 0 else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS if achieved else None,
                "traffic": profiled_traffic(args.workload),
                "kernel": sweep_kernel_name(1, base["n_windows"] * base["walkers_per_window"]),
                "sweep_avg_us": 1e3 * sweep_ms / launches if launches else None,
                "valu_slots_per_attempt": slots}
    out = {
        "metric": "spin-flip attempts/sec (1 GPU) + p50/p99 time-to-converged ln g, "
                  "batched vs plain",
        "value": attempts / wall, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "form": "plain",
                   "walkers": base["n_windows"] * base["walkers_per_window"],
                   "L": base["L"], "q": base["q"], "seeds": list(range(1, args.steps + 1))},
        "time_to_dos_s": {"p50": percentile(times, 50), "p99": percentile(times, 99),
                          "rounds": [r["rounds"] for r in runs]},
        "max_abs_dlng_vs_exact": [exact_error(base, r["lng"]) for r in runs],
        "roofline": roofline,
    }
    if args.batch > 0:
        params = [run_params(args.workload, seed=1 + i) for i in range(args.batch)]
        P = args.walkers_per_wave or autotune(rewl, params)
        bres = gpu_batched(rewl, params, P, args.graph, args.max_rounds)
        dts = [d for d in bres["done_at"] if d is not None]
        out["batched"] = {"runs": args.batch, "walkers_per_wave": P, "graph_rounds": args.graph,
                          "value": bres["attempts"] / bres["wall"], "unit": "attempts/s",
                          "wall_s": bres["wall"], "converged": len(dts),
                          "time_to_dos_s": {"p50": percentile(dts, 50),
                                            "p99": percentile(dts, 99)},
                          "seeds": list(range(1, args.batch + 1))}
        import numpy as np

        done_lng = [x for x in bres["lng"] if x is not None]
        errs = [exact_error(params[i], x) for i, x in enumerate(bres["lng"]) if x is not None]
        if len(done_lng) >= 2 and all(e is not None for e in errs):
            # independent runs: the mean ln g and its jackknife error bar
            mean, jk = rewl.jackknife(np.array(done_lng))
            fin = np.isfinite(mean)
            out["batched"]["max_abs_dlng_vs_exact"] = {
                "per_run": errs, "mean_of_runs": exact_error(params[0], mean),
                "max_jackknife_error_of_mean": float(np.nanmax(jk[fin]))}
        log(f"batched: {args.batch} runs, P={P}, {bres['wall']:.1f} s, "
            f"{bres['attempts'] / bres['wall'] / 1e9:.3f} G attempts/s")
    if args.glasses > 0:
        g = gpu_glasses(rewl, args.glasses, args.glass_rounds)
        ach = VALU_SLOTS_PER_ATTEMPT["ea"] * g["attempts"] / (g["sweep_ms"] * 1e-3) / 1e12
        out["batched_glasses"] = {
            "workload": f"{args.glasses} independent 2D +-J EA glasses L=24, 8 windows x 4 "
                        f"walkers each, {args.glass_rounds * 10_000} attempts/walker timed, "
                        "one batch",
            "walkers_per_wave": g["P"], "attempts_per_round": g["S"],
            "value": g["attempts"] / g["wall"],
            "unit": "attempts/s",
            "roofline": {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TOPS,
                         "unit": "TOP/s", "frac": ach / VALU_PEAK_TOPS,
                         # state in and out once per launch: the same bytes at any S
                         "traffic": profiled_traffic(f"ea24x{args.glasses}_P{g['P']}"),
                         "kernel": sweep_kernel_name(g["P"], args.glasses * 32 // g["P"]),
                         "sweep_avg_us": 1e3 * g["sweep_ms"] / max(g["launches"], 1),
                         "valu_slots_per_attempt": VALU_SLOTS_PER_ATTEMPT["ea"]}}
        log(f"glasses: {args.glasses} runs, P={g['P']}, S={g['S']}, "
            f"{g['attempts'] / g['wall'] / 1e9:.2f} G attempts/s")
    if not args.no_cpu:
        p = dict(run_params(args.workload, seed=1))
        p["name"] = args.workload
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else \
            (os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds, runs[0]["finish"], threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
