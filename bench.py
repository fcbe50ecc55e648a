#!/usr/bin/env python3
"""Benchmark: replica-exchange Wang-Landau on one MI355X.

One step = one complete REWL run of the workload: start-up on the device,
rounds until every window has reached ln f_final, stitching of ln g on the
host.  Each step uses a fresh seed.  Reported:
  value        sweep attempts per second over the timed steps (every attempt
               counts, accepted or not), wall clock around all timed steps;
  time_to_dos  per-run seconds from creation to the stitched ln g on the host
               (p50 / p99 over the steps);
  roofline     the sweep kernel's VALU work per attempt times the attempts it
               made, over its own time measured with HIP events on the run's
               stream (rewl_set_timing), against the MI355X vector-ALU peak;
  cpu_baseline the CPU oracle on a bounded sample of the same workload, all
               host cores.
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ising32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU lane-slots one sweep attempt needs (Ising; quarter-rate 32-bit
# multiplies count 4): Philox4x32-10 100, site draw 4, ln u 50, neighbours 20,
# the accept/update chain 20.  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_ATTEMPT = {"ising": 194, "ea": 200, "potts": 204}
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
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def run_kwargs(p):
    keys = ("model", "L", "q", "couplings", "e_min", "e_max", "n_windows", "overlap",
            "walkers_per_window", "flatness", "lnf_init", "lnf_final", "S", "seed")
    return {k: p[k] for k in keys if k in p}


def gpu_full_run(rewl, p, max_rounds):
    """One complete run; returns (seconds, attempts, rounds, sweep_ms, launches, converged)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = rewl.Run(**run_kwargs(p))
    r.set_timing(True)
    ok, issued = False, 0
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
    r.close()
    assert lng.shape[0] == info["n_bins"]
    return t1 - t0, info["attempts"], rounds, ms, n, ok


def cpu_baseline(p, seconds):
    """The oracle on the same workload: start-up, then rounds until ~`seconds`."""
    from oracle import core

    threads = os.cpu_count() or 1
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
    return {"value": att / el, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"{p['name']} seed {p['seed']}: first {rounds} rounds after start-up "
                      f"({att} sweep attempts, {el:.1f} s, OpenMP over walkers)",
            "seconds_per_round": el / rounds}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="ising32", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--max-rounds", type=int, default=200000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rounds", type=int, default=0,
                    help="profile mode: one run, this many rounds after start-up, then exit")
    ap.add_argument("--batch", type=int, default=0,
                    help="profile mode: this many runs of the workload (seeds 1..n) in one batch")
    ap.add_argument("--walkers-per-wave", type=int, default=1)
    ap.add_argument("--graph", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: each REWL run lives on one device and "
              "this build has no multi-GPU path (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    import paper_1305_5615_amd as rewl
    from workloads import run_params

    base = dict(run_params(args.workload, seed=1))
    model = base["model"]

    if args.rounds > 0 and args.batch > 0:
        runs = [run_kwargs(run_params(args.workload, seed=1 + i)) for i in range(args.batch)]
        b = rewl.Batch(runs, walkers_per_wave=args.walkers_per_wave, graph_rounds=args.graph)
        if not args.graph:
            b.set_timing(True)
        b.step(1)
        torch.cuda.synchronize()
        a0 = sum(b[i].info()["attempts"] for i in range(len(b)))
        t0 = time.perf_counter()
        b.step(args.rounds)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ms, n = b.timing()
        att = sum(b[i].info()["attempts"] for i in range(len(b))) - a0
        log(f"profile: {args.batch} x {args.workload}, P={args.walkers_per_wave}, "
            f"graph={args.graph}, {args.rounds} rounds, {att} attempts, {dt:.3f} s, "
            f"{att / dt / 1e9:.3f} G attempts/s, sweep avg {1e3 * ms / max(n, 1):.1f} us")
        b.close()
        return
    if args.rounds > 0:
        r = rewl.Run(**run_kwargs(base))
        r.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.step(args.rounds)
        ms, n = r.timing()
        dt = time.perf_counter() - t0
        att = r.info()["attempts"]
        log(f"profile: {args.workload}, {args.rounds} rounds, {att} attempts, {dt:.3f} s, "
            f"{att / dt / 1e9:.3f} G attempts/s, sweep avg {1e3 * ms / max(n, 1):.1f} us")
        r.close()
        return

    for i in range(args.warmup):
        p = run_params(args.workload, seed=900 + i)
        dt, att, rounds, _, _, ok = gpu_full_run(rewl, p, args.max_rounds)
        log(f"warmup {i}: {dt:.2f} s, {rounds} rounds, converged={ok}")

    times, attempts, rounds_l, sweep_ms, launches = [], 0, [], 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        p = run_params(args.workload, seed=1 + i)
        dt, att, rounds, ms, n, ok = gpu_full_run(rewl, p, args.max_rounds)
        if not ok:
            log(f"step {i}: not converged within {args.max_rounds} rounds")
        times.append(dt)
        attempts += att
        rounds_l.append(rounds)
        sweep_ms += ms
        launches += n
        log(f"step {i}: {dt:.2f} s, {rounds} rounds, {att / dt / 1e9:.3f} G attempts/s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    value = attempts / wall
    slots = VALU_SLOTS_PER_ATTEMPT[model]
    achieved = slots * attempts / (sweep_ms * 1e-3) / 1e12 if sweep_ms > 0 else None
    roofline = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS if achieved else None, "traffic": None,
                "kernel": f"sweep_kernel<{model}>",
                "sweep_avg_us": 1e3 * sweep_ms / launches if launches else None,
                "valu_slots_per_attempt": slots}
    out = {
        "metric": "spin-flip attempts/sec (1 GPU) + p50/p99 time-to-converged ln g, "
                  "batched vs plain",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "form": "plain",
                   "walkers": base["n_windows"] * base["walkers_per_window"],
                   "L": base["L"], "q": base["q"], "seeds": list(range(1, args.steps + 1))},
        "time_to_dos_s": {"p50": percentile(times, 50), "p99": percentile(times, 99),
                          "rounds": rounds_l},
        "roofline": roofline,
    }
    if not args.no_cpu:
        p = dict(run_params(args.workload, seed=1))
        p["name"] = args.workload
        cb = cpu_baseline(p, args.cpu_seconds)
        cb.pop("seconds_per_round")
        # the oracle makes exactly the GPU's attempts (bit-identical runs)
        cb["time_to_dos_s_extrapolated"] = (attempts / args.steps) / cb["value"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
