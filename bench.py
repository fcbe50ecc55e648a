#!/usr/bin/env python3
"""Benchmark: replica-exchange Wang-Landau on one MI355X.

Headline (the JSON line's `value`): the batched spin-glass workload, 256
independent 2D +-J Edwards-Anderson glasses L = 24 (couplings +-1 with p = 1/2,
one coupling seed per instance), 8 windows x 4 walkers each, overlap 0.75,
flatness 0.8, ln f 1 -> 1e-6, 10^4 attempts per walker between exchange steps.
One step = one round of every run: 8192 walkers x 10^4 sweep attempts, then
flatness, merges and one exchange step.  `value` = sweep attempts (accepted or
not; start-up excluded) per second of wall clock over the K timed steps, after
W untimed ones; the launch form (per-round kernels, or one persistent
work-group per run looping the rounds in LDS) and the walkers per wave come
from the package's autotuner unless given.

  roofline      the dominant kernel of the timed steps (the persistent kernel,
                or the sweep kernel of the per-round form): VALU lane-slots per
                sweep attempt (170, the upper end of the algorithmic 150-170
                estimate for the model with couplings) x attempts per launch,
                over the launch's average duration from HIP events recorded on
                the batch's stream around each launch, against 256 CUs x 4
                SIMDs x 16 lanes x 2.4 GHz; traffic = HBM bytes per launch from
                the committed rocprofv3 counter summary while the device
                sources are unchanged (null otherwise);
  cpu_baseline  the CPU oracle on the same workload (a few of the instances,
                a few rounds each), all host threads; single-core and all-core
                rates for the other workloads under `per_workload`;
  legs          bounded sub-measurements, each with its own wall-clock budget:
                the other launch form at the same setting; the 32x32 Ising and
                64x64 q=10 Potts single runs (attempts/s over rounds with every
                window running, sweep kernel time); p50/p99 time-to-converged
                ln g of the 8x8 Ising workload over 20 seeds arriving together:
                plain runs one after another (each run's own duration, and its
                completion time counting the runs before it) vs all 20 in one
                batch (autotuned launch setting).
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--form auto|rounds|persistent]
                       [--walkers-per-wave P] [--legs all|headline] [--no-cpu]
Other modes (one JSON line each): --rounds R (profile: fixed rounds of one
workload), --served N, --balanced, --errors R, --time-to-dos N, --copy-mb M
(counter calibration).
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

# VALU lane-slots one sweep attempt needs, the algorithmic estimate (quarter-
# rate 32-bit multiplies count 4): Philox4x32-10 ~100-110, site 4, neighbours
# and energy change ~20, the decision 2, the acceptance function ~16, updates
# ~5: 150-170; the upper end is taken for every model.  This implementation
# spends ~194-212 (it draws ln u, ~50 slots, for every attempt; reported beside
# it as the recount).  Peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_SLOTS_PER_ATTEMPT = 170
VALU_SLOTS_RECOUNT = {"ising": 194, "ea": 200, "potts": 204, "ea3": 212}
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
HEADLINE = ("256 independent 2D +-J EA glasses L=24 periodic (couplings +-1, p=0.5, seeds "
            "1-256), 8 windows x 4 walkers each, overlap 0.75, flatness 0.8, ln f 1 -> 1e-6, "
            "1e4 attempts/walker between exchanges; one step = one round of all 256 runs")


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
    """HBM bytes per launch of the profiled kernel from profiles/<tag>.md
    (FETCH_SIZE and WRITE_SIZE scaled by a device copy of known size), or None
    when the file is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{tag}.md")
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


def percentile(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs, dtype=float), q)) if xs else None


def run_kwargs(p):
    keys = ("model", "L", "q", "couplings", "e_min", "e_max", "n_windows", "overlap",
            "walkers_per_window", "flatness", "lnf_init", "lnf_final", "S", "seed", "schedule",
            "windows")
    return {k: p[k] for k in keys if k in p}


class Budget:
    """Wall-clock allowance of the optional legs: a leg runs only while the
    time spent so far leaves its own allowance."""

    def __init__(self, total_s):
        self.t0 = time.perf_counter()
        self.total = total_s

    def left(self):
        return self.total - (time.perf_counter() - self.t0)

    def allows(self, need_s, name):
        if self.left() >= need_s:
            return True
        log(f"leg {name}: skipped ({self.left():.0f} s of the budget left, needs {need_s:.0f} s)")
        return False


def roofline(attempts, launches, launch_ms, traffic, kernel):
    """VALU roofline of the dominant kernel from its HIP-event launch times."""
    if launches <= 0 or launch_ms <= 0:
        return None
    per_launch = attempts / launches
    avg_s = launch_ms * 1e-3 / launches
    achieved = VALU_SLOTS_PER_ATTEMPT * per_launch / avg_s / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic, "kernel": kernel,
            "launch_avg_us": avg_s * 1e6, "attempts_per_launch": per_launch,
            "valu_slots_per_attempt": VALU_SLOTS_PER_ATTEMPT,
            "frac_at_recount": achieved / VALU_PEAK_TOPS * VALU_SLOTS_RECOUNT["ea"] /
            VALU_SLOTS_PER_ATTEMPT,
            "valu_slots_recount": VALU_SLOTS_RECOUNT["ea"]}


def kernel_name(rewl, form, P, waves):
    """The instantiation a launch runs: the per-step bin records sit in
    registers when waves outnumber the compute units."""
    import torch

    cus = torch.cuda.get_device_properties(0).multi_processor_count
    rp = "true" if waves > cus else "false"
    return f"persist_kernel<{P}, {rp}>" if form == "persistent" else f"sweep_kernel<{P}, {rp}>"


def attempts_of(views):
    return sum(v.info()["attempts"] for v in views)


def glass_runs(n, S=10_000):
    from workloads import run_params

    return [dict(run_kwargs(run_params("ea24", seed=1 + i)), S=S) for i in range(n)]


def timed_batch(rewl, runs, setting, steps, warmup):
    """W untimed rounds, then K rounds bracketed by device synchronisations,
    with HIP events around each launch of the dominant kernel."""
    import torch

    b = rewl.Batch(runs, walkers_per_wave=setting.walkers_per_wave,
                   graph_rounds=setting.graph_rounds, form=setting.form)
    views = [b[i] for i in range(len(runs))]
    b.set_timing(True)
    if warmup:
        b.step(warmup)
    torch.cuda.synchronize()
    ms0, n0 = b.timing()
    a0 = attempts_of(views)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = b.timing()
    att = attempts_of(views) - a0
    b.close()
    return dict(wall=wall, attempts=att, launch_ms=ms - ms0, launches=n - n0)


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


def profile(rewl, args, run_params):
    """Fixed rounds of one run (or of a batch) after start-up, for profilers."""
    import torch

    over = {"S": args.attempts_per_round} if args.attempts_per_round else {}
    if args.batch > 1 and args.walkers_per_wave > 0:
        runs = [run_kwargs(run_params(args.workload, seed=1 + i, **over))
                for i in range(args.batch)]
        P = args.walkers_per_wave
        r = rewl.Batch(runs, walkers_per_wave=P, graph_rounds=0,
                       form=args.form if args.form != "auto" else "rounds")
        label = f"{len(runs)} x {args.workload}, P={P}, {args.form}"
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


def accuracy(rewl, args):
    """One run of a workload to convergence (possibly over several invocations:
    it checkpoints after --max-rounds rounds and --resume continues), then max
    |ln g - ln g_exact| where an exact DOS is stored.  Walkers per window and
    the ln f schedule may differ from the workload's (--accuracy-m, --schedule,
    --lnf-final)."""
    from workloads import run_params

    p = run_params(args.workload, seed=1)
    over = {"schedule": args.schedule}
    if args.accuracy_m:
        over["walkers_per_window"] = args.accuracy_m
    if args.lnf_final:
        over["lnf_final"] = args.lnf_final
    p.update(over)
    t0 = time.perf_counter()
    r = rewl.Run.load(args.resume) if args.resume else rewl.Run(**run_kwargs(p))
    issued, ok, rounds = 0, False, 0
    while issued < args.max_rounds and not ok:
        n = min(20_000, args.max_rounds - issued)
        ok, rounds = r.run(n)
        issued += n
        ws = r.windows()
        log(f"{time.perf_counter() - t0:.0f} s: rounds {r.info()['rounds']}, windows done "
            f"{sum(w['done'] for w in ws)}/{len(ws)}, largest ln f {max(w['lnf'] for w in ws):.3g}")
    out = {"metric": "max |ln g - ln g_exact| of one run to convergence",
           "workload": WORKLOAD_TEXT[args.workload], "overrides": over,
           "seconds_this_invocation": time.perf_counter() - t0, "converged": ok}
    if ok:
        out["rounds"] = rounds
        lng = r.lng()
        out["max_abs_dlng_vs_exact"] = exact_error(p, lng)
        out["checks"] = dos_checks(p, r, lng)
    else:
        r.save(args.checkpoint)
        out["checkpoint"] = args.checkpoint
        out["rounds_so_far"] = r.info()["rounds"]
    r.close()
    print(json.dumps(out), flush=True)


def dos_checks(p, r, lng):
    """Checks of a converged ln g that need no exact DOS: the log of the total
    number of states against N ln(states per site), and the peak of the
    specific heat per site C/N = beta^2 var(E) / N on a temperature scan (for
    first-order transitions a known finite-size law places it)."""
    import numpy as np

    n, states = r.N, (p.get("q") or 2) if p["model"] == "potts" else 2
    E = r.energies().astype(float)
    fin = np.isfinite(lng)
    E, g = E[fin], lng[fin]
    m = g.max()
    out = {"log_total_states": float(m + math.log(np.exp(g - m).sum())),
           "n_ln_states_per_site": n * math.log(states)}

    def heat(T):
        w = g - E / T
        wm = w.max()
        pr = np.exp(w - wm)
        z = pr.sum()
        e1 = (pr * E).sum() / z
        return ((pr * E * E).sum() / z - e1 * e1) / (T * T) / n

    Ts = np.linspace(0.2, 5.0, 4801)
    cs = np.array([heat(T) for T in Ts])
    i = int(cs.argmax())
    fine = np.linspace(Ts[max(i - 1, 0)], Ts[min(i + 1, len(Ts) - 1)], 2001)
    cf = np.array([heat(T) for T in fine])
    j = int(cf.argmax())
    out["specific_heat_peak"] = {"T": float(fine[j]), "C_per_site": float(cf[j])}
    return out


def calibrate_copy(mb):
    """One device-to-device copy of `mb` MiB (read mb, write mb) for scaling
    the FETCH_SIZE / WRITE_SIZE counters.  The source is written first and then
    pushed out of the last-level cache (256 MB) by writing 1 GiB elsewhere, so
    the copy's reads come from HBM; use a copy several times larger than that
    cache."""
    import torch

    src = torch.ones(mb << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    flush.fill_(2.0)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy: {mb} MiB read, {mb} MiB written (after a 1 GiB fill)")



def plain_rate(rewl, name, rounds):
    """One plain run of a workload: attempts/s and the sweep kernel's average
    launch over `rounds` rounds right after start-up (every window running)."""
    import torch

    from workloads import run_params

    r = rewl.Run(**run_kwargs(run_params(name, seed=1)))
    r.set_timing(True)
    r.step(1)
    torch.cuda.synchronize()
    a0 = r.info()["attempts"]
    ms0, n0 = r.timing()
    t0 = time.perf_counter()
    r.step(rounds)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = r.timing()
    att = r.info()["attempts"] - a0
    r.close()
    return {"workload": WORKLOAD_TEXT[name], "rounds": rounds, "attempts_per_s": att / wall,
            "sweep_avg_us": 1e3 * (ms - ms0) / max(n - n0, 1)}


def time_to_dos(rewl, seeds, budget_plain_s, workload="ising8", max_rounds=100_000,
                verbose=False):
    """p50/p99 time-to-converged ln g of a workload: each seed as a plain run,
    one after another (time from creation to the stitched ln g on the host),
    and all seeds in one batch, launched as the autotuner picks and polled every
    16 rounds (time from the batch's creation to the run's stitched ln g on
    the host)."""
    import numpy as np
    import torch

    from paper_1305_5615_amd import autotune
    from workloads import run_params

    params = [run_params(workload, seed=s) for s in seeds]
    plain, plain_err, plain_att = [], [], 0
    t_start = time.perf_counter()
    for p in params:
        if time.perf_counter() - t_start > budget_plain_s:
            log(f"time-to-DOS: plain runs stopped after {len(plain)} seeds (budget)")
            break
        res = gpu_full_run(rewl, p, max_rounds)
        if verbose:
            log(f"time-to-DOS: plain {workload} seed {p['seed']}: {res['seconds']:.2f} s")
        plain.append(res["seconds"])
        plain_att += res["attempts"]
        plain_err.append(exact_error(p, res["lng"]))
    kws = [run_kwargs(p) for p in params]
    setting, _, _ = autotune.tune(kws, P_options=(1, 2, 8), forms=("rounds", "persistent"),
                                  graph_options=(0, 16), rounds=8, log=log)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = rewl.Batch(kws, walkers_per_wave=setting.walkers_per_wave,
                   graph_rounds=setting.graph_rounds, form=setting.form)
    done_at = [None] * len(params)
    errs = [None] * len(params)
    issued = 0
    while issued < max_rounds:
        b.step(16)
        issued += 16
        d = b.done()
        for i in np.nonzero(d)[0]:
            if done_at[i] is None:
                lng = b[int(i)].lng()
                done_at[i] = time.perf_counter() - t0
                if verbose:
                    log(f"time-to-DOS: batched run {int(i)} done at {done_at[i]:.2f} s")
                errs[i] = exact_error(params[i], lng)
        if d.all():
            break
    wall = time.perf_counter() - t0
    att = attempts_of([b[i] for i in range(len(params))])
    b.close()
    got = [x for x in done_at if x is not None]
    # the same requests all arriving at once and served one after another:
    # a run's time-to-DOS then includes waiting for the runs before it
    fifo = list(np.cumsum(plain))
    return {"workload": WORKLOAD_TEXT[workload], "seeds": [int(s) for s in seeds],
            "plain_fifo": {"runs": len(fifo), "p50_s": percentile(fifo, 50),
                           "p99_s": percentile(fifo, 99)},
            "plain": {"runs": len(plain), "p50_s": percentile(plain, 50),
                      "p99_s": percentile(plain, 99), "wall_s": sum(plain),
                      "attempts_per_s": plain_att / sum(plain) if plain else None,
                      "max_abs_dlng_vs_exact": plain_err},
            "batched": {"runs": len(got), "p50_s": percentile(got, 50),
                        "p99_s": percentile(got, 99), "wall_s": wall,
                        "attempts_per_s": att / wall, "setting": setting._asdict(),
                        "max_abs_dlng_vs_exact": errs}}


def oracle_rate(params, threads, seconds, max_rounds=10**9):
    """The oracle's sweep attempts per second on `params` (one run after
    another, start-up untimed), stepping rounds until `seconds` have passed or
    the run has converged."""
    from oracle import core

    att, el, rounds = 0, 0.0, 0
    for p in params:
        o = core.Run(**run_kwargs(p), n_threads=threads)
        a0 = o.stats()["attempts"]
        t0 = time.perf_counter()
        r = 0
        while r < max_rounds and not o.info()["done"]:
            o.step(1)
            r += 1
            if time.perf_counter() - t0 >= seconds / len(params):
                break
        el += time.perf_counter() - t0
        att += o.stats()["attempts"] - a0
        rounds += r
    return att / el, rounds, att, el


def cpu_baseline(threads, seconds):
    """The oracle on the headline workload (two of the 256 instances, a few
    rounds each, all host threads), plus single-core and all-core rates on
    every workload."""
    from workloads import run_params

    glass = [run_params("ea24", seed=s) for s in (1, 2)]
    v, rounds, att, el = oracle_rate(glass, threads, seconds)
    out = {"value": v, "unit": "attempts/s", "cores": threads, "kind": "oracle",
           "sample": f"instances 1-2 of the 256 24x24 +-J glasses, {rounds} rounds after "
                     f"start-up ({att} sweep attempts in {el:.1f} s), OpenMP over each "
                     f"instance's 32 walkers, {threads} threads",
           "per_workload": {}}
    for name in ("ising8", "ising32", "potts64", "ea24"):
        p = [run_params(name, seed=1)]
        rec = {}
        for label, th in (("one_core", 1), ("all_cores", threads)):
            r, n, a, e = oracle_rate(p, th, seconds / 4)
            rec[label] = {"attempts_per_s": r, "rounds": n, "threads": th}
        out["per_workload"][name] = rec
        log(f"cpu: {name}: 1 core {rec['one_core']['attempts_per_s']:.3g}, "
            f"{threads} threads {rec['all_cores']['attempts_per_s']:.3g} attempts/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--form", default="auto", choices=("auto", "rounds", "persistent"),
                    help="launch form of the headline batch (auto: the autotuner's choice)")
    ap.add_argument("--walkers-per-wave", type=int, default=0,
                    help="walkers per wave of the headline batch (0: autotune); in profile "
                         "mode with --batch, the batch's setting")
    ap.add_argument("--legs", default="all", choices=("all", "headline"),
                    help="headline only, or the bounded sub-measurements too")
    ap.add_argument("--budget", type=float, default=150.0,
                    help="wall-clock seconds for the optional legs and the CPU baseline")
    ap.add_argument("--glasses", type=int, default=256, help="runs in the headline batch")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="ising32", choices=sorted(WORKLOAD_TEXT),
                    help="profile / balanced / errors modes: the workload")
    ap.add_argument("--batch", type=int, default=0,
                    help="profile mode: this many runs of the workload in one batch")
    ap.add_argument("--max-rounds", type=int, default=400000)
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
    ap.add_argument("--time-to-dos", type=int, default=0,
                    help="time-to-DOS mode: seeds 1..N of --workload as plain runs one after "
                         "another (within --budget seconds) and all in one batch")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="counter calibration: one device copy of this many MiB")
    ap.add_argument("--accuracy", action="store_true",
                    help="accuracy mode: one run of --workload to convergence (checkpointed "
                         "after --max-rounds rounds; --resume continues) and its max |d ln g|")
    ap.add_argument("--accuracy-m", type=int, default=0,
                    help="accuracy mode: walkers per window (0: the workload's)")
    ap.add_argument("--schedule", default="halving", choices=("halving", "1/t"),
                    help="accuracy mode: ln f schedule")
    ap.add_argument("--lnf-final", type=float, default=0.0,
                    help="accuracy mode: ln f_final (0: the workload's)")
    ap.add_argument("--resume", default="", help="accuracy mode: checkpoint to continue from")
    ap.add_argument("--checkpoint", default="accuracy.rewl",
                    help="accuracy mode: where to write the checkpoint")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: each REWL run lives on one device and "
              "the library has no multi-GPU path (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    import paper_1305_5615_amd as rewl
    from paper_1305_5615_amd import autotune
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
    if args.accuracy:
        accuracy(rewl, args)
        return
    if args.time_to_dos > 0:
        out = time_to_dos(rewl, range(1, args.time_to_dos + 1), args.budget,
                          workload=args.workload, max_rounds=args.max_rounds, verbose=True)
        out["metric"] = "time-to-converged ln g, plain one after another vs batched"
        print(json.dumps(out), flush=True)
        return

    budget = Budget(args.budget)
    runs = glass_runs(args.glasses)
    # the launch setting: walkers per wave (8 or 4 fill the chip's SIMDs with
    # 8192 walkers) and the form; graphs are left out because the timed region
    # records HIP events around every launch
    forms = ("rounds", "persistent") if args.form == "auto" else (args.form,)
    Ps = (args.walkers_per_wave,) if args.walkers_per_wave else (4, 8)
    if len(forms) * len(Ps) > 1:
        setting, rate, table = autotune.tune(runs, P_options=Ps, forms=forms, graph_options=(0,),
                                             rounds=2, log=log)
        tuned = [{"setting": c._asdict(), "attempts_per_s": r} for c, r in table]
    else:
        setting = autotune.Setting(Ps[0], forms[0], 0, None)
        tuned = []
    log(f"headline: {setting}")
    res = timed_batch(rewl, runs, setting, args.steps, args.warmup)
    waves = len(runs) * 32 // setting.walkers_per_wave
    kname = kernel_name(rewl, setting.form, setting.walkers_per_wave, waves)
    tag = f"{'persist' if setting.form == 'persistent' else 'sweep'}_ea24x256_P{setting.walkers_per_wave}"
    value = res["attempts"] / res["wall"]
    log(f"headline: {args.steps} rounds, {res['attempts']} attempts in {res['wall']:.4f} s = "
        f"{value / 1e9:.2f} G attempts/s; {res['launches']} launches, "
        f"{res['launch_ms']:.3f} ms")
    out = {
        "metric": "spin-flip attempts/sec (1 GPU) + p50/p99 time-to-converged ln g, "
                  "batched vs plain",
        "value": value, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * res["wall"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE, "form": setting.form,
                   "walkers_per_wave": setting.walkers_per_wave, "runs": len(runs),
                   "walkers": len(runs) * 32, "attempts_per_step": res["attempts"] / args.steps},
        "roofline": roofline(res["attempts"], res["launches"], res["launch_ms"],
                             profiled_traffic(tag), kname),
        "autotune": tuned,
    }
    legs = {}
    if args.legs == "all":
        other = "rounds" if setting.form == "persistent" else "persistent"
        if budget.allows(10, "other form"):
            try:
                o = timed_batch(rewl, runs, setting._replace(form=other), args.steps, args.warmup)
                legs["other_form"] = {
                    "form": other, "walkers_per_wave": setting.walkers_per_wave,
                    "attempts_per_s": o["attempts"] / o["wall"],
                    "launch_avg_us": 1e3 * o["launch_ms"] / max(o["launches"], 1),
                    "launches": o["launches"]}
            except rewl.RewlError as e:
                legs["other_form"] = {"form": other, "error": str(e)}
        for name, rounds in (("ising32", 300), ("potts64", 60)):
            if budget.allows(15, name):
                legs[f"plain_{name}"] = plain_rate(rewl, name, rounds)
                log(f"plain {name}: {legs[f'plain_{name}']['attempts_per_s'] / 1e9:.3f} G/s")
        if budget.allows(45, "time-to-DOS"):
            legs["time_to_dos_ising8"] = time_to_dos(rewl, range(1, 21),
                                                          min(30.0, budget.left() - 15))
            t = legs["time_to_dos_ising8"]
            log(f"time-to-DOS 8x8 Ising: plain alone p50 {t['plain']['p50_s']:.3f} s p99 "
                f"{t['plain']['p99_s']:.3f} s; plain one after another p50 "
                f"{t['plain_fifo']['p50_s']:.2f} s p99 {t['plain_fifo']['p99_s']:.2f} s; "
                f"batched p50 {t['batched']['p50_s']:.3f} s p99 {t['batched']['p99_s']:.3f} s")
    out["legs"] = legs
    if not args.no_cpu and budget.allows(args.cpu_seconds * 2 + 5, "cpu baseline"):
        threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else \
            (os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(threads, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
