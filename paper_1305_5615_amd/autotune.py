"""Launch-setting search for batched REWL runs.

The results of a batch do not depend on how its rounds are launched: walkers
per wave (how many walkers share one wave's instructions in the sweep), the
form of a round (separate kernel launches, optionally replayed from a captured
HIP graph of several rounds, or one persistent launch per work-group that loops
rounds with the whole run in LDS) change only the speed.  The attempts per
walker between exchange steps (S) do change the walk; they are searched only
when the caller says the workload leaves them open, and then every candidate
is compared over the same number of attempts per walker.

Each candidate is timed on a fresh batch built from the same run parameters:
one round to warm up, then `rounds` rounds (scaled by 10^4 / S when S is
searched) bracketed by stream synchronisations.  The fastest, by sweep
attempts per second, is kept and cached per run shape for the life of the
process, so a Batch or Server created later for the same shape reuses it.
"""
from __future__ import annotations

import itertools
import time
from typing import Callable, Dict, Iterable, List, NamedTuple, Optional, Sequence, Tuple


class Setting(NamedTuple):
    walkers_per_wave: int
    form: str              # "rounds" (kernel launches per round) or "persistent"
    graph_rounds: int      # rounds per captured graph in the "rounds" form (0: direct)
    S: Optional[int]       # attempts per walker per round, None: the runs' own


_cache: Dict[tuple, Tuple[Setting, float]] = {}


def shape_key(runs: Sequence[dict], open_S: bool = False) -> tuple:
    """What the speed of a batch depends on: each run's model, lattice,
    windows and walkers (not its seed or couplings), and S unless S is
    searched."""
    items = []
    for kw in runs:
        items.append((kw["model"], kw["L"], kw.get("q", 2), kw.get("n_windows", 4),
                      kw.get("walkers_per_window", 2), kw.get("e_min"), kw.get("e_max"),
                      round(float(kw.get("overlap", 0.75)), 6),
                      None if open_S else kw.get("S", 10_000)))
    return tuple(sorted(items)) + ((len(runs),),)


def candidates(P_options: Iterable[int] = (1, 2, 4, 8), forms: Iterable[str] = ("rounds",),
               graph_options: Iterable[int] = (0, 16),
               S_options: Optional[Iterable[int]] = None) -> List[Setting]:
    """The search space: persistent launches take no graph."""
    out = []
    S_list = list(S_options) if S_options else [None]
    for S, form, P in itertools.product(S_list, forms, P_options):
        graphs = list(graph_options) if form == "rounds" else [0]
        for gr in graphs:
            out.append(Setting(int(P), form, int(gr), S))
    return out


def search(cands: Sequence[Setting], measure: Callable[[Setting], Optional[float]],
           log: Optional[Callable[[str], None]] = None) -> Tuple[Setting, float, list]:
    """Rate every candidate (attempts/s; None: the setting is not valid for
    these runs) and return the fastest, its rate and the whole table.  Ties go
    to the earlier candidate."""
    best, best_rate, table = None, -1.0, []
    for c in cands:
        rate = measure(c)
        table.append((c, rate))
        if log:
            log(f"autotune: {c} -> " + ("invalid" if rate is None else f"{rate / 1e9:.3f} G/s"))
        if rate is not None and rate > best_rate:
            best, best_rate = c, rate
    if best is None:
        raise ValueError("autotune: no candidate setting is valid for these runs")
    return best, best_rate, table


def batch_rate(runs: Sequence[dict], setting: Setting, rounds: int = 4,
               make_batch: Optional[Callable] = None, sync: Optional[Callable] = None,
               timer: Callable[[], float] = time.perf_counter) -> Optional[float]:
    """Sweep attempts per second of a fresh batch of `runs` launched with
    `setting`: one round to warm up, then `rounds` rounds (times 10^4 / S when
    the setting overrides S, so that every S covers the same attempts)."""
    if make_batch is None:
        from . import Batch as make_batch
    if sync is None:
        import torch

        sync = torch.cuda.synchronize
    from . import RewlError

    kws = [dict(kw, S=setting.S) if setting.S else dict(kw) for kw in runs]
    try:
        b = make_batch(kws, walkers_per_wave=setting.walkers_per_wave,
                       graph_rounds=setting.graph_rounds, form=setting.form)
    except RewlError:
        return None
    try:
        n = len(kws)
        S = setting.S or kws[0].get("S", 10_000)
        steps = max(1, rounds * 10_000 // S) if setting.S else rounds
        b.step(1)
        sync()
        a0 = sum(b[i].info()["attempts"] for i in range(n))
        t0 = timer()
        b.step(steps)
        sync()
        dt = timer() - t0
        att = sum(b[i].info()["attempts"] for i in range(n)) - a0
    finally:
        b.close()
    return att / dt if dt > 0 else None


def tune(runs: Sequence[dict], P_options: Iterable[int] = (1, 2, 4, 8),
         forms: Iterable[str] = ("rounds", "persistent"), graph_options: Iterable[int] = (0, 16),
         S_options: Optional[Iterable[int]] = None, rounds: int = 4,
         measure: Optional[Callable[[Setting], Optional[float]]] = None,
         log: Optional[Callable[[str], None]] = None, use_cache: bool = True):
    """The fastest setting for this batch of runs (cached per run shape).
    Returns (setting, attempts/s, table); the table is empty on a cache hit."""
    key = shape_key(runs, open_S=S_options is not None) + (
        tuple(P_options), tuple(forms), tuple(graph_options),
        tuple(S_options) if S_options else None)
    if use_cache and key in _cache:
        s, r = _cache[key]
        return s, r, []
    if measure is None:
        def measure(c):
            return batch_rate(runs, c, rounds=rounds)
    best, rate, table = search(candidates(P_options, forms, graph_options, S_options), measure,
                               log)
    _cache[key] = (best, rate)
    return best, rate, table


def clear_cache():
    _cache.clear()
