"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds no part of the method's arithmetic: it only names the
workloads (lattice model, size, windows, walkers, schedule) and draws the random
inputs that are not part of the Monte Carlo itself -- the +-J couplings of the
spin-glass instances and the arrival stream of the served workload -- from
numpy's seeded generator.  The oracle and the GPU library both receive these as
plain arrays and numbers.
"""
from __future__ import annotations

import numpy as np

# Workload parameters.  Energies: Ising and +-J span [-2N, 2N] in steps of 4,
# Potts [-2N, 0] in steps of 1 (N = L*L); the 3D +-J glass [-3N, 3N] in steps
# of 4 (N = L^3).
CONFIGS = {
    # 2D Ising 8x8, 4 windows x 2 walkers, ln f 1 -> 1e-6 (the small parity case)
    "ising8": dict(model="ising", L=8, q=2, n_windows=4, overlap=0.75, walkers_per_window=2,
                   flatness=0.8, lnf_init=1.0, lnf_final=1e-6, S=10_000),
    # 2D Ising 32x32, 16 windows x 4 walkers, exchange every 1e4 attempts, ln f final 1e-8
    "ising32": dict(model="ising", L=32, q=2, n_windows=16, overlap=0.75, walkers_per_window=4,
                    flatness=0.8, lnf_init=1.0, lnf_final=1e-8, S=10_000),
    # 2D 10-state Potts 64x64, 32 windows x 8 walkers, ln f final 1e-8
    "potts64": dict(model="potts", L=64, q=10, n_windows=32, overlap=0.75, walkers_per_window=8,
                    flatness=0.8, lnf_init=1.0, lnf_final=1e-8, S=10_000),
    # one 2D +-J Edwards-Anderson glass 24x24, 8 windows x 4 walkers (256 of them batched)
    "ea24": dict(model="ea", L=24, q=2, n_windows=8, overlap=0.75, walkers_per_window=4,
                 flatness=0.8, lnf_init=1.0, lnf_final=1e-6, S=10_000),
    # one 3D +-J glass 12x12x12 (the paper's ground-state test size), 8 windows
    # x 4 walkers, ln f final 1e-6
    "ea3d12": dict(model="ea3", L=12, q=2, n_windows=8, overlap=0.75, walkers_per_window=4,
                   flatness=0.8, lnf_init=1.0, lnf_final=1e-6, S=10_000),
}


def ea_couplings(L, seed):
    """+-1 couplings with p = 1/2, laid out [2i] = J(i, right), [2i+1] = J(i, down)."""
    rng = np.random.default_rng(np.random.SeedSequence([0xEA, int(seed)]))
    return np.where(rng.random(2 * L * L) < 0.5, 1, -1).astype(np.int8)


def ea3_couplings(L, seed):
    """+-1 couplings with p = 1/2 on the L^3 torus, laid out [3i + a] = J(i,
    next site along axis a = x, y, z), sites i = (z L + y) L + x."""
    rng = np.random.default_rng(np.random.SeedSequence([0xEA3, int(seed)]))
    return np.where(rng.random(3 * L ** 3) < 0.5, 1, -1).astype(np.int8)


def full_range(model, L):
    if model == "ea3":
        return (-3 * L ** 3, 3 * L ** 3)
    N = L * L
    return (-2 * N, 0) if model == "potts" else (-2 * N, 2 * N)


def run_params(name, seed=1, **over):
    """Complete parameter dict for a named workload (couplings drawn for EA)."""
    p = dict(CONFIGS[name])
    p.update(over)
    e_min, e_max = full_range(p["model"], p["L"])
    p.setdefault("e_min", e_min)
    p.setdefault("e_max", e_max)
    p["seed"] = int(seed)
    if p["model"] == "ea" and "couplings" not in p:
        p["couplings"] = ea_couplings(p["L"], seed)
    elif p["model"] == "ea3" and "couplings" not in p:
        p["couplings"] = ea3_couplings(p["L"], seed)
    elif p["model"] not in ("ea", "ea3"):
        p["couplings"] = None
    return p


SERVED_SIZES = {
    # Ising L choices, Potts L range, +-J L range, windows range (inclusive)
    "full": ((16, 24, 32, 48, 64), (16, 48), (16, 32), (4, 32)),
    "small": ((8, 12, 16), (8, 16), (8, 16), (4, 16)),
}


def served_stream(n_requests, rate_per_s, seed=7, lnf_choices=(1e-4, 1e-5, 1e-6), sizes="full"):
    """Poisson arrivals of REWL requests with a mix of models and sizes.

    sizes="full": Ising L in {16,24,32,48,64}; Potts q in 2..10, L in 16..48;
    +-J L in 16..32 on |E| <= 1.5 N; windows 4..32.  sizes="small": the same mix on L <= 16 and
    4..16 windows, for runs of seconds.  Walkers 2, 4 or 8 per window.  Returns
    a list of dicts with an 'arrival' time in seconds and the run parameters.
    """
    ising_L, potts_L, ea_L, hs = SERVED_SIZES[sizes]
    rng = np.random.default_rng(np.random.SeedSequence([0x5E, int(seed)]))
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        kind = ("ising", "potts", "ea")[rng.integers(3)]
        if kind == "ising":
            L = int(rng.choice(list(ising_L)))
            q = 2
        elif kind == "potts":
            L = int(rng.integers(potts_L[0], potts_L[1] + 1))
            q = int(rng.integers(2, 11))
        else:
            L = int(rng.integers(ea_L[0], ea_L[1] + 1))
            q = 2
        h = int(rng.integers(hs[0], hs[1] + 1))
        m = int(rng.choice([2, 4, 8]))
        e_min, e_max = full_range(kind, L)
        if kind == "ea":
            # +-J: |E| <= 1.5 N holds every state an instance can reach (the
            # ground state is near -1.40 N), so no window lies wholly below it
            e_min, e_max = -(3 * L * L) // 2, (3 * L * L) // 2
        p = dict(model=kind, L=L, q=q, n_windows=h, overlap=0.75, walkers_per_window=m,
                 flatness=0.8, lnf_init=1.0, lnf_final=float(rng.choice(lnf_choices)),
                 S=10_000, e_min=e_min, e_max=e_max, seed=1000 + i)
        p["couplings"] = ea_couplings(L, 1000 + i) if kind == "ea" else None
        out.append(dict(arrival=t, params=p))
    return out
