"""ctypes binding of the C oracle (rewl_oracle.c) -- TEST INFRASTRUCTURE ONLY.

Argument marshalling only; every step of the algorithm runs in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rewl_oracle.c")
# REWL_ORACLE_LIB: load another build of the oracle (the tests that plant a
# mistake in a copy of the C file and check that the pins catch it)
LIB = os.environ.get("REWL_ORACLE_LIB") or os.path.join(HERE, "librewl_oracle.so")

MODELS = {"ising": 0, "potts": 1, "ea": 2, "ea3": 3}


def n_sites(model, L):
    return L ** 3 if model == "ea3" else L * L


def bonds_per_site(model):
    return 3 if model == "ea3" else 2
SCHEDULES = {"halving": 0, "1/t": 1}


def build(force=False):
    """Compile the oracle with gcc (plain C11, no contraction of a*b+c)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        i64, u64, i32, u32, dbl = C.c_int64, C.c_uint64, C.c_int, C.c_uint32, C.c_double
        P = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(P), i32, i32, i32, P, i64, i64, i32, dbl, i32,
                                 dbl, dbl, dbl, i64, u64, i32, i32, P, P]
        L.orc_first_merge.argtypes = [P, P]
        L.orc_partition_balanced.argtypes = [i64, i32, dbl, i32, P, P, P, P, P]
        L.orc_destroy.argtypes = [P]
        L.orc_step.argtypes = [P, i64]
        L.orc_run_to.argtypes = [P, i64]
        L.orc_info.argtypes = [P] + [P] * 8
        L.orc_window.argtypes = [P, i32, P, P, P, P, P]
        L.orc_walker.argtypes = [P, i32, P, P, P, P, P, P, P]
        L.orc_set_lng.argtypes = [P, i32, P]
        L.orc_get_lng.argtypes = [P, P, i64]
        L.orc_stats.argtypes = [P, P, P, P, P]
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_ln_u.argtypes = [dbl]
        L.orc_ln_u.restype = dbl
        L.orc_uniform.argtypes = [u32, u32]
        L.orc_uniform.restype = dbl
        L.orc_energy.argtypes = [i32, i32, i32, P, P]
        L.orc_energy.restype = i64
        L.orc_partition.argtypes = [i64, i32, dbl, P, P]
        L.orc_stitch.argtypes = [i32, P, P, P, i64, P, i64, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def ln_u(u):
    return lib().orc_ln_u(float(u))


def uniform(hi, lo):
    return lib().orc_uniform(int(hi), int(lo))


def energy(model, L, spins, couplings=None, q=2):
    s = np.ascontiguousarray(spins, dtype=np.int8)
    J = None if couplings is None else np.ascontiguousarray(couplings, dtype=np.int8)
    return lib().orc_energy(MODELS[model], L, q, _p(s), _p(J))


def partition(n_bins, n_windows, overlap):
    lo = np.zeros(n_windows, dtype=np.int64)
    hi = np.zeros(n_windows, dtype=np.int64)
    rc = lib().orc_partition(n_bins, n_windows, overlap, _p(lo), _p(hi))
    if rc:
        raise ValueError("invalid partition")
    return lo, hi


def partition_balanced(n_bins, n_windows, overlap, pre_lo, pre_hi, first_rounds):
    """Run-time balanced windows from a pre-run's windows and first-iteration
    rounds (T_k = rounds until window k's first merge)."""
    pl = np.ascontiguousarray(pre_lo, dtype=np.int64)
    ph = np.ascontiguousarray(pre_hi, dtype=np.int64)
    T = np.ascontiguousarray(first_rounds, dtype=np.int64)
    lo = np.zeros(n_windows, dtype=np.int64)
    hi = np.zeros(n_windows, dtype=np.int64)
    rc = lib().orc_partition_balanced(n_bins, n_windows, overlap, len(pl), _p(pl), _p(ph), _p(T),
                                      _p(lo), _p(hi))
    if rc:
        raise ValueError("invalid balanced partition")
    return lo, hi


def stitch(lo, hi, pieces, visited, n_bins):
    lo = np.ascontiguousarray(lo, dtype=np.int64)
    hi = np.ascontiguousarray(hi, dtype=np.int64)
    P = np.ascontiguousarray(pieces, dtype=np.float64)
    V = np.ascontiguousarray(visited, dtype=np.uint8)
    out = np.zeros(n_bins)
    joins = np.zeros(max(1, len(lo) - 1), dtype=np.int64)
    rc = lib().orc_stitch(len(lo), _p(lo), _p(hi), _p(P), P.shape[1], _p(V), n_bins, _p(out),
                          _p(joins))
    if rc:
        raise ValueError(f"stitch failed ({rc})")
    return out, joins[: len(lo) - 1]


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


class Run:
    """One REWL run in the C oracle."""

    def __init__(self, model, L, q=2, couplings=None, e_min=None, e_max=None, n_windows=4,
                 overlap=0.75, walkers_per_window=2, flatness=0.8, lnf_init=1.0,
                 lnf_final=1e-6, S=10_000, seed=1, n_threads=1, schedule="halving",
                 windows=None):
        N = n_sites(model, L)
        nb = bonds_per_site(model)
        if e_min is None:
            e_min = -nb * N
        if e_max is None:
            e_max = 0 if model == "potts" else nb * N
        J = None if couplings is None else np.ascontiguousarray(couplings, dtype=np.int8)
        wl = wh = None
        if windows is not None:
            wl = np.ascontiguousarray(windows[0], dtype=np.int64)
            wh = np.ascontiguousarray(windows[1], dtype=np.int64)
            if len(wl) != n_windows or len(wh) != n_windows:
                raise OracleError(-1, "orc_create")
        h = C.c_void_p()
        rc = lib().orc_create(C.byref(h), MODELS[model], L, q, _p(J), e_min, e_max, n_windows,
                              overlap, walkers_per_window, flatness, lnf_init, lnf_final, S,
                              seed, n_threads, SCHEDULES[schedule], _p(wl), _p(wh))
        if rc:
            raise OracleError(rc, "orc_create")
        self._h = h
        self.model, self.L, self.N = model, L, N
        info = self.info()
        self.n_bins, self.e_min, self.e_step = info["n_bins"], info["e_min"], info["e_step"]
        self.h, self.m = info["n_windows"], info["m"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def info(self):
        v = [C.c_int64(), C.c_int64(), C.c_int64(), C.c_int(), C.c_int(), C.c_int(), C.c_int64(),
             C.c_int()]
        lib().orc_info(self._h, *[C.byref(x) for x in v])
        keys = ["n_bins", "e_min", "e_step", "n_windows", "m", "n_sites", "round", "done"]
        return {k: x.value for k, x in zip(keys, v)}

    def step(self, rounds):
        lib().orc_step(self._h, rounds)

    def run(self, max_rounds=-1):
        return lib().orc_run_to(self._h, max_rounds) == 0

    def window(self, k):
        lo, hi, lnf, done, fin = (C.c_int64(), C.c_int64(), C.c_double(), C.c_int(),
                                  C.c_int64())
        lib().orc_window(self._h, k, C.byref(lo), C.byref(hi), C.byref(lnf), C.byref(done),
                         C.byref(fin))
        return {"lo": lo.value, "hi": hi.value, "lnf": lnf.value, "done": bool(done.value),
                "finish_round": fin.value}

    def windows(self):
        return [self.window(k) for k in range(self.h)]

    def walker(self, w):
        k = w // self.m
        win = self.window(k)
        W = win["hi"] - win["lo"] + 1
        spins = np.zeros(self.N, dtype=np.int8)
        lng = np.zeros(W)
        H = np.zeros(W, dtype=np.uint32)
        vis = np.zeros(W, dtype=np.uint8)
        E, t, flat = C.c_int64(), C.c_uint64(), C.c_int()
        lib().orc_walker(self._h, w, _p(spins), C.byref(E), C.byref(t), C.byref(flat), _p(lng),
                         _p(H), _p(vis))
        return {"spins": spins, "E": E.value, "t": t.value, "flat": bool(flat.value),
                "lng": lng, "H": H, "visited": vis}

    def set_lng(self, w, lng):
        a = np.ascontiguousarray(lng, dtype=np.float64)
        lib().orc_set_lng(self._h, w, _p(a))

    def lng(self):
        out = np.zeros(self.n_bins)
        rc = lib().orc_get_lng(self._h, _p(out), self.n_bins)
        if rc:
            raise OracleError(rc, "orc_get_lng")
        return out

    def energies(self):
        return self.e_min + self.e_step * np.arange(self.n_bins)

    def first_merge(self):
        out = np.zeros(self.h, dtype=np.int64)
        lib().orc_first_merge(self._h, _p(out))
        return out

    def stats(self):
        v = [C.c_uint64() for _ in range(4)]
        lib().orc_stats(self._h, *[C.byref(x) for x in v])
        return dict(zip(["attempts", "accepts", "ex_prop", "ex_acc"], [x.value for x in v]))
