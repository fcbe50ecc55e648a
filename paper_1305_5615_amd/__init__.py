"""MI355X-native replica-exchange Wang-Landau sampling (arXiv:1305.5615).

Thin Python binding of librewl.so (C ABI in include/rewl.h).  Argument
marshalling only: every step of the method runs in the library's HIP kernels.
PyTorch supplies the device memory (a uint8 tensor of rewl_footprint() bytes)
and the stream the kernels are queued on.  There is no CPU fallback: without
the built library, or without a GPU, creating a run raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librewl.so")

MODELS = {"ising": 0, "potts": 1, "ea": 2, "ea3": 3}


def n_sites(model, L):
    """Sites of the lattice: L^2, or L^3 for the 3D glass."""
    return L ** 3 if model == "ea3" else L * L
ERRORS = {1: "REWL_NOT_CONVERGED", -1: "REWL_EINVAL", -2: "REWL_ENOMEM", -3: "REWL_EDEVICE",
          -4: "REWL_EINIT", -5: "REWL_ECORRUPT", -6: "REWL_EBUSY", -7: "REWL_ESTITCH"}


class RewlError(RuntimeError):
    def __init__(self, code, what, detail=""):
        super().__init__(f"{what}: {ERRORS.get(code, code)} {detail}".strip())
        self.code = code


class Params(C.Structure):
    _fields_ = [("model", C.c_int), ("L", C.c_int), ("q", C.c_int),
                ("couplings", C.c_void_p), ("e_min", C.c_int64), ("e_max", C.c_int64),
                ("n_windows", C.c_int), ("overlap", C.c_double),
                ("walkers_per_window", C.c_int), ("flatness", C.c_double),
                ("lnf_init", C.c_double), ("lnf_final", C.c_double),
                ("attempts_per_round", C.c_int64), ("seed", C.c_uint64),
                ("schedule", C.c_int), ("window_lo", C.c_void_p), ("window_hi", C.c_void_p)]

SCHEDULES = {"halving": 0, "1/t": 1}


_lib = None


def lib():
    """Load librewl.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with "
                              "python -m paper_1305_5615_amd.build (hipcc, gfx950)")
        L = C.CDLL(LIB)
        P, i64, u64, i32, dbl = C.c_void_p, C.c_int64, C.c_uint64, C.c_int, C.c_double
        L.rewl_last_error.restype = C.c_char_p
        L.rewl_footprint.argtypes = [C.POINTER(Params), C.POINTER(C.c_size_t),
                                     C.POINTER(C.c_size_t)]
        L.rewl_create_ex.argtypes = [C.POINTER(P), C.POINTER(Params), P, C.c_size_t, P]
        L.rewl_create.argtypes = [C.POINTER(P), i32, i32, i32, P, i64, i64, i32, dbl, i32, dbl,
                                  dbl, u64]
        L.rewl_run.argtypes = [P, i64, C.POINTER(i64)]
        L.rewl_step.argtypes = [P, i64]
        L.rewl_get_lng.argtypes = [P, P, i64, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
        L.rewl_get_walker.argtypes = [P, i32, P, P, P, P, P, P, P]
        L.rewl_get_window.argtypes = [P, i32, P, P, P, P, P]
        L.rewl_get_info.argtypes = [P] + [P] * 11
        L.rewl_destroy.argtypes = [P]
        L.rewl_destroy.restype = None
        L.rewl_set_timing.argtypes = [P, i32]
        L.rewl_get_first_merge.argtypes = [P, P, i32]
        L.rewl_jackknife.argtypes = [P, i32, i64, P, P]
        L.rewl_save.argtypes = [P, C.c_char_p]
        L.rewl_load.argtypes = [C.POINTER(P), C.c_char_p, P, C.c_size_t, P]
        L.rewl_partition_balanced.argtypes = [i64, i32, dbl, i32, P, P, P, P, P]
        L.rewl_get_timing.argtypes = [P, C.POINTER(dbl), C.POINTER(i64)]
        L.rewl_batch_create.argtypes = [C.POINTER(P), P, i32, i32, P]
        L.rewl_batch_get_run.argtypes = [P, i32, C.POINTER(P)]
        L.rewl_batch_set_walkers_per_wave.argtypes = [P, i32]
        L.rewl_batch_set_graph.argtypes = [P, i32]
        L.rewl_batch_set_form.argtypes = [P, i32]
        L.rewl_run_noalloc.argtypes = [C.POINTER(Params), i64, P, P, i64, P, P, i64, P]
        L.rewl_batch_step.argtypes = [P, i64]
        L.rewl_batch_run.argtypes = [P, i64, C.POINTER(i64)]
        L.rewl_batch_done.argtypes = [P, P, i32]
        L.rewl_batch_set_timing.argtypes = [P, i32]
        L.rewl_batch_get_timing.argtypes = [P, C.POINTER(dbl), C.POINTER(i64)]
        L.rewl_batch_destroy.argtypes = [P]
        L.rewl_batch_destroy.restype = None
        L.rewl_server_create.argtypes = [C.POINTER(P), C.c_size_t, i32, i32, P]
        L.rewl_server_submit.argtypes = [P, C.POINTER(Params), C.POINTER(i64)]
        L.rewl_server_tick.argtypes = [P, C.POINTER(i32), C.POINTER(i32)]
        L.rewl_server_next_done.argtypes = [P, C.POINTER(i64), C.POINTER(i64)]
        L.rewl_server_result.argtypes = [P, i64, P, i64, C.POINTER(i64), C.POINTER(i64),
                                         C.POINTER(i64)]
        L.rewl_server_release.argtypes = [P, i64]
        L.rewl_server_destroy.argtypes = [P]
        L.rewl_server_destroy.restype = None
        L.rewl_selftest_philox.argtypes = [P, P, P, i32]
        L.rewl_selftest_ln_u.argtypes = [P, P, i32]
        _lib = L
    return _lib


def _check(rc, what):
    if rc < 0:
        raise RewlError(rc, what, lib().rewl_last_error().decode())
    return rc


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def make_params(model, L, q=2, couplings=None, e_min=None, e_max=None, n_windows=4,
                overlap=0.75, walkers_per_window=2, flatness=0.8, lnf_init=1.0,
                lnf_final=1e-6, S=10_000, seed=1, schedule="halving", windows=None):
    """rewl_params for the arguments, and the arrays it points to (keep them
    alive until the library has copied them).  windows: (lo, hi) bin arrays of
    an explicit partition, or None for the equal partition."""
    N = n_sites(model, L)
    nb = 3 if model == "ea3" else 2
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
            raise RewlError(-1, "make_params", "windows must have n_windows entries")
    p = Params(MODELS[model], L, q, None if J is None else J.ctypes.data, int(e_min),
               int(e_max), n_windows, overlap, walkers_per_window, flatness, lnf_init,
               lnf_final, int(S), int(seed), SCHEDULES[schedule],
               None if wl is None else wl.ctypes.data, None if wh is None else wh.ctypes.data)
    return p, (J, wl, wh)


def partition_balanced(n_bins, n_windows, overlap, pre_lo, pre_hi, first_rounds):
    """Run-time balanced windows (rewl_partition_balanced) from a pre-run's
    windows and first-iteration rounds."""
    pl = np.ascontiguousarray(pre_lo, dtype=np.int64)
    ph = np.ascontiguousarray(pre_hi, dtype=np.int64)
    T = np.ascontiguousarray(first_rounds, dtype=np.int64)
    lo = np.zeros(n_windows, dtype=np.int64)
    hi = np.zeros(n_windows, dtype=np.int64)
    _check(lib().rewl_partition_balanced(int(n_bins), n_windows, float(overlap), len(pl), _p(pl),
                                         _p(ph), _p(T), _p(lo), _p(hi)),
           "rewl_partition_balanced")
    return lo, hi


def jackknife(lng_runs):
    """Jackknife mean and error of ln g per bin over independent runs
    (rewl_jackknife); lng_runs: runs x bins."""
    x = np.ascontiguousarray(lng_runs, dtype=np.float64)
    mean = np.empty(x.shape[1])
    err = np.empty(x.shape[1])
    _check(lib().rewl_jackknife(_p(x), x.shape[0], x.shape[1], _p(mean), _p(err)),
           "rewl_jackknife")
    return mean, err


def balanced_windows(chunk=16, max_rounds=1_000_000, **kw):
    """Run-time balanced windows for the run described by kw: a pre-run on the
    equal partition (same parameters and seed) is stepped `chunk` rounds at a
    time until every window has merged once; each window's first iteration
    took first_merge + 1 rounds, which rewl_partition_balanced turns into the
    new windows.  Returns (lo, hi, pre-run rounds stepped)."""
    kw = {k: v for k, v in kw.items() if k != "windows"}
    pre = Run(**kw)
    try:
        issued = 0
        while True:
            f = pre.first_merge()
            if (f >= 0).all():
                break
            if issued >= max_rounds:
                raise RewlError(1, "balanced_windows", "pre-run did not finish its first iteration")
            pre.step(chunk)
            issued += chunk
        wins = pre.windows()
        lo_pre = np.array([w["lo"] for w in wins], dtype=np.int64)
        hi_pre = np.array([w["hi"] for w in wins], dtype=np.int64)
        lo, hi = partition_balanced(pre.n_bins, pre.h, kw.get("overlap", 0.75), lo_pre, hi_pre,
                                    f + 1)
    finally:
        pre.close()
    return lo, hi, issued


def footprint(**kw):
    p, _J = make_params(**kw)
    dev, lds = C.c_size_t(), C.c_size_t()
    _check(lib().rewl_footprint(C.byref(p), C.byref(dev), C.byref(lds)), "rewl_footprint")
    return dev.value, lds.value


class RunView:
    """Readers of one run's state (a run made alone, or run i of a batch)."""

    def _attach(self, h, model, L, params):
        self._h = h
        self.model, self.L, self.N = model, L, n_sites(model, L)
        self.params = params
        info = self.info()
        self.n_bins, self.e_min, self.e_step = info["n_bins"], info["e_min"], info["e_step"]
        self.h, self.m = info["n_windows"], info["m"]

    def info(self):
        v = [C.c_int64(), C.c_int64(), C.c_int64(), C.c_int(), C.c_int(), C.c_int(),
             C.c_int64(), C.c_uint64(), C.c_uint64(), C.c_uint64(), C.c_uint64()]
        _check(lib().rewl_get_info(self._h, *[C.cast(C.byref(x), C.c_void_p) for x in v]),
               "rewl_get_info")
        keys = ["n_bins", "e_min", "e_step", "n_windows", "m", "n_sites", "rounds", "attempts",
                "accepts", "ex_prop", "ex_acc"]
        return {k: x.value for k, x in zip(keys, v)}

    def stats(self):
        i = self.info()
        return {k: i[k] for k in ("attempts", "accepts", "ex_prop", "ex_acc")}

    def window(self, k):
        lo, hi, lnf, done, fin = C.c_int64(), C.c_int64(), C.c_double(), C.c_int(), C.c_int64()
        _check(lib().rewl_get_window(self._h, k, *[C.cast(C.byref(x), C.c_void_p)
                                                   for x in (lo, hi, lnf, done, fin)]),
               "rewl_get_window")
        return {"lo": lo.value, "hi": hi.value, "lnf": lnf.value, "done": bool(done.value),
                "finish_round": fin.value}

    def first_merge(self):
        """Round of each window's first merge (-1 where none yet)."""
        out = np.zeros(self.h, dtype=np.int64)
        _check(lib().rewl_get_first_merge(self._h, _p(out), self.h), "rewl_get_first_merge")
        return out

    def windows(self):
        return [self.window(k) for k in range(self.h)]

    def walker(self, w):
        win = self.window(w // self.m)
        W = win["hi"] - win["lo"] + 1
        spins = np.zeros(self.N, dtype=np.int8)
        lng = np.zeros(W)
        H = np.zeros(W, dtype=np.uint32)
        vis = np.zeros(W, dtype=np.uint8)
        E, t, flat = C.c_int64(), C.c_uint64(), C.c_int()
        _check(lib().rewl_get_walker(self._h, w, _p(spins), C.cast(C.byref(E), C.c_void_p),
                                     C.cast(C.byref(t), C.c_void_p),
                                     C.cast(C.byref(flat), C.c_void_p), _p(lng), _p(H), _p(vis)),
               "rewl_get_walker")
        return {"spins": spins, "E": E.value, "t": t.value, "flat": bool(flat.value),
                "lng": lng, "H": H, "visited": vis}

    def lng(self):
        out = np.zeros(self.n_bins)
        nb, em, es = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().rewl_get_lng(self._h, _p(out), self.n_bins, C.byref(nb), C.byref(em),
                                  C.byref(es)), "rewl_get_lng")
        return out

    def energies(self):
        return self.e_min + self.e_step * np.arange(self.n_bins)


class Run(RunView):
    """One REWL run on the GPU (see rewl_create_ex)."""

    def __init__(self, model, L, q=2, couplings=None, e_min=None, e_max=None, n_windows=4,
                 overlap=0.75, walkers_per_window=2, flatness=0.8, lnf_init=1.0,
                 lnf_final=1e-6, S=10_000, seed=1, schedule="halving", windows=None,
                 stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the REWL library runs on the GPU only")
        p, keep = make_params(model, L, q, couplings, e_min, e_max, n_windows, overlap,
                              walkers_per_window, flatness, lnf_init, lnf_final, S, seed,
                              schedule, windows)
        dev, lds = C.c_size_t(), C.c_size_t()
        _check(lib().rewl_footprint(C.byref(p), C.byref(dev), C.byref(lds)), "rewl_footprint")
        self._buf = torch.empty(dev.value, dtype=torch.uint8, device="cuda")
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().rewl_create_ex(C.byref(h), C.byref(p), C.c_void_p(self._buf.data_ptr()),
                                    dev.value, C.c_void_p(self._stream.cuda_stream)),
               "rewl_create_ex")
        self._attach(h, model, L, dict(model=model, L=L, q=q, n_windows=n_windows,
                                       overlap=overlap, walkers_per_window=walkers_per_window,
                                       flatness=flatness, lnf_init=lnf_init,
                                       lnf_final=lnf_final, S=S, seed=seed,
                                       schedule=schedule))

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().rewl_destroy(h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        try:
            self.close()
        except Exception:
            pass

    def step(self, rounds):
        _check(lib().rewl_step(self._h, int(rounds)), "rewl_step")

    def run(self, max_rounds=-1):
        """Rounds to convergence (or max_rounds); returns (converged, rounds)."""
        r = C.c_int64()
        rc = _check(lib().rewl_run(self._h, int(max_rounds), C.byref(r)), "rewl_run")
        return rc == 0, r.value

    def set_timing(self, on=True):
        _check(lib().rewl_set_timing(self._h, 1 if on else 0), "rewl_set_timing")

    def timing(self):
        """(summed sweep-kernel milliseconds, sweep launches) since set_timing."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().rewl_get_timing(self._h, C.byref(ms), C.byref(n)), "rewl_get_timing")
        return ms.value, n.value

    def save(self, path):
        """Checkpoint the run (rewl_save)."""
        _check(lib().rewl_save(self._h, os.fsencode(path)), "rewl_save")

    @classmethod
    def load(cls, path, stream=None):
        """Resume a run from a checkpoint (rewl_load) into a torch-owned buffer."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the REWL library runs on the GPU only")
        self = cls.__new__(cls)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        # the state's size is known only from the file: the library allocates
        self._buf = None
        h = C.c_void_p()
        _check(lib().rewl_load(C.byref(h), os.fsencode(path), None, 0,
                               C.c_void_p(self._stream.cuda_stream)), "rewl_load")
        # model and L follow the 8-byte tag of the file (int32 each)
        with open(path, "rb") as f:
            head = f.read(16)
        model, L = np.frombuffer(head[8:16], dtype="<i4")
        names = {v: k for k, v in MODELS.items()}
        self._attach(h, names[int(model)], int(L), dict(checkpoint=str(path)))
        return self


FORMS = {"rounds": 0, "persistent": 1}


class Batch:
    """Many independent runs advanced together (see rewl_batch_create).

    runs: list of keyword dicts as for Run (model, L, q, couplings, ...).
    walkers_per_wave: 1, 2, 4 or 8; 0 lets the autotuner (autotune.tune) pick
    walkers per wave, the form and the rounds per graph for this shape of
    batch (the choice is cached per shape; results never depend on it).
    form: "rounds" (kernel launches per round, graph_rounds > 0 replays a
    captured graph of that many rounds) or "persistent" (one work-group per run
    loops the rounds with the run in LDS).
    """

    def __init__(self, runs, walkers_per_wave=1, graph_rounds=0, stream=None, form="rounds"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the REWL library runs on the GPU only")
        self.setting = None
        if walkers_per_wave == 0:
            from .autotune import tune

            self.setting = tune(runs)[0]
            walkers_per_wave = self.setting.walkers_per_wave
            graph_rounds = self.setting.graph_rounds
            form = self.setting.form
        self._keep = []
        arr = (Params * len(runs))()
        for i, kw in enumerate(runs):
            p, J = make_params(**kw)
            self._keep.append(J)
            arr[i] = p
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().rewl_batch_create(C.byref(h), C.cast(arr, C.c_void_p), len(runs),
                                       int(walkers_per_wave), C.c_void_p(self._stream.cuda_stream)),
               "rewl_batch_create")
        self._h = h
        self.n = len(runs)
        self._views = []
        for i, kw in enumerate(runs):
            rh = C.c_void_p()
            _check(lib().rewl_batch_get_run(self._h, i, C.byref(rh)), "rewl_batch_get_run")
            v = RunView()
            v._attach(rh, kw["model"], kw["L"], dict(kw))
            self._views.append(v)
        if graph_rounds:
            self.set_graph(graph_rounds)
        if form != "rounds":
            try:
                self.set_form(form)
            except RewlError:
                self.close()
                raise

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().rewl_batch_destroy(h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        try:
            self.close()
        except Exception:
            pass

    def __getitem__(self, i):
        return self._views[i]

    def __len__(self):
        return self.n

    def set_walkers_per_wave(self, P):
        _check(lib().rewl_batch_set_walkers_per_wave(self._h, int(P)), "set_walkers_per_wave")

    def set_graph(self, rounds):
        _check(lib().rewl_batch_set_graph(self._h, int(rounds)), "rewl_batch_set_graph")

    def set_form(self, form):
        """"rounds" or "persistent" (rewl_batch_set_form)."""
        _check(lib().rewl_batch_set_form(self._h, FORMS[form]), "rewl_batch_set_form")

    def step(self, rounds):
        _check(lib().rewl_batch_step(self._h, int(rounds)), "rewl_batch_step")

    def run(self, max_rounds=-1):
        r = C.c_int64()
        rc = _check(lib().rewl_batch_run(self._h, int(max_rounds), C.byref(r)), "rewl_batch_run")
        return rc == 0, r.value

    def done(self):
        f = np.zeros(self.n, dtype=np.int32)
        _check(lib().rewl_batch_done(self._h, _p(f), self.n), "rewl_batch_done")
        return f.astype(bool)

    def set_timing(self, on=True):
        _check(lib().rewl_batch_set_timing(self._h, 1 if on else 0), "rewl_batch_set_timing")

    def timing(self):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().rewl_batch_get_timing(self._h, C.byref(ms), C.byref(n)), "timing")
        return ms.value, n.value


class Server:
    """Continuous batching of arriving runs (see rewl_server_create).

    walkers_per_wave=0 lets the autotuner pick it from `sample`, a list of run
    keyword dicts shaped like the expected requests (timed as one batch in
    the per-round form the server uses; cached per shape)."""

    def __init__(self, device_budget_bytes=8 << 30, walkers_per_wave=1, rounds_per_tick=8,
                 stream=None, sample=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the REWL library runs on the GPU only")
        self.setting = None
        if walkers_per_wave == 0:
            if not sample:
                raise ValueError("walkers_per_wave=0 needs a sample of requests to tune on")
            from .autotune import tune

            self.setting = tune(sample, forms=("rounds",), graph_options=(0,))[0]
            walkers_per_wave = self.setting.walkers_per_wave
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _check(lib().rewl_server_create(C.byref(h), int(device_budget_bytes),
                                        int(walkers_per_wave), int(rounds_per_tick),
                                        C.c_void_p(self._stream.cuda_stream)),
               "rewl_server_create")
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            lib().rewl_server_destroy(h)
            self._h = None

    def __del__(self):
        # at interpreter exit the module's globals may already be gone
        try:
            self.close()
        except Exception:
            pass

    def submit(self, **kw):
        p, J = make_params(**kw)
        rid = C.c_int64()
        _check(lib().rewl_server_submit(self._h, C.byref(p), C.byref(rid)), "rewl_server_submit")
        return rid.value

    def tick(self):
        """Retire finished runs, admit waiting ones, advance; returns (running, queued)."""
        r, q = C.c_int(), C.c_int()
        _check(lib().rewl_server_tick(self._h, C.byref(r), C.byref(q)), "rewl_server_tick")
        return r.value, q.value

    def next_done(self):
        """(id, rounds) of the next finished run, or None."""
        rid, rounds = C.c_int64(), C.c_int64()
        rc = _check(lib().rewl_server_next_done(self._h, C.byref(rid), C.byref(rounds)),
                    "rewl_server_next_done")
        return None if rc == 1 else (rid.value, rounds.value)

    def result(self, rid):
        nb, em, es = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().rewl_server_result(self._h, int(rid), None, 0, C.byref(nb), C.byref(em),
                                        C.byref(es)), "rewl_server_result")
        out = np.zeros(nb.value)
        _check(lib().rewl_server_result(self._h, int(rid), _p(out), nb.value, C.byref(nb),
                                        C.byref(em), C.byref(es)), "rewl_server_result")
        return out

    def release(self, rid):
        _check(lib().rewl_server_release(self._h, int(rid)), "rewl_server_release")


def run_noalloc(rounds, E, spins, lng, H, stream=None, **kw):
    """rewl_run_noalloc: the run of kw stepped `rounds` rounds into the caller's
    torch tensors E (int32, walkers), spins (int8, walkers x stride), lng
    (float64, walkers x bins) and H (int32, walkers x bins), without any
    allocation by the library (argument marshalling only)."""
    import torch

    p, keep = make_params(**kw)
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().rewl_run_noalloc(C.byref(p), int(rounds), C.c_void_p(E.data_ptr()),
                                  C.c_void_p(spins.data_ptr()), int(spins.shape[1]),
                                  C.c_void_p(lng.data_ptr()), C.c_void_p(H.data_ptr()),
                                  int(lng.shape[1]), C.c_void_p(s.cuda_stream)),
           "rewl_run_noalloc")
    del keep


def selftest_philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    _check(lib().rewl_selftest_philox(_p(c), _p(k), _p(out), c.shape[0]), "selftest_philox")
    return out


def selftest_ln_u(words):
    w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros(w.shape[0])
    _check(lib().rewl_selftest_ln_u(_p(w), _p(out), w.shape[0]), "selftest_ln_u")
    return out
