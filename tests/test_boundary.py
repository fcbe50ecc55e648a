"""The C-ABI library loads on a machine without a GPU, exports every function
include/rewl.h declares, and validates parameters on the host."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from conftest import ROOT


@pytest.fixture(scope="module")
def rewl():
    import paper_1305_5615_amd as rewl

    if not os.path.exists(rewl.LIB):
        from paper_1305_5615_amd import build

        build.build()
    return rewl


def declared_functions():
    src = open(os.path.join(ROOT, "include", "rewl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rewl_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(rewl):
    names = declared_functions()
    assert "rewl_create" in names and "rewl_run" in names and "rewl_get_lng" in names
    lib = rewl.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_footprint_validates_on_host(rewl):
    dev, lds = rewl.footprint(model="ising", L=32, n_windows=16, walkers_per_window=4)
    assert dev > 64 * 1024 and 0 < lds < 160 * 1024
    for bad in (dict(model="ising", L=2), dict(model="potts", L=8, q=1),
                dict(model="ising", L=8, overlap=1.0), dict(model="ising", L=8, n_windows=64),
                dict(model="ising", L=8, walkers_per_window=0),
                dict(model="ising", L=8, lnf_final=0.0), dict(model="ising", L=8, S=0)):
        with pytest.raises(rewl.RewlError) as e:
            rewl.footprint(**bad)
        assert e.value.code == -1, bad
    with pytest.raises(rewl.RewlError):
        rewl.footprint(model="ea", L=8)             # couplings missing
    # one window spanning a whole 128x128 Ising range does not fit the LDS of a CU
    with pytest.raises(rewl.RewlError):
        rewl.footprint(model="ising", L=128, n_windows=1)


def test_validation_matches_oracle(rewl, oracle_lib):
    """Every parameter set the oracle refuses, the library refuses too (host
    validation, no GPU): empty window sets, degenerate overlaps and flatness,
    non-positive ln f, zero attempts, unknown schedule, bad couplings, sizes
    out of range, inconsistent explicit windows."""
    from workloads import ea3_couplings, ea_couplings

    J = ea_couplings(6, 1)
    bad_J = J.copy()
    bad_J[3] = 2
    lo, hi = oracle_lib.partition(37, 3, 0.75)
    bad_hi = hi.copy()
    bad_hi[0] = lo[1]                  # windows 0 and 1 would share one bin
    cases = [
        dict(model="ising", L=6, n_windows=0),
        dict(model="ising", L=6, overlap=0.0),
        dict(model="ising", L=6, flatness=0.0),
        dict(model="ising", L=6, flatness=1.5),
        dict(model="ising", L=6, lnf_final=-1.0),
        dict(model="ising", L=6, lnf_init=0.0),
        dict(model="ising", L=6, S=0),
        dict(model="ea", L=6, couplings=bad_J),
        dict(model="ea3", L=33, couplings=ea3_couplings(33, 1)),
        dict(model="ea3", L=1, couplings=np.ones(3, np.int8)),
        dict(model="ising", L=6, n_windows=3, windows=(lo, bad_hi)),
        dict(model="ising", L=6, e_min=40, e_max=40),
    ]
    for kw in cases:
        with pytest.raises(oracle_lib.OracleError):
            oracle_lib.Run(**kw)
        with pytest.raises(rewl.RewlError) as e:
            rewl.footprint(**kw)
        assert e.value.code == -1, kw
    # and the same explicit windows, when valid, are accepted by both
    rewl.footprint(model="ising", L=6, n_windows=3, windows=(lo, hi))
    oracle_lib.Run(model="ising", L=6, n_windows=3, windows=(lo, hi))
    with pytest.raises(rewl.RewlError):
        rewl.footprint(model="ising", L=6, schedule="1/t", n_windows=3,
                       windows=(lo[:2], hi[:2]))


def test_footprint_grows_with_walkers(rewl):
    a, _ = rewl.footprint(model="potts", L=64, q=10, n_windows=32, walkers_per_window=8)
    b, _ = rewl.footprint(model="potts", L=64, q=10, n_windows=32, walkers_per_window=4)
    assert a > b


def test_balanced_partition_matches_oracle(oracle_lib):
    """rewl_partition_balanced is host code: on random pre-runs it returns the
    oracle's windows exactly, and refuses the same invalid cases."""
    import paper_1305_5615_amd as rewl

    rng = np.random.default_rng(11)
    agree = 0
    for _ in range(200):
        B = int(rng.integers(20, 4000))
        h = int(rng.integers(1, 40))
        ph = int(rng.integers(1, 40))
        o = float(rng.choice([0.5, 0.6, 0.75, 0.8]))
        try:
            plo, phi = oracle_lib.partition(B, ph, 0.75)
        except ValueError:
            continue
        T = rng.integers(1, 10 ** 6, size=ph)
        try:
            want = oracle_lib.partition_balanced(B, h, o, plo, phi, T)
        except ValueError:
            want = None
        try:
            got = rewl.partition_balanced(B, h, o, plo, phi, T)
        except rewl.RewlError:
            got = None
        assert (want is None) == (got is None), (B, h, ph, o)
        if want is not None:
            assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])
            agree += 1
    assert agree > 100


def test_jackknife_matches_oracle():
    """rewl_jackknife (host code) against the oracle's definition."""
    import paper_1305_5615_amd as rewl
    from oracle.errors import jackknife

    rng = np.random.default_rng(7)
    x = rng.normal(size=(6, 300)) * 0.05 + np.linspace(0, 700, 300)
    x[2, 5] = -np.inf
    m1, e1 = jackknife(x)
    m2, e2 = rewl.jackknife(x)
    fin = np.isfinite(m1)
    assert np.array_equal(fin, np.isfinite(m2)) and np.isnan(e2[5])
    assert np.allclose(m1[fin], m2[fin], rtol=1e-14, atol=0)
    assert np.allclose(e1[fin], e2[fin], rtol=1e-9, atol=1e-13)


def test_load_rejects_non_checkpoints(tmp_path):
    """rewl_load refuses a file that is not a checkpoint before touching the
    GPU (REWL_ECORRUPT), and a missing file with REWL_EINVAL."""
    import ctypes as C

    import paper_1305_5615_amd as rewl

    junk = tmp_path / "junk.rewl"
    junk.write_bytes(b"not a checkpoint at all" * 10)
    h = C.c_void_p()
    assert rewl.lib().rewl_load(C.byref(h), str(junk).encode(), None, 0, None) == -5
    assert rewl.lib().rewl_load(C.byref(h), str(tmp_path / "none").encode(), None, 0, None) == -1
    # a valid tag with a wrong checksum
    junk.write_bytes(b"REWLSAV1" + bytes(64))
    assert rewl.lib().rewl_load(C.byref(h), str(junk).encode(), None, 0, None) == -5


@pytest.mark.parametrize("sizes", ["small", "full"])
def test_served_streams_are_valid(rewl, sizes):
    """The served benchmark's request streams: arrivals increase, all three
    models appear, every request passes host validation and fits a CU's LDS,
    and +-J requests stay within |E| <= 1.5 N (to the integer below for odd N)."""
    import bench
    from workloads import served_stream

    reqs = served_stream(48, 4.0, seed=7, lnf_choices=(1e-3, 1e-4), sizes=sizes)
    arr = [r["arrival"] for r in reqs]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    assert {r["params"]["model"] for r in reqs} == {"ising", "potts", "ea"}
    for r in reqs:
        p = r["params"]
        dev, lds = rewl.footprint(**bench.run_kwargs(p))
        assert dev > 0 and 0 < lds <= 160 * 1024
        if p["model"] == "ea":
            N = p["L"] ** 2
            assert -1.5 * N - 0.5 <= p["e_min"] < p["e_max"] <= 1.5 * N


def test_oracle_refuses_an_unstartable_glass(oracle_lib):
    """A +-J window wholly below any reachable energy (8x8, E <= -100 where
    the ground state is near -90) fails the start-up with REWL_EINIT (-4) in
    the oracle, which the served GPU test relies on."""
    from workloads import ea_couplings

    with pytest.raises(oracle_lib.OracleError) as e:
        oracle_lib.Run(model="ea", L=8, couplings=ea_couplings(8, 5), e_min=-128, e_max=-100,
                       n_windows=2, walkers_per_window=2, S=1000, lnf_final=1e-2, seed=5)
    assert e.value.code == -4


def test_no_cpu_fallback_without_a_gpu(rewl):
    """Without a visible GPU, runs, batches and servers refuse to exist: there
    is no CPU path behind the binding."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    kw = dict(model="ising", L=8, n_windows=2, walkers_per_window=1)
    with pytest.raises(RuntimeError, match="no GPU"):
        rewl.Run(**kw)
    with pytest.raises(RuntimeError, match="no GPU"):
        rewl.Batch([kw], walkers_per_wave=1)
    with pytest.raises(RuntimeError, match="no GPU"):
        rewl.Server(device_budget_bytes=1 << 20)


def test_plain_c_program_uses_the_library(tmp_path):
    """A C11 program (tests/c_abi_probe.c) compiles against include/rewl.h with
    gcc, links librewl.so and runs the host-only entry points without a GPU."""
    import subprocess

    import paper_1305_5615_amd as rewl

    if not os.path.exists(rewl.LIB):
        from paper_1305_5615_amd import build

        build.build()
    exe = tmp_path / "probe"
    libdir = os.path.dirname(rewl.LIB)
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror",
                    "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c_abi_probe.c"), "-o", str(exe),
                    "-L", libdir, "-lrewl", "-Wl,-rpath," + libdir, "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c-abi probe: ok" in r.stdout


def test_missing_library_fails_loudly():
    """Without librewl.so the binding raises at the first call: nothing falls
    back to another implementation."""
    import subprocess
    import sys

    code = ("import paper_1305_5615_amd as r\n"
            "r.LIB = '/nonexistent/librewl.so'\n"
            "try:\n"
            "    r.footprint(model='ising', L=8)\n"
            "except ImportError as e:\n"
            "    print('refused:', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0 and "refused:" in out.stdout, out.stdout + out.stderr


def _fnv1a(data):
    h = 1469598103934665603
    for b in data:
        h ^= b
        h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def _checkpoint_bytes(model, L, q, h, m, lo, hi, couplings, slab, nc=None):
    """A file in the checkpoint format (the fields rewl_save writes, in order)
    with a valid checksum."""
    import struct

    s = b"REWLSAV1" + struct.pack("<6i", model, L, q, h, m, 0)
    N = L * L
    s += struct.pack("<2q4dqQ", -2 * N, 2 * N if model != 1 else 0, 0.75, 0.8, 1.0, 1e-3,
                     1000, 1)
    s += struct.pack("<Q", len(couplings) if nc is None else nc) + bytes(couplings)
    s += struct.pack(f"<{h}q", *lo) + struct.pack(f"<{h}q", *hi)
    s += struct.pack("<Q", len(slab)) + slab
    return s + struct.pack("<Q", _fnv1a(s))


def test_load_refuses_a_made_up_state(tmp_path, rewl, oracle_lib):
    """A file with a valid checksum whose device state does not fit its own
    parameters (windows, energies, spins, couplings), or whose lengths are
    absurd, is refused on the host with REWL_ECORRUPT before any GPU work."""
    import ctypes as C

    lo, hi = oracle_lib.partition(65, 4, 0.75)              # 8x8 Ising, 4 windows
    dev, _ = rewl.footprint(model="ising", L=8, n_windows=4, walkers_per_window=2)
    h = C.c_void_p()
    f = tmp_path / "made_up.rewl"
    # garbage state of the right size
    f.write_bytes(_checkpoint_bytes(0, 8, 2, 4, 2, lo, hi, b"", b"\x7f" * dev))
    assert rewl.lib().rewl_load(C.byref(h), str(f).encode(), None, 0, None) == -5
    assert b"window" in rewl.lib().rewl_last_error()
    # a state of the wrong size
    f.write_bytes(_checkpoint_bytes(0, 8, 2, 4, 2, lo, hi, b"", bytes(dev - 256)))
    assert rewl.lib().rewl_load(C.byref(h), str(f).encode(), None, 0, None) == -5
    # couplings claimed for a model without them, and an absurd couplings length
    f.write_bytes(_checkpoint_bytes(0, 8, 2, 4, 2, lo, hi, b"\x01" * 128, bytes(dev)))
    assert rewl.lib().rewl_load(C.byref(h), str(f).encode(), None, 0, None) == -5
    f.write_bytes(_checkpoint_bytes(0, 8, 2, 4, 2, lo, hi, b"", bytes(dev), nc=(1 << 63)))
    assert rewl.lib().rewl_load(C.byref(h), str(f).encode(), None, 0, None) == -5


def test_load_survives_corrupted_fields(tmp_path, rewl, oracle_lib):
    """Checkpoints with random bytes changed, fields set to extreme values or the
    body cut short, each with its checksum recomputed so the reader gets past it,
    are all refused on the host (REWL_ECORRUPT, or REWL_EINVAL for parameters
    that are not a valid run) with a message, and never crash the reader."""
    lo, hi = oracle_lib.partition(65, 4, 0.75)              # 8x8 Ising, 4 windows
    dev, _ = rewl.footprint(model="ising", L=8, n_windows=4, walkers_per_window=2)
    base = _checkpoint_bytes(0, 8, 2, 4, 2, lo, hi, b"", b"\x7f" * dev)[:-8]
    rng = np.random.default_rng(21)
    extremes = [0, 2 ** 64 - 1, 2 ** 63, 2 ** 63 - 1, 2 ** 31 - 1, 2 ** 31]
    f = tmp_path / "fuzzed.rewl"
    h = C.c_void_p()
    seen = set()
    for it in range(400):
        body = bytearray(base)
        kind = it % 3
        if kind == 0:                      # change 1-4 bytes of the parameters and windows
            for _ in range(int(rng.integers(1, 5))):
                body[int(rng.integers(8, 200))] ^= int(rng.integers(1, 256))
        elif kind == 1:                    # an 8-byte field set to an extreme value
            at = int(rng.integers(8, 190))
            body[at:at + 8] = int(extremes[it % len(extremes)]).to_bytes(8, "little")
        else:                              # the body cut short
            body = body[:int(rng.integers(8, len(body)))]
        f.write_bytes(bytes(body) + int(_fnv1a(body)).to_bytes(8, "little"))
        rc = rewl.lib().rewl_load(C.byref(h), str(f).encode(), None, 0, None)
        assert rc in (-1, -5), (it, rc)
        assert h.value is None
        assert rewl.lib().rewl_last_error()
        seen.add(rc)
    assert seen == {-1, -5}


def test_random_parameters_validate_like_the_oracle(rewl, oracle_lib):
    """Random small runs with up to two fields pushed to edge or invalid values
    (NaN and boundary overlaps and flatness, non-positive ln f, zero attempts,
    too many windows, empty or inverted energy ranges, q and L out of range,
    couplings that are not +-1, unknown schedules): the library's host
    validation refuses exactly the sets the oracle refuses (code -1 on both
    sides).  Small lattices keep every accepted window inside the LDS limit,
    which the oracle does not have; more than 64 walkers per window is the
    library's own limit and refused there alone."""
    from workloads import ea3_couplings, ea_couplings

    rng = np.random.default_rng(31)
    nan = float("nan")
    perturb = {
        "overlap": [nan, 0.0, 1.0, 1e-3, 0.5, 0.999],
        "flatness": [nan, 0.0, 1.0, 1.0001, 0.5],
        "lnf_init": [0.0, -1.0, 1e-12, 2.0],
        "lnf_final": [0.0, -1e-8, 1e-12, 3.0],
        "S": [0, -5, 1, 7],
        "n_windows": [0, -1, 1, 2, 5, 9, 40],
        "walkers_per_window": [0, 1, 3, 64, 65],
        "e_min": [-10 ** 6, -3, 0, 5, 40],
        "e_max": [10 ** 6, 5, 0, -3, -40],
        "schedule": [2, -1],
        "bad_coupling": [0, 2, -2],
        "L": [2, 257, 1],
        "q": [1, 0, 128, 127],
    }
    models = ["ising", "potts", "ea", "ea3"]
    disagree = []
    n_ok = n_bad = 0
    for it in range(300):
        model = models[it % 4]
        L = int(rng.integers(2, 4)) if model == "ea3" else int(rng.integers(3, 9))
        kw = dict(model=model, L=L, n_windows=int(rng.integers(1, 4)),
                  walkers_per_window=int(rng.integers(1, 3)), S=100, seed=int(it))
        if model == "potts":
            kw["q"] = int(rng.integers(2, 6))
        fields = rng.choice(sorted(perturb), size=int(rng.integers(0, 3)), replace=False)
        sched = None
        for f in fields:
            v = perturb[f][int(rng.integers(len(perturb[f])))]
            if f == "schedule":
                sched = v
            elif f != "bad_coupling":
                kw[f] = v
        if kw["L"] < 1 or (model != "ea3" and kw["L"] > 256) or kw["L"] > 64:
            L_cpl = 3
        else:
            L_cpl = kw["L"]
        if model == "ea":
            kw["couplings"] = ea_couplings(L_cpl, it)
        elif model == "ea3":
            kw["couplings"] = ea3_couplings(L_cpl, it)
        if "bad_coupling" in fields and model in ("ea", "ea3"):
            kw["couplings"] = kw["couplings"].copy()
            kw["couplings"][int(rng.integers(kw["couplings"].size))] = perturb["bad_coupling"][it % 3]
        if L_cpl != kw["L"]:
            continue    # couplings of the documented length cannot be made for this L
        p, keep = rewl.make_params(**kw)
        dev, lds = C.c_size_t(), C.c_size_t()
        if sched is not None:
            # an unknown schedule number (the Python bindings only pass known names)
            p.schedule = sched
            assert rewl.lib().rewl_footprint(C.byref(p), C.byref(dev), C.byref(lds)) == -1
            n_bad += 1
            continue
        r = rewl.lib().rewl_footprint(C.byref(p), C.byref(dev), C.byref(lds))
        if kw["walkers_per_window"] > 64:
            # the library's own limit: the exchange step keeps a window pair's
            # partner permutation in 64-entry work-group arrays
            assert r == -1 and b"walkers_per_window" in rewl.lib().rewl_last_error()
            n_bad += 1
            continue
        try:
            oracle_lib.Run(**kw)
            o = 0
        except oracle_lib.OracleError as e:
            o = e.code
        if (o == -1) != (r == -1):
            disagree.append((kw, o, r, rewl.lib().rewl_last_error()))
        if r == 0:
            n_ok += 1
            assert 0 < lds.value <= 160 * 1024
        else:
            n_bad += 1
    assert not disagree, disagree[:3]
    assert n_ok > 50 and n_bad > 50, (n_ok, n_bad)


def test_last_error_is_per_thread(rewl):
    """rewl_last_error describes the calling thread's last failure: two threads
    failing validation for different reasons at the same time (ctypes releases
    the interpreter lock during the calls) each read back their own message."""
    import threading

    cases = {"L": (dict(model="ising", L=2), b"L must"),
             "q": (dict(model="potts", L=8, q=1), b"q must")}
    bad = []
    barrier = threading.Barrier(2)

    def work(name):
        kw, want = cases[name]
        p, keep = rewl.make_params(**kw)
        dev, lds = C.c_size_t(), C.c_size_t()
        barrier.wait()
        for _ in range(20000):
            if rewl.lib().rewl_footprint(C.byref(p), C.byref(dev), C.byref(lds)) != -1 or \
                    want not in rewl.lib().rewl_last_error():
                bad.append(name)
                return

    ts = [threading.Thread(target=work, args=(n,)) for n in cases]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not bad, bad
