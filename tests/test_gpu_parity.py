"""GPU path against the CPU oracle, element by element (needs an MI355X).

The GPU library and the oracle share no code; they are fed the same seeded
parameters (and the same +-J couplings from workloads.py) and must agree
bit for bit on every walker's spins, energy, attempt counter, flat flag, ln g,
H and visited set, on every window's ln f / done flag / finishing round, and
on the counters, after a fixed number of rounds.  The stitched ln g of a
converged run must agree too.
"""
import numpy as np
import pytest

from workloads import ea3_couplings, ea_couplings, run_params


def _with_couplings(kw):
    kw = dict(kw)
    if kw["model"] == "ea":
        kw["couplings"] = ea_couplings(kw["L"], kw["seed"])
    elif kw["model"] == "ea3":
        kw["couplings"] = ea3_couplings(kw["L"], kw["seed"])
    return kw

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1305_5615_amd as rewl

    rewl.lib()
    return rewl


@pytest.fixture(scope="module")
def orc(oracle_lib):
    return oracle_lib


def _kw(p):
    keys = ("model", "L", "q", "couplings", "e_min", "e_max", "n_windows", "overlap",
            "walkers_per_window", "flatness", "lnf_init", "lnf_final", "S", "seed")
    return {k: p[k] for k in keys if k in p}


def _pair(gpu, orc, **kw):
    print("case:", {k: v for k, v in kw.items() if k != "couplings"}, flush=True)
    return gpu.Run(**kw), orc.Run(**kw)


def assert_same_state(g, o, label=""):
    assert g.n_bins == o.n_bins and g.e_min == o.e_min and g.e_step == o.e_step
    for k in range(o.h):
        wg, wo = g.window(k), o.window(k)
        assert wg == wo, (label, "window", k, wg, wo)
    for w in range(o.h * o.m):
        a, b = g.walker(w), o.walker(w)
        for key in ("E", "t", "flat"):
            assert a[key] == b[key], (label, "walker", w, key, a[key], b[key])
        for key in ("spins", "H", "visited"):
            assert np.array_equal(a[key], b[key]), (label, "walker", w, key)
        # ln g bit for bit
        assert np.array_equal(a["lng"].view(np.uint64), b["lng"].view(np.uint64)), \
            (label, "walker", w, "lng", np.abs(a["lng"] - b["lng"]).max())
    sg, so = g.stats(), o.stats()
    assert sg == so, (label, sg, so)


def test_philox_bitexact(gpu, orc):
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    key = np.array([0x12345678, 0x9ABCDEF0], dtype=np.uint32)
    out = gpu.selftest_philox(ctr, key)
    for i in range(0, 4096, 37):
        assert np.array_equal(out[i], orc.philox(ctr[i], key))


def test_ln_u_bitexact(gpu, orc):
    rng = np.random.default_rng(2)
    words = rng.integers(0, 2 ** 32, size=(20000, 2), dtype=np.uint64).astype(np.uint32)
    words[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0x80000000, 0], [0xB504F333, 0xF9DE6000]]
    got = gpu.selftest_ln_u(words)
    ref = np.array([orc.ln_u(orc.uniform(int(h), int(lo))) for h, lo in words])
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


CASES = [
    # name, parameters (small sizes that still span several 64-attempt blocks,
    # a ragged last block, merges and finished windows)
    ("ising8", dict(model="ising", L=8, n_windows=4, walkers_per_window=2, S=1000,
                    lnf_final=1e-2, seed=3)),
    ("potts12q5", dict(model="potts", L=12, q=5, n_windows=5, walkers_per_window=2, S=777,
                       lnf_final=1e-2, seed=4)),
    ("ea10", dict(model="ea", L=10, n_windows=4, walkers_per_window=4, S=1000, lnf_final=1e-2,
                  seed=5)),
    ("ising5_odd", dict(model="ising", L=5, n_windows=3, walkers_per_window=3, S=65,
                        lnf_final=1e-2, seed=6)),
    ("potts6q2_m1", dict(model="potts", L=6, q=2, n_windows=2, walkers_per_window=1, S=1,
                         lnf_final=0.3, seed=7)),
    ("ising12_range", dict(model="ising", L=12, n_windows=3, walkers_per_window=2, S=500,
                           e_min=-240, e_max=40, lnf_final=1e-2, seed=8)),
    ("ea3_4", dict(model="ea3", L=4, n_windows=3, walkers_per_window=2, S=700, lnf_final=1e-2,
                   seed=13)),
    ("ea3_3_odd", dict(model="ea3", L=3, n_windows=2, walkers_per_window=3, S=130,
                       lnf_final=1e-2, seed=14)),
    # one window: no exchange partner, plain WL with m walkers
    ("ising6_h1", dict(model="ising", L=6, n_windows=1, walkers_per_window=2, S=300,
                       lnf_final=1e-2, seed=15)),
]


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_rounds_bitexact(gpu, orc, name, kw):
    kw = _with_couplings(kw)
    g, o = _pair(gpu, orc, **kw)
    assert_same_state(g, o, "start-up")
    done_rounds = 0
    for rounds in (1, 2, 7, 40, 150):
        g.step(rounds)
        o.step(rounds)
        done_rounds += rounds
        assert_same_state(g, o, f"{name} after {done_rounds} rounds")


ONE_OVER_T = [
    # name, parameters, round increments: the checkpoints fall before, across
    # and after each window's switch from halving to the 1/t rule, and after
    # the windows finish
    ("ising6_1t", dict(model="ising", L=6, n_windows=3, walkers_per_window=2, S=300,
                       flatness=0.6, lnf_final=2e-4, seed=9), (1, 270, 20, 30, 100)),
    ("ea6_1t", dict(model="ea", L=6, n_windows=3, walkers_per_window=3, S=129, flatness=0.6,
                    lnf_final=1e-4, seed=10), (1, 900, 400, 700, 100)),
    ("potts5q3_1t", dict(model="potts", L=5, q=3, n_windows=2, walkers_per_window=2, S=200,
                         flatness=0.6, lnf_final=1e-4, seed=11), (1, 530, 170, 1400)),
]


@pytest.mark.parametrize("name,kw,steps", ONE_OVER_T, ids=[c[0] for c in ONE_OVER_T])
def test_one_over_t_rounds_bitexact(gpu, orc, name, kw, steps):
    kw = _with_couplings(dict(kw, schedule="1/t"))
    g, o = _pair(gpu, orc, **kw)
    done_rounds = 0
    for rounds in steps:
        g.step(rounds)
        o.step(rounds)
        done_rounds += rounds
        assert_same_state(g, o, f"{name} after {done_rounds} rounds")
    assert o.info()["done"]
    lg, lo = g.lng(), o.lng()
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(lg), fin)
    assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64))


WIDE = [
    # windows wider than the 256 threads of the flatness/merge work-group, so
    # its reductions and its merge loop take two or three strides; flatness 0.5
    # and ln f_final 0.1 give four merges per window (flags set, cleared, set
    # again) within a few hundred to a few thousand rounds
    ("ising24_368bins", dict(model="ising", L=24, n_windows=2, walkers_per_window=2, S=5000,
                             e_min=-1100, e_max=1100, overlap=0.5, flatness=0.5, lnf_final=0.1,
                             seed=21), (1, 60, 300)),
    ("potts16q10_343bins", dict(model="potts", L=16, q=10, n_windows=2, walkers_per_window=2,
                                S=5000, overlap=0.5, flatness=0.5, lnf_final=0.1, seed=22),
     (1, 250, 1300)),
    ("ising32_676bins_h1", dict(model="ising", L=32, n_windows=1, walkers_per_window=2, S=5000,
                                e_min=-1300, e_max=1400, flatness=0.5, lnf_final=0.1, seed=23),
     (1, 400, 200)),
]


@pytest.mark.parametrize("name,kw,steps", WIDE, ids=[c[0] for c in WIDE])
def test_wide_windows_bitexact(gpu, orc, name, kw, steps):
    """Windows of 343 to 676 bins through several merges to convergence: every
    walker's state after each checkpoint, then the stitched ln g."""
    g, o = _pair(gpu, orc, **kw)
    widths = [w["hi"] - w["lo"] + 1 for w in o.windows()]
    assert min(widths) > 256, widths
    done_rounds = 0
    for rounds in steps:
        g.step(rounds)
        o.step(rounds)
        done_rounds += rounds
        assert_same_state(g, o, f"{name} after {done_rounds} rounds")
    assert any(f >= 0 for f in o.first_merge()), "no window merged yet"
    ok_g, rounds_g = g.run()
    assert ok_g and o.run()
    assert rounds_g == max(w["finish_round"] for w in o.windows()) + 1
    assert_same_state(g, o, f"{name} converged")
    assert all(w["lnf"] == 0.0625 for w in o.windows())   # four merges: 1 -> 1/16
    lg, lo = g.lng(), o.lng()
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(lg), fin)
    assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64))


@pytest.mark.parametrize("model,L,q", [("ising", 8, 2), ("potts", 6, 4)])
def test_balanced_partition_run_bitexact(gpu, orc, model, L, q):
    """Run-time balanced windows: the pre-run's first-merge rounds agree with
    the oracle's, both derive the same windows, and the run on them is
    bit-exact with the oracle to convergence, stitched ln g included."""
    kw = dict(model=model, L=L, q=q, n_windows=4, walkers_per_window=2, S=1500,
              lnf_final=1e-3, seed=12)
    g, o = _pair(gpu, orc, **kw)
    for _ in range(2000):
        if (o.first_merge() >= 0).all():
            break
        g.step(4)
        o.step(4)
    f = o.first_merge()
    assert (f >= 0).all()
    assert np.array_equal(g.first_merge(), f)
    plo = np.array([w["lo"] for w in o.windows()])
    phi = np.array([w["hi"] for w in o.windows()])
    want = orc.partition_balanced(o.n_bins, 4, 0.75, plo, phi, f + 1)
    got = gpu.partition_balanced(g.n_bins, 4, 0.75, plo, phi, f + 1)
    assert np.array_equal(want[0], got[0]) and np.array_equal(want[1], got[1])
    lo, hi, _ = gpu.balanced_windows(chunk=4, **kw)
    assert np.array_equal(lo, want[0]) and np.array_equal(hi, want[1])
    print("balanced windows:", list(zip(lo, hi)), flush=True)
    gb, ob = _pair(gpu, orc, windows=(lo, hi), **kw)
    assert_same_state(gb, ob, "balanced start-up")
    for rounds in (1, 10, 60):
        gb.step(rounds)
        ob.step(rounds)
        assert_same_state(gb, ob, f"balanced after {rounds}")
    ok_g, _ = gb.run()
    assert ok_g and ob.run()
    assert_same_state(gb, ob, "balanced converged")
    lg, lo_ = gb.lng(), ob.lng()
    fin = np.isfinite(lo_)
    assert np.array_equal(np.isfinite(lg), fin)
    assert np.array_equal(lg[fin].view(np.uint64), lo_[fin].view(np.uint64))


@pytest.mark.parametrize("kw", [
    dict(model="ising", L=8, n_windows=4, walkers_per_window=2, S=1000, lnf_final=1e-3, seed=31),
    dict(model="ea3", L=4, n_windows=3, walkers_per_window=2, S=700, lnf_final=1e-3, seed=32),
    dict(model="potts", L=6, q=3, n_windows=3, walkers_per_window=2, S=500, lnf_final=1e-3,
         seed=33, schedule="1/t"),
], ids=["ising8", "ea3_4", "potts6_1t"])
def test_checkpoint_resume_bitexact(gpu, orc, tmp_path, kw):
    """A run saved after some rounds and loaded again continues exactly as the
    saved run and as the oracle do, through convergence."""
    kw = _with_couplings(kw)
    g, o = _pair(gpu, orc, **kw)
    g.step(7)
    o.step(7)
    path = tmp_path / "run.rewl"
    g.save(path)
    r = gpu.Run.load(path)
    assert_same_state(r, o, "loaded")
    for rounds in (1, 25):
        g.step(rounds)
        r.step(rounds)
        o.step(rounds)
        assert_same_state(r, o, f"resumed +{rounds}")
        assert_same_state(g, o, f"original +{rounds}")
    ok, _ = r.run()
    assert ok and o.run()
    assert_same_state(r, o, "resumed converged")
    lr, lo_ = r.lng(), o.lng()
    fin = np.isfinite(lo_)
    assert np.array_equal(lr[fin].view(np.uint64), lo_[fin].view(np.uint64))
    # a flipped byte is caught by the checksum
    data = bytearray(path.read_bytes())
    data[len(data) // 2] ^= 0x40
    bad = tmp_path / "bad.rewl"
    bad.write_bytes(bytes(data))
    with pytest.raises(gpu.RewlError) as e:
        gpu.Run.load(bad)
    assert e.value.code == -5


def test_largest_lattice_bitexact(gpu, orc):
    """The largest square lattice one walker's window fits in a CU's LDS with
    32 windows (Ising 120x120: 151.8 KB), two rounds against the oracle; one
    size up is refused."""
    kw = dict(model="ising", L=120, n_windows=32, walkers_per_window=1, S=2000, seed=16)
    g = gpu.Run(**kw)
    o = orc.Run(**kw, n_threads=0)
    print("case: ising 120x120, 32 windows x 1", flush=True)
    assert_same_state(g, o, "start-up")
    g.step(2)
    o.step(2)
    assert_same_state(g, o, "2 rounds")
    g.close()
    with pytest.raises(gpu.RewlError):
        gpu.Run("ising", 128, n_windows=32, walkers_per_window=1)


def test_concurrent_use_is_refused(gpu):
    """A second host thread calling into a run while the first is stepping it
    gets REWL_EBUSY; the run is unaffected and usable afterwards.  The first
    thread signals right before it enters a long call (3000 rounds, about 3 s);
    the second polls a read-only call (which changes nothing when it gets in
    first) until it is refused, while the first is still inside."""
    import threading

    r = gpu.Run("ising", 32, n_windows=16, walkers_per_window=4, seed=41)
    r.step(1)
    errors = []
    entering = threading.Event()

    def long_run():
        try:
            entering.set()
            r.run(3000)
        except gpu.RewlError as e:
            errors.append(e)

    th = threading.Thread(target=long_run)
    th.start()
    assert entering.wait(30)
    refused = None
    for _ in range(100_000):
        try:
            r.info()
        except gpu.RewlError as e:
            refused = e
            break
        if not th.is_alive():
            break
    assert refused is not None and refused.code == -6, "no REWL_EBUSY while the run was busy"
    th.join()
    assert not errors
    assert r.info()["rounds"] == 3001
    r.step(1)
    assert r.info()["rounds"] == 3002
    r.close()


def test_ising8_full_run_bitexact(gpu, orc):
    """The small Ising workload run to convergence: same rounds, same stitched ln g."""
    p = run_params("ising8", seed=2)
    g, o = _pair(gpu, orc, **_kw(p))
    ok_g, rounds_g = g.run()
    ok_o = o.run()
    assert ok_g and ok_o
    assert rounds_g == max(w["finish_round"] for w in o.windows()) + 1
    assert_same_state(g, o, "converged")
    lg, lo = g.lng(), o.lng()
    assert np.array_equal(np.isfinite(lg), np.isfinite(lo))
    fin = np.isfinite(lo)
    assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64))


@pytest.mark.parametrize("name,rounds", [("ising32", 3), ("potts64", 1), ("ea24", 2),
                                         ("ea3d12", 2)])
def test_full_size_rounds_bitexact(gpu, orc, name, rounds):
    """The full-size workloads (32x32 Ising 16x4, 64x64 q=10 Potts 32x8, 24x24
    +-J 8x4, 12x12x12 +-J 8x4) for a few rounds of 10^4 attempts per walker,
    in the launch configuration the benchmark times."""
    p = run_params(name, seed=1)
    kw = _kw(p)
    print("case:", name, flush=True)
    g = gpu.Run(**kw)
    o = orc.Run(**kw, n_threads=0)
    assert_same_state(g, o, f"{name} start-up")
    g.step(rounds)
    o.step(rounds)
    assert_same_state(g, o, f"{name} after {rounds} rounds")


def test_zero_rounds_change_nothing(gpu, orc):
    """Stepping or running zero rounds leaves a run as it was."""
    kw = dict(model="ising", L=8, n_windows=4, walkers_per_window=2, S=500, seed=51)
    g, o = _pair(gpu, orc, **kw)
    g.step(3)
    o.step(3)
    g.step(0)
    ok, rounds = g.run(0)
    assert not ok and rounds == 3
    assert_same_state(g, o, "after zero rounds")


def test_invalid_arguments_rejected(gpu):
    with pytest.raises(gpu.RewlError) as e:
        gpu.Run("ising", 2)
    assert e.value.code == -1
    with pytest.raises(gpu.RewlError):
        gpu.Run("potts", 8, q=1)
    with pytest.raises(gpu.RewlError):
        gpu.Run("ising", 8, n_windows=64)
    with pytest.raises(gpu.RewlError):
        gpu.Run("ising", 8, walkers_per_window=65)


# ------------------------------------------------------------------ batches
MIXED = [
    dict(model="ising", L=8, n_windows=4, walkers_per_window=2, S=1000, lnf_final=1e-2, seed=21),
    dict(model="potts", L=10, q=4, n_windows=3, walkers_per_window=4, S=700, lnf_final=1e-2,
         seed=22),
    dict(model="ea", L=8, n_windows=5, walkers_per_window=2, S=1000, lnf_final=1e-2, seed=23),
    dict(model="ising", L=6, n_windows=2, walkers_per_window=1, S=333, lnf_final=1e-2, seed=24),
    dict(model="ea3", L=4, n_windows=3, walkers_per_window=2, S=500, lnf_final=1e-2, seed=25),
]


def _mixed():
    return [_with_couplings(kw) for kw in MIXED]


@pytest.mark.parametrize("P", [1, 2, 4, 8])
def test_batch_runs_match_oracle(gpu, orc, P):
    """Runs of different models and sizes in one batch, P walkers per wave:
    each run equals the same run in the oracle, bit for bit."""
    runs = _mixed()
    print("case: mixed batch, walkers per wave", P, flush=True)
    b = gpu.Batch(runs, walkers_per_wave=P)
    oracles = [orc.Run(**kw) for kw in runs]
    for rounds in (1, 6, 30):
        b.step(rounds)
        for o in oracles:
            o.step(rounds)
        for i, o in enumerate(oracles):
            assert_same_state(b[i], o, f"batch P={P} run {i}")
    b.close()


def test_batch_graph_replays(gpu, orc):
    """Rounds replayed from a captured graph, with eager reads between replays,
    equal the oracle after every replay."""
    runs = _mixed()
    print("case: mixed batch with a 4-round graph", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=2, graph_rounds=4)
    oracles = [orc.Run(**kw) for kw in runs]
    for rounds in (4, 4, 6, 8):
        b.step(rounds)
        for o in oracles:
            o.step(rounds)
        for i, o in enumerate(oracles):
            assert_same_state(b[i], o, f"graph run {i}")
    b.close()


def test_batch_to_convergence(gpu, orc):
    """A batch run to convergence: every run done, stitched ln g identical to
    the oracle's."""
    runs = _mixed()
    print("case: mixed batch to convergence", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=4, graph_rounds=8)
    ok, _ = b.run()
    assert ok and b.done().all()
    for i, kw in enumerate(runs):
        o = orc.Run(**kw)
        assert o.run()
        assert_same_state(b[i], o, f"converged run {i}")
        lg, lo = b[i].lng(), o.lng()
        fin = np.isfinite(lo)
        assert np.array_equal(np.isfinite(lg), fin)
        assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64))
    b.close()


def test_batch_full_size_glasses(gpu, orc):
    """16 +-J 24x24 glasses (8 windows x 4 walkers each), 4 walkers per wave,
    2 rounds of 10^4 attempts: every run equals the oracle."""
    runs = [_kw(run_params("ea24", seed=s)) for s in range(16)]
    print("case: 16 x ea24 batch", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=4)
    b.step(2)
    for i in (0, 7, 15):
        o = orc.Run(**runs[i], n_threads=0)
        o.step(2)
        assert_same_state(b[i], o, f"ea24 run {i}")
    b.close()


def _cus():
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


def test_batch_more_waves_than_cus_one_walker_per_wave(gpu, orc):
    """Eight copies (new seeds) of the mixed runs, one walker per wave: more
    waves than the device has compute units, which selects the sweep form that
    keeps the per-step bin records in registers; every run equals the oracle."""
    runs = []
    for c in range(8):
        for kw in MIXED:
            runs.append(_with_couplings(dict(kw, seed=kw["seed"] + 100 * (c + 1))))
    walkers = sum(kw["n_windows"] * kw["walkers_per_window"] for kw in runs)
    assert walkers > _cus()
    print("case: 8 x mixed batch, P=1,", walkers, "waves", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=1)
    oracles = [orc.Run(**kw) for kw in runs]
    for rounds in (1, 5):
        b.step(rounds)
        for o in oracles:
            o.step(rounds)
        for i, o in enumerate(oracles):
            assert_same_state(b[i], o, f"many-wave batch run {i}")
    b.close()


def test_batch_full_glass_workload_samples(gpu, orc):
    """The 256-glass workload as the benchmark times it (8 walkers per wave,
    1024 waves): 2 rounds, then sampled runs against the oracle."""
    runs = [_kw(run_params("ea24", seed=1 + s)) for s in range(256)]
    assert 256 * 32 // 8 > _cus()
    print("case: 256 x ea24 batch, P=8", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=8)
    b.step(2)
    for i in (0, 101, 255):
        o = orc.Run(**runs[i], n_threads=0)
        o.step(2)
        assert_same_state(b[i], o, f"ea24 run {i} of 256")
    b.close()


# ------------------------------------------------------------------- server
def test_server_results_equal_alone(gpu, orc):
    """Runs submitted while others are on the device, admitted at round
    boundaries under a device budget: each stitched ln g equals the same run
    alone in the oracle, bit for bit."""
    reqs = _mixed() + [
        dict(model="potts", L=6, q=3, n_windows=2, walkers_per_window=2, S=500, lnf_final=3e-2,
             seed=31),
        dict(model="ising", L=10, n_windows=3, walkers_per_window=4, S=900, lnf_final=3e-2,
             seed=32),
    ]
    print("case: server with staggered submissions", flush=True)
    srv = gpu.Server(device_budget_bytes=3 * 1024 * 1024, walkers_per_wave=2, rounds_per_tick=3)
    ids, done = {}, {}
    pending = list(range(len(reqs)))
    ticks = 0
    while len(done) < len(reqs):
        if pending and ticks % 2 == 0:
            i = pending.pop(0)
            ids[srv.submit(**reqs[i])] = i
        srv.tick()
        while True:
            d = srv.next_done()
            if d is None:
                break
            done[d[0]] = d[1]
        ticks += 1
        assert ticks < 5000
    for rid, i in ids.items():
        o = orc.Run(**reqs[i])
        assert o.run()
        assert done[rid] == max(w["finish_round"] for w in o.windows()) + 1
        lg, lo = srv.result(rid), o.lng()
        fin = np.isfinite(lo)
        assert np.array_equal(np.isfinite(lg), fin), i
        assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64)), i
    srv.close()


def test_server_unstartable_request_finishes_alone(gpu, orc):
    """A request no walker can start (a +-J window entirely below the ground
    state) finishes at once with REWL_EINIT, as the oracle refuses it too; the
    runs around it are unaffected and equal the oracle."""
    bad = _with_couplings(dict(model="ea", L=8, e_min=-128, e_max=-100, n_windows=2,
                               walkers_per_window=2, S=1000, lnf_final=1e-2, seed=5))
    with pytest.raises(Exception):
        orc.Run(**bad)
    good = [_with_couplings(kw) for kw in MIXED[:2]]
    print("case: server with one unstartable request", flush=True)
    srv = gpu.Server(device_budget_bytes=64 << 20, walkers_per_wave=1, rounds_per_tick=4)
    ids = [srv.submit(**good[0]), srv.submit(**bad), srv.submit(**good[1])]
    done = {}
    ticks = 0
    while len(done) < 3:
        srv.tick()
        while True:
            d = srv.next_done()
            if d is None:
                break
            done[d[0]] = d[1]
        ticks += 1
        assert ticks < 5000
    assert done[ids[1]] == 0
    with pytest.raises(gpu.RewlError) as e:
        srv.result(ids[1])
    assert e.value.code == -4
    for rid, kw in ((ids[0], good[0]), (ids[2], good[1])):
        o = orc.Run(**kw)
        assert o.run()
        lg, lo = srv.result(rid), o.lng()
        fin = np.isfinite(lo)
        assert np.array_equal(np.isfinite(lg), fin)
        assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64))
    srv.close()
