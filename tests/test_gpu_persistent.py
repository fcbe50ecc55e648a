"""The persistent form (one work-group per run, the run held in LDS across
rounds) against the CPU oracle, bit for bit (needs an MI355X).

Each case steps a batch in the persistent form and the same runs in the
oracle, then compares every walker's spins, energy, attempt counter, flat
flag, ln g, H and visited set, every window's ln f / done / finishing round and
the counters; converged runs also compare their stitched ln g.
"""
import numpy as np
import pytest

from test_gpu_parity import (MIXED, ONE_OVER_T, WIDE, _kw, _with_couplings,
                             assert_same_state)
from workloads import run_params

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


def _same_lng(g, o, label):
    lg, lo = g.lng(), o.lng()
    fin = np.isfinite(lo)
    assert np.array_equal(np.isfinite(lg), fin), label
    assert np.array_equal(lg[fin].view(np.uint64), lo[fin].view(np.uint64)), label


@pytest.mark.parametrize("P", [2, 4, 8])
def test_persistent_mixed_batch_bitexact(gpu, orc, P):
    """Ising, Potts, +-J and 3D +-J runs of different sizes in one persistent
    launch per step; 1, 6 and 30 rounds per launch."""
    runs = [_with_couplings(kw) for kw in MIXED]
    print("case: persistent mixed batch, walkers per wave", P, flush=True)
    b = gpu.Batch(runs, walkers_per_wave=P, form="persistent")
    oracles = [orc.Run(**kw) for kw in runs]
    for rounds in (1, 6, 30):
        b.step(rounds)
        for o in oracles:
            o.step(rounds)
        for i, o in enumerate(oracles):
            assert_same_state(b[i], o, f"persistent P={P} run {i}")
    b.close()


def test_persistent_mixed_batch_to_convergence(gpu, orc):
    """The mixed runs to convergence in the persistent form (windows finish,
    and whole runs finish, inside launches): same rounds, same stitched ln g."""
    runs = [_with_couplings(kw) for kw in MIXED]
    print("case: persistent mixed batch to convergence", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=4, form="persistent")
    ok, _ = b.run()
    assert ok and b.done().all()
    for i, kw in enumerate(runs):
        o = orc.Run(**kw)
        assert o.run()
        assert_same_state(b[i], o, f"converged run {i}")
        _same_lng(b[i], o, f"run {i}")
    b.close()


def test_persistent_one_over_t_bitexact(gpu, orc):
    """The 1/t cases (halving, switch to W/t, merges every round, done) in one
    persistent batch, checked across the switch and after convergence."""
    runs = [_with_couplings(dict(kw, schedule="1/t")) for _, kw, _ in ONE_OVER_T]
    print("case: persistent 1/t batch", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=2, form="persistent")
    oracles = [orc.Run(**kw) for kw in runs]
    for rounds in (1, 300, 700, 1500):
        b.step(rounds)
        for o in oracles:
            o.step(rounds)
        for i, o in enumerate(oracles):
            assert_same_state(b[i], o, f"1/t run {i}")
    for i, o in enumerate(oracles):
        assert o.info()["done"], i
        _same_lng(b[i], o, f"1/t run {i}")
    b.close()


def test_persistent_wide_windows_bitexact(gpu, orc):
    """Windows of 343 to 676 bins (flatness and merge loops of several strides
    over the work-group) through their merges to convergence."""
    runs = [kw for _, kw, _ in WIDE]
    print("case: persistent wide-window batch", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=2, form="persistent")
    oracles = [orc.Run(**kw) for kw in runs]
    b.step(200)
    for o in oracles:
        o.step(200)
    for i, o in enumerate(oracles):
        assert_same_state(b[i], o, f"wide run {i} after 200")
    ok, _ = b.run()
    assert ok
    for i, o in enumerate(oracles):
        assert o.run()
        assert_same_state(b[i], o, f"wide run {i} converged")
        _same_lng(b[i], o, f"wide run {i}")
    b.close()


def test_persistent_full_glass_workload_samples(gpu, orc):
    """The 256-glass workload (24x24 +-J, 8 windows x 4 walkers each) in the
    persistent form at 8 walkers per wave: 3 rounds in one launch, then 2 more;
    sampled runs against the oracle."""
    runs = [_kw(run_params("ea24", seed=1 + s)) for s in range(256)]
    print("case: 256 x ea24 persistent, P=8", flush=True)
    b = gpu.Batch(runs, walkers_per_wave=8, form="persistent")
    b.step(3)
    b.step(2)
    for i in (0, 77, 255):
        o = orc.Run(**runs[i], n_threads=0)
        o.step(5)
        assert_same_state(b[i], o, f"ea24 run {i} of 256")
    b.close()


def test_persistent_equals_round_launches(gpu):
    """Twenty 8x8 Ising runs (the small Ising workload's shape, seeds 1-20):
    the persistent form and the per-round launches leave identical states."""
    runs = [_kw(run_params("ising8", seed=s)) for s in range(1, 21)]
    print("case: 20 x ising8, persistent vs rounds", flush=True)
    a = gpu.Batch(runs, walkers_per_wave=1, form="persistent")
    c = gpu.Batch(runs, walkers_per_wave=2, graph_rounds=8)
    for rounds in (3, 40, 100):
        a.step(rounds)
        c.step(rounds)
        for i in range(len(runs)):
            for w in range(8):
                x, y = a[i].walker(w), c[i].walker(w)
                assert x["E"] == y["E"] and x["t"] == y["t"] and x["flat"] == y["flat"]
                assert np.array_equal(x["spins"], y["spins"])
                assert np.array_equal(x["H"], y["H"])
                assert np.array_equal(x["lng"].view(np.uint64), y["lng"].view(np.uint64))
            assert a[i].stats() == c[i].stats()
            assert a[i].windows() == c[i].windows()
    a.close()
    c.close()


def test_persistent_refuses_runs_too_large(gpu):
    """A run that needs more than 8 waves (12 walkers at one walker per wave)
    or more than one CU's LDS is refused for the persistent form, and the batch
    keeps working in the per-round form."""
    runs = [_with_couplings(kw) for kw in MIXED]
    b = gpu.Batch(runs, walkers_per_wave=1)
    with pytest.raises(gpu.RewlError) as e:
        b.set_form("persistent")
    assert e.value.code == -1
    b.step(1)
    b.close()
    big = [_kw(run_params("ising32", seed=1))]     # 64 walkers of 1024 spins
    with pytest.raises(gpu.RewlError):
        gpu.Batch(big, walkers_per_wave=8, form="persistent")
