"""The allocation-free entry point rewl_run_noalloc against rewl_create_ex +
rewl_step on the same runs, bit for bit (needs an MI355X).

Two calls in a row, the second on a smaller run, so that the second shows
nothing of the first survives in the library's static scratch; then a run too
large for the scratch is refused.
"""
import numpy as np
import pytest

from workloads import ea_couplings

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_1305_5615_amd as rewl

    rewl.lib()
    return rewl


def _noalloc(gpu, rounds, kw):
    """Outputs allocated by the caller (here torch), the call, then a sync."""
    import torch

    ref = gpu.Run(**kw)
    nw = ref.h * ref.m
    W = max(w["hi"] - w["lo"] + 1 for w in ref.windows())
    ref.close()
    stride = (ref.N + 3) // 4 * 4 + 4          # a stride wider than the sites
    dev = torch.device("cuda")
    E = torch.full((nw,), -7, dtype=torch.int32, device=dev)
    spins = torch.full((nw, stride), 5, dtype=torch.int8, device=dev)
    lng = torch.full((nw, W + 3), 123.0, dtype=torch.float64, device=dev)
    H = torch.full((nw, W + 3), 77, dtype=torch.int32, device=dev)
    gpu.run_noalloc(rounds, E, spins, lng, H, **kw)
    torch.cuda.synchronize()
    return E.cpu().numpy(), spins.cpu().numpy(), lng.cpu().numpy(), H.cpu().numpy()


def _check_against_run(gpu, rounds, kw, out):
    E, spins, lng, H = out
    r = gpu.Run(**kw)
    r.step(rounds)
    nw = r.h * r.m
    for w in range(nw):
        st = r.walker(w)
        W = len(st["lng"])
        assert E[w] == st["E"], (w, E[w], st["E"])
        assert np.array_equal(spins[w, : r.N], st["spins"]), w
        assert np.array_equal(lng[w, :W].view(np.uint64), st["lng"].view(np.uint64)), w
        assert np.array_equal(H[w, :W].astype(np.uint32), st["H"]), w
    r.close()


def test_noalloc_equals_create_and_step_twice(gpu):
    first = dict(model="ea", L=12, couplings=ea_couplings(12, 3), n_windows=4,
                 walkers_per_window=4, S=1500, lnf_final=1e-2, seed=3)
    second = dict(model="ising", L=6, n_windows=2, walkers_per_window=2, S=700,
                  lnf_final=1e-2, seed=4)
    print("case: noalloc ea 12x12 4x4, 40 rounds", flush=True)
    out1 = _noalloc(gpu, 40, first)
    _check_against_run(gpu, 40, first, out1)
    print("case: noalloc ising 6x6 2x2 (smaller), 60 rounds", flush=True)
    out2 = _noalloc(gpu, 60, second)
    _check_against_run(gpu, 60, second, out2)


def test_noalloc_potts_through_merges(gpu):
    kw = dict(model="potts", L=10, q=4, n_windows=3, walkers_per_window=2, S=900,
              lnf_final=1e-2, seed=8)
    print("case: noalloc potts 10x10 q=4, 200 rounds", flush=True)
    _check_against_run(gpu, 200, kw, _noalloc(gpu, 200, kw))


def test_noalloc_refuses_what_does_not_fit(gpu):
    import torch

    dev = torch.device("cuda")
    E = torch.zeros(8, dtype=torch.int32, device=dev)
    spins = torch.zeros((8, 256), dtype=torch.int8, device=dev)
    lng = torch.zeros((8, 64), dtype=torch.float64, device=dev)
    H = torch.zeros((8, 64), dtype=torch.int32, device=dev)
    # 64 windows x 64 walkers: the walkers' bookkeeping exceeds the 128 KiB
    # scratch (refused before any output is touched)
    kw = dict(model="ising", L=16, n_windows=64, walkers_per_window=64, S=10, seed=1)
    with pytest.raises(gpu.RewlError) as e:
        gpu.run_noalloc(1, E, spins, lng, H, **kw)
    assert e.value.code == -1 and "128 KiB" in str(e.value)
    # more than 64 windows
    kw = dict(model="ising", L=64, n_windows=65, walkers_per_window=1, S=10, seed=1)
    with pytest.raises(gpu.RewlError) as e:
        gpu.run_noalloc(1, E, spins, lng, H, **kw)
    assert e.value.code == -1
    # an output stride narrower than the lattice
    kw = dict(model="ising", L=16, n_windows=2, walkers_per_window=1, S=10, seed=1)
    with pytest.raises(gpu.RewlError):
        gpu.run_noalloc(1, E, spins[:, :252], lng, H, **kw)
