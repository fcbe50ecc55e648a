"""Accuracy of the GPU path against the exact DOS (needs an MI355X).

The GPU path is bit-identical to the oracle (test_gpu_parity.py), so these
runs are the oracle's too; they are only too long to repeat on the CPU here.
"""
import numpy as np
import pytest

from conftest import load_ising_golden
from workloads import run_params

pytestmark = pytest.mark.gpu


def test_ising8_one_over_t_within_002():
    """8x8 Ising, 4 windows x 2 walkers, overlap 0.75, flatness 0.8, halving
    from ln f = 1 and then the 1/t rule down to ln f = 1e-7: the stitched ln g,
    normalised to ln g(-2N) = ln 2, lies within 0.02 of the exact DOS in every
    bin, for 5 seeds run side by side in one batch."""
    import torch

    import paper_1305_5615_amd as rewl

    assert torch.cuda.is_available()
    _, ref = load_ising_golden(8)
    fin = np.isfinite(ref)
    keys = ("model", "L", "q", "e_min", "e_max", "n_windows", "overlap", "walkers_per_window",
            "flatness", "lnf_init", "S", "seed")
    runs = []
    for seed in range(1, 6):
        p = run_params("ising8", seed=seed)
        kw = {k: p[k] for k in keys if k in p}
        kw.update(schedule="1/t", lnf_final=1e-7)
        runs.append(kw)
    print("case: ising8 1/t to 1e-7, seeds 1-5", flush=True)
    b = rewl.Batch(runs, walkers_per_wave=1, graph_rounds=16)
    issued = 0
    while not b.done().all():
        b.step(256)
        issued += 256
        assert issued < 100_000
    errs = []
    for i in range(len(runs)):
        lg = b[i].lng()
        assert lg[0] == np.log(2)
        assert np.array_equal(np.isfinite(lg), fin)
        errs.append(float(np.abs(lg[fin] - ref[fin]).max()))
    b.close()
    print("max |d ln g| per seed:", errs, flush=True)
    assert max(errs) <= 0.02, errs
