"""The seeded inputs: couplings are +-1 with p = 1/2, reproducible from their
seed and distinct between seeds; the named workloads carry the stated sizes;
their parameter sets pass the oracle's and the library's host validation."""
import numpy as np
import pytest

import workloads


@pytest.mark.parametrize("fn,L,per_site", [(workloads.ea_couplings, 24, 2),
                                           (workloads.ea3_couplings, 12, 3)])
def test_couplings_are_seeded_pm1(fn, L, per_site):
    N = L ** (3 if per_site == 3 else 2)
    a, b, c = fn(L, 1), fn(L, 1), fn(L, 2)
    assert a.dtype == np.int8 and a.shape == (per_site * N,)
    assert set(np.unique(a)) == {-1, 1}
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    # p = 1/2: the fraction of -1 bonds within 5 standard deviations
    frac = float((a == -1).mean())
    assert abs(frac - 0.5) < 5 * 0.5 / np.sqrt(a.size)


def test_named_workloads():
    c = workloads.CONFIGS
    assert (c["ising32"]["L"], c["ising32"]["n_windows"], c["ising32"]["walkers_per_window"],
            c["ising32"]["lnf_final"], c["ising32"]["S"]) == (32, 16, 4, 1e-8, 10_000)
    assert (c["potts64"]["q"], c["potts64"]["L"], c["potts64"]["n_windows"],
            c["potts64"]["walkers_per_window"]) == (10, 64, 32, 8)
    assert (c["ea24"]["L"], c["ea24"]["n_windows"], c["ea24"]["walkers_per_window"]) == (24, 8, 4)
    assert all(v["overlap"] == 0.75 and v["flatness"] == 0.8 for v in c.values())
    assert workloads.full_range("ising", 32) == (-2048, 2048)
    assert workloads.full_range("potts", 64) == (-8192, 0)
    assert workloads.full_range("ea3", 12) == (-5184, 5184)


@pytest.mark.parametrize("name", sorted(workloads.CONFIGS))
def test_named_workloads_validate(name):
    import bench
    import paper_1305_5615_amd as rewl

    p = workloads.run_params(name, seed=3)
    dev, lds = rewl.footprint(**bench.run_kwargs(p))
    assert dev > 0 and 0 < lds <= 160 * 1024
