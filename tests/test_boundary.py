"""The C-ABI library loads on a machine without a GPU, exports every function
include/rewl.h declares, and validates parameters on the host."""
import ctypes as C
import os
import re

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


def test_footprint_grows_with_walkers(rewl):
    a, _ = rewl.footprint(model="potts", L=64, q=10, n_windows=32, walkers_per_window=8)
    b, _ = rewl.footprint(model="potts", L=64, q=10, n_windows=32, walkers_per_window=4)
    assert a > b
