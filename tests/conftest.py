import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import core
    core.build()
    return core


def load_ising_golden(L):
    """Exact ln g(E) of the L x L Ising torus from tests/golden (-inf where g = 0)."""
    import math

    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", f"ising_exact_L{L}.txt")
    E, lg = [], []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                continue
            e, v = line.split()
            E.append(int(e))
            if L <= 16:
                n = int(v)
                lg.append(math.log(n) if n > 0 else -math.inf)
            else:
                lg.append(float(v))
    return np.array(E), np.array(lg)
