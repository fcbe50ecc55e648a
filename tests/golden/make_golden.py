"""Write the exact densities of states used by the tests.

Calls only oracle.exact.  2D Ising: Kaufman's finite-torus partition function,
inverted as Beale did; one line per energy level, "E g(E)" for L <= 16 (exact
integers) and "E ln g(E)" with 17 significant digits for larger L.  3D +-J
glass, 3x3x3, couplings workloads.ea3_couplings(3, 1): enumeration of all 2^27
configurations (a few minutes), "E g(E)".  2D q = 3 Potts, 4x4: enumeration of all
3^16 configurations, "E g(E)".
Usage: python tests/golden/make_golden.py [L ... | ea3 | potts]   (default: 8 16 32)
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402
from workloads import ea3_couplings  # noqa: E402


def write(L):
    g = exact.ising_dos_exact(L)
    N = L * L
    assert sum(g) == 2 ** N
    path = os.path.join(HERE, f"ising_exact_L{L}.txt")
    with open(path, "w") as f:
        f.write(f"# exact 2D Ising DOS, {L}x{L} torus, E = -sum s_i s_j; "
                f"written by tests/golden/make_golden.py from oracle.exact\n")
        if L <= 16:
            f.write("# columns: E g(E)\n")
            for j, n in enumerate(g):
                f.write(f"{-2 * N + 4 * j} {n}\n")
        else:
            f.write("# columns: E ln_g(E) (-inf where g = 0)\n")
            for j, n in enumerate(g):
                v = repr(math.log(n)) if n > 0 else "-inf"
                f.write(f"{-2 * N + 4 * j} {v}\n")
    print("wrote", path)


def write_ea3(L=3, seed=1):
    g = exact.brute_dos("ea3", L, couplings=ea3_couplings(L, seed))
    assert sum(g.values()) == 2 ** (L ** 3)
    path = os.path.join(HERE, f"ea3_L{L}_seed{seed}.txt")
    with open(path, "w") as f:
        f.write(f"# exact DOS of the 3D +-J glass {L}x{L}x{L}, couplings "
                f"workloads.ea3_couplings({L}, {seed}), E = -sum J s_i s_j; written by "
                f"tests/golden/make_golden.py from oracle.exact\n# columns: E g(E)\n")
        for e in sorted(g):
            f.write(f"{e} {g[e]}\n")
    print("wrote", path)


def write_potts(L=4, q=3):
    g = exact.brute_dos("potts", L, q=q)
    assert sum(g.values()) == q ** (L * L)
    path = os.path.join(HERE, f"potts_L{L}_q{q}.txt")
    with open(path, "w") as f:
        f.write(f"# exact DOS of the 2D {q}-state Potts model, {L}x{L} torus, "
                f"E = -sum delta(s_i, s_j); written by tests/golden/make_golden.py from "
                f"oracle.exact\n# columns: E g(E)\n")
        for e in sorted(g):
            f.write(f"{e} {g[e]}\n")
    print("wrote", path)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args == ["ea3"]:
        write_ea3()
    elif args == ["potts"]:
        write_potts()
    else:
        for L in [int(a) for a in args] or [8, 16, 32]:
            write(L)
