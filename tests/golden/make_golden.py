"""Write the exact 2D Ising densities of states used by the tests.

Calls only oracle.exact (Kaufman's finite-torus partition function, inverted as
Beale did).  Output per L: one line per energy level, "E g(E)" for L <= 16
(exact integers) and "E ln g(E)" with 17 significant digits for larger L.
Usage: python tests/golden/make_golden.py [L ...]   (default: 8 16 32)
"""
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import exact  # noqa: E402


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


if __name__ == "__main__":
    for L in [int(a) for a in sys.argv[1:]] or [8, 16, 32]:
        write(L)
