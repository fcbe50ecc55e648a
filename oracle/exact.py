"""Exact densities of states for small lattices -- TEST INFRASTRUCTURE ONLY.

These are the truth sources the oracle is pinned against (the paper compares its
2D Ising results with exact ones, in the paragraph on the Ising and Potts tests):

* ``brute_dos``: enumeration of every configuration (Ising, q-state Potts and
  +-J models on L x L tori, and the +-J model on L x L x L tori, with at most a
  few tens of millions of states).
* ``ising_dos_transfer``: the 2D Ising DOS on an L x L torus by a row-to-row
  transfer matrix over polynomials in the number of unsatisfied bonds, in exact
  integer arithmetic (independent of the closed form below).
* ``potts_dos_transfer``: the 2D q-state Potts DOS on an L x L torus by a row
  transfer matrix (exact while q^N < 2^53: 5 x 5 at q = 3, 4 x 4 at q = 4).
* ``ea_dos_transfer``: the 2D +-J DOS on an L x L torus for given couplings by
  a row transfer matrix with one matrix per row (exact for L <= 7).
* ``ea3_dos_layers``: the 3D +-J DOS on the 3 x 3 x 3 torus by summing over
  its three layers (independent of enumeration).
* ``ising_dos_exact``: the 2D Ising DOS on an L x L torus (L even) from
  Kaufman's closed-form partition function of the finite torus (B. Kaufman,
  Phys. Rev. 76, 1232 (1949)), turned into the integer coefficients g(E) the way
  P. D. Beale did (Phys. Rev. Lett. 76, 78 (1996)): Z is evaluated at M = N+1
  points on the unit circle of x = exp(-4K) and the polynomial coefficients are
  recovered by an inverse discrete Fourier transform, in high precision.

Energies are E = -sum over bonds; the Ising DOS is returned over
E = -2N, -2N+4, ..., 2N (N+1 entries).
"""
from __future__ import annotations

import numpy as np


def _bonds(L):
    """(site, right neighbour) and (site, lower neighbour) index arrays."""
    idx = np.arange(L * L).reshape(L, L)
    right = np.roll(idx, -1, axis=1).ravel()
    down = np.roll(idx, -1, axis=0).ravel()
    return idx.ravel(), right, down


def _bonds3(L):
    """(site, +x, +y, +z neighbour) index arrays on the L^3 torus, sites
    i = (z L + y) L + x."""
    idx = np.arange(L ** 3).reshape(L, L, L)  # [z, y, x]
    return (idx.ravel(), np.roll(idx, -1, axis=2).ravel(), np.roll(idx, -1, axis=1).ravel(),
            np.roll(idx, -1, axis=0).ravel())


def brute_dos(model, L, q=2, couplings=None):
    """Exact DOS by enumerating all configurations.

    model: 'ising' | 'potts' | 'ea' | 'ea3'.  couplings (ea): int8 array of 2N
    values, [2i] = J(i, right), [2i+1] = J(i, down); (ea3): 3N values,
    [3i + a] = J(i, next site along axis a = x, y, z).  Returns a dict
    {E: count}.
    """
    N = L ** 3 if model == "ea3" else L * L
    nstates = 2 if model in ("ising", "ea", "ea3") else q
    # +-1 models: E is even under flipping every spin, so the last spin is held
    # at +1 and every count doubled
    half = nstates == 2
    total = nstates ** (N - 1) if half else nstates ** N
    if total > 80_000_000:
        raise ValueError("too many states for enumeration")
    site, right, down = _bonds(L)
    if model == "ea":
        J = np.asarray(couplings, dtype=np.int64).reshape(N, 2)
    if model == "ea3":
        site, xp, yp, zp = _bonds3(L)
        J = np.asarray(couplings, dtype=np.int64).reshape(N, 3)
    counts = {}
    chunk = 1 << 20
    for start in range(0, total, chunk):
        codes = np.arange(start, min(total, start + chunk), dtype=np.int64)
        digits = np.empty((codes.size, N), dtype=np.int64)
        c = codes.copy()
        for i in range(N - 1 if half else N):
            digits[:, i] = c % nstates
            c //= nstates
        if half:
            digits[:, N - 1] = 1
        if model == "potts":
            E = -((digits[:, site] == digits[:, right]).sum(1)
                  + (digits[:, site] == digits[:, down]).sum(1))
        else:
            s = 2 * digits - 1
            if model == "ising":
                E = -((s[:, site] * s[:, right]).sum(1) + (s[:, site] * s[:, down]).sum(1))
            elif model == "ea3":
                E = -((J[:, 0] * s[:, site] * s[:, xp]).sum(1)
                      + (J[:, 1] * s[:, site] * s[:, yp]).sum(1)
                      + (J[:, 2] * s[:, site] * s[:, zp]).sum(1))
            else:
                E = -((J[:, 0] * s[:, site] * s[:, right]).sum(1)
                      + (J[:, 1] * s[:, site] * s[:, down]).sum(1))
        vals, cnt = np.unique(E, return_counts=True)
        for v, n in zip(vals.tolist(), cnt.tolist()):
            counts[v] = counts.get(v, 0) + (2 * n if half else n)
    return counts


def ising_dos_transfer(L):
    """Exact 2D Ising DOS on the L x L torus by a row transfer matrix.

    Each row state is an L-bit integer; a polynomial in y counts unsatisfied
    bonds.  Rows are added one by one from a fixed first row, and the periodic
    closure with the first row is added at the end.  Python integers are exact.
    Returns a list over E = -2N, -2N+4, ..., 2N.
    """
    N = L * L
    nrow = 1 << L
    rows = [[1 if (s >> c) & 1 else -1 for c in range(L)] for s in range(nrow)]
    intra = [sum(rows[s][c] != rows[s][(c + 1) % L] for c in range(L)) for s in range(nrow)]
    inter = [[sum(rows[a][c] != rows[b][c] for c in range(L)) for b in range(nrow)]
             for a in range(nrow)]
    D = 2 * N + 1
    total = [0] * D
    for s0 in range(nrow):
        vec = {s0: {intra[s0]: 1}}
        for _ in range(L - 1):
            new = {}
            for a, poly in vec.items():
                for b in range(nrow):
                    add = inter[a][b] + intra[b]
                    tgt = new.setdefault(b, {})
                    for u, n in poly.items():
                        tgt[u + add] = tgt.get(u + add, 0) + n
            vec = new
        for a, poly in vec.items():
            add = inter[a][s0]
            for u, n in poly.items():
                total[u + add] += n
    # E = -2N + 2u; the number u of unsatisfied bonds is even on the torus
    out = []
    for j in range(N + 1):
        out.append(total[2 * j])
    assert all(total[u] == 0 for u in range(1, D, 2))
    return out


def potts_dos_transfer(L, q):
    """Exact 2D q-state Potts DOS on the L x L torus by a row transfer matrix.

    Row states are L-digit base-q integers; the weight counts the bonds whose
    two spins are equal (u of them, E = -u).  Rows are added one by one after
    every fixed first row, and the periodic closure with the first row is added
    at the end.  The counts are integers below 2^53 (checked: q^N < 2^53), so
    the float64 matrix products, whose partial sums are integers no larger than
    the total, are exact.  Returns a dict {E: count}.
    """
    N = L * L
    if q ** N >= 2 ** 53:
        raise ValueError("counts too large for exact float64 sums")
    R = q ** L
    digits = np.array([[(s // q ** c) % q for c in range(L)] for s in range(R)])
    intra = (digits == np.roll(digits, -1, axis=1)).sum(1)          # equal bonds in a row
    inter = (digits[:, None, :] == digits[None, :, :]).sum(2)        # equal bonds between rows
    D = 2 * N + 1                                                     # u = 0 .. 2N
    V = np.zeros((R, D, R))                                           # [first row, u, last row]
    V[np.arange(R), intra, np.arange(R)] = 1.0
    for _ in range(L - 1):
        new = np.zeros_like(V)
        for v in range(L + 1):
            K = (inter == v).astype(np.float64)
            P = (V.reshape(R * D, R) @ K).reshape(R, D, R)
            for h in np.unique(intra):
                cols = intra == h
                sh = v + int(h)
                new[:, sh:, cols] += P[:, :D - sh, cols]
        V = new
    total = np.zeros(D)
    for r0 in range(R):
        for v in range(L + 1):
            cols = inter[:, r0] == v
            total[v:] += V[r0, :D - v, :][:, cols].sum(1)
    out = {-u: int(n) for u, n in enumerate(total) if n}
    assert sum(out.values()) == q ** N
    return out


def _add_shifted(dst, src, shift, cols):
    """dst[:, u + shift, cols] += src[:, u, cols] over every u that stays in range."""
    D = dst.shape[1]
    if shift >= 0:
        dst[:, shift:, cols] += src[:, :D - shift, cols]
    else:
        dst[:, :D + shift, cols] += src[:, -shift:, cols]


def ea_dos_transfer(L, couplings):
    """Exact DOS of the 2D +-J model on the L x L torus by a row transfer matrix.

    couplings: 2N values +-1, [2i] = J(i, right), [2i+1] = J(i, down), site
    i = row * L + column; E = -sum J s s.  Row r's own bonds and its bonds to the
    row above differ from row to row, so each added row has its own matrix; the
    periodic closure with the first row uses the last row's downward bonds.
    Index u = E + 2N stays in [0, 4N] for every partial sum of bonds.  The counts
    are integers below 2^N < 2^53 (L <= 7), so the float64 products are exact.
    Returns a dict {E: count}.
    """
    N = L * L
    if N >= 53:
        raise ValueError("counts too large for exact float64 sums")
    J = np.asarray(couplings, dtype=np.int64).reshape(L, L, 2)      # [row, column, right/down]
    R = 1 << L
    spins = np.array([[1 if (a >> c) & 1 else -1 for c in range(L)] for a in range(R)])
    nxt = np.roll(spins, -1, axis=1)
    # energy of a row's own bonds, per row index: -sum_c J[r, c, right] s_c s_{c+1}
    intra = [-(spins * nxt * J[r, :, 0]).sum(1) for r in range(L)]
    # energy of the bonds from row r (state a) down to the next row (state b)
    def inter(r):
        return -(spins[:, None, :] * spins[None, :, :] * J[r, :, 1]).sum(2)

    D = 4 * N + 1
    V = np.zeros((R, D, R))                                           # [first row, u, last row]
    V[np.arange(R), 2 * N + intra[0], np.arange(R)] = 1.0
    for r in range(1, L):
        X = inter(r - 1)
        new = np.zeros_like(V)
        for v in np.unique(X):
            P = (V.reshape(R * D, R) @ (X == v).astype(np.float64)).reshape(R, D, R)
            for h in np.unique(intra[r]):
                _add_shifted(new, P, int(v + h), intra[r] == h)
        V = new
    X = inter(L - 1)                                                  # last row down to the first
    total = np.zeros(D)
    for r0 in range(R):
        for v in np.unique(X[:, r0]):
            cols = X[:, r0] == v
            part = V[r0][:, cols].sum(1)
            if v >= 0:
                total[v:] += part[:D - v]
            else:
                total[:D + v] += part[-v:]
    out = {u - 2 * N: int(n) for u, n in enumerate(total) if n}
    assert sum(out.values()) == 2 ** N
    return out


def ea3_dos_layers(couplings):
    """Exact DOS of the 3D +-J model on the 3 x 3 x 3 torus by summing over its
    three layers z = 0, 1, 2 (512 states each).

    couplings: 3N values +-1, [3i + a] = J(i, next site along axis a = x, y, z),
    site i = (z L + y) L + x; E = -sum J s s.  E splits into each layer's own
    bonds (x and y), and the z bonds from layer 0 to 1, 1 to 2 and 2 back to 0.
    For every pair (layer 0, layer 2) the middle layer's sum is a polynomial in
    its energy, built from 0/1 matrices grouped by energy value; the ends are
    added last.  Counts are integers below 2^27, exact in float64.  Returns a
    dict {E: count}.
    """
    L = 3
    N = L ** 3
    J = np.asarray(couplings, dtype=np.int64).reshape(L, L, L, 3)   # [z, y, x, axis]
    S = 1 << (L * L)
    lay = np.array([[1 if (a >> j) & 1 else -1 for j in range(L * L)] for a in range(S)])
    lay = lay.reshape(S, L, L)                                         # [state, y, x]
    xn = np.roll(lay, -1, axis=2)
    yn = np.roll(lay, -1, axis=1)
    intra = [-(lay * xn * J[z, :, :, 0] + lay * yn * J[z, :, :, 1]).sum((1, 2))
             for z in range(L)]
    inter = [-(lay[:, None] * lay[None, :] * J[z, :, :, 2]).sum((2, 3)) for z in range(L)]
    M = 2 * L * L + 2 * L * L                                          # bonds in the middle sum
    P = np.zeros((S, S, 2 * M + 1))                                    # [layer 0, layer 2, m + M]
    for h in np.unique(intra[1]):
        cols = intra[1] == h
        for v1 in np.unique(inter[0][:, cols]):
            A = (inter[0][:, cols] == v1).astype(np.float64)
            for v2 in np.unique(inter[1][cols, :]):
                B = (inter[1][cols, :] == v2).astype(np.float64)
                P[:, :, int(h + v1 + v2) + M] += A @ B
    Q = intra[0][:, None] + intra[2][None, :] + inter[2].T             # [layer 0, layer 2]
    total = {}
    for t in np.unique(Q):
        part = P[Q == t].sum(0)
        for m in np.flatnonzero(part):
            e = int(t) + int(m) - M
            total[e] = total.get(e, 0) + int(part[m])
    assert sum(total.values()) == 2 ** N
    return total


def ising_dos_exact(L, extra_digits=40):
    """Exact 2D Ising DOS on the L x L torus (L even) from Kaufman's formula.

    Z(K) = 1/2 (2 sinh 2K)^(N/2) (Z1 + Z2 + Z3 + Z4) with, for L even,
      Z1 = prod_{k odd < L} 2 (T_L(c_k) + 1),  Z2 = prod_{k odd < L} 2 (T_L(c_k) - 1),
      Z3 = 2cosh(L g0/2) 2cosh(L gL/2) prod_{k even, 0<k<L} 2 (T_L(c_k) + 1),
      Z4 = 2sinh(L g0/2) 2sinh(L gL/2) prod_{k even, 0<k<L} 2 (T_L(c_k) - 1),
    where c_k = cosh 2K coth 2K - cos(pi k / L) is cosh(gamma_k), T_L is the
    Chebyshev polynomial (cosh(L gamma) = T_L(cosh gamma)), and the two unpaired
    factors use exp(g0) = exp(2K) tanh K and exp(gL) = exp(2K) / tanh K.  The
    products over k and 2L-k coincide, which is why they appear squared, and
    every factor is then an entire function of K without branch choices.
    P(x) = exp(-2NK) Z is a polynomial of degree N in x = exp(-4K) whose
    coefficient j is g(E = -2N + 4j); it is sampled at x_m = exp(2 pi i (m+1/2)/M),
    M = N + 1, and inverted by a DFT.  Returns a list of Python ints.
    """
    import mpmath as mp

    if L % 2:
        raise ValueError("L must be even")
    N = L * L
    M = N + 1
    with mp.workdps(int(N * 0.30103) + extra_digits):
        cos_k = [mp.cos(mp.pi * k / L) for k in range(L + 1)]

        def cheb(c):
            t0, t1 = mp.mpf(1), c
            for _ in range(L - 1):
                t0, t1 = t1, 2 * c * t1 - t0
            return t1

        values = []
        for m in range(M):
            theta = 2 * mp.pi * (m + mp.mpf(1) / 2) / M
            K = mp.mpc(0, -theta / 4)
            s2 = mp.sinh(2 * K)
            ch2 = mp.cosh(2 * K)
            base = ch2 * ch2 / s2
            t = mp.tanh(K)
            eLK = mp.exp(L * K)
            th = t ** (L // 2)
            e0 = eLK * th          # exp(L g0 / 2)
            eL = eLK / th          # exp(L gL / 2)
            z1 = z2 = mp.mpc(1)
            z3 = (e0 + 1 / e0) * (eL + 1 / eL)
            z4 = (e0 - 1 / e0) * (eL - 1 / eL)
            for k in range(1, L):
                T = cheb(base - cos_k[k])
                if k % 2:
                    z1 *= 2 * (T + 1)
                    z2 *= 2 * (T - 1)
                else:
                    z3 *= 2 * (T + 1)
                    z4 *= 2 * (T - 1)
            Z = (2 * s2) ** (N // 2) * (z1 + z2 + z3 + z4) / 2
            values.append(mp.exp(-2 * N * K) * Z)
        # x_m^-j = exp(-i pi (2m+1) j / M): one table of the 2M-th roots of unity
        roots = [mp.expjpi(-mp.mpf(r) / M) for r in range(2 * M)]
        out = []
        worst = mp.mpf(0)
        for j in range(M):
            acc = mp.mpc(0)
            for m in range(M):
                acc += values[m] * roots[((2 * m + 1) * j) % (2 * M)]
            acc /= M
            n = int(mp.nint(acc.real))
            err = abs(acc - n)
            if err > worst:
                worst = err
            out.append(n)
        if worst > 1e-6:
            raise ArithmeticError(f"DFT residue {worst} too large; raise extra_digits")
    return out


def ln_dos(counts_by_e):
    """{E: count} or list -> (E array, ln g array) over the nonzero entries."""
    import math

    items = sorted(counts_by_e.items())
    E = np.array([e for e, n in items if n > 0], dtype=np.int64)
    lg = np.array([math.log(n) for e, n in items if n > 0])
    return E, lg


def ising_list_to_dict(L, g):
    N = L * L
    return {-2 * N + 4 * j: n for j, n in enumerate(g)}


__all__ = ["brute_dos", "ising_dos_transfer", "ising_dos_exact", "ln_dos",
           "ising_list_to_dict"]
