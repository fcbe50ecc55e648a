"""Pins of the CPU oracle against facts fixed outside it (no GPU needed).

Each test checks a piece of the oracle against the mathematics, an exact
enumeration, an independent library, or an exact density of states, so that a
dropped term, a wrong sign or a swapped index in the oracle fails one of them.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import ROOT, load_ising_golden


# ------------------------------------------------------------------ Philox --
def test_philox_matches_rocrand(oracle_lib, tmp_path):
    """Philox4x32-10 (Salmon et al., SC'11) agrees with rocRAND's implementation.

    rocRAND keeps counter = (offset/4, subsequence) and key = seed, so the oracle's
    block for counter (t_lo, t_hi, walker, stream) is rocRAND's four draws after
    rocrand_init(seed, walker | stream << 32, 4 t)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND probe")
    exe = tmp_path / "anchor"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-o", str(exe),
                    os.path.join(ROOT, "tests", "rocrand_anchor.hip")], check=True)
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(200):
        seed = int(rng.integers(0, 2 ** 63))
        t = int(rng.integers(0, 2 ** 40))
        walker = int(rng.integers(0, 2 ** 32))
        stream = int(rng.integers(0, 8))
        cases.append((seed, t, walker, stream))
    cases += [(0, 0, 0, 0), (2 ** 64 - 1, 2 ** 62 - 1, 2 ** 32 - 1, 3)]
    inp = "\n".join(f"{s} {w | (st << 32)} {4 * t}" for s, t, w, st in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    for (seed, t, w, st), ref in zip(cases, got):
        ours = oracle_lib.philox([t & 0xFFFFFFFF, t >> 32, w, st],
                                 [seed & 0xFFFFFFFF, seed >> 32])
        assert list(map(int, ours)) == ref, (seed, t, w, st)


def test_philox_counter_sensitivity(oracle_lib):
    base = oracle_lib.philox([1, 2, 3, 4], [5, 6])
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(oracle_lib.philox(c, [5, 6]), base)


# ------------------------------------------------------------- uniform, ln --
def test_uniform_range(oracle_lib):
    assert oracle_lib.uniform(0, 0) == 2.0 ** -53
    assert oracle_lib.uniform(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle_lib.uniform(0x80000000, 0) == 0.5 + 2.0 ** -53
    # the low 12 bits of the second word are unused
    assert oracle_lib.uniform(123, 0xFFF) == oracle_lib.uniform(123, 0)


def _ulp(x):
    return math.ulp(x)


def test_ln_u_accuracy(oracle_lib):
    """ln u within 2 ulp of the exact logarithm (mpmath, 40 digits) over (0,1)."""
    import mpmath as mp

    rng = np.random.default_rng(11)
    hi = rng.integers(0, 2 ** 32, size=4000, dtype=np.uint64)
    lo = rng.integers(0, 2 ** 32, size=4000, dtype=np.uint64)
    us = [oracle_lib.uniform(int(a), int(b)) for a, b in zip(hi, lo)]
    us += [0.5 + 2.0 ** -53, 1 - 2.0 ** -53, 2.0 ** -53, 1 / math.sqrt(2),
           math.sqrt(2) / 2 + 1e-16, 0.75, 0.25, 1e-10, 0.999999]
    us += list(np.exp(-rng.uniform(0, 36, 2000)))
    worst = 0.0
    with mp.workdps(40):
        for u in us:
            ref = mp.log(mp.mpf(u))
            got = oracle_lib.ln_u(u)
            err = abs(mp.mpf(got) - ref) / _ulp(float(ref))
            worst = max(worst, float(err))
            assert got < 0.0
    assert worst <= 2.0, worst


def test_ln_u_monotone(oracle_lib):
    xs = np.sort(np.random.default_rng(3).uniform(1e-12, 1 - 1e-12, 3000))
    ys = [oracle_lib.ln_u(float(x)) for x in xs]
    assert all(a <= b for a, b in zip(ys, ys[1:]))


def test_ln2_split_constants():
    """The two halves of ln 2 used by ln u: 32 fractional bits, then the rest."""
    import mpmath as mp

    src = open(os.path.join(ROOT, "oracle", "rewl_oracle.c")).read()
    hi = float.fromhex(src.split("LN2_HI = ")[1].split(";")[0])
    lo = float.fromhex(src.split("LN2_LO = ")[1].split(";")[0])
    with mp.workdps(50):
        ln2 = mp.log(2)
        assert hi == float(mp.nint(ln2 * 2 ** 32) / 2 ** 32)
        assert lo == float(ln2 - mp.mpf(hi))


# ------------------------------------------------------------------ models --
def test_energy_reference_states(oracle_lib):
    L = 6
    N = L * L
    up = np.ones(N, dtype=np.int8)
    chk = np.array([1 if (i // L + i % L) % 2 == 0 else -1 for i in range(N)], dtype=np.int8)
    assert oracle_lib.energy("ising", L, up) == -2 * N
    assert oracle_lib.energy("ising", L, chk) == 2 * N
    assert oracle_lib.energy("potts", L, np.zeros(N, np.int8), q=3) == -2 * N
    stripes = np.array([i % 3 for i in range(N)], dtype=np.int8)  # rows alike, columns differ
    assert oracle_lib.energy("potts", L, stripes, q=3) == -N
    J = -np.ones(2 * N, dtype=np.int8)
    assert oracle_lib.energy("ea", L, up, J) == 2 * N
    # one flipped spin in the ferromagnet costs 8
    one = up.copy()
    one[7] = -1
    assert oracle_lib.energy("ising", L, one) == -2 * N + 8


def test_energy_matches_brute_force_definition(oracle_lib):
    """orc_energy against an independent numpy bond sum on random states."""
    from workloads import ea_couplings

    rng = np.random.default_rng(2)
    for L in (3, 4, 7):
        N = L * L
        idx = np.arange(N).reshape(L, L)
        rt = np.roll(idx, -1, 1).ravel()
        dn = np.roll(idx, -1, 0).ravel()
        J = ea_couplings(L, L).astype(np.int64).reshape(N, 2)
        for _ in range(20):
            s = rng.choice([-1, 1], N).astype(np.int8)
            si = s.astype(np.int64)
            assert oracle_lib.energy("ising", L, s) == -(si * si[rt] + si * si[dn]).sum()
            assert oracle_lib.energy("ea", L, s, J.ravel().astype(np.int8)) == \
                -(J[:, 0] * si * si[rt] + J[:, 1] * si * si[dn]).sum()
            p = rng.integers(0, 5, N).astype(np.int8)
            assert oracle_lib.energy("potts", L, p, q=5) == -((p == p[rt]).sum() + (p == p[dn]).sum())


@pytest.mark.parametrize("model,q,L", [("ising", 2, 6), ("potts", 4, 6), ("ea", 2, 6),
                                       ("ea3", 2, 4), ("ea3", 2, 3)])
def test_walker_energy_tracks_spins(oracle_lib, model, q, L):
    """After rounds of sweeps and exchanges every walker's E equals E(spins)."""
    from workloads import ea3_couplings, ea_couplings

    J = {"ea": lambda: ea_couplings(L, 3), "ea3": lambda: ea3_couplings(L, 3)}.get(
        model, lambda: None)()
    run = oracle_lib.Run(model, L, q=q, couplings=J, n_windows=3, walkers_per_window=2,
                         S=500, seed=9)
    for _ in range(5):
        run.step(3)
        for w in range(run.h * run.m):
            st = run.walker(w)
            assert st["E"] == oracle_lib.energy(model, L, st["spins"], J, q=q)
            win = run.window(w // run.m)
            b = (st["E"] - run.e_min) // run.e_step
            assert win["lo"] <= b <= win["hi"]
            if model == "potts":
                assert st["spins"].min() >= 0 and st["spins"].max() < q
            else:
                assert set(np.unique(st["spins"])) <= {-1, 1}


# --------------------------------------------------------------- partition --
def test_partition_examples(oracle_lib):
    lo, hi = oracle_lib.partition(65, 4, 0.75)          # 8x8 Ising
    assert list(zip(lo, hi)) == [(0, 37), (9, 46), (18, 55), (27, 64)]
    lo, hi = oracle_lib.partition(1025, 16, 0.75)       # 32x32 Ising
    assert (hi - lo + 1).max() == 218 and lo[0] == 0 and hi[-1] == 1024
    assert (hi[:-1] - lo[1:] + 1).min() >= 163
    lo, hi = oracle_lib.partition(8193, 32, 0.75)       # 64x64 Potts
    assert (hi - lo + 1).max() == 939


def test_partition_invariants(oracle_lib):
    for B in (20, 65, 257, 1025, 4097):
        for h in (1, 2, 3, 5, 8, 16):
            for o in (0.5, 0.75, 0.9):
                try:
                    lo, hi = oracle_lib.partition(B, h, o)
                except ValueError:
                    continue
                assert lo[0] == 0 and hi[-1] == B - 1
                assert np.all(np.diff(lo) > 0) and np.all(np.diff(hi) >= 0)
                assert np.all(hi[:-1] >= lo[1:] + 1)         # overlap of at least 2 bins
                covered = np.zeros(B, bool)
                for a, b in zip(lo, hi):
                    covered[a:b + 1] = True
                assert covered.all()


# ---------------------------------------------------------- exact DOS tools --
def test_balanced_partition_uniform_is_equal(oracle_lib):
    """With first-iteration time proportional to window width (a uniform time
    density) the run-time balanced partition is the equal partition, exactly."""
    for B, h, o in [(65, 4, 0.75), (1025, 16, 0.75), (8193, 32, 0.75), (577, 8, 0.6),
                    (300, 7, 0.5)]:
        lo, hi = oracle_lib.partition(B, h, o)
        lo2, hi2 = oracle_lib.partition_balanced(B, h, o, lo, hi, hi - lo + 1)
        assert np.array_equal(lo, lo2) and np.array_equal(hi, hi2), (B, h, o)


def test_balanced_partition_equalises_time(oracle_lib):
    """A pre-run whose low windows took 9x longer per bin: the balanced windows
    are narrower there, and every window holds the same first-iteration time
    up to the density of one bin at each end."""
    B, h, o = 1025, 16, 0.75
    plo, phi = oracle_lib.partition(B, h, o)
    T = np.where(np.arange(h) < h // 2, 9, 1) * (phi - plo + 1)
    lo, hi = oracle_lib.partition_balanced(B, h, o, plo, phi, T)
    assert lo[0] == 0 and hi[-1] == B - 1
    assert np.all(np.diff(lo) > 0) and np.all(np.diff(hi) > 0)
    # the time density the partition sees, rebuilt from its definition
    t = np.zeros(B)
    for b in range(B):
        ks = [k for k in range(h) if plo[k] <= b <= phi[k]]
        t[b] = np.mean([T[k] / (phi[k] - plo[k] + 1) for k in ks])
    F = np.concatenate([[0.0], np.cumsum((t[:-1] + t[1:]) / 2)])
    w = F[-1] / (1 + (h - 1) * (1 - o))
    spans = F[hi] - F[lo]
    assert np.all(np.abs(spans[:-1] - w) <= 2 * t.max() + 1e-9), (spans, w)
    widths = hi - lo + 1
    assert widths[-1] > 3 * widths[0] and widths[-2] > 2 * widths[0]


def test_first_merge_round(oracle_lib):
    """The round of each window's first merge is the round in which its ln f
    first dropped below ln f_init."""
    run = oracle_lib.Run("ising", 6, n_windows=3, walkers_per_window=2, S=500, seed=3,
                         lnf_final=0.1)
    seen = [-1] * 3
    for r in range(2000):
        run.step(1)
        for k in range(3):
            if seen[k] < 0 and run.window(k)["lnf"] < 1.0:
                seen[k] = r
        if min(seen) >= 0:
            break
    assert list(run.first_merge()) == seen


def test_explicit_windows_match_equal_partition(oracle_lib):
    """A run given the equal partition explicitly evolves exactly as the
    default run; an invalid explicit partition is refused."""
    lo, hi = oracle_lib.partition(65, 4, 0.75)
    a = oracle_lib.Run("ising", 8, n_windows=4, walkers_per_window=2, S=700, seed=5)
    b = oracle_lib.Run("ising", 8, n_windows=4, walkers_per_window=2, S=700, seed=5,
                       windows=(lo, hi))
    a.step(20)
    b.step(20)
    for w in range(8):
        x, y = a.walker(w), b.walker(w)
        assert np.array_equal(x["lng"], y["lng"]) and np.array_equal(x["spins"], y["spins"])
    bad_hi = hi.copy()
    bad_hi[1] = lo[2]          # windows 1 and 2 would share one bin
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ising", 8, n_windows=4, windows=(lo, bad_hi))


def test_jackknife_identities():
    """The jackknife error of a mean is the standard error of the mean,
    s / sqrt(R) with the unbiased s (an identity); two runs give |a - b| / 2;
    equal runs give 0; a bin some run never visited gives -inf and NaN."""
    from oracle.errors import jackknife

    rng = np.random.default_rng(5)
    x = rng.normal(size=(9, 40)) * 3 + 100
    mean, err = jackknife(x)
    assert np.allclose(mean, x.mean(0), rtol=0, atol=1e-12)
    assert np.allclose(err, x.std(0, ddof=1) / 3.0, rtol=1e-12, atol=0)
    two = np.array([[1.0, 5.0], [4.0, 5.0]])
    m2, e2 = jackknife(two)
    assert np.allclose(e2, [1.5, 0.0], atol=1e-15)
    x[3, 7] = -np.inf
    m3, e3 = jackknife(x)
    assert m3[7] == -np.inf and np.isnan(e3[7]) and np.isfinite(e3[8])


def test_exact_ising_three_ways():
    """Kaufman's closed form = transfer matrix = enumeration (L = 4); L = 6 = transfer."""
    from oracle import exact

    g4 = exact.ising_dos_exact(4)
    brute = exact.brute_dos("ising", 4)
    assert g4 == [brute.get(-32 + 4 * j, 0) for j in range(17)]
    assert g4 == exact.ising_dos_transfer(4)
    assert exact.ising_dos_exact(6) == exact.ising_dos_transfer(6)


@pytest.mark.parametrize("L", [8, 16])
def test_exact_ising_golden_sum_rules(L):
    """Golden tables: sum 2^N, g(E) = g(-E), and the low-energy counts 2, 0, 2N, 4N."""
    path = os.path.join(ROOT, "tests", "golden", f"ising_exact_L{L}.txt")
    g = [int(line.split()[1]) for line in open(path) if not line.startswith("#")]
    N = L * L
    assert sum(g) == 2 ** N
    assert g == g[::-1]
    assert g[0] == 2 and g[1] == 0 and g[2] == 2 * N and g[3] == 4 * N


def test_exact_ising_golden_L8_regenerates():
    from oracle import exact

    path = os.path.join(ROOT, "tests", "golden", "ising_exact_L8.txt")
    g = [int(line.split()[1]) for line in open(path) if not line.startswith("#")]
    assert g == exact.ising_dos_exact(8)


def test_exact_ising_golden_L32_shape():
    E, lg = load_ising_golden(32)
    N = 1024
    assert len(E) == N + 1 and E[0] == -2 * N
    assert abs(lg[0] - math.log(2)) < 1e-15 and lg[1] == -math.inf
    assert abs(lg[2] - math.log(2 * N)) < 1e-12 and abs(lg[3] - math.log(4 * N)) < 1e-12
    fin = np.isfinite(lg)
    rev = lg[::-1]
    assert np.array_equal(np.isfinite(rev), fin)
    assert np.allclose(lg[fin], rev[fin], atol=1e-12)
    # sum g = 2^N
    mx = lg[fin].max()
    assert abs(mx + math.log(np.exp(lg[fin] - mx).sum()) - N * math.log(2)) < 1e-9


def test_brute_force_potts_q2_is_ising():
    """delta(s,s') = (1 + s s')/2 gives E_Potts = -N + E_Ising / 2 at q = 2."""
    from oracle import exact

    ising = exact.brute_dos("ising", 4)
    potts = exact.brute_dos("potts", 4, q=2)
    assert potts == {-16 + e // 2: n for e, n in ising.items()}


def test_brute_force_potts_counts():
    from oracle import exact

    L, q = 3, 3
    N = L * L
    g = exact.brute_dos("potts", L, q=q)
    assert sum(g.values()) == q ** N
    assert g[-2 * N] == q
    assert all(g.get(-2 * N + d, 0) == 0 for d in (1, 2, 3))
    assert g[-2 * N + 4] == q * N * (q - 1)


def _potts_golden(L, q):
    rows = [line.split() for line in open(os.path.join(ROOT, "tests", "golden",
                                                       f"potts_L{L}_q{q}.txt"))
            if not line.startswith("#")]
    return {int(e): int(n) for e, n in rows}


_POTTS_EXACT = {}


def _potts_exact(L, q):
    """The stored enumeration for 4x4 q = 3, else the transfer matrix (cached)."""
    if (L, q) == (4, 3):
        return _potts_golden(4, 3)
    if (L, q) not in _POTTS_EXACT:
        from oracle import exact

        _POTTS_EXACT[(L, q)] = exact.potts_dos_transfer(L, q)
    return _POTTS_EXACT[(L, q)]


def test_potts_transfer_matrix_agrees_with_enumeration():
    """Two independent exact methods for the Potts DOS agree: the row transfer
    matrix equals enumeration (3x3 at q = 3 and 4, the stored 4x4 q = 3 table of
    all 3^16 configurations), and at q = 2 it equals Kaufman's Ising DOS through
    E_P = -N + E_I / 2 (4x4, 6x6)."""
    from oracle import exact

    for q in (3, 4):
        assert exact.potts_dos_transfer(3, q) == exact.brute_dos("potts", 3, q=q)
    assert exact.potts_dos_transfer(4, 3) == _potts_golden(4, 3)
    for L in (4, 6):
        N = L * L
        ising = exact.ising_dos_exact(L)
        want = {-N + (-2 * N + 4 * j) // 2: n for j, n in enumerate(ising) if n}
        assert exact.potts_dos_transfer(L, 2) == want


@pytest.mark.parametrize("L,q", [(4, 3), (5, 3), (4, 4), (3, 10)])
def test_potts_low_levels_closed_form(L, q):
    """Sum rule and the lowest levels, counted by hand on the torus: the q ordered
    states; one site of another state breaks 4 bonds (qN(q-1) states); a
    two-site domino breaks 6 when both sites share a new state (2N q(q-1)) and
    7 when they differ from each other too (2N q(q-1)(q-2)); 1, 2, 3 and 5
    broken bonds are impossible.  On the 3x3 torus a whole row or column of
    one new state also breaks just 6 bonds (2L q(q-1) more)."""
    N = L * L
    g = _potts_exact(L, q)
    assert sum(g.values()) == q ** N
    lo = -2 * N
    assert g[lo] == q
    assert all(lo + d not in g for d in (1, 2, 3, 5))
    assert g[lo + 4] == q * N * (q - 1)
    lines = 2 * L * q * (q - 1) if L == 3 else 0
    assert g[lo + 6] == 2 * N * q * (q - 1) + lines
    assert g[lo + 7] == 2 * N * q * (q - 1) * (q - 2)


def test_potts_converges_to_exact(oracle_lib):
    """REWL on Potts lattices beyond enumeration's reach for a test, against the
    exact DOS: 4x4 q = 3 under halving to ln f = 1e-6 (measured 0.075, 0.061 for
    seeds 1, 2); 5x5 q = 3 and 4x4 q = 4 under the 1/t rule to 1e-5 (measured
    0.037-0.067 over seeds 1-3); 3x3 at the workload's q = 10 (halving 0.086,
    1/t 0.045).  Every exactly reachable level is visited, and no other."""
    cases = [(4, 3, 3, "halving", 1e-6, 1, 0.2), (4, 3, 3, "halving", 1e-6, 2, 0.2),
             (5, 3, 4, "1/t", 1e-5, 1, 0.1), (4, 4, 3, "1/t", 1e-5, 2, 0.1),
             (3, 10, 2, "halving", 1e-6, 1, 0.2), (3, 10, 2, "1/t", 1e-5, 2, 0.1)]
    for L, q, h, sched, lf, seed, tol in cases:
        g = _potts_exact(L, q)
        run = oracle_lib.Run("potts", L, q=q, n_windows=h, walkers_per_window=2, lnf_final=lf,
                             S=5_000, seed=seed, schedule=sched, n_threads=4)
        assert run.run()
        ref = np.array([math.log(g[e]) if e in g else -np.inf for e in run.energies()])
        lng = run.lng()
        assert np.array_equal(np.isfinite(lng), np.isfinite(ref)), (L, q, seed)
        assert _max_err(lng, ref) < tol, (L, q, sched, seed, _max_err(lng, ref))


def test_ea_transfer_matrix_agrees_with_enumeration():
    """The +-J transfer matrix (one matrix per row, since the couplings change
    from row to row) equals enumeration on 3x3 and 4x4 instances, and with every
    coupling +1 equals Kaufman's Ising DOS (4x4, 6x6)."""
    from oracle import exact
    from workloads import ea_couplings

    for L in (3, 4):
        for seed in (1, 2, 3):
            J = ea_couplings(L, seed)
            assert exact.ea_dos_transfer(L, J) == exact.brute_dos("ea", L, couplings=J)
    for L in (4, 6):
        N = L * L
        ising = exact.ising_dos_exact(L)
        assert exact.ea_dos_transfer(L, np.ones(2 * N, np.int8)) == \
            {-2 * N + 4 * j: n for j, n in enumerate(ising) if n}


@pytest.mark.parametrize("L", [5, 6])
def test_ea_converges_to_exact(oracle_lib, L):
    """REWL on +-J instances beyond the enumerated 4x4 against the transfer-matrix
    DOS (5x5: odd, no E -> -E symmetry; 6x6: symmetric), range |E| <= 1.5 N, so
    the lowest visited level is the reference (ln g = 0 there).  Measured max
    errors, halving to ln f = 1e-6: 0.17, 0.09 (5x5), 0.12, 0.25 (6x6)."""
    from oracle import exact
    from workloads import ea_couplings

    N = L * L
    J = ea_couplings(L, 1)
    g = exact.ea_dos_transfer(L, J)
    assert sum(g.values()) == 2 ** N
    n_neg = int((J < 0).sum())
    assert all((e + 2 * N - 2 * n_neg) % 4 == 0 for e in g)
    if L % 2 == 0:
        assert all(g.get(-e) == n for e, n in g.items())
    for seed in (1, 2):
        run = oracle_lib.Run("ea", L, couplings=J, e_min=-(3 * N) // 2, e_max=(3 * N) // 2,
                             n_windows=4, walkers_per_window=2, lnf_final=1e-6, S=5_000,
                             seed=seed, n_threads=4)
        assert run.run()
        ref = np.array([math.log(g[e]) if e in g else -np.inf for e in run.energies()])
        ref = ref - ref[np.isfinite(ref)][0]
        assert _max_err(run.lng(), ref) < 0.35, (L, seed, _max_err(run.lng(), ref))


def test_brute_force_ea_symmetry():
    """On an even torus g(E) = g(-E) for any +-J couplings (flip one sublattice)."""
    from oracle import exact
    from workloads import ea_couplings

    J = ea_couplings(4, 1)
    g = exact.brute_dos("ea", 4, couplings=J)
    assert sum(g.values()) == 2 ** 16
    assert all(g[e] == g.get(-e, 0) for e in g)
    n_neg = int((J < 0).sum())
    assert all((e - (-32 + 2 * n_neg)) % 4 == 0 for e in g)


# --------------------------------------------------------------- stitching --
def test_stitch_recovers_exact_pieces(oracle_lib):
    """Exact ln g pieces with arbitrary offsets are joined back to ln g + const."""
    E, lg = load_ising_golden(16)
    B = len(lg)
    lo, hi = oracle_lib.partition(B, 6, 0.75)
    W = int((hi - lo + 1).max())
    P = np.zeros((6, W))
    V = np.zeros((6, W), np.uint8)
    rng = np.random.default_rng(4)
    for k in range(6):
        seg = lg[lo[k]:hi[k] + 1]
        fin = np.isfinite(seg)
        P[k, :len(seg)][fin] = seg[fin] + rng.uniform(-50, 50)
        V[k, :len(seg)] = fin
    out, joins = oracle_lib.stitch(lo, hi, P, V, B)
    fin = np.isfinite(lg)
    assert np.array_equal(np.isfinite(out), fin)
    d = out[fin] - lg[fin]
    assert d.max() - d.min() < 1e-9
    for k, j in enumerate(joins):
        assert lo[k + 1] <= j <= hi[k]


def test_stitch_picks_matching_slope(oracle_lib):
    """Where the two pieces agree in slope only at one place, the join is there."""
    B = 12
    lo = np.array([0, 4])
    hi = np.array([7, 11])
    base = np.arange(B, dtype=float) ** 1.5
    P = np.zeros((2, 8))
    P[0] = base[0:8]
    P[1] = base[4:12] + 3.0
    P[1, 0:2] += np.array([5.0, 0.0])   # bin 4 disagrees in slope with piece 0
    P[1, 3] += 7.0                      # slopes around bin 7 disagree too
    V = np.ones((2, 8), np.uint8)
    out, joins = oracle_lib.stitch(lo, hi, P, V, B)
    assert joins[0] == 5
    assert np.allclose(out[:5], base[:5]) and np.allclose(out[5:7], base[5:7])


# ------------------------------------------------------- Markov-chain pins --
def _fixed_weight_run(oracle_lib, lg_exact, tilt, h, m, S, seed, L=4):
    """Walkers with ln g frozen at exact + tilt * E: visits must follow exp(-tilt E)."""
    run = oracle_lib.Run("ising", L, n_windows=h, overlap=0.75, walkers_per_window=m,
                         flatness=1.0, lnf_init=1e-300, lnf_final=1e-310, S=S, seed=seed)
    E = run.energies()
    for w in range(h * m):
        win = run.window(w // m)
        seg = slice(win["lo"], win["hi"] + 1)
        vals = lg_exact[seg] + tilt[w // m] * E[seg]
        vals = np.where(np.isfinite(vals), vals - np.nanmin(np.where(np.isfinite(vals), vals, np.nan)) + 1.0, 0.0)
        run.set_lng(w, vals)
    return run, E


def test_sweep_samples_inverse_dos(oracle_lib):
    """With ln g fixed at the exact DOS the energy histogram is flat (A1, A3)."""
    from oracle import exact

    g = exact.ising_dos_exact(4)
    lg = np.array([math.log(x) if x else -np.inf for x in g])
    for tilt in (0.0, 0.06):
        run, E = _fixed_weight_run(oracle_lib, lg, [tilt], 1, 1, 20_000, 3)
        run.step(100)
        H = run.walker(0)["H"].astype(float)
        reach = np.isfinite(lg)
        target = np.exp(-tilt * E[reach])
        target *= H[reach].sum() / target.sum()
        rel = np.abs(H[reach] / target - 1.0)
        assert rel.max() < 0.05, (tilt, rel.max())
        assert H[~reach].sum() == 0


def test_exchange_keeps_detailed_balance(oracle_lib):
    """Frequent exchanges between tilted walkers keep each one's exp(-tilt E) law (Eq. (1))."""
    from oracle import exact

    g = exact.ising_dos_exact(4)
    lg = np.array([math.log(x) if x else -np.inf for x in g])
    tilts = [0.05, -0.05]
    run, E = _fixed_weight_run(oracle_lib, lg, tilts, 2, 2, 20, 5)
    run.step(100_000)
    st = run.stats()
    assert st["ex_acc"] > 0.05 * st["ex_prop"]
    for w in range(4):
        k = w // 2
        win = run.window(k)
        seg = slice(win["lo"], win["hi"] + 1)
        H = run.walker(w)["H"].astype(float)
        reach = np.isfinite(lg[seg])
        target = np.exp(-tilts[k] * E[seg][reach])
        target *= H[reach].sum() / target.sum()
        rel = np.abs(H[reach] / target - 1.0)
        # statistical scatter stays near 0.1; a sign error in Eq. (1) gives ~3
        assert rel.max() < 0.25, (w, rel.max())


def test_exchange_pairs_alternate(oracle_lib):
    """Exchanges run between neighbouring windows, the pairs (k, k+1) with
    k = round mod 2, one proposal per walker of the lower window: with 4 windows
    of 3 walkers that is 2 pairs (6 proposals) in even rounds and 1 pair
    (3 proposals) in odd ones."""
    run = oracle_lib.Run("ising", 6, n_windows=4, walkers_per_window=3, S=200, seed=9,
                         lnf_final=1e-12)
    prev = run.stats()["ex_prop"]
    for r in range(12):
        run.step(1)
        assert not any(w["done"] for w in run.windows())
        now = run.stats()["ex_prop"]
        assert now - prev == (6 if r % 2 == 0 else 3), (r, now - prev)
        prev = now


def _observed_partners(oracle_lib, m, rounds, seed):
    """Partner permutations of the exchange step, read off a run in which every
    exchange is accepted: two windows that both cover every level the walk can
    reach from random spins (6x6 Ising, overlap 0.95: bins [0, 35] and [1, 36],
    which leave out only the two ordered states), ln f = 1e-30 so that every Eq. (1) log-ratio is far above any
    ln u (<= ln(1 - 2^-53)), flatness 1 so that merges stay rare, one attempt per
    walker per round.  In an even round (pair (0, 1)) walker a of window 0 hands
    its configuration to walker pi[a] of window 1; after one attempt each
    configuration is within one flipped spin of what it was before the round,
    which identifies pi[a]."""
    run = oracle_lib.Run("ising", 6, n_windows=2, walkers_per_window=m, overlap=0.95,
                         flatness=1.0, lnf_init=1e-30, lnf_final=1e-300, S=1, seed=seed)
    win = [run.window(k) for k in range(2)]
    assert (win[0]["lo"], win[0]["hi"], win[1]["lo"], win[1]["hi"]) == (0, 35, 1, 36)
    perms = []
    for r in range(rounds):
        before = [run.walker(w)["spins"].copy() for w in range(2 * m)]
        run.step(1)
        if r % 2:
            continue
        after = [run.walker(w)["spins"] for w in range(2 * m)]
        pi = []
        for a in range(m):
            hits = [b for b in range(m) if np.sum(after[m + b] != before[a]) <= 1]
            pi.append(hits[0] if len(hits) == 1 else None)
        if None not in pi:
            perms.append(tuple(pi))
    return perms, run.stats()


@pytest.mark.parametrize("m,rounds", [(2, 800), (3, 2400), (4, 4800)])
def test_exchange_partner_is_uniform(oracle_lib, m, rounds):
    """The paper lets each walker pick its exchange partner in the neighbouring
    window at random (parallel-scheme paragraph).  The partners of one exchange
    step form a permutation of the m walkers of the upper window; every one of the
    m! permutations must come out equally often.  Chi-square over the observed
    permutations, p > 1e-6.  (A shuffle that never leaves an element in place
    yields only the (m-1)! cyclic orders; pairing a with a yields the identity.)"""
    import itertools

    from scipy import stats

    perms = []
    ex = 0
    for seed in (3, 4):
        p, st = _observed_partners(oracle_lib, m, rounds // 2, seed)
        perms += p
        ex += st["ex_acc"]
    n_pairs = 2 * (rounds // 4) * m
    assert ex == n_pairs and len(perms) > 0.99 * (n_pairs // m), (ex, n_pairs, len(perms))
    for p in perms:
        assert sorted(p) == list(range(m)), p
    cats = list(itertools.permutations(range(m)))
    counts = np.array([perms.count(c) for c in cats], dtype=float)
    chi2, pval = stats.chisquare(counts)
    assert pval > 1e-6, (m, counts, chi2, pval)


@pytest.mark.parametrize("model,q,L", [("ising", 2, 6), ("potts", 3, 5), ("ea", 2, 6)])
def test_walkers_stay_in_their_windows(oracle_lib, model, q, L):
    """A move or an exchange that would take a walker out of its window is
    rejected, so every walker's energy stays in its window through rounds of
    sweeps and exchanges (Eq. (1) is applied only when both energies lie in both
    windows); exchanges do get accepted."""
    from workloads import ea_couplings

    J = ea_couplings(L, 5) if model == "ea" else None
    run = oracle_lib.Run(model, L, q=q, couplings=J, n_windows=4, walkers_per_window=2,
                         overlap=0.5, S=300, seed=11, lnf_final=1e-12)
    for _ in range(40):
        run.step(1)
        for w in range(run.h * run.m):
            win = run.window(w // run.m)
            E = run.walker(w)["E"]
            assert (E - run.e_min) % run.e_step == 0
            assert win["lo"] <= (E - run.e_min) // run.e_step <= win["hi"], (w, E, win)
    assert run.stats()["ex_acc"] > 0


# -------------------------------------------------------------- schedule --
def _flat_by_definition(st, p):
    """The flatness criterion written out: over the visited bins of the window,
    the smallest histogram entry is at least p times the mean entry (compared as
    min * n >= p * sum, free of the division's rounding)."""
    h = st["H"][st["visited"] > 0].astype(np.float64)
    return bool(h.size > 0 and h.min() * h.size >= p * h.sum())


def test_merge_and_schedule(oracle_lib):
    """Windows merge only when all m walkers are flat; ln f halves; H resets."""
    run = oracle_lib.Run("ising", 6, n_windows=2, walkers_per_window=2, S=2000, seed=4,
                         lnf_final=1e-3)
    prev = [1.0, 1.0]
    was_flat = [False] * 4
    for _ in range(400):
        run.step(1)
        for k in range(2):
            win = run.window(k)
            sts = [run.walker(2 * k + s) for s in range(2)]
            if win["lnf"] != prev[k]:
                assert win["lnf"] == prev[k] * 0.5
                assert np.array_equal(sts[0]["lng"], sts[1]["lng"])
                assert np.array_equal(sts[0]["visited"], sts[1]["visited"])
                if not win["done"]:
                    # fresh iteration: only the exchange step ran after the merge
                    assert all(s["H"].sum() == 0 for s in sts)
                    assert not any(s["flat"] for s in sts)
                prev[k] = win["lnf"]
            elif not win["done"]:
                # no merge: a walker's flag is the flatness of its histogram over
                # the bins it visited (min H >= p * mean H, p = 0.8) the first
                # time that holds, and stays set until the window merges
                for s, st in enumerate(sts):
                    w = 2 * k + s
                    if not was_flat[w]:
                        assert st["flat"] == _flat_by_definition(st, 0.8), (w, st["H"])
                    else:
                        assert st["flat"]
            for s, st in enumerate(sts):
                was_flat[2 * k + s] = st["flat"]
            assert np.array_equal(sts[0]["visited"] > 0, sts[0]["lng"] > 0)
        if run.info()["done"]:
            break
    assert run.info()["done"]
    for k in range(2):
        w = run.window(k)
        assert w["done"] and w["lnf"] < 1e-3 <= 2 * w["lnf"]


def test_one_over_t_schedule(oracle_lib):
    """1/t rule: ln f halves until a halving would drop below W/t; from then on
    ln f = W/t exactly (W window bins, t attempts per walker), the walkers of
    the window are averaged every round, and the window ends once W/t is below
    the final ln f."""
    S, final = 5000, 1e-6
    run = oracle_lib.Run("ising", 6, n_windows=2, walkers_per_window=2, S=S, seed=4,
                         lnf_final=final, schedule="1/t")
    prev = [1.0, 1.0]
    switched = [None, None]
    ended = [False, False]
    for _ in range(10_000):
        run.step(1)
        for k in range(2):
            if ended[k]:
                continue
            win = run.window(k)
            W = win["hi"] - win["lo"] + 1
            sts = [run.walker(2 * k + s) for s in range(2)]
            t = sts[0]["t"]
            assert sts[1]["t"] == t
            if switched[k] is not None:
                assert win["lnf"] == W / t
                assert np.array_equal(sts[0]["lng"], sts[1]["lng"])
            elif win["lnf"] != prev[k]:
                if win["lnf"] == prev[k] * 0.5:
                    assert prev[k] * 0.5 >= W / t
                else:
                    assert win["lnf"] == W / t and prev[k] * 0.5 < W / t
                    switched[k] = t
            prev[k] = win["lnf"]
            ended[k] = win["done"]
            if win["done"]:
                assert win["lnf"] < final
                if switched[k] is not None:   # ended on the first W/t below final
                    assert final <= W / (t - S)
        if run.info()["done"]:
            break
    assert run.info()["done"]
    assert all(x is not None for x in switched), switched


def test_one_over_t_increments(oracle_lib):
    """In the 1/t phase the j-th attempt of a walker (j counted after the
    attempt) adds W/j to ln g of the bin it ends in, so one round of S attempts
    raises the sum of a walker's ln g over the window by the sum of W/j for
    j = t0+1 .. t0+S; the end-of-round average over the window's walkers, which
    all share t, and the exchange step (no ln g update) keep that sum."""
    S = 3000
    run = oracle_lib.Run("ising", 6, n_windows=2, walkers_per_window=2, S=S, seed=7,
                         lnf_final=1e-9, schedule="1/t")
    checked = 0
    prev = [None, None]   # (t, sum of ln g) once the window runs the 1/t rule
    for _ in range(4000):
        run.step(1)
        for k in range(2):
            win = run.window(k)
            W = win["hi"] - win["lo"] + 1
            st = run.walker(2 * k)
            total = math.fsum(st["lng"])
            if prev[k] is not None and not prev[k][2]:
                t0, before, _ = prev[k]
                assert st["t"] == t0 + S
                want = math.fsum(W / j for j in range(t0 + 1, t0 + S + 1))
                assert abs((total - before) - want) < 1e-8, (k, total - before, want)
                checked += 1
            if win["lnf"] == W / st["t"]:   # in the 1/t phase (set at this merge)
                prev[k] = (st["t"], total, win["done"])
        if checked >= 20 or run.info()["done"]:
            break
    assert checked >= 20, checked


def test_one_over_t_removes_saturation(oracle_lib):
    """6x6 Ising against the exact DOS: halving to ln f = 1e-6 stalls at errors
    of 0.1-0.2, the 1/t rule reaches a few hundredths by ln f = 1e-5."""
    _E, ref = None, None
    from oracle import exact

    ref = np.array([math.log(n) if n > 0 else -np.inf for n in exact.ising_dos_exact(6)])
    errs = {"halving": [], "1/t": []}
    for sched, lf in (("halving", 1e-6), ("1/t", 1e-5)):
        for seed in (1, 2, 3):
            run = oracle_lib.Run("ising", 6, n_windows=4, walkers_per_window=2, lnf_final=lf,
                                 S=10_000, seed=seed, schedule=sched)
            assert run.run()
            errs[sched].append(_max_err(run.lng(), ref))
    assert max(errs["1/t"]) < 0.08, errs
    assert np.mean(errs["1/t"]) < 0.5 * np.mean(errs["halving"]), errs


def test_histogram_counts_attempts(oracle_lib):
    run = oracle_lib.Run("potts", 5, q=3, n_windows=3, walkers_per_window=2, S=777, seed=8)
    run.step(1)
    for w in range(6):
        st = run.walker(w)
        assert st["H"].sum() == 777 and st["t"] == 777


def test_deterministic_and_thread_independent(oracle_lib):
    from workloads import ea_couplings

    J = ea_couplings(8, 2)
    a = oracle_lib.Run("ea", 8, couplings=J, n_windows=4, walkers_per_window=2, S=3000, seed=6,
                       n_threads=1)
    b = oracle_lib.Run("ea", 8, couplings=J, n_windows=4, walkers_per_window=2, S=3000, seed=6,
                       n_threads=4)
    a.step(30)
    b.step(30)
    for w in range(8):
        x, y = a.walker(w), b.walker(w)
        for key in ("spins", "lng", "H", "visited"):
            assert np.array_equal(x[key], y[key])
        assert x["E"] == y["E"] and x["t"] == y["t"]


def test_descent_reaches_every_window(oracle_lib):
    """Start-up puts each walker inside its window, the lowest q=10 Potts windows
    through the ordered-state restart."""
    run = oracle_lib.Run("potts", 16, q=10, n_windows=8, walkers_per_window=2, seed=3)
    for w in range(16):
        st = run.walker(w)
        win = run.window(w // 2)
        b = (st["E"] - run.e_min) // run.e_step
        assert win["lo"] <= b <= win["hi"]


def test_ea3_energy_definition(oracle_lib):
    """3D glass energy -sum over the 3N bonds (site, +x / +y / +z neighbour) of
    J s s, against a numpy evaluation of that definition, and the reference
    states: all spins up gives -sum J."""
    from workloads import ea3_couplings

    rng = np.random.default_rng(4)
    for L in (2, 3, 5):
        N = L ** 3
        J = ea3_couplings(L, L)
        idx = np.arange(N).reshape(L, L, L)
        nbr = [np.roll(idx, -1, axis=ax).ravel() for ax in (2, 1, 0)]
        Jr = J.reshape(N, 3).astype(np.int64)
        for _ in range(20):
            s = rng.choice(np.array([-1, 1], dtype=np.int8), size=N)
            ref = -sum((Jr[:, a] * s * s[nbr[a]]).sum() for a in range(3))
            assert oracle_lib.energy("ea3", L, s, J) == ref
        assert oracle_lib.energy("ea3", L, np.ones(N, np.int8), J) == -int(J.astype(int).sum())


def test_ea3_brute_force_pins():
    """The 2x2x2 glass enumerated: sum g = 2^N, g(E) = g(-E) (the cubic torus of
    even L is bipartite: flipping one sublattice maps E to -E), energies on the
    class -3N + 2 n_neg (mod 4)."""
    from oracle import exact
    from workloads import ea3_couplings

    for seed in (1, 2, 3):
        J = ea3_couplings(2, seed)
        g = exact.brute_dos("ea3", 2, couplings=J)
        assert sum(g.values()) == 2 ** 8
        assert all(g[e] == g.get(-e, 0) for e in g)
        n_neg = int((J < 0).sum())
        assert all((e - (-24 + 2 * n_neg)) % 4 == 0 for e in g)


def test_ea3_converges_to_brute_force(oracle_lib):
    """REWL on 2x2x2 glasses against exact enumeration."""
    from oracle import exact
    from workloads import ea3_couplings

    for seed in (1, 2):
        J = ea3_couplings(2, seed)
        g = exact.brute_dos("ea3", 2, couplings=J)
        run = oracle_lib.Run("ea3", 2, couplings=J, n_windows=2, walkers_per_window=2,
                             S=3000, lnf_final=1e-6, seed=seed)
        assert run.run()
        E = run.energies()
        ref = np.array([math.log(g[e]) if g.get(e, 0) else -np.inf for e in E])
        assert _max_err(run.lng(), ref) < 0.05


def _load_ea3_golden():
    path = os.path.join(ROOT, "tests", "golden", "ea3_L3_seed1.txt")
    g = {}
    with open(path) as f:
        for line in f:
            if not line.startswith("#"):
                e, n = line.split()
                g[int(e)] = int(n)
    return g


def test_ea3_golden_3x3x3(oracle_lib):
    """The stored 3x3x3 glass DOS (all 2^27 configurations enumerated): sum rule,
    energy class, and REWL in the oracle converging to it (4 windows x 4
    walkers, ln f to 1e-6; seeds 2-4 give 0.06-0.08)."""
    from workloads import ea3_couplings

    g = _load_ea3_golden()
    J = ea3_couplings(3, 1)
    assert sum(g.values()) == 2 ** 27
    n_neg = int((J < 0).sum())
    assert all((e - (-81 + 2 * n_neg)) % 4 == 0 for e in g)
    run = oracle_lib.Run("ea3", 3, couplings=J, n_windows=4, walkers_per_window=4, S=5000,
                         lnf_final=1e-6, seed=2)
    assert run.run()
    E = run.energies()
    ref = np.array([math.log(g[e]) if g.get(e, 0) else -np.inf for e in E])
    assert _max_err(run.lng(), ref) < 0.15


def test_ea3_layer_sum_agrees_with_enumeration():
    """A second exact method for the 3x3x3 glass, summing over its three layers,
    reproduces the stored enumeration; with every coupling +1 (the 3D Ising
    torus) its lowest levels are the hand counts: 2 ground states, 2N single
    flips (6 broken bonds, E + 12), 2 x 3N dominoes (10 broken bonds, E + 20) and
    nothing between."""
    from oracle import exact
    from workloads import ea3_couplings

    assert exact.ea3_dos_layers(ea3_couplings(3, 1)) == _load_ea3_golden()
    N = 27
    g = exact.ea3_dos_layers(np.ones(3 * N, np.int8))
    lo = -3 * N
    assert g[lo] == 2 and g[lo + 12] == 2 * N and g[lo + 20] == 2 * 3 * N
    assert all(lo + d not in g for d in (4, 8, 16))


@pytest.mark.parametrize("coupling_seed", [2, 3])
def test_ea3_converges_to_layer_sum(oracle_lib, coupling_seed):
    """REWL on two more 3x3x3 glasses against their exact DOS from the layer sum
    (4 windows x 4 walkers, ln f to 1e-6; measured 0.055-0.087)."""
    from oracle import exact
    from workloads import ea3_couplings

    J = ea3_couplings(3, coupling_seed)
    g = exact.ea3_dos_layers(J)
    n_neg = int((J < 0).sum())
    assert all((e - (-81 + 2 * n_neg)) % 4 == 0 for e in g)
    run = oracle_lib.Run("ea3", 3, couplings=J, n_windows=4, walkers_per_window=4, S=5000,
                         lnf_final=1e-6, seed=1, n_threads=4)
    assert run.run()
    ref = np.array([math.log(g[e]) if e in g else -np.inf for e in run.energies()])
    assert _max_err(run.lng(), ref) < 0.15


def test_invalid_arguments(oracle_lib):
    from workloads import ea3_couplings

    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ea3", 33, couplings=ea3_couplings(33, 1))
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ea3", 4)                       # no couplings
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ising", 2)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("potts", 8, q=1)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ising", 8, overlap=1.0)
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.Run("ising", 8, n_windows=64)   # windows narrower than 2 bins


# ----------------------------------------------------- convergence to truth --
def _max_err(lg, ref):
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(lg), fin)
    return np.abs(lg[fin] - ref[fin]).max()


def test_ising8_converges_to_exact(oracle_lib):
    """Ising 8x8, 4 windows x 2 walkers, ln f 1 -> 1e-6: ln g within WL's
    statistical error of the exact DOS, normalised ln g(-2N) = ln 2."""
    _, ref = load_ising_golden(8)
    errs = []
    for seed in (1, 2, 3):
        run = oracle_lib.Run("ising", 8, n_windows=4, walkers_per_window=2, lnf_final=1e-6,
                             S=10_000, seed=seed)
        assert run.run()
        lg = run.lng()
        assert lg[0] == math.log(2)
        errs.append(_max_err(lg, ref))
    assert max(errs) < 0.3, errs


def test_small_models_converge_to_brute_force(oracle_lib):
    """3x3 q=3 Potts and a 4x4 +-J glass against exact enumeration."""
    from oracle import exact
    from workloads import ea_couplings

    g = exact.brute_dos("potts", 3, q=3)
    run = oracle_lib.Run("potts", 3, q=3, n_windows=2, walkers_per_window=2, lnf_final=1e-6,
                         S=5_000, seed=2)
    assert run.run()
    E = run.energies()
    ref = np.array([math.log(g[e]) if g.get(e, 0) else -np.inf for e in E])
    ref = ref - ref[0] + math.log(3)
    assert _max_err(run.lng(), ref) < 0.25

    J = ea_couplings(4, 1)
    g = exact.brute_dos("ea", 4, couplings=J)
    run = oracle_lib.Run("ea", 4, couplings=J, n_windows=2, walkers_per_window=2,
                         lnf_final=1e-6, S=5_000, seed=2)
    assert run.run()
    E = run.energies()
    ref = np.array([math.log(g[e]) if g.get(e, 0) else -np.inf for e in E])
    assert _max_err(run.lng(), ref) < 0.25
