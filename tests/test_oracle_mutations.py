"""The pins catch plausible mistakes: copies of the oracle, each with one
planted mistake, are compiled on the CPU, and the fast pins of
test_oracle_pins.py must fail on every copy while passing on an unmodified
copy built the same way.  The oracle file itself is not touched."""
import os
import subprocess
import sys

import pytest

from conftest import ROOT

SRC = os.path.join(ROOT, "oracle", "rewl_oracle.c")

# the fast pins that check the walk, the schedule, the exchange and energies
WALK = ("sweep_samples_inverse_dos or exchange_keeps_detailed_balance or merge_and_schedule "
        "or walker_energy_tracks_spins or small_models_converge_to_brute_force")

# planted mistake: (text in the oracle, replacement, pins expected to catch it)
MUTATIONS = {
    "acceptance difference with its operands swapped": (
        "double d = lng[bin_of(run, E) - lo] - lng[bin_of(run, En) - lo];",
        "double d = lng[bin_of(run, En) - lo] - lng[bin_of(run, E) - lo];", WALK),
    "acceptance test reversed": (
        "if (orc_ln_u(u) < d) {",
        "if (orc_ln_u(u) > d) {", WALK),
    "ln f quartered instead of halved": (
        "run->lnf[k] = run->lnf[k] * 0.5;",
        "run->lnf[k] = run->lnf[k] * 0.25;", WALK),
    "a wrong neighbour in the Ising energy change": (
        "return 2 * (int64_t)s[i] * (s[rt] + s[lf] + s[dn] + s[up]);",
        "return 2 * (int64_t)s[i] * (s[rt] + s[rt] + s[dn] + s[up]);", WALK),
    "the second term of Eq. (1) with its sign flipped": (
        "(gj[bin_of(run, EY) - lj] - gj[bin_of(run, EX) - lj]);",
        "(gj[bin_of(run, EX) - lj] - gj[bin_of(run, EY) - lj]);", WALK),
    "the merge summing ln g instead of averaging": (
        "double mean = pow2 ? sum * inv : sum / (double)m;",
        "double mean = sum;", WALK),
    "flatness without the threshold p": (
        "return (double)hmin * (double)n >= run->p * (double)sum;",
        "return (double)hmin * (double)n >= (double)sum;", WALK),
    "a Philox round multiplier off by two": (
        "uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;",
        "uint64_t p0 = (uint64_t)0xD2511F55u * (uint64_t)c0;", "philox_matches_rocrand"),
    "the ln u series shifted by one term": (
        "Q = horner(Q, z, 1.0 / (double)(2 * i + 1));",
        "Q = horner(Q, z, 1.0 / (double)(2 * i + 3));", "ln_u_accuracy"),
    "the joining point one bin late": (
        "if (diff < best_diff) { best_diff = diff; best = prev; }",
        "if (diff < best_diff) { best_diff = diff; best = b; }",
        "stitch_picks_matching_slope or stitch_recovers_exact_pieces"),
    "windows rounded the wrong way": (
        "lo[k] = (int64_t)floor(x);",
        "lo[k] = (int64_t)ceil(x);", "partition_examples"),
    "the +-J energy change using the site's own coupling to the left": (
        "(J[2 * i] * s[rt] + J[2 * lf] * s[lf] + J[2 * i + 1] * s[dn] + J[2 * up + 1] * s[up]);",
        "(J[2 * i] * s[rt] + J[2 * i] * s[lf] + J[2 * i + 1] * s[dn] + J[2 * up + 1] * s[up]);",
        WALK),
    "the +-J energy change using the site's own coupling upwards": (
        "(J[2 * i] * s[rt] + J[2 * lf] * s[lf] + J[2 * i + 1] * s[dn] + J[2 * up + 1] * s[up]);",
        "(J[2 * i] * s[rt] + J[2 * lf] * s[lf] + J[2 * i + 1] * s[dn] + J[2 * i + 1] * s[up]);",
        "ea_converges_to_exact"),
    "the Potts energy change with its sign flipped": (
        "return (int64_t)same_old - same_new;",
        "return (int64_t)same_new - same_old;", WALK),
    "the Potts energy change counting one neighbour twice for the new state": (
        "int same_new = (s[rt] == nw) + (s[lf] == nw) + (s[dn] == nw) + (s[up] == nw);",
        "int same_new = (s[rt] == nw) + (s[lf] == nw) + (s[dn] == nw) + (s[dn] == nw);",
        "potts_converges_to_exact"),
    "the 3D glass taking the coupling of the wrong site backwards": (
        "h += (int64_t)J[3 * i + a] * s[up] + (int64_t)J[3 * dn + a] * s[dn];",
        "h += (int64_t)J[3 * i + a] * s[up] + (int64_t)J[3 * i + a] * s[dn];", WALK),
    "the ground state normalised to ln(q + 1)": (
        "target = log(run->model == ORC_POTTS ? (double)run->q : 2.0);",
        "target = log((double)run->q + 1.0);", "small_models_converge_to_brute_force"),
    "the glass normalisation missing the log of its sum": (
        "ref = mx + log(sum);",
        "ref = mx;", "small_models_converge_to_brute_force"),
    "an accepted move not updating the walker's energy": (
        "E = En;\n                acc += 1;",
        "acc += 1;", WALK),
    "exchanges always starting from the lowest window pair": (
        "for (int k = (int)(round % 2); k + 1 < run->h; k += 2) {",
        "for (int k = 0; k + 1 < run->h; k += 2) {", "exchange_pairs_alternate"),
    "exchanges proposed between every neighbouring pair each round": (
        "for (int k = (int)(round % 2); k + 1 < run->h; k += 2) {",
        "for (int k = 0; k + 1 < run->h; k += 1) {", "exchange_pairs_alternate"),
    "a merge leaving the walkers' flatness flags set": (
        "for (int s = 0; s < m; ++s) run->flat[k * m + s] = 0;",
        "", "merge_and_schedule"),
    "flatness counting bins the walker never visited": (
        "if (!vis[b]) continue;",
        "", "merge_and_schedule"),
    "balanced windows sized as if they did not overlap": (
        "double w = F[B - 1] / (1.0 + (double)(h - 1) * (1.0 - o));",
        "double w = F[B - 1] / (double)h;", "balanced_partition_uniform_is_equal"),
    "the 1/t increment taken with t counted before the attempt": (
        "if (one_over_t) lnf = Wd / (double)run->t[w];",
        "if (one_over_t) lnf = Wd / (double)(run->t[w] - 1);", "one_over_t_increments"),
    "the 1/t increment taken as W/(t+1)": (
        "if (one_over_t) lnf = Wd / (double)run->t[w];",
        "if (one_over_t) lnf = Wd / (double)(run->t[w] + 1);", "one_over_t_increments"),
    "the partner shuffle never leaving a walker in place": (
        "int j = (int)mulhi32(next_word(&ws), (uint32_t)(a + 1));",
        "int j = (int)mulhi32(next_word(&ws), (uint32_t)(a));", "exchange_partner_is_uniform"),
    "exchange partners paired by slot instead of by the permutation": (
        "int wi = k * m + a, wj = (k + 1) * m + perm[a];",
        "int wi = k * m + a, wj = (k + 1) * m + a;", "exchange_partner_is_uniform"),
    "the 1/t rule never switched on": (
        "if (run->schedule == 1 && run->lnf[k] < Wt) {",
        "if (run->schedule == 2 && run->lnf[k] < Wt) {", "one_over_t_schedule"),
}
PINS = " or ".join(sorted({m[2] for m in MUTATIONS.values()}))


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-shared", "-fPIC", "-I", os.path.join(ROOT, "oracle"), "-o", str(lib),
                    str(src), "-lm"], check=True)
    return lib


def _pins_pass(lib, pins):
    env = dict(os.environ, REWL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", pins],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    return r.returncode == 0, r.stdout[-2000:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, "clean", open(SRC).read()), PINS)
    assert ok, out


@pytest.mark.parametrize("what", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, what):
    old, new, pins = MUTATIONS[what]
    text = open(SRC).read()
    assert text.count(old) == 1, what
    ok, out = _pins_pass(_build(tmp_path, "mutant", text.replace(old, new)), pins)
    assert not ok, f"the pins did not catch: {what}"
