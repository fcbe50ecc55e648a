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
PINS = ("sweep_samples_inverse_dos or exchange_keeps_detailed_balance or merge_and_schedule "
        "or walker_energy_tracks_spins or small_models_converge_to_brute_force")

MUTATIONS = {
    "acceptance difference with its operands swapped": (
        "double d = lng[bin_of(run, E) - lo] - lng[bin_of(run, En) - lo];",
        "double d = lng[bin_of(run, En) - lo] - lng[bin_of(run, E) - lo];"),
    "acceptance test reversed": (
        "if (orc_ln_u(u) < d) {",
        "if (orc_ln_u(u) > d) {"),
    "ln f quartered instead of halved": (
        "run->lnf[k] = run->lnf[k] * 0.5;",
        "run->lnf[k] = run->lnf[k] * 0.25;"),
    "a wrong neighbour in the Ising energy change": (
        "return 2 * (int64_t)s[i] * (s[rt] + s[lf] + s[dn] + s[up]);",
        "return 2 * (int64_t)s[i] * (s[rt] + s[rt] + s[dn] + s[up]);"),
    "the second term of Eq. (1) with its sign flipped": (
        "(gj[bin_of(run, EY) - lj] - gj[bin_of(run, EX) - lj]);",
        "(gj[bin_of(run, EX) - lj] - gj[bin_of(run, EY) - lj]);"),
}


def _build(tmp_path, name, text):
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    lib = tmp_path / f"{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-shared", "-fPIC", "-I", os.path.join(ROOT, "oracle"), "-o", str(lib),
                    str(src), "-lm"], check=True)
    return lib


def _pins_pass(lib):
    env = dict(os.environ, REWL_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", PINS],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    return r.returncode == 0, r.stdout[-2000:]


def test_unmodified_copy_passes(tmp_path):
    ok, out = _pins_pass(_build(tmp_path, "clean", open(SRC).read()))
    assert ok, out


@pytest.mark.parametrize("what", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, what):
    old, new = MUTATIONS[what]
    text = open(SRC).read()
    assert text.count(old) == 1, what
    ok, out = _pins_pass(_build(tmp_path, "mutant", text.replace(old, new)))
    assert not ok, f"the pins did not catch: {what}"
