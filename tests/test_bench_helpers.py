"""Host-side helpers of bench.py that its reported figures rest on (no GPU)."""
import numpy as np

from conftest import load_ising_golden


def test_exact_error_measures_the_largest_deviation():
    import bench
    from workloads import run_params

    p = run_params("ising32", seed=1)
    _, ref = load_ising_golden(32)
    assert bench.exact_error(p, ref) == 0.0
    off = ref.copy()
    b = int(np.flatnonzero(np.isfinite(ref))[100])
    off[b] += 0.015
    assert abs(bench.exact_error(p, off) - 0.015) < 1e-12
    # a visited set different from the exact support is an infinite error
    bad = ref.copy()
    bad[b] = -np.inf
    assert bench.exact_error(p, bad) == float("inf")
    # no stored exact DOS for other models
    assert bench.exact_error(run_params("potts64", seed=1), ref) is None


def test_percentile_and_roofline_constants():
    import bench

    assert bench.percentile([], 50) is None
    assert bench.percentile([1.0, 2.0, 3.0], 50) == 2.0
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, in T lane-slots/s
    assert abs(bench.VALU_PEAK_TOPS - 256 * 4 * 16 * 2.4e9 / 1e12) < 1e-9


def test_committed_profiles_match_the_kernel_sources():
    """The HBM traffic the benchmark reports comes from profiles/ only while
    they were taken on the current device sources (a kernel change without new
    profiles leaves it null, which this test reports as a skip)."""
    import os

    import pytest

    import bench

    for tag in ("sweep_ea24x256_P8",):
        assert os.path.exists(os.path.join(bench.ROOT, "profiles", f"{tag}.md")), tag
        if bench.profiled_traffic(tag) is None:
            pytest.skip(f"profiles/{tag}.md was taken on other kernel sources")


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    """bench.py measures one GPU: --gpus N with N > 1 (or a multi-rank launch)
    exits with status 2 and a message saying so, before it imports torch."""
    import os
    import subprocess
    import sys

    from conftest import ROOT

    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                           env=dict(os.environ, **env), capture_output=True, text=True,
                           timeout=120, cwd=ROOT)
        assert r.returncode == 2, (argv, env, r.stderr)
        assert "exactly one GPU" in r.stderr and "--gpus 1" in r.stderr
        assert r.stdout == ""



def test_profile_commands_run_committed_files_within_counter_limits():
    """Every rocprofv3 command recorded in profiles/ runs bench.py (a committed
    file) with arguments bench.py accepts, puts the program right after `--`,
    and keeps each counter pass within one pass's hardware limits (at most 8 SQ
    and 2 GRBM counters, FETCH_SIZE and WRITE_SIZE in passes of their own) and
    free of trace domains."""
    import glob
    import os
    import shlex
    import subprocess
    import sys

    from conftest import ROOT

    cmds = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        cmds += [(path, line.strip()) for line in open(path)
                 if line.strip().startswith("rocprofv3 ")]
    assert len(cmds) >= 8
    for path, line in cmds:
        argv = shlex.split(line)
        prog = argv[argv.index("--") + 1:]
        assert prog[:2] == ["python3", "bench.py"], (path, line)
        opts = argv[1:argv.index("--")]
        for bad in ("-s", "--sys-trace", "-r", "--runtime-trace", "--hip-trace", "--hsa-trace"):
            assert not ("--pmc" in opts and bad in opts), (path, line)
        if "--pmc" in opts:
            i = opts.index("--pmc") + 1
            counters = []
            while i < len(opts) and not opts[i].startswith("-"):
                counters.append(opts[i])
                i += 1
            assert sum(c.startswith("SQ_") for c in counters) <= 8, line
            assert sum(c.startswith("GRBM_") for c in counters) <= 2, line
            assert not ({"FETCH_SIZE", "WRITE_SIZE"} <= set(counters)), line
        # bench.py parses the arguments (then stops at the one-GPU check, before
        # any GPU work): an unknown or malformed argument would exit with "error:"
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *prog[2:],
                            "--gpus", "2"], capture_output=True, text=True, timeout=120, cwd=ROOT)
        assert r.returncode == 2 and "error:" not in r.stderr and "exactly one GPU" in r.stderr, \
            (path, line, r.stderr[-500:])


def test_roofline_arithmetic():
    """achieved = 170 lane-slots x attempts per launch / average launch time,
    against 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz; the recount scales it."""
    import bench

    r = bench.roofline(attempts=20 * 81_920_000, launches=20, launch_ms=20 * 2.0,
                       traffic=123.0, kernel="k")
    ach = 170 * 81_920_000 / 2.0e-3 / 1e12
    assert abs(r["achieved"] - ach) < 1e-9
    assert abs(r["frac"] - ach / bench.VALU_PEAK_TOPS) < 1e-12
    assert abs(r["launch_avg_us"] - 2000.0) < 1e-9
    assert r["bound"] == "alu" and r["unit"] == "TOP/s" and r["traffic"] == 123.0
    assert abs(r["frac_at_recount"] - r["frac"] * 200 / 170) < 1e-12
    assert bench.roofline(attempts=1, launches=0, launch_ms=0.0, traffic=None, kernel="k") is None


def test_dos_checks_on_the_exact_ising_density_of_states():
    """The accuracy mode's checks that need no exact DOS, applied to the exact
    8x8 Ising DOS: the total count is 2^N exactly, and the specific heat peaks
    above the infinite-lattice T_c = 2/ln(1+sqrt 2) (finite-size shift of the
    8x8 torus) with the value a direct evaluation gives there."""
    import math

    import bench

    E, ref = load_ising_golden(8)

    class R:
        N = 64

        def energies(self):
            return np.asarray(E)

    out = bench.dos_checks({"model": "ising", "L": 8}, R(), ref)
    assert abs(out["log_total_states"] - 64 * math.log(2)) < 1e-9
    assert out["n_ln_states_per_site"] == 64 * math.log(2)
    T = out["specific_heat_peak"]["T"]
    assert 2 / math.log(1 + math.sqrt(2)) < T < 2.6
    fin = np.isfinite(ref)
    e, g = np.asarray(E, dtype=float)[fin], ref[fin]
    w = g - e / T
    pr = np.exp(w - w.max())
    mean = (pr * e).sum() / pr.sum()
    var = (pr * (e - mean) ** 2).sum() / pr.sum()
    assert abs(out["specific_heat_peak"]["C_per_site"] - var / T ** 2 / 64) < 1e-9
