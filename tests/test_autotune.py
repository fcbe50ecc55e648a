"""The launch-setting search of paper_1305_5615_amd.autotune, with a stubbed
batch and timer (no GPU): it must time every candidate over the same work,
keep the fastest, skip settings the library refuses, compare attempts-per-round
candidates over equal attempts, and cache its choice per run shape."""
import pytest

from paper_1305_5615_amd import autotune
from paper_1305_5615_amd.autotune import Setting


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def make_fake(clock, cost, refuse=()):
    """A stand-in for Batch: every round advances `clock` by cost(setting, S)
    seconds and adds S attempts per walker to every run."""
    from paper_1305_5615_amd import RewlError

    made = []

    class View:
        def __init__(self, b, i):
            self.b, self.i = b, i

        def info(self):
            return {"attempts": self.b.attempts[self.i]}

    class FakeBatch:
        def __init__(self, runs, walkers_per_wave, graph_rounds, form):
            s = Setting(walkers_per_wave, form, graph_rounds, None)
            if (walkers_per_wave, form) in refuse:
                raise RewlError(-1, "fake", "refused")
            self.runs = runs
            self.s = s
            self.attempts = [0] * len(runs)
            self.rounds = 0
            self.closed = False
            made.append(self)

        def step(self, n):
            S = self.runs[0]["S"]
            for i, kw in enumerate(self.runs):
                self.attempts[i] += n * S * kw["n_windows"] * kw["walkers_per_window"]
            self.rounds += n
            clock.t += n * cost(self.s, S)

        def __getitem__(self, i):
            return View(self, i)

        def close(self):
            self.closed = True

    return FakeBatch, made


RUNS = [dict(model="ea", L=24, n_windows=8, walkers_per_window=4, S=10_000, seed=s)
        for s in range(1, 5)]


def test_search_keeps_the_fastest_and_skips_refused():
    clock = FakeClock()

    def cost(s, S):     # seconds per round: P=8 persistent fastest, P=1 refused
        return {("rounds", 4): 3.0, ("rounds", 8): 2.0, ("persistent", 4): 2.5,
                ("persistent", 8): 1.0}[(s.form, s.walkers_per_wave)]

    fake, made = make_fake(clock, cost, refuse={(1, "persistent"), (1, "rounds")})
    cands = autotune.candidates((1, 4, 8), ("rounds", "persistent"), (0,))
    best, rate, table = autotune.search(
        cands, lambda c: autotune.batch_rate(RUNS, c, rounds=4, make_batch=fake,
                                             sync=lambda: None, timer=clock))
    assert best == Setting(8, "persistent", 0, None)
    walkers = sum(kw["n_windows"] * kw["walkers_per_window"] for kw in RUNS)
    assert rate == pytest.approx(walkers * 10_000 / 1.0)
    refused = [c for c, r in table if r is None]
    assert {c.walkers_per_wave for c in refused} == {1} and len(refused) == 2
    # every valid candidate: one warm-up round plus the same 4 timed rounds
    assert [b.rounds for b in made] == [5] * 4 and all(b.closed for b in made)


def test_ties_go_to_the_earlier_candidate():
    c = autotune.candidates((2, 4), ("rounds",), (0,))
    best, _, _ = autotune.search(c, lambda s: 1.0)
    assert best == c[0]
    with pytest.raises(ValueError):
        autotune.search(c, lambda s: None)


def test_candidates_space():
    c = autotune.candidates((1, 8), ("rounds", "persistent"), (0, 16), S_options=(1000, 10_000))
    # rounds: 2 P x 2 graphs, persistent: 2 P x no graph; times 2 S
    assert len(c) == 2 * (4 + 2)
    assert all(s.graph_rounds == 0 for s in c if s.form == "persistent")
    assert {s.S for s in c} == {1000, 10_000}


def test_open_attempts_per_round_compared_over_equal_attempts():
    """With S searched, a candidate with S = 1000 is timed over ten times the
    rounds of one with S = 10^4: the same attempts, so the rate compares the
    cost per attempt (here the per-round overhead favours the larger S)."""
    clock = FakeClock()

    def cost(s, S):
        return 0.001 + S * 1e-6      # 1 ms of overhead per round + 1 us per attempt

    fake, made = make_fake(clock, cost)
    cands = autotune.candidates((8,), ("rounds",), (0,), S_options=(1000, 10_000))
    best, _, table = autotune.search(
        cands, lambda c: autotune.batch_rate(RUNS, c, rounds=2, make_batch=fake,
                                             sync=lambda: None, timer=clock))
    assert best.S == 10_000
    timed = [b.rounds - 1 for b in made]
    assert timed == [20, 2]
    assert [b.runs[0]["S"] for b in made] == [1000, 10_000]


def test_choice_cached_per_shape():
    autotune.clear_cache()
    calls = []

    def measure(c):
        calls.append(c)
        return float(c.walkers_per_wave)

    s1, _, t1 = autotune.tune(RUNS, P_options=(2, 4), forms=("rounds",), graph_options=(0,),
                              measure=measure)
    n = len(calls)
    assert s1.walkers_per_wave == 4 and len(t1) == 2
    # other seeds and couplings, same shape: cached, nothing measured
    other = [dict(kw, seed=kw["seed"] + 100) for kw in RUNS]
    s2, _, t2 = autotune.tune(other, P_options=(2, 4), forms=("rounds",), graph_options=(0,),
                              measure=measure)
    assert s2 == s1 and t2 == [] and len(calls) == n
    # a different shape is searched again
    bigger = [dict(kw, L=32) for kw in RUNS]
    autotune.tune(bigger, P_options=(2, 4), forms=("rounds",), graph_options=(0,),
                  measure=measure)
    assert len(calls) == 2 * n
    autotune.clear_cache()
