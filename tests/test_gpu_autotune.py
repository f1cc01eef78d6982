"""NS_FLAG_AUTOTUNE: the launch shape of each kernel group's chains chosen by timing (chains
per workgroup 1..4, and for mixture chains in a 16-bit mode the tests planned per round:
4, 8 or 16), at the context's iterations 0, 32 and 96, ranked by summed time.

Every candidate is timed on the same iteration (the state the chains change is saved and
restored around each timed launch), and a chain's decisions and arithmetic do not depend on
the launch shape, so a tuned run must equal the untuned run bit for bit (points, logL,
evidence, iteration count); the tuner must actually time its candidates at each point the run
reaches (counted launches) and a later context of the same shape must reuse the choice
without timing anything.
"""

TUNE_AT = (0, 32, 96)


def _points(iterations):
    """Tuning points a run of this many iterations reaches (at most: the third is skipped when
    the leader is clear after two)."""
    return sum(a < iterations for a in TUNE_AT)


def _points_ok(launches, per_point, iterations):
    """The launches match the points reached, the later ones possibly skipped once the leader
    was clear: per_point times a count between 1 and the points reached."""
    n = _points(iterations)
    return launches % per_point == 0 and 1 <= launches // per_point <= n
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


@pytest.fixture(autouse=True)
def empty_cache(N):
    """Every test starts with an empty process-wide tuning cache."""
    assert N.ns_tune_clear()[0] == N.NS_OK
    yield
    N.ns_tune_clear()


def _same_state(a, b):
    sa, sb = a.state(), b.state()
    assert sa["iter"] == sb["iter"]
    assert np.array_equal(sa["perm"], sb["perm"])
    assert np.array_equal(sa["x"], sb["x"])
    assert np.array_equal(sa["logL"], sb["logL"])
    assert sa["logZ"] == sb["logZ"] and sa["logX"] == sb["logX"]


def test_autotune_config1_full_run_identical(N):
    """config 1 (k = 50, FP64: 4 candidates, 2 timed launches each per point): the tuned run
    equals the untuned one, timing at every tuning point the run reaches; a second context of
    the same shape starts with the cached choice and times nothing."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    a = N.NSRun(prob, seed=5, autotune=True)
    b = N.NSRun(prob, seed=5)
    assert b.chains_per_workgroup() == 1   # the rule: ceil(50 / 256)
    a.step()
    b.step()
    assert a.stats()["tune_launches"] == 8
    _same_state(a, b)
    ia, ib = a.run(), b.run()
    assert ia == ib
    _same_state(a, b)
    assert a.logz() == b.logz()
    n_it = a.state()["iter"]
    assert n_it > 32
    assert _points_ok(a.stats()["tune_launches"], 8, n_it)
    c, plan = a.launch_shape()
    assert 1 <= c <= 4 and plan == 4
    again = N.NSRun(prob, seed=6, autotune=True)
    assert again.launch_shape() == (c, plan)
    again.step()
    assert again.stats()["tune_launches"] == 0
    for r in (a, b, again):
        r.close()


def test_autotune_mixture_full_size_identical(N):
    """The d = 64 mixture (k = 1000, BF16x3, chains of 64 steps): 12 candidates (chains per
    workgroup x 4, 8 or 16 planned tests), ten iterations equal to the untuned ones."""
    from paper_2601_23252_amd import problems as G
    prob = G.config3()
    a = N.NSRun(prob, p=64, seed=2, precision="bf16x3", autotune=True)
    b = N.NSRun(prob, p=64, seed=2, precision="bf16x3")
    assert b.launch_shape() == (4, 16)
    for _ in range(10):
        a.step()
        b.step()
    _same_state(a, b)
    assert a.stats()["evals"] == b.stats()["evals"]
    assert a.stats()["tune_launches"] == 24
    c, plan = a.launch_shape()
    assert 1 <= c <= 4 and plan in (4, 8, 16)
    a.close()
    b.close()


def test_autotune_batch_with_graphs_identical(N):
    """Two kernel groups (a d = 8 Gaussian and d = 16 funnels) in one batch, with HIP graphs:
    every run's evidence equals the untuned batch's."""
    from paper_2601_23252_amd import problems as G
    runs = [(G.config2(3, d=8, m=120, k=40), dict(seed=1, run_id=0)),
            (G.funnel(16, m=100, k=30), dict(seed=1, run_id=1)),
            (G.funnel(16, m=90, k=45), dict(seed=2, run_id=2))]
    tuned = N.NSBatch([(p, dict(kw, autotune=True, graph=True)) for p, kw in runs])
    plain = N.NSBatch([(p, dict(kw, graph=True)) for p, kw in runs])
    tuned.run()
    plain.run()
    zt, zp = tuned.logz(), plain.logz()
    for r in range(3):
        assert zt[0][r] == zp[0][r] and zt[2][r] == zp[2][r]
        st, sp = tuned.state(r), plain.state(r)
        assert np.array_equal(st["x"], sp["x"]) and st["iter"] == sp["iter"]
        assert 1 <= N.ns_chains_per_workgroup(tuned.ctx, r) <= 4
    # two groups, 4 candidates, 2 launches each, at every point a group's runs reach
    tl = tuned.stats(0)["tune_launches"]
    assert tl >= 16 and tl % 8 == 0
    assert tl <= 16 * _points(max(tuned.state(r)["iter"] for r in range(3)))  # an upper bound
    tuned.close()
    plain.close()


@pytest.mark.parametrize("kw", [dict(outer="smc", m=300, p=10), dict(replacement="rw", p=20)])
def test_autotune_smc_and_random_walk_identical(N, kw):
    """The tempered-SMC outer loop and the random-walk replacement under the tuner: ten
    iterations (the first one tuning) equal the untuned ones."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    a = N.NSRun(prob, seed=9, autotune=True, **kw)
    b = N.NSRun(prob, seed=9, **kw)
    for _ in range(10):
        da = a.step()
        db = b.step()
        assert da == db
        if da:
            break
    _same_state(a, b)
    assert a.stats()["evals"] == b.stats()["evals"]
    assert a.stats()["tune_launches"] == 8
    assert 1 <= a.chains_per_workgroup() <= 4
    a.close()
    b.close()


def test_autotune_cache_file_is_used(N, tmp_path):
    """A tuning cache written and loaded back: a context of a cached shape starts with the
    cached launch shape and times nothing (its result equals the plain run's)."""
    import json
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    path = tmp_path / "tune.json"
    # config 1's shape in FP64: padded dimension 32, mixture, 1 fragment unit, slice sampling
    entry = dict(D=32, lik=1, mode=0, upw=1, rw=0, chains=50, planned=0, C=3, plan=0)
    path.write_text('{"nss_tune": 2, "entries": [\n  ' + json.dumps(entry) + "\n]}\n")
    assert N.ns_tune_load(path)[0] == N.NS_OK
    a = N.NSRun(prob, seed=4, autotune=True)
    assert a.chains_per_workgroup() == 3
    b = N.NSRun(prob, seed=4)
    for _ in range(3):
        a.step()
        b.step()
    _same_state(a, b)
    assert a.chains_per_workgroup() == 3
    assert a.stats()["tune_launches"] == 0
    st, n = N.ns_tune_save(tmp_path / "saved.json")
    assert st == N.NS_OK and n >= 1
    saved = json.loads((tmp_path / "saved.json").read_text())
    assert entry in saved["entries"]
    a.close()
    b.close()


def test_autotune_points_follow_the_schedule(N):
    """The d = 32 correlated Gaussian in BF16x3 (4 candidates per point, or 12 where the plan
    kernel applies): timing happens only at iterations 0, 32 and 96 (the later points skipped
    once the leader is clear), and the run equals the untuned one throughout."""
    from paper_2601_23252_amd import problems as G
    prob = G.config2()
    a = N.NSRun(prob, p=32, seed=3, precision="bf16x3", autotune=True)
    b = N.NSRun(prob, p=32, seed=3, precision="bf16x3")
    per_point = None
    prev = 0
    for it in range(100):
        da = a.step()
        assert b.step() == da
        tl = a.stats()["tune_launches"]
        if it == 0:
            per_point = tl
            assert per_point in (8, 24)
        assert _points_ok(tl, per_point, it + 1), f"iteration {it}"
        # points are only ever taken at the scheduled iterations
        if it + 1 not in (1, 33, 97):
            assert tl == prev, f"iteration {it}: timing outside the schedule"
        prev = tl
        if da:
            break
    assert it >= 96
    _same_state(a, b)
    a.close()
    b.close()
