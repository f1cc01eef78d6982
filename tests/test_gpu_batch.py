"""Batched serving of independent runs (ns_init_batch) on the GPU, through the C ABI.

Bars:
  - a run inside a batch follows exactly the trajectory it has alone: identical iteration
    count, deleted order and evaluation counts, and bit-identical ln Z (the same kernels do the
    same arithmetic on the same Philox counters; only the launch grouping differs);
  - against the FP64 oracle: end to end |d logZ| <= 1e-9 with identical iteration counts for
    small runs, and at the full batched-serving size (256 runs of d in {8..128}, n_live=500,
    k=250) the state after one iteration of a stratified subset of 16 runs (identical parents
    and deleted order, points and logL within 1e-10 relative).
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def _small_batch():
    from paper_2601_23252_amd import problems as G
    from oracle import theory as T
    runs = [
        (G.config1(), dict(seed=3, run_id=0)),
        (G.config2(7, d=24, m=200, k=100), dict(seed=3, run_id=1, precision="bf16x3")),
        (G.funnel(8, m=100, k=50), dict(seed=4, run_id=2)),
        (G.funnel(40, m=120, k=60), dict(seed=4, run_id=3)),
        (G.mixture_problem(5, 70, 2, m=200, k=100), dict(seed=5, run_id=4, precision="fp16x3")),
        (G.config1(), dict(seed=3, run_id=9, width=T.width_whitened(5))),
        (G.config2(8, d=48, m=150, k=149), dict(seed=6, run_id=5)),
    ]
    return runs


def test_batch_runs_equal_single_runs(N):
    runs = _small_batch()
    B = N.NSBatch(runs)
    assert N.ns_num_runs(B.ctx) == len(runs)
    B.run()
    zb, eb, hb = B.logz()
    for r, (prob, kw) in enumerate(runs):
        kw = dict(kw)
        S = N.NSRun(prob, **kw)
        it = S.run()
        zs, es, hs = S.logz()
        sb, ss = B.state(r), S.state()
        assert sb["done"] == 1 and ss["done"] == 1, r
        assert sb["iter"] == ss["iter"], (r, sb["iter"], ss["iter"], it)
        assert np.array_equal(sb["perm"], ss["perm"]), r
        assert np.array_equal(sb["logL"], ss["logL"]), r
        assert zb[r] == zs and eb[r] == es and hb[r] == hs, (r, zb[r], zs)
        stb, sts = B.stats(r), S.stats()
        for key in ("evals", "tests", "prior_rejects", "stepout_caps", "shrink_caps",
                    "rechecks", "n_dead"):
            assert stb[key] == sts[key], (r, key, stb[key], sts[key])
        S.close()
    B.close()


def test_batch_step_and_reset(N):
    """ns_step advances every unfinished run by one iteration; ns_reset restarts run r with
    (seed, run_id + r)."""
    runs = _small_batch()[:3]
    B = N.NSBatch(runs)
    B.step()
    for r in range(len(runs)):
        assert B.state(r)["iter"] == 1
    B.reset(11, 20)
    B.step()
    B.step()
    for r, (prob, kw) in enumerate(runs):
        kw = dict(kw, seed=11, run_id=20 + r)
        S = N.NSRun(prob, **kw)
        S.step()
        S.step()
        sb, ss = B.state(r), S.state()
        assert sb["iter"] == ss["iter"] == 2
        assert np.array_equal(sb["perm"], ss["perm"])
        assert np.array_equal(sb["x"], ss["x"])
        S.close()
    B.close()


def test_batch_end_to_end_matches_oracle(N, O):
    from oracle import theory as T
    from paper_2601_23252_amd import problems as G
    probs = [G.config1(), G.funnel(4, m=80, k=40), G.config2(9, d=6, m=100, k=30)]
    runs = [(p, dict(seed=21, run_id=r, width=T.width_whitened(p["d"])))
            for r, p in enumerate(probs)]
    B = N.NSBatch(runs)
    B.run()
    zb, _, _ = B.logz()
    for r, p in enumerate(probs):
        o = O.Run(O.Problem(p), p["m"], p["k"], p["p"], T.width_whitened(p["d"]), 21, run_id=r,
                  threads=8)
        o.init()
        it = o.run()
        zo, _, _ = o.logz()
        assert B.state(r)["iter"] == o.state()["iter"], (r, it)
        assert abs(zb[r] - zo) <= 1e-9, (r, zb[r], zo)
    B.close()


def _config5_runs(precision_gauss):
    from oracle import theory as T
    from paper_2601_23252_amd import problems as G
    probs = G.config5()
    runs = [(p, dict(seed=5, run_id=r, precision=precision_gauss if p["lik"] == "mixture"
                     else "fp64", max_iter=3000, width=T.width_whitened(p["d"])))
            for r, p in enumerate(probs)]
    return probs, runs


def _stratified(probs, n=16):
    """n runs spread over dimension and likelihood: sort by (lik, d) and take evenly spaced."""
    order = sorted(range(len(probs)), key=lambda r: (probs[r]["lik"], probs[r]["d"], r))
    idx = np.linspace(0, len(order) - 1, n).round().astype(int)
    return [order[i] for i in idx]


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_config5_full_size_first_iteration_matches_oracle(N, O, prec):
    from oracle import theory as T
    probs, runs = _config5_runs(prec)
    print(f"[config5] 256 runs, Gaussians in {prec}", flush=True)
    B = N.NSBatch(runs)
    B.step()
    for r in _stratified(probs):
        p = probs[r]
        print(f"[config5] run {r}: {p['name']}", flush=True)
        o = O.Run(O.Problem(p), p["m"], p["k"], p["p"], T.width_whitened(p["d"]), 5, run_id=r,
                  threads=8)
        o.init()
        o.step()
        g, s = B.state(r), o.state()
        assert g["iter"] == s["iter"] == 1
        assert np.array_equal(g["parents"], o.aux()[1]), r
        assert np.array_equal(g["perm"], s["perm"]), r
        assert np.allclose(g["x"], s["x"], rtol=1e-10, atol=1e-12), r
        assert np.allclose(g["logL"], s["logL"], rtol=1e-10, atol=1e-10), r
        assert abs(g["logZ"] - s["logZ"]) <= 1e-12 * abs(s["logZ"]) + 1e-12, r
    B.close()


def test_graph_replay_matches_eager(N):
    """NS_FLAG_GRAPH: batches of 16 iterations captured once per block-map epoch and replayed
    (with host copies and synchronisation between replays) give the eager trajectories bit for
    bit, through several re-captures as runs finish."""
    runs = _small_batch()
    A = N.NSBatch(runs)
    G = N.NSBatch([(p, dict(kw, graph=True)) for p, kw in runs])
    A.run()
    G.run()
    za, _, _ = A.logz()
    zg, _, _ = G.logz()
    assert np.array_equal(za, zg)
    for r in range(len(runs)):
        sa, sg = A.state(r), G.state(r)
        assert sa["iter"] == sg["iter"]
        assert np.array_equal(sa["perm"], sg["perm"]) and np.array_equal(sa["x"], sg["x"])
    # a second run on the same contexts replays the cached graphs of the first epochs
    A.reset(31)
    G.reset(31)
    A.run()
    G.run()
    assert np.array_equal(A.logz()[0], G.logz()[0])
    A.close()
    G.close()


@pytest.mark.parametrize("graph", [False, True])
def test_concurrent_groups_equal_serial_groups(N, graph):
    """The small batch compiles to several chain kernels; launched concurrently on side streams
    (the default, eager iterations) or one after the other (NS_FLAG_SERIAL_GROUPS, and every
    graph-captured iteration), every run's trajectory is the same bit for bit."""
    runs = _small_batch()
    Sr = N.NSBatch([(p, dict(kw, serial_groups=True, graph=graph)) for p, kw in runs])
    Cc = N.NSBatch([(p, dict(kw, graph=graph)) for p, kw in runs])
    Sr.run()
    Cc.run()
    assert np.array_equal(Sr.logz()[0], Cc.logz()[0])
    for r in range(len(runs)):
        a, b = Sr.state(r), Cc.state(r)
        assert a["iter"] == b["iter"] and a["done"] == b["done"] == 1
        assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["logL"], b["logL"])
        assert Sr.stats(r)["evals"] == Cc.stats(r)["evals"]
    Sr.close()
    Cc.close()


def test_dead_record_growth_in_a_graph_batch(N):
    """A batch with graphs in which one run (config 1 at k = 2, ~1,700 iterations) outgrows its
    dead record's initial 512 iterations while another finishes early: every run's evidence,
    death count and post-hoc replicas over the whole dead record equal its single run's (the
    growth replaces the record between graph replays; the kernels read its address from the
    run's descriptor)."""
    from paper_2601_23252_amd import problems as G
    from oracle import theory as T
    w = T.width_whitened(5)
    runs = [(G.config1(), dict(k=2, p=10, width=w, seed=3, run_id=0, graph=True)),
            (G.funnel(8, m=100, k=50), dict(seed=4, run_id=1, graph=True))]
    B = N.NSBatch(runs)
    B.run()
    for r, (prob, kw) in enumerate(runs):
        S = N.NSRun(prob, **{a: b for a, b in kw.items() if a != "graph"})
        S.run()
        assert B.state(r)["iter"] == S.state()["iter"]
        assert B.logz()[0][r] == S.logz()[0]
        assert B.stats(r)["n_dead"] == S.stats()["n_dead"]
        gb, gs = B.geom(r, R=8, seed=2, run_id=0), S.geom(R=8, seed=2, run_id=0)
        assert np.array_equal(gb["logz"], gs["logz"])   # over the whole dead record
        S.close()
    assert B.state(0)["iter"] > 1024
    B.close()
