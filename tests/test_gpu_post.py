"""Post-hoc geometric uncertainty on the GPU (ns_geom_uncertainty) against the FP64 oracle.

Both sides draw the same shrinkages (Philox, purpose 6) and evaluate the same expression
log w = beta logL + log X + log1p(-t t') - log 2; they differ in the order of the prefix sums
of log t (sequential in the oracle; chunk sums, scans and per-thread runs on the GPU), in
log(u) / n against log(u) * (1/n), and in the order of the evidence and mean sums.  With
|log X| the size of the prefix, each log weight moves by a few ulp of |log X| times the depth
of the sums, by a few ulp of t t' over 1 - t t' >= ~1/n in the log1p term, and by the
rounding of beta logL + log dX; the mean over R replicas of values of size |log w| adds at most
eps R |log w| / 2 (R additions of partial sums up to R |log w|, divided by R).  The bars:
  - log weights (geometric means):  |d| <= 1e-12 (1 + |log X|) + eps R |log w| + 8 eps n_max,
    with |log X| <= |log w - beta L| + log(2 n_max) bounding the prefix;
  - log Z per replica: the same bound at the largest |log X| and |log w|;
  - Kish ESS: relative 1e-10 (twice the weight error, with room).
"""
import math

import numpy as np
import pytest

from tests import oracle_runs

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def _width(d):
    from oracle import theory as T
    return T.width_whitened(d)


def _compare(O, run, orc, R, beta, seed, run_id):
    """The GPU's geometric uncertainty of its run against the oracle's, computed from the
    oracle's own run of the same problem and seeds (same trajectory: the dead records agree to
    the likelihoods' rounding, which the bars below add as beta |dL|)."""
    dead_o, fin_o, _ = oracle_runs.deaths(orc)
    s = run.state()
    dead_g = run.dead()
    fin_g = np.sort(s["logL"][s["perm"][run.k:]])
    assert len(dead_g) == len(dead_o)
    assert np.allclose(dead_g, dead_o, rtol=1e-10, atol=1e-10)
    assert np.allclose(fin_g, fin_o, rtol=1e-10, atol=1e-10)
    dL = np.abs(np.concatenate([dead_g, fin_g]) - np.concatenate([dead_o, fin_o]))
    g = run.geom(R=R, beta=beta, seed=seed, run_id=run_id)
    z, lw, ess = O.geom(dead_o, fin_o, run.m, run.k, R, beta, seed, run_id)
    L = np.concatenate([dead_o, fin_o])
    assert len(g["logw_mean"]) == len(L)
    tl = np.zeros_like(L) if beta == 0 else beta * L
    scale = 1.0 + np.abs(lw - tl) + math.log(2 * run.m)
    tol = 1e-12 * scale + EPS * R * np.abs(lw) + 8 * EPS * run.m + beta * dL
    fin_w = np.isfinite(lw)
    assert np.array_equal(fin_w, np.isfinite(g["logw_mean"]))
    d = np.abs(g["logw_mean"][fin_w] - lw[fin_w])
    assert np.all(d <= tol[fin_w]), (np.max(d / tol[fin_w]), np.argmax(d / tol[fin_w]))
    ztol = 1e-12 * np.max(scale[fin_w]) + EPS * np.max(np.abs(lw[fin_w])) + 8 * EPS * run.m \
        + beta * np.max(dL)
    assert np.all(np.abs(g["logz"] - z) <= ztol), np.max(np.abs(g["logz"] - z))
    assert abs(g["ess"] - ess) <= 1e-10 * ess + 2 * beta * np.max(dL) * ess, (g["ess"], ess)
    return g, z


_FULL = {}


def _config1_full(O):
    """The oracle's config-1 run (seed 11) to termination, shared by the tests below."""
    if "run" not in _FULL:
        from paper_2601_23252_amd import problems as G
        prob = G.config1()
        _FULL["run"] = oracle_runs.run_iterations(O, prob, prob["m"], prob["k"], prob["p"],
                                                  _width(5), 11, 100_000)[1]
    return _FULL["run"]


@pytest.mark.parametrize("R,beta", [(1, 1.0), (7, 1.0), (100, 1.0), (100, 0.0), (33, 0.37),
                                    (100, 2.5)])
def test_geom_matches_oracle_after_full_run(N, oracle_lib, R, beta):
    """config 1 (d = 5, m = 200, k = 50) run to termination: several chunks of deaths with a
    ragged tail; R = 100 spreads replicas over several groups of workgroups."""
    from paper_2601_23252_amd import problems as G
    run = N.NSRun(G.config1(), width=_width(5), seed=11)
    run.run()
    orc = _config1_full(oracle_lib)
    assert orc.done and run.state()["done"] == 1
    _compare(oracle_lib, run, orc, R, beta, seed=5, run_id=2)
    run.close()


def test_geom_right_after_init_and_edge_counts(N, oracle_lib):
    """Right after initialisation (one accounted batch), k = 1, and a single survivor
    (k = m - 1)."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    for m, k in ((200, 50), (64, 1), (40, 39)):
        run = N.NSRun(prob, m=m, k=k, p=5, width=_width(5), seed=3)
        orc = oracle_lib.Run(oracle_lib.Problem(prob), m, k, 5, _width(5), 3,
                             threads=oracle_runs.THREADS)
        orc.init()
        _compare(oracle_lib, run, orc, 9, 1.0, seed=1, run_id=0)
        for _ in range(6):
            if orc.done:
                break
            orc.step()
            run.step()
        _compare(oracle_lib, run, orc, 9, 1.0, seed=1, run_id=0)
        run.close()


def test_geom_full_size_mixture(N, oracle_lib):
    """The mixture workload at full size (d = 64, m = 2000, k = 1000; chains of 64 steps) after
    40 iterations, R = 100: 41 chunks of deaths per replica."""
    from paper_2601_23252_amd import problems as G
    prob = G.config3()
    run = N.NSRun(prob, p=64, width=_width(64), precision="bf16x3", seed=4)
    for _ in range(40):
        run.step()
    _, orc = oracle_runs.run_iterations(oracle_lib, prob, prob["m"], prob["k"], 64, _width(64),
                                        4, 40)
    g, z = _compare(oracle_lib, run, orc, 100, 1.0, seed=9, run_id=0)
    assert np.std(z) > 0
    run.close()


def test_geom_batch_run_and_truncated_record(N, oracle_lib):
    """A run inside a batch uses its own dead record; a truncated record is refused."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    B = N.NSBatch([(prob, dict(seed=7, run_id=0)), (G.funnel(8, m=100, k=25), dict(seed=7))])
    for _ in range(5):
        B.step()
    s = B.state(1)
    m, k = 100, 25
    dead_n = N.ns_stats_run(B.ctx, 1)[1]["n_dead"]
    g = B.geom(1, R=5, beta=1.0, seed=3)
    assert len(g["logw_mean"]) == dead_n + m - k
    B.close()
    run = N.NSRun(prob, seed=1, max_iter=2)
    for _ in range(4):
        run.step()
    st = N.ns_geom_uncertainty(run.ctx, 0, 4, 1.0, 0, 0)[0]
    assert st == N.NS_ESTATE
    run.close()


def test_posterior_samples_match_oracle(N, oracle_lib):
    """Config 1 run to termination with the dead coordinates recorded: the GPU's posterior
    samples are those the oracle draws from its own run (same deaths; coordinates within FP64
    rounding of the chains)."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    run = N.NSRun(prob, width=_width(5), seed=11, record_points=True)
    run.run()
    x, idx = run.posterior_samples(3000, R=50, beta=1.0, seed=4, run_id=1)
    orc = _config1_full(oracle_lib)
    dead_o, fin_o, finx_o = oracle_runs.deaths(orc)
    n_dead = len(dead_o)
    assert len(run.dead()) == n_dead
    assert np.all((idx >= 0) & (idx < n_dead + len(fin_o)))
    ox, oidx = oracle_lib.posterior_samples(dead_o, orc.dead_x(), fin_o, finx_o, run.m, run.k,
                                            50, 3000, 1.0, seed=4, run_id=1)
    assert np.array_equal(idx, oidx)
    assert np.allclose(x, ox, rtol=1e-10, atol=1e-12)
    # the sampled dead points' coordinates reproduce the oracle's recorded logL
    dmask = idx < n_dead
    L = oracle_lib.Problem(prob).loglik(ox[dmask])
    assert np.array_equal(L, dead_o[idx[dmask]])
    run.close()


def test_posterior_samples_multi_block_scan(N, oracle_lib):
    """Config 2 (m = 1000, k = 500) run to termination: about 57,000 deaths, so the normalised
    cumulative weights span several scan blocks of 8192; the samples equal the oracle's."""
    from paper_2601_23252_amd import problems as G
    prob = G.config2()
    run = N.NSRun(prob, width=_width(32), seed=2, record_points=True)
    run.run()
    _, orc = oracle_runs.run_iterations(oracle_lib, prob, prob["m"], prob["k"], prob["p"],
                                        _width(32), 2, 100_000)
    assert orc.done and run.state()["done"] == 1
    dead_o, fin_o, finx_o = oracle_runs.deaths(orc)
    n_all = len(dead_o) + len(fin_o)
    assert n_all > 3 * 8192
    x, idx = run.posterior_samples(20000, R=20, beta=1.0, seed=6, run_id=0)
    ox, oidx = oracle_lib.posterior_samples(dead_o, orc.dead_x(), fin_o, finx_o, run.m, run.k,
                                            20, 20000, 1.0, seed=6, run_id=0)
    assert np.array_equal(idx, oidx)
    assert np.allclose(x, ox, rtol=1e-10, atol=1e-12)
    assert len(np.unique(idx // 8192)) >= 2   # the samples come from several scan blocks
    run.close()


def test_posterior_samples_need_recorded_points(N):
    from paper_2601_23252_amd import problems as G
    run = N.NSRun(G.config1(), seed=1)
    run.step()
    st, _, _ = N.ns_posterior_samples(run.ctx, 0, 10, 1.0, 0, 0, 100, 5)
    assert st == N.NS_ESTATE
    run.close()
