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

pytestmark = pytest.mark.gpu

EPS = np.finfo(float).eps


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def _deaths(run):
    s = run.state()
    k = run.k
    fin = s["logL"][s["perm"][k:]]
    return run.dead(), fin


def _compare(O, run, R, beta, seed, run_id):
    dead, fin = _deaths(run)
    g = run.geom(R=R, beta=beta, seed=seed, run_id=run_id)
    z, lw, ess = O.geom(dead, fin, run.m, run.k, R, beta, seed, run_id)
    L = np.concatenate([dead, np.sort(fin)])
    assert len(g["logw_mean"]) == len(L)
    tl = np.zeros_like(L) if beta == 0 else beta * L
    scale = 1.0 + np.abs(lw - tl) + math.log(2 * run.m)
    tol = 1e-12 * scale + EPS * R * np.abs(lw) + 8 * EPS * run.m
    fin_w = np.isfinite(lw)
    assert np.array_equal(fin_w, np.isfinite(g["logw_mean"]))
    d = np.abs(g["logw_mean"][fin_w] - lw[fin_w])
    assert np.all(d <= tol[fin_w]), (np.max(d / tol[fin_w]), np.argmax(d / tol[fin_w]))
    ztol = 1e-12 * np.max(scale[fin_w]) + EPS * np.max(np.abs(lw[fin_w])) + 8 * EPS * run.m
    assert np.all(np.abs(g["logz"] - z) <= ztol), np.max(np.abs(g["logz"] - z))
    assert abs(g["ess"] - ess) <= 1e-10 * ess, (g["ess"], ess)
    return g, z


@pytest.mark.parametrize("R,beta", [(1, 1.0), (7, 1.0), (100, 1.0), (100, 0.0), (33, 0.37),
                                    (100, 2.5)])
def test_geom_matches_oracle_after_full_run(N, oracle_lib, R, beta):
    """config 1 (d = 5, m = 200, k = 50) run to termination: several chunks of deaths with a
    ragged tail; R = 100 spreads replicas over several groups of workgroups."""
    from paper_2601_23252_amd import problems as G
    run = N.NSRun(G.config1(), seed=11)
    run.run()
    _compare(oracle_lib, run, R, beta, seed=5, run_id=2)
    run.close()


def test_geom_right_after_init_and_edge_counts(N, oracle_lib):
    """Right after initialisation (one accounted batch), k = 1, and a single survivor
    (k = m - 1)."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    for m, k in ((200, 50), (64, 1), (40, 39)):
        run = N.NSRun(prob, m=m, k=k, p=5, seed=3)
        _compare(oracle_lib, run, 9, 1.0, seed=1, run_id=0)
        for _ in range(6):
            run.step()
        _compare(oracle_lib, run, 9, 1.0, seed=1, run_id=0)
        run.close()


def test_geom_full_size_mixture(N, oracle_lib):
    """The mixture workload at full size (d = 64, m = 2000, k = 1000) after 40 iterations,
    R = 100: tens of chunks per replica."""
    from paper_2601_23252_amd import problems as G
    run = N.NSRun(G.config3(), precision="bf16x3", seed=4)
    for _ in range(40):
        run.step()
    g, z = _compare(oracle_lib, run, 100, 1.0, seed=9, run_id=0)
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
    samples are the oracle's (same deaths, coordinates within FP64 rounding); the recorded
    coordinates reproduce the dead record's logL."""
    from paper_2601_23252_amd import problems as G
    prob = G.config1()
    run = N.NSRun(prob, seed=11, record_points=True)
    run.run()
    s = run.state()
    dead = run.dead()
    x, idx = run.posterior_samples(3000, R=50, beta=1.0, seed=4, run_id=1)
    k = run.k
    fin = s["perm"][k:]
    n_dead = len(dead)
    assert np.all((idx >= 0) & (idx < n_dead + len(fin)))
    # the dead rows among the samples reproduce their recorded logL
    dmask = idx < n_dead
    L = oracle_lib.Problem(prob).loglik(x[dmask])
    assert np.allclose(L, dead[idx[dmask]], rtol=1e-12, atol=1e-12)
    # the oracle, fed the GPU's deaths and coordinates, draws the same samples
    dead_x = np.zeros((n_dead, prob["d"]))
    dead_x[idx[dmask]] = x[dmask]
    ox, oidx = oracle_lib.posterior_samples(dead, dead_x, s["logL"][fin], s["x"][fin], run.m, k,
                                            50, 3000, 1.0, seed=4, run_id=1)
    assert np.array_equal(idx, oidx)
    assert np.allclose(x, ox, rtol=0, atol=0)
    run.close()


def test_posterior_samples_need_recorded_points(N):
    from paper_2601_23252_amd import problems as G
    run = N.NSRun(G.config1(), seed=1)
    run.step()
    st, _, _ = N.ns_posterior_samples(run.ctx, 0, 10, 1.0, 0, 0, 100, 5)
    assert st == N.NS_ESTATE
    run.close()
