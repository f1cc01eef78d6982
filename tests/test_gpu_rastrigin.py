"""Gaussian-Rastrigin test likelihood on the GPU against the FP64 oracle, through the C ABI.

Bars: the two sides differ in how cos(2 pi x) is formed (the oracle reduces x to the nearest
integer first, the GPU uses cospi(2x)), in summation order and in libm against device math,
each a few ulp per coordinate, scaled by A = 10 in the Rastrigin term:
  - likelihood values: |d log L| <= 1e-12 (1 + |log L|) + 1e-14 A d;
  - per-iteration state on identical Philox streams: identical parents, deleted order,
    evaluation counts and per-step decision traces; points and logL within 1e-10 relative;
  - end to end (d = 2, 4): identical stop iteration, |d ln Z| <= 1e-9, and ln Z within
    3.5 sigma of the semi-analytic evidence (Bessel-function one-dimensional integrals).
"""
import math

import numpy as np
import pytest

from tests import oracle_runs, truth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def _width(d):
    from oracle import theory as T
    return T.width_whitened(d)


@pytest.mark.parametrize("d,alpha", [(1, 0.5), (2, 0.0), (10, 0.3), (33, 1.0), (100, 0.5),
                                     (128, 0.0), (129, 0.7), (300, 0.5)])
def test_rastrigin_loglik_matches_oracle(N, oracle_lib, d, alpha):
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(d, alpha, m=64, k=16)
    rng = np.random.default_rng(d)
    X = rng.uniform(-5.14, 5.14, (200, d))
    X[:50] = np.round(X[:50]) + 0.05 * rng.standard_normal((50, d))   # near the lattice
    X[50:60] = 0.0
    R = N.NSRun(prob, m=64, k=16, p=1, seed=0)
    g = R.eval_loglik(X, "fp64")
    o = oracle_lib.Problem(prob).loglik(X)
    tol = 1e-12 * (1 + np.abs(o)) + 1e-14 * 10 * d
    assert np.all(np.abs(g - o) <= tol), np.max(np.abs(g - o) / tol)
    R.close()


def _parity(N, O, prob, m, k, p, seed, n_iter):
    width = _width(prob["d"])
    orc = O.Run(O.Problem(prob), m, k, p, width, seed, threads=8)
    orc.init()
    gpu = N.NSRun(prob, m=m, k=k, p=p, width=width, seed=seed, trace=True)
    g, o = gpu.state(), orc.state()
    assert np.array_equal(g["perm"], o["perm"])
    done_o = orc.done
    for it in range(n_iter):
        if done_o:
            break
        done_o = orc.step()
        done_g = gpu.step()
        g, o = gpu.state(), orc.state()
        _, par_o = orc.aux()
        assert np.array_equal(g["parents"], par_o), f"iter {it}: parents"
        assert np.array_equal(g["perm"], o["perm"]), f"iter {it}: delete-k order"
        assert np.allclose(g["x"], o["x"], rtol=1e-10, atol=1e-12), f"iter {it}: points"
        assert np.allclose(g["logL"], o["logL"], rtol=1e-10, atol=1e-10), f"iter {it}: logL"
        sg = gpu.stats()
        assert sg["evals"] == o["evals"] and sg["tests"] == o["tests"], f"iter {it}: counts"
        assert done_g == done_o
    return gpu, orc


def test_rastrigin_parity_d10(N, oracle_lib):
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(10, 0.3)
    _parity(N, oracle_lib, prob, m=200, k=50, p=50, seed=4, n_iter=8)


@pytest.mark.parametrize("d,alpha", [(2, 0.0), (2, 0.5), (4, 0.1)])
def test_rastrigin_end_to_end_lnz(N, oracle_lib, d, alpha):
    """Whole runs, GPU against the oracle iteration by iteration, then ln Z against the
    semi-analytic evidence."""
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(d, alpha, m=500, k=100)
    gpu, orc = _parity(N, oracle_lib, prob, m=500, k=100, p=5 * d, seed=7, n_iter=100_000)
    assert gpu.state()["done"] == 1
    zg, eg, _ = gpu.logz()
    zo, _, _ = orc.logz()
    assert abs(zg - zo) <= 1e-9
    tz = truth.lnz_rastrigin_gauss(d, alpha)
    assert abs(zg - tz) < 3.5 * eg, (zg, tz, eg)


def _sampled_chains(N, O, prob, seed, chains):
    """The first iteration at full size against the oracle's: every new point and logL, and
    the sampled chains' decision traces recomputed from the oracle's own state, whitening and
    parents."""
    width = _width(prob["d"])
    gpu = N.NSRun(prob, width=width, seed=seed, trace=True)
    s0 = gpu.state()
    gpu.step()
    s1 = gpu.state()
    tr = gpu.trace()
    P, _, o0, o1, Ls_o, par_o = oracle_runs.first_iteration(O, prob, prob["m"], prob["k"],
                                                            prob["p"], width, seed)
    assert np.array_equal(s0["perm"], o0["perm"])
    assert np.array_equal(s1["parents"], par_o)
    assert np.allclose(s1["x"], o1["x"], rtol=1e-10, atol=1e-12)
    assert np.allclose(s1["logL"], o1["logL"], rtol=1e-10, atol=1e-10)
    for j in chains:
        parent = par_o[j]
        x, logL, _, trace = P.hrss_chain(o0["x"][parent], o0["logL"][parent], o0["Lstar"],
                                         Ls_o, width, prob["p"], seed, 0, 1, j, trace=True)
        slot = o0["perm"][j]
        assert np.array_equal(tr[j], trace), f"chain {j}: decisions"
        assert np.allclose(s1["x"][slot], x, rtol=1e-10, atol=1e-12), f"chain {j}"
        assert math.isclose(s1["logL"][slot], logL, rel_tol=1e-10, abs_tol=1e-10)
    gpu.close()


def test_rastrigin_full_size_d100_sampled_chains(N, oracle_lib):
    """d = 100, 1000 live points, k = 500, p = 25 d."""
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(100, 0.5)
    _sampled_chains(N, oracle_lib, prob, 3, (0, 137, prob["k"] - 1))


def test_rastrigin_parity_d150(N, oracle_lib):
    """d = 150 runs on the padded-320 kernels (global-memory Cholesky, 32-row direction
    blocks, five coordinates per lane): per-iteration parity with the oracle.  The survivors
    (300) outnumber the dimensions, so the whitening covariance is well conditioned."""
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(150, 0.5)
    _parity(N, oracle_lib, prob, m=400, k=100, p=30, seed=4, n_iter=4)


def test_rastrigin_full_size_d300_sampled_chains(N, oracle_lib):
    """d = 300 (the largest dimension of the paper's comparison), 1000 live points, k = 500,
    300 steps per chain."""
    from paper_2601_23252_amd import problems as G
    prob = G.rastrigin_gauss(300, 0.5, p=300)
    _sampled_chains(N, oracle_lib, prob, 5, (0, 250, prob["k"] - 1))
