"""Edge cases of the GPU path against the FP64 oracle, through the C ABI, from injected states
(ns_set_state on the GPU, the same state in the oracle): ties at the threshold, a total plateau,
NaN / +inf stored log-likelihoods and a singular survivor set (the whitening fallback).

Bars as in the per-iteration parity tests: identical delete-k order, parents and counters;
points and logL within 1e-10 relative; L*, ln Z, ln X within 1e-12 relative.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

D, M, K, P_STEPS, SEED = 5, 40, 10, 10, 13


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def _prob():
    from paper_2601_23252_amd import problems as G
    return G.gaussian_problem(D, np.zeros(D), 0.01 * np.eye(D), "box", -1.0, 1.0, m=M, k=K)


def _width():
    from oracle import theory as T
    return T.width_whitened(D)


def _pair(N, O, x, logL, it=3, logZ=-7.0, logX=-2.0, Mv=-3.0):
    """An oracle run and a GPU run holding the same injected state."""
    prob = _prob()
    orc = O.Run(O.Problem(prob), M, K, P_STEPS, _width(), SEED, term_frac=0.0)
    orc.init()
    orc.set_state(x, logL, logZ, logX, Mv, it)
    gpu = N.NSRun(prob, width=_width(), seed=SEED, p=P_STEPS, term_frac=0.0, trace=True)
    gpu.set_state(x, logL, logZ, logX, Mv, it)
    return orc, gpu


def _cmp(g, o, label):
    assert np.array_equal(g["perm"], o["perm"]), label
    assert np.allclose(g["x"], o["x"], rtol=1e-10, atol=1e-12), label
    assert np.array_equal(np.isneginf(g["logL"]), np.isneginf(o["logL"])), label
    f = np.isfinite(o["logL"])
    assert np.allclose(g["logL"][f], o["logL"][f], rtol=1e-10, atol=1e-10), label
    for key in ("Lstar", "logZ", "logX", "M"):
        if math.isinf(o[key]):
            assert g[key] == o[key], (label, key)
        else:
            assert math.isclose(g[key], o[key], rel_tol=1e-12, abs_tol=1e-11), (label, key)
    assert g["iter"] == o["iter"], label


def _base_state(O):
    prob = _prob()
    orc = O.Run(O.Problem(prob), M, K, P_STEPS, _width(), SEED)
    orc.init()
    s = orc.state()
    return s["x"].copy(), s["logL"].copy()


def _steps(N, O, orc, gpu, n, label):
    _cmp(gpu.state(), orc.state(), f"{label}: injected")
    for it in range(n):
        orc.step()
        gpu.step()
        g, o = gpu.state(), orc.state()
        _, par = orc.aux()
        assert np.array_equal(g["parents"], par), f"{label} iter {it}: parents"
        _cmp(g, o, f"{label} iter {it}")
        sg = gpu.stats()
        assert sg["evals"] == o["evals"] and sg["tests"] == o["tests"], f"{label} iter {it}"
        assert sg["nonfinite"] == o["nonfinite"], f"{label} iter {it}"


def test_ties_at_the_threshold(N, oracle_lib):
    """Sec. 3.1: survivors tied with the k-th worst point get no parent weight (strict
    threshold); the tie is broken by index in the delete-k order."""
    O = oracle_lib
    x, logL = _base_state(O)
    order = np.argsort(logL, kind="stable")
    tied = logL.copy()
    tied[order[K:K + 6]] = logL[order[K - 1]]       # six survivors tie with L*
    tied[order[2]] = tied[order[3]]                 # and two of the deleted points tie
    orc, gpu = _pair(N, O, x, tied)
    st = gpu.state()
    assert st["Lstar"] == logL[order[K - 1]]
    _steps(N, O, orc, gpu, 3, "ties")
    gpu.close()


def test_first_step_parents_skip_tied_survivors(N, oracle_lib):
    O = oracle_lib
    x, logL = _base_state(O)
    order = np.argsort(logL, kind="stable")
    tied = logL.copy()
    tied[order[K:K + 6]] = logL[order[K - 1]]
    orc, gpu = _pair(N, O, x, tied)
    s0 = gpu.state()
    gpu.step()
    orc.step()
    par = gpu.state()["parents"]
    assert np.all(tied[par] > s0["Lstar"])
    assert np.array_equal(par, orc.aux()[1])
    gpu.close()


def test_total_plateau_is_a_state_error(N, oracle_lib):
    """Every live point at the same log L: no survivor lies strictly above L*, so no parent
    exists; the GPU step returns NS_ESTATE and the oracle refuses the step."""
    O = oracle_lib
    x, _ = _base_state(O)
    flat = np.full(M, -4.25)
    orc, gpu = _pair(N, O, x, flat)
    with pytest.raises(RuntimeError):
        orc.step()
    with pytest.raises(N.NSError) as e:
        gpu.step()
    assert e.value.status == N.NS_ESTATE
    gpu.close()


def test_nonfinite_stored_loglik_is_rejected_and_counted(N, oracle_lib):
    """NaN and +inf log L are taken as -inf (rejected), die first and are counted; the run
    then continues exactly as the oracle's."""
    O = oracle_lib
    x, logL = _base_state(O)
    bad = logL.copy()
    bad[[3, 17, 29]] = np.nan
    bad[[8, 35]] = np.inf
    orc, gpu = _pair(N, O, x, bad)
    assert gpu.stats()["nonfinite"] == 5 == orc.state()["nonfinite"]
    st = gpu.state()
    assert set(st["perm"][:5].tolist()) == {3, 8, 17, 29, 35}
    _steps(N, O, orc, gpu, 3, "nonfinite")
    dg, do = gpu.dead(), orc.dead()
    assert np.allclose(dg, do, rtol=1e-10, atol=1e-10)
    gpu.close()


def test_nonfinite_loglik_from_evaluation_is_rejected(N):
    """A non-finite coordinate evaluates to -inf, not NaN (the evaluator's sanitising)."""
    prob = _prob()
    gpu = N.NSRun(prob, width=_width(), seed=SEED, p=P_STEPS)
    x = np.zeros((4, D))
    x[1, 2] = np.nan
    x[2, 0] = np.inf
    out = gpu.eval_loglik(x, "fp64")
    assert np.isfinite(out[0]) and np.isfinite(out[3])
    assert np.isneginf(out[1]) and np.isneginf(out[2])
    gpu.close()


def test_singular_survivors_take_the_diagonal_fallback(N, oracle_lib):
    """Every survivor at one point: the covariance is zero (its jitter too), the factorisation
    fails and the whitening falls back to the diagonal (unit where a variance is zero); counted
    once per failed factorisation."""
    O = oracle_lib
    x, logL = _base_state(O)
    order = np.argsort(logL, kind="stable")
    xs = x.copy()
    xs[order[K:]] = x[order[-1]]
    orc, gpu = _pair(N, O, xs, logL)
    orc.step()
    gpu.step()
    Ls_o, par = orc.aux()
    g = gpu.state()
    assert np.array_equal(Ls_o, np.eye(D))
    assert np.array_equal(g["Lsig"], np.eye(D))
    assert gpu.stats()["whiten_fallbacks"] == 1
    assert np.array_equal(g["parents"], par)
    _cmp(g, orc.state(), "fallback")
    gpu.close()


def test_dead_record_grows_past_its_initial_size(N, oracle_lib):
    """A run of ~1,400 iterations (config 1 with k = 2) outgrows the dead record's initial 512
    iterations twice; the whole record equals the oracle's, and posterior samples drawn over it
    (the dead points' coordinates, grown alongside) are the oracle's.  With max_iter = 600 the
    record stops at 601 iterations: its stored part still equals the oracle's and the
    geometric-uncertainty call reports the truncation."""
    from paper_2601_23252_amd import problems as G
    from oracle import theory as T
    from tests import oracle_runs
    prob = G.config1()
    w = T.width_whitened(5)
    orc = oracle_lib.Run(oracle_lib.Problem(prob), 200, 2, 10, w, 3, threads=8)
    orc.init()
    orc.run()
    gpu = N.NSRun(prob, k=2, p=10, width=w, seed=3, record_points=True)
    gpu.run()
    it = gpu.state()["iter"]
    assert it == orc.state()["iter"] and it > 1024
    dg, do = gpu.dead(), orc.dead()
    assert dg.shape == do.shape == (2 * (it + 1),)
    assert np.allclose(dg, do, rtol=1e-10, atol=1e-10)
    assert abs(gpu.logz()[0] - orc.logz()[0]) <= 1e-9
    x, idx = gpu.posterior_samples(2000, R=10, beta=1.0, seed=2, run_id=0)
    dead_o, fin_o, finx_o = oracle_runs.deaths(orc)
    ox, oidx = oracle_lib.posterior_samples(dead_o, orc.dead_x(), fin_o, finx_o, 200, 2, 10,
                                            2000, 1.0, seed=2, run_id=0)
    assert np.array_equal(idx, oidx)
    assert np.allclose(x, ox, rtol=1e-10, atol=1e-12)
    gpu.close()
    short = N.NSRun(prob, k=2, p=10, width=w, seed=3, max_iter=600)
    short.run()
    assert short.state()["iter"] == it
    ds = short.dead()
    assert np.allclose(ds[:1202], do[:1202], rtol=1e-10, atol=1e-10)
    with pytest.raises(N.NSError):
        short.geom(R=4)
    short.close()
