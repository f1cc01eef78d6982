"""Adaptive tempered SMC with the slice-sampling mutation (NS_OUTER_SMC) on the GPU against the
FP64 oracle, through the C ABI.

Both sides run the same algorithm on the same Philox streams.  They differ in the order of the
ESS and weight sums (parallel on the GPU, sequential in the oracle), so the bisected inverse
temperature agrees to a few ulp and the resampling positions (u + j)/m fall on the same side of
the cumulative weights except at rounding-level ties; the chains then differ only by FP64
rounding as in the nested-sampling parity tests.  Bars: beta within 1e-12 relative; identical
parents, evaluation and test counts and per-step traces; points and logL within 1e-10; log Z
within 1e-10 per step and 1e-9 end to end.
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


def _parity(N, O, prob, m, p, seed, n_steps, rho=0.5, trace=False):
    width = _width(prob["d"])
    orc = O.SMC(O.Problem(prob), m, p, width, seed, ess_frac=rho, threads=8)
    orc.init()
    gpu = N.NSRun(prob, m=m, p=p, width=width, seed=seed, outer="smc", ess_frac=rho,
                  trace=trace)
    g, o = gpu.state(), orc.state()
    assert np.allclose(g["x"], o["x"], rtol=1e-10, atol=1e-12) and g["Lstar"] == 0.0
    for st in range(n_steps):
        done_o = orc.step()
        done_g = gpu.step()
        g, o = gpu.state(), orc.state()
        _, par_o = orc.aux()
        assert math.isclose(g["Lstar"], o["Lstar"], rel_tol=1e-12, abs_tol=1e-15), \
            f"step {st}: beta {g['Lstar']} vs {o['Lstar']}"
        assert np.array_equal(g["parents"], par_o), f"step {st}: parents"
        assert np.allclose(g["x"], o["x"], rtol=1e-10, atol=1e-12), f"step {st}: particles"
        assert np.allclose(g["logL"], o["logL"], rtol=1e-10, atol=1e-10), f"step {st}: logL"
        assert math.isclose(g["logZ"], o["logZ"], rel_tol=1e-10, abs_tol=1e-10), f"step {st}"
        sg = gpu.stats()
        assert sg["evals"] == o["evals"] and sg["tests"] == o["tests"], f"step {st}: counts"
        assert done_g == done_o
        if done_o:
            break
    return gpu, orc


def test_smc_parity_config1_end_to_end(N, oracle_lib):
    from paper_2601_23252_amd import problems as G
    gpu, orc = _parity(N, oracle_lib, G.config1(), m=300, p=10, seed=3, n_steps=100)
    assert gpu.state()["done"] == 1 and gpu.state()["Lstar"] == 1.0
    zg, eg, hg = gpu.logz()
    zo = orc.state()["logZ"]
    assert abs(zg - zo) <= 1e-9 and math.isnan(eg) and math.isnan(hg)
    tz = truth.lnz_gauss_box_isotropic(5, 0.1, 1.0)
    assert abs(zg - tz) < 0.6


def test_smc_parity_gaussian_prior_and_rho(N, oracle_lib):
    """Gaussian prior (tempered slice over log Pi + beta log L) and a different ESS target."""
    from paper_2601_23252_amd import problems as G
    prob = G.config2(d=12, m=200, k=100)
    _parity(N, oracle_lib, prob, m=200, p=12, seed=5, n_steps=6, rho=0.3)


def test_smc_parity_rastrigin_and_funnel(N, oracle_lib):
    from paper_2601_23252_amd import problems as G
    _parity(N, oracle_lib, G.rastrigin_gauss(4, 0.5), m=256, p=20, seed=2, n_steps=5)
    _parity(N, oracle_lib, G.funnel(6, box=10.0), m=130, p=12, seed=8, n_steps=5)


def test_smc_chain_traces_full_size(N, oracle_lib):
    """config 3 (d = 64 mixture, 2000 particles): the first step against the oracle's (beta,
    parents, every particle), and sampled tempered chains recomputed by the oracle from its own
    particles, temperature, whitening and parents take the same decisions."""
    from paper_2601_23252_amd import problems as G
    prob = G.config3()
    width = _width(64)
    gpu = N.NSRun(prob, m=2000, p=64, width=width, seed=4, outer="smc", trace=True)
    gpu.step()
    s1 = gpu.state()
    tr = gpu.trace()
    P = oracle_lib.Problem(prob)
    orc = oracle_lib.SMC(P, 2000, 64, width, 4, threads=oracle_runs.THREADS)
    orc.init()
    o0 = orc.state()
    orc.step()
    o1 = orc.state()
    Ls_o, par_o = orc.aux()
    beta = o1["Lstar"]
    assert 0.0 < beta < 1.0
    assert math.isclose(s1["Lstar"], beta, rel_tol=1e-12, abs_tol=1e-15)
    assert np.array_equal(s1["parents"], par_o)
    assert np.allclose(s1["x"], o1["x"], rtol=1e-10, atol=1e-12)
    assert np.allclose(s1["logL"], o1["logL"], rtol=1e-10, atol=1e-10)
    for j in (0, 777, 1999):
        par = par_o[j]
        x, lx, _, otr = P.hrss_chain_tempered(o0["x"][par], o0["logL"][par], beta, Ls_o,
                                              width, 64, 4, 0, 1, j, trace=True)
        assert np.array_equal(tr[j], otr), f"chain {j}"
        assert np.allclose(s1["x"][j], x, rtol=1e-10, atol=1e-12)
        assert math.isclose(s1["logL"][j], lx, rel_tol=1e-10, abs_tol=1e-10)
    gpu.close()


def test_smc_rejects_unsupported_combinations(N):
    from paper_2601_23252_amd import problems as G
    p1 = G.config1()
    runs = [(p1, dict(seed=1)), (p1, dict(seed=2, outer="smc"))]
    with pytest.raises(N.NSError) as e:
        N.NSBatch(runs)
    assert e.value.status == N.NS_EINVAL
    R = N.NSRun(p1, m=100, p=5, outer="smc")
    R.step()
    st = N.ns_geom_uncertainty(R.ctx, 0, 4, 1.0, 0, 0)[0]
    assert st == N.NS_EUNSUPPORTED
    R.close()


def test_smc_graph_replay_equals_eager(N):
    """ns_run with NS_FLAG_GRAPH (batches of 16 steps captured and replayed) reproduces the
    eager SMC run bit for bit."""
    from paper_2601_23252_amd import problems as G
    prob = G.config2(d=12, m=300, k=100)
    a = N.NSRun(prob, m=300, p=24, seed=9, outer="smc")
    b = N.NSRun(prob, m=300, p=24, seed=9, outer="smc", graph=True)
    a.run()
    b.run()
    sa, sb = a.state(), b.state()
    assert sa["done"] == sb["done"] == 1 and sa["iter"] == sb["iter"]
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["logL"], sb["logL"])
    assert a.logz()[0] == b.logz()[0]
    a.close()
    b.close()
