"""The 16-bit mixture chains with hypothesis plans (16 or 8 planned tests per round) against the
4-test kernel (NS_FLAG_SHALLOW_PLAN), through the C ABI.  Both take every decision as FP64
does, so their trajectories are identical: the same delete-k order, points bit for bit, the
same per-step decision traces and the same evaluation counters.  The 4-test kernel is itself
checked against the oracle (test_gpu_parity.py, test_gpu_fullsize.py)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def _problems():
    from paper_2601_23252_amd import problems as G
    return {
        "mix8_d64": (G.config3(), dict(m=400, k=200, p=64)),
        "corr32_gauss_prior": (G.config2(), dict(m=300, k=150, p=40)),
        "mix3_d48": (G.mixture_problem(5, 48, 3, m=300, k=100), dict(p=48)),
        "mix2_d100": (G.mixture_problem(11, 100, 2, m=200, k=64), dict(p=30)),
        "mix12_d20": (G.mixture_problem(9, 20, 12, m=256, k=128), dict(p=20)),
    }


@pytest.mark.parametrize("plan8", [False, True])
@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "bf16", "fp16"])
@pytest.mark.parametrize("name", ["mix8_d64", "corr32_gauss_prior", "mix3_d48", "mix2_d100",
                                  "mix12_d20"])
def test_plan_equals_shallow_kernel(N, name, prec, plan8):
    prob, kw = _problems()[name]
    print(f"plan vs shallow: {name} {prec} plan8={plan8}", flush=True)
    a = N.NSRun(prob, seed=3, precision=prec, trace=True, plan8=plan8, **kw)
    assert a.launch_shape()[1] == (8 if plan8 else 16)
    b = N.NSRun(prob, seed=3, precision=prec, trace=True, shallow_plan=True, **kw)
    for it in range(6):
        da, db = a.step(), b.step()
        assert da == db
        sa, sb = a.state(), b.state()
        assert np.array_equal(sa["perm"], sb["perm"]), (name, prec, it)
        assert np.array_equal(sa["x"], sb["x"]), (name, prec, it)
        assert np.array_equal(sa["logL"], sb["logL"]), (name, prec, it)
        assert np.array_equal(a.trace(), b.trace()), (name, prec, it)
        ta, tb = a.stats(), b.stats()
        for key in ("evals", "tests", "prior_rejects", "stepout_caps", "shrink_caps",
                    "nonfinite", "band_violations"):
            assert ta[key] == tb[key], (name, prec, it, key, ta[key], tb[key])
        if da:
            break
    a.close()
    b.close()


def test_plan_caps_and_short_chains(N):
    """Small step-out and shrink caps (a cap inside a plan's stepping-out or shrink slots) and
    chains of a single step: still identical."""
    prob, kw = _problems()["mix3_d48"]
    for caps in (dict(stepout_cap=1, shrink_cap=3), dict(stepout_cap=2, shrink_cap=1),
                 dict(stepout_cap=0, shrink_cap=5), dict(p=1)):
        k2 = dict(kw, **caps)
        a = N.NSRun(prob, seed=8, precision="bf16x3", trace=True, plan8=caps.get("p") == 1, **k2)
        b = N.NSRun(prob, seed=8, precision="bf16x3", trace=True, shallow_plan=True, **k2)
        for _ in range(3):
            a.step()
            b.step()
        sa, sb = a.state(), b.state()
        assert np.array_equal(sa["x"], sb["x"]), caps
        assert np.array_equal(a.trace(), b.trace()), caps
        ta, tb = a.stats(), b.stats()
        for key in ("evals", "tests", "prior_rejects", "stepout_caps", "shrink_caps"):
            assert ta[key] == tb[key], (caps, key)
        a.close()
        b.close()


@pytest.mark.parametrize("prec", ["fp16x3", "bf16"])
@pytest.mark.parametrize("plan8", [False, True])
def test_two_workgroups_per_cu_variant_is_identical(N, prec, plan8):
    """A batch whose plan-kernel launch has more workgroups than CUs (six d = 48 mixtures with
    k = 200: 1,200 chains, 300 workgroups) runs the variant compiled for two workgroups per CU;
    each run's trajectory equals its single run's (200 chains, one workgroup per CU)."""
    from paper_2601_23252_amd import problems as G
    runs = [(G.mixture_problem(20 + r, 48, 3, m=400, k=200),
             dict(p=24, seed=5, run_id=r, precision=prec, plan8=plan8)) for r in range(6)]
    B = N.NSBatch(runs)
    assert N.ns_chains_per_workgroup(B.ctx, 0) == 4
    for _ in range(5):
        B.step()
    for r, (prob, kw) in enumerate(runs):
        S = N.NSRun(prob, **kw)
        assert S.chains_per_workgroup() == 1
        for _ in range(5):
            S.step()
        sb, ss = B.state(r), S.state()
        assert np.array_equal(sb["perm"], ss["perm"]), r
        assert np.array_equal(sb["x"], ss["x"]), r
        assert np.array_equal(sb["logL"], ss["logL"]), r
        assert B.stats(r)["evals"] == S.stats()["evals"]
        S.close()
    B.close()
