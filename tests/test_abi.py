"""C ABI checks that need no GPU: the library loads, exports every function include/nss.h
declares, and rejects invalid arguments before touching a device."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def N():
    from paper_2601_23252_amd import nss
    nss.load()
    return nss


def test_exports_every_declared_function(N):
    L = N.load()
    names = N.header_functions()
    for required in ("ns_init", "ns_step", "ns_run", "ns_logz", "ns_reset", "ns_free",
                     "ns_stats", "ns_get_state", "ns_set_state", "ns_eval_loglik"):
        assert required in names
    for f in names:
        assert hasattr(L, f), f


def test_config_defaults(N):
    c = N.ns_config_default()
    assert (c.stepout_cap, c.shrink_cap) == (10, 100)
    assert abs(c.term_frac - 1e-3) < 1e-15 and c.precision == N.NS_FP64


def _structs(N, prob):
    return N.make_structs(prob)


@pytest.mark.parametrize("m,k,p", [(10, 10, 5), (10, 0, 5), (1, 1, 5), (10, 3, 0), (9000, 10, 5)])
def test_invalid_run_shape(N, m, k, p):
    from paper_2601_23252_amd import problems as G
    pr, en, keep = _structs(N, G.config1())
    cfg = N.ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = m, k, p
    st, ctx = N.ns_init(pr, en, cfg, None)
    assert ctx is None
    assert st == (N.NS_EUNSUPPORTED if m > 8192 else N.NS_EINVAL)
    assert N.ns_last_error(None)


def test_invalid_problem(N):
    from paper_2601_23252_amd import problems as G
    cfg = N.ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = 50, 10, 5
    pr, en, keep = _structs(N, G.funnel(330))
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED   # d > 320
    pr, en, keep = _structs(N, G.mixture_problem(3, 200, 1))
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED   # d > 128: not mixtures
    pr, en, keep = _structs(N, G.funnel(200))
    cfg.flags = N.NS_FLAG_INLINE_DIRECTIONS
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED   # d > 128: direction buffer
    cfg.flags = 0
    pr, en, keep = _structs(N, G.funnel(1 + 1))
    en.d = 3
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL          # dimension mismatch
    pr, en, keep = _structs(N, G.config1())
    en.n_comp = 0
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    pr, en, keep = _structs(N, G.config1())
    cfg.precision = 9
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    pr, en, keep = _structs(N, G.funnel(8))
    cfg.precision = N.NS_MIXED_BF16
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # mixed: mixtures only
    assert N.ns_init(None, en, cfg, None)[0] == N.NS_EINVAL


def test_null_context_calls(N):
    assert N.ns_step(None)[0] == N.NS_EINVAL
    assert N.ns_run(None, 1)[0] == N.NS_EINVAL
    assert N.ns_logz(None)[0] == N.NS_EINVAL
    assert N.ns_reset(None, 0) == N.NS_EINVAL
    assert N.ns_geom_uncertainty(None, 0, 100, 1.0, 0, 0)[0] == N.NS_EINVAL
    assert N.ns_chains_per_workgroup(None, 0) == 0
    N.ns_free(None)


def test_invalid_gp_and_batch_arguments(N):
    from paper_2601_23252_amd import problems as G
    cfg = N.ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = 50, 10, 5
    gp = G.gp_problem(4, n=20)
    pr, en, keep = _structs(N, gp)
    en.n_obs = 300
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # n_obs > 256
    pr, en, keep = _structs(N, gp)
    en.n_obs = 0
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    pr, en, keep = _structs(N, gp)
    cfg.precision = N.NS_MIXED_BF16X3
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # GP: FP64 or FP32
    pr, en, keep = _structs(N, G.config1())
    cfg.precision = N.NS_MIXED_FP32
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # FP32: GP only
    cfg.precision = N.NS_FP64
    # batch: every run is validated and the failing run is named
    pr2, en2, keep2 = _structs(N, G.funnel(8))
    bad = N.ns_config_default()
    bad.n_live, bad.k, bad.chain_len = 50, 50, 5                   # k > n_live - 1
    st, ctx = N.ns_init_batch([pr, pr2], [en, en2], [cfg, bad], None)
    assert st == N.NS_EINVAL and ctx is None
    assert "run 1" in N.ns_last_error(None)
    assert N.ns_init_batch([], [], [], None)[0] == N.NS_EINVAL
    assert N.ns_num_runs(None) == 0


def test_invalid_replacement_and_rastrigin_arguments(N):
    from paper_2601_23252_amd import problems as G
    cfg = N.ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = 50, 10, 5
    assert cfg.replacement == N.NS_REPLACE_HRSS
    pr, en, keep = _structs(N, G.config1())
    cfg.replacement = 7
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    cfg.replacement = N.NS_REPLACE_RW
    pr, en, keep = _structs(N, G.gp_problem(4, n=20))
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # RW: not for the GP
    cfg.replacement = N.NS_REPLACE_HRSS
    for alpha, amp in ((-0.1, 10.0), (1.5, 10.0), (0.5, -1.0), (0.5, float("inf"))):
        pr, en, keep = _structs(N, G.rastrigin_gauss(4, 0.5))
        en.alpha, en.amp = alpha, amp
        assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    pr, en, keep = _structs(N, G.rastrigin_gauss(4, 0.5))
    cfg.precision = N.NS_MIXED_BF16X3
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED    # Rastrigin: FP64 only


def test_invalid_smc_arguments(N):
    from paper_2601_23252_amd import problems as G
    cfg = N.ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = 50, 10, 5
    assert cfg.outer == N.NS_OUTER_NESTED and cfg.ess_frac == 0.5
    pr, en, keep = _structs(N, G.config1())
    cfg.outer = 5
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    cfg.outer = N.NS_OUTER_SMC
    for rho in (0.0, 1.0, -0.2):
        cfg.ess_frac = rho
        assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EINVAL
    cfg.ess_frac = 0.5
    cfg.precision = N.NS_MIXED_BF16X3
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED     # SMC: FP64 only
    cfg.precision = N.NS_FP64
    cfg.replacement = N.NS_REPLACE_RW
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED     # SMC: slice mutation
    cfg.replacement = N.NS_REPLACE_HRSS
    pr, en, keep = _structs(N, G.gp_problem(4, n=20))
    assert N.ns_init(pr, en, cfg, None)[0] == N.NS_EUNSUPPORTED     # SMC: not for the GP


def test_tune_cache_json_round_trip(N, tmp_path):
    """The autotuner's cache file (host only): a file in the saved format merges into the
    cache and is written back with the same entries; a malformed file is refused whole; the
    cache can be emptied."""
    import json
    assert N.ns_tune_clear()[0] == N.NS_OK
    src = tmp_path / "tune.json"
    entries = [dict(D=64, lik=1, mode=3, upw=8, rw=0, chains=1000, planned=1, C=4, plan=16),
               dict(D=32, lik=2, mode=0, upw=1, rw=1, chains=77, planned=0, C=2, plan=0)]
    body = ",".join("\n  " + json.dumps(e) for e in entries)
    src.write_text('{"nss_tune": 2, "entries": [' + body + "\n]}\n")
    st, n = N.ns_tune_load(src)
    assert st == N.NS_OK and n == 2
    out = tmp_path / "out.json"
    st, n2 = N.ns_tune_save(out)
    assert st == N.NS_OK and n2 == n
    saved = json.loads(out.read_text())
    assert saved["nss_tune"] == 2 and len(saved["entries"]) == n
    for e in entries:
        assert e in saved["entries"]
    bad = tmp_path / "bad.json"
    good = entries[0]
    for e in (dict(good, C=9), dict(good, C=3.7), dict(good, extra=1), dict(good, D=48),
              dict(good, upw=5), dict(good, plan=12), dict(good, mode=9),
              dict(good, planned=0, plan=16), dict(good, lik=7)):
        bad.write_text('{"nss_tune": 2, "entries": [' + json.dumps(e) + "]}")
        assert N.ns_tune_load(bad)[0] == N.NS_EINVAL, e
    assert N.ns_tune_load(tmp_path / "missing.json")[0] == N.NS_EINVAL
    assert N.ns_tune_load(None)[0] == N.NS_EINVAL
    st, n3 = N.ns_tune_save(tmp_path / "again.json")
    assert st == N.NS_OK and n3 == n
    st, n4 = N.ns_tune_clear()
    assert st == N.NS_OK and n4 == n
    assert N.ns_tune_save(tmp_path / "empty.json") == (N.NS_OK, 0)


def test_binding_constants_match_the_header(N):
    """Every NS_FLAG_* / NS_* integer constant the binding defines has the value the header
    #defines or enumerates, and the flags are distinct single bits."""
    import re
    txt = open(N.HEADER).read()
    defined = {m.group(1): int(m.group(2))
               for m in re.finditer(r"#define\s+(NS_FLAG_\w+)\s+(\d+)", txt)}
    assert len(defined) >= 12
    for name, val in defined.items():
        assert getattr(N, name) == val, name
        assert val & (val - 1) == 0, name
    assert len(set(defined.values())) == len(defined)
    enums = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(NS_\w+)\s*=\s*(-?\d+)", txt)}
    for name, val in enums.items():
        if hasattr(N, name):
            assert getattr(N, name) == val, name
