"""Python binding of libnss.so (include/nss.h): argument marshalling only.

Every step of the sampler runs in the HIP kernels behind the C ABI; this module converts
numpy arrays and problem dictionaries to the ABI's structs and back.  The functions carry the
ABI's names (ns_init, ns_step, ns_run, ns_logz, ...); ``NSRun`` bundles them for convenience.
If the library is missing it is built with hipcc; if it cannot be loaded an ImportError is
raised: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnss.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nss.h")

NS_OK, NS_DONE, NS_EINVAL, NS_ENOMEM, NS_EDEVICE, NS_ESTATE, NS_EUNSUPPORTED = 0, 1, -1, -2, -3, -4, -5
NS_PRIOR_BOX, NS_PRIOR_GAUSS_DIAG = 0, 1
NS_LIK_MIXTURE, NS_LIK_FUNNEL, NS_LIK_GP, NS_LIK_GAUSS_RASTRIGIN = 1, 2, 3, 4
NS_REPLACE_HRSS, NS_REPLACE_RW = 0, 1
NS_OUTER_NESTED, NS_OUTER_SMC = 0, 1
OUTERS = {"ns": NS_OUTER_NESTED, "smc": NS_OUTER_SMC}
REPLACEMENTS = {"hrss": NS_REPLACE_HRSS, "rw": NS_REPLACE_RW}
NS_FP64, NS_MIXED_BF16, NS_MIXED_FP16, NS_MIXED_BF16X3, NS_MIXED_FP16X3, NS_MIXED_FP32 = 0, 1, 2, 3, 4, 5
NS_FLAG_TRACE, NS_FLAG_TIMING, NS_FLAG_INLINE_DIRECTIONS, NS_FLAG_GRAPH = 1, 2, 4, 8
NS_FLAG_RECORD_POINTS = 16
NS_FLAG_AUTOTUNE = 32
NS_FLAG_SHALLOW_PLAN = 64
NS_FLAG_PLAN8 = 128
NS_FLAG_GP_NO_WAIT = 256
NS_FLAG_FREEZE_WHITENING = 512
NS_FLAG_DIAGONAL_METRIC = 1024
NS_FLAG_SERIAL_GROUPS = 2048
PRECISIONS = {"fp64": NS_FP64, "bf16": NS_MIXED_BF16, "fp16": NS_MIXED_FP16,
              "bf16x3": NS_MIXED_BF16X3, "fp16x3": NS_MIXED_FP16X3, "fp32": NS_MIXED_FP32}
# guard band of each mixed mode: (rel, abs) as set by the library
GUARD = {"bf16": (0.025, 2e-3), "fp16": (0.0032, 2e-3), "bf16x3": (4e-5, 2e-4),
         "fp16x3": (6e-6, 2e-4)}
# GP FP32 mode: rel |L| + abs + c * n * s, s = (sf^2 + sn^2) / sn^2; FP64 beyond n s = 1e5
GP_GUARD = (1e-6, 4e-3, 1e-6)
GP_MAX_COND = 1e5

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)


class ns_prior(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("a", _d), ("b", _d)]


class ns_energy(C.Structure):
    _fields_ = [("kind", C.c_int32), ("d", C.c_int32), ("n_comp", C.c_int32), ("logw", _d),
                ("mean", _d), ("cov", _d), ("n_obs", C.c_int32), ("x_obs", _d), ("y_obs", _d),
                ("alpha", C.c_double), ("amp", C.c_double)]


class ns_config(C.Structure):
    _fields_ = [("n_live", C.c_int32), ("k", C.c_int32), ("chain_len", C.c_int32),
                ("width", C.c_double), ("stepout_cap", C.c_int32), ("shrink_cap", C.c_int32),
                ("term_frac", C.c_double), ("seed", C.c_uint64), ("run_id", C.c_uint32),
                ("precision", C.c_int32), ("max_iter", C.c_int32), ("flags", C.c_int32),
                ("replacement", C.c_int32), ("outer", C.c_int32), ("ess_frac", C.c_double)]


class ns_stats_t(C.Structure):
    _fields_ = [("iterations", C.c_int64), ("evals", C.c_int64), ("tests", C.c_int64),
                ("prior_rejects", C.c_int64), ("stepout_caps", C.c_int64),
                ("shrink_caps", C.c_int64), ("nonfinite", C.c_int64), ("rechecks", C.c_int64),
                ("band_violations", C.c_int64), ("whiten_fallbacks", C.c_int64),
                ("n_dead", C.c_int64), ("hrss_ms", C.c_double), ("hrss_launches", C.c_int64),
                ("width", C.c_double), ("tune_launches", C.c_int64),
                ("gp_wait_timeouts", C.c_int64)]


class ns_state_view(C.Structure):
    _fields_ = [("x", _d), ("logL", _d), ("perm", _i32), ("Lsig", _d), ("parents", _i32),
                ("Lstar", C.c_double), ("logZ", C.c_double), ("logX", C.c_double),
                ("M", C.c_double), ("iter", C.c_int64), ("done", C.c_int32)]


def header_functions() -> list[str]:
    """Names of the functions include/nss.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ns_[a-z_]+)\s*\(", txt)))


_lib = None


def load(build_if_missing: bool = True):
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own libamdhip64 whose dependents ask for
    # the unversioned name, so loading /opt/rocm's copy first would put two runtimes in the
    # process.  Importing torch first makes libnss.so bind to the copy torch already loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        if not build_if_missing:
            raise ImportError(f"{LIB_PATH} is not built")
        from . import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ns_init.restype = C.c_int
    L.ns_init.argtypes = [C.POINTER(ns_prior), C.POINTER(ns_energy), C.POINTER(ns_config), vp,
                          C.POINTER(vp)]
    L.ns_reset.restype = C.c_int
    L.ns_reset.argtypes = [vp, C.c_uint64, C.c_uint32]
    L.ns_step.restype = C.c_int
    L.ns_step.argtypes = [vp, _i32]
    L.ns_run.restype = C.c_int
    L.ns_run.argtypes = [vp, C.c_int32, _i32]
    L.ns_logz.restype = C.c_int
    L.ns_logz.argtypes = [vp, _d, _d, _d]
    L.ns_stats.restype = C.c_int
    L.ns_stats.argtypes = [vp, C.POINTER(ns_stats_t)]
    L.ns_get_state.restype = C.c_int
    L.ns_get_state.argtypes = [vp, C.POINTER(ns_state_view)]
    L.ns_set_state.restype = C.c_int
    L.ns_set_state.argtypes = [vp, C.POINTER(ns_state_view)]
    L.ns_get_dead.restype = C.c_int
    L.ns_get_dead.argtypes = [vp, _d, C.c_int64, C.POINTER(C.c_int64)]
    L.ns_get_trace.restype = C.c_int
    L.ns_get_trace.argtypes = [vp, _i32]
    L.ns_eval_loglik.restype = C.c_int
    L.ns_eval_loglik.argtypes = [vp, _d, C.c_int32, C.c_int32, _d]
    L.ns_free.restype = None
    L.ns_free.argtypes = [vp]
    L.ns_last_error.restype = C.c_char_p
    L.ns_last_error.argtypes = [vp]
    L.ns_config_default.restype = None
    L.ns_config_default.argtypes = [C.POINTER(ns_config)]
    L.ns_init_batch.restype = C.c_int
    L.ns_init_batch.argtypes = [C.c_int32, C.POINTER(ns_prior), C.POINTER(ns_energy),
                                C.POINTER(ns_config), vp, C.POINTER(vp)]
    L.ns_num_runs.restype = C.c_int32
    L.ns_num_runs.argtypes = [vp]
    L.ns_chains_per_workgroup.restype = C.c_int32
    L.ns_chains_per_workgroup.argtypes = [vp, C.c_int32]
    for fn in (L.ns_tune_save, L.ns_tune_load):
        fn.restype = C.c_int
        fn.argtypes = [C.c_char_p, _i32]
    L.ns_tune_clear.restype = C.c_int
    L.ns_tune_clear.argtypes = [_i32]
    L.ns_launch_shape.restype = C.c_int
    L.ns_launch_shape.argtypes = [vp, C.c_int32, _i32, _i32]
    L.ns_logz_batch.restype = C.c_int
    L.ns_logz_batch.argtypes = [vp, _d, _d, _d]
    L.ns_stats_run.restype = C.c_int
    L.ns_stats_run.argtypes = [vp, C.c_int32, C.POINTER(ns_stats_t)]
    L.ns_get_state_run.restype = C.c_int
    L.ns_get_state_run.argtypes = [vp, C.c_int32, C.POINTER(ns_state_view)]
    L.ns_posterior_samples.restype = C.c_int
    L.ns_posterior_samples.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_uint64,
                                       C.c_uint32, C.c_int32, _d, C.POINTER(C.c_int64)]
    L.ns_geom_uncertainty.restype = C.c_int
    L.ns_geom_uncertainty.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_uint64,
                                      C.c_uint32, _d, _d, C.c_int64, _d, C.POINTER(C.c_int64),
                                      _d]
    L.ns_geom_uncertainty_noalloc.restype = C.c_int
    L.ns_geom_uncertainty_noalloc.argtypes = [vp, C.c_int32, C.c_int32, C.c_double, C.c_uint64,
                                              C.c_uint32, vp, vp, C.c_int64, vp,
                                              C.POINTER(C.c_int64)]
    _lib = L
    return L


class NSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def _ptr(a, t=_d):
    return a.ctypes.data_as(t) if a is not None else None


def _check(st, ctx=None, ok=(NS_OK,)):
    if st not in ok:
        raise NSError(st, load().ns_last_error(ctx).decode())
    return st


# ---- the ABI's calls -------------------------------------------------------------------------
def ns_config_default() -> ns_config:
    c = ns_config()
    load().ns_config_default(C.byref(c))
    return c


def ns_init(prior: ns_prior, energy: ns_energy, cfg: ns_config, stream=None):
    """Returns (status, ctx); ctx is None unless status is NS_OK."""
    ctx = C.c_void_p()
    ref = lambda o: C.byref(o) if o is not None else None
    st = load().ns_init(ref(prior), ref(energy), ref(cfg), stream, C.byref(ctx))
    return st, (ctx.value if st == NS_OK else None)


def ns_reset(ctx, seed, run_id=0):
    return load().ns_reset(ctx, int(seed), int(run_id))


def ns_step(ctx):
    done = C.c_int32(0)
    st = load().ns_step(ctx, C.byref(done))
    return st, int(done.value)


def ns_run(ctx, max_iter):
    it = C.c_int32(0)
    st = load().ns_run(ctx, int(max_iter), C.byref(it))
    return st, int(it.value)


def ns_logz(ctx):
    z, e, h = C.c_double(), C.c_double(), C.c_double()
    st = load().ns_logz(ctx, C.byref(z), C.byref(e), C.byref(h))
    return st, z.value, e.value, h.value


def ns_stats(ctx):
    s = ns_stats_t()
    st = load().ns_stats(ctx, C.byref(s))
    return st, {f: getattr(s, f) for f, _ in ns_stats_t._fields_}


def ns_init_batch(priors, energies, cfgs, stream=None):
    """priors, energies, cfgs: equal-length lists of structs.  Returns (status, ctx)."""
    n = len(priors)
    if not (len(energies) == n and len(cfgs) == n):
        raise ValueError("priors, energies and cfgs must have equal length")
    pa = (ns_prior * max(n, 1))(*priors)
    ea = (ns_energy * max(n, 1))(*energies)
    ca = (ns_config * max(n, 1))(*cfgs)
    ctx = C.c_void_p()
    st = load().ns_init_batch(n, pa, ea, ca, stream, C.byref(ctx))
    return st, (ctx.value if st == NS_OK else None)


def ns_num_runs(ctx) -> int:
    return int(load().ns_num_runs(ctx))


def ns_chains_per_workgroup(ctx, run=0) -> int:
    return int(load().ns_chains_per_workgroup(ctx, run))


def ns_tune_save(path):
    n = C.c_int32(0)
    st = load().ns_tune_save(None if path is None else str(path).encode(), C.byref(n))
    return st, n.value


def ns_tune_load(path):
    n = C.c_int32(0)
    st = load().ns_tune_load(None if path is None else str(path).encode(), C.byref(n))
    return st, n.value


def ns_tune_clear():
    n = C.c_int32(0)
    st = load().ns_tune_clear(C.byref(n))
    return st, n.value


def ns_launch_shape(ctx, run=0):
    """Returns (status, chains per workgroup, tests planned per round)."""
    c, p = C.c_int32(0), C.c_int32(0)
    st = load().ns_launch_shape(ctx, int(run), C.byref(c), C.byref(p))
    return st, c.value, p.value


def ns_logz_batch(ctx):
    n = ns_num_runs(ctx)
    z, e, h = np.zeros(n), np.zeros(n), np.zeros(n)
    st = load().ns_logz_batch(ctx, _ptr(z), _ptr(e), _ptr(h))
    return st, z, e, h


def ns_stats_run(ctx, run):
    s = ns_stats_t()
    st = load().ns_stats_run(ctx, int(run), C.byref(s))
    return st, {f: getattr(s, f) for f, _ in ns_stats_t._fields_}


def ns_free(ctx):
    if ctx:
        load().ns_free(ctx)


def ns_last_error(ctx=None) -> str:
    return load().ns_last_error(ctx).decode()


# ---- problem marshalling ---------------------------------------------------------------------
def make_structs(prob: dict):
    """(ns_prior, ns_energy, keep-alive arrays) from a problem dictionary."""
    d = int(prob["d"])
    pa = np.ascontiguousarray(prob["prior_a"], np.float64)
    pb = np.ascontiguousarray(prob["prior_b"], np.float64)
    pr = ns_prior(NS_PRIOR_BOX if prob["prior"] == "box" else NS_PRIOR_GAUSS_DIAG, d, _ptr(pa),
                  _ptr(pb))
    keep = [pa, pb]
    if prob["lik"] == "mixture":
        K = int(prob["K"])
        lw = np.ascontiguousarray(prob["logw"], np.float64)
        mu = np.ascontiguousarray(prob["mu"], np.float64).reshape(K, d)
        cov = np.ascontiguousarray(prob["cov"], np.float64).reshape(K, d, d)
        keep += [lw, mu, cov]
        en = ns_energy(NS_LIK_MIXTURE, d, K, _ptr(lw), _ptr(mu), _ptr(cov))
    elif prob["lik"] == "funnel":
        en = ns_energy(NS_LIK_FUNNEL, d, 0, None, None, None)
    elif prob["lik"] == "rastrigin":
        en = ns_energy(NS_LIK_GAUSS_RASTRIGIN, d, 0, None, None, None, 0, None, None,
                       float(prob["alpha"]), float(prob["amp"]))
    elif prob["lik"] == "gp":
        gx = np.ascontiguousarray(prob["gp_x"], np.float64)
        gy = np.ascontiguousarray(prob["gp_y"], np.float64)
        keep += [gx, gy]
        en = ns_energy(NS_LIK_GP, d, 0, None, None, None, len(gy), _ptr(gx), _ptr(gy))
    else:
        raise ValueError(prob["lik"])
    return pr, en, keep


def current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


def make_config(m, k, p, width=0.0, seed=0, run_id=0, precision="fp64", term_frac=1e-3,
                stepout_cap=10, shrink_cap=100, max_iter=100000, trace=False, timing=False,
                inline_directions=False, graph=False, replacement="hrss", outer="ns",
                ess_frac=0.5, record_points=False, autotune=False,
                shallow_plan=False, plan8=False, gp_no_wait=False,
                freeze_whitening=False, diagonal_metric=False,
                serial_groups=False) -> ns_config:
    cfg = ns_config_default()
    cfg.n_live, cfg.k, cfg.chain_len = int(m), int(k), int(p)
    cfg.width = float(width)
    cfg.stepout_cap, cfg.shrink_cap = int(stepout_cap), int(shrink_cap)
    cfg.term_frac = float(term_frac)
    cfg.seed, cfg.run_id = int(seed), int(run_id)
    cfg.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.max_iter = int(max_iter)
    cfg.flags = ((NS_FLAG_TRACE if trace else 0) | (NS_FLAG_TIMING if timing else 0)
                 | (NS_FLAG_INLINE_DIRECTIONS if inline_directions else 0)
                 | (NS_FLAG_GRAPH if graph else 0)
                 | (NS_FLAG_RECORD_POINTS if record_points else 0)
                 | (NS_FLAG_AUTOTUNE if autotune else 0)
                 | (NS_FLAG_SHALLOW_PLAN if shallow_plan else 0)
                 | (NS_FLAG_PLAN8 if plan8 else 0)
                 | (NS_FLAG_GP_NO_WAIT if gp_no_wait else 0)
                 | (NS_FLAG_FREEZE_WHITENING if freeze_whitening else 0)
                 | (NS_FLAG_DIAGONAL_METRIC if diagonal_metric else 0)
                 | (NS_FLAG_SERIAL_GROUPS if serial_groups else 0))
    cfg.replacement = REPLACEMENTS[replacement] if isinstance(replacement, str) else int(replacement)
    cfg.outer = OUTERS[outer] if isinstance(outer, str) else int(outer)
    cfg.ess_frac = float(ess_frac)
    return cfg


def _state_of(ctx, run, m, d, k):
    x = np.zeros((m, d)); logL = np.zeros(m); perm = np.zeros(m, np.int32)
    Ls = np.zeros((d, d)); par = np.zeros(k, np.int32)
    v = ns_state_view(_ptr(x), _ptr(logL), _ptr(perm, _i32), _ptr(Ls), _ptr(par, _i32),
                      0.0, 0.0, 0.0, 0.0, 0, 0)
    _check(load().ns_get_state_run(ctx, int(run), C.byref(v)), ctx)
    return dict(x=x, logL=logL, perm=perm, Lsig=Ls, parents=par, Lstar=v.Lstar, logZ=v.logZ,
                logX=v.logX, M=v.M, iter=int(v.iter), done=int(v.done))


def ns_geom_uncertainty(ctx, run, R, beta, seed, run_id, n_deaths=None, timing=False):
    """One call of the C function.  With n_deaths (= dead points + n_live - k) the mean log
    weights are returned too.  Returns (status, logz[R], logw_mean or None, ess, N,
    device_ms or None)."""
    L = load()
    n = C.c_int64(0)
    logz = np.zeros(max(int(R), 1))
    ess = C.c_double(0.0)
    ms = C.c_double(0.0)
    lw = None if n_deaths is None else np.zeros(int(n_deaths))
    st = L.ns_geom_uncertainty(ctx, int(run), int(R), float(beta), int(seed), int(run_id),
                               _ptr(logz), _ptr(lw), 0 if lw is None else len(lw),
                               C.byref(ess), C.byref(n), C.byref(ms) if timing else None)
    if lw is not None and st == NS_OK and n.value != len(lw):
        raise NSError(NS_EINVAL, f"{n.value} deaths, {len(lw)} expected")
    return st, logz[:int(R)], lw, ess.value, n.value, (ms.value if timing else None)


def ns_geom_uncertainty_noalloc(ctx, run, R, beta, seed, run_id, logz_ptr, logw_mean_ptr, cap,
                                ess_ptr):
    """One call of the C function with caller-owned device outputs (integer device addresses).
    Returns (status, N)."""
    n = C.c_int64(0)
    st = load().ns_geom_uncertainty_noalloc(ctx, int(run), int(R), float(beta), int(seed),
                                            int(run_id), C.c_void_p(logz_ptr),
                                            C.c_void_p(logw_mean_ptr), int(cap),
                                            C.c_void_p(ess_ptr), C.byref(n))
    return st, n.value


def ns_posterior_samples(ctx, run, R, beta, seed, run_id, n, d):
    """Returns (status, x[n, d], idx[n])."""
    x = np.zeros((max(int(n), 1), int(d)))
    idx = np.zeros(max(int(n), 1), np.int64)
    st = load().ns_posterior_samples(ctx, int(run), int(R), float(beta), int(seed), int(run_id),
                                     int(n), _ptr(x), idx.ctypes.data_as(C.POINTER(C.c_int64)))
    return st, x[:int(n)], idx[:int(n)]


def _geom(ctx, run, cfg, R, beta, seed, run_id, weights, timing):
    seed = cfg.seed if seed is None else seed
    run_id = cfg.run_id if run_id is None else run_id
    nd = None
    if weights:
        st, s = ns_stats_run(ctx, run)
        _check(st, ctx)
        nd = int(s["n_dead"]) + cfg.n_live - cfg.k
    st, logz, lw, ess, _, ms = ns_geom_uncertainty(ctx, run, R, beta, seed, run_id, nd, timing)
    _check(st, ctx)
    out = dict(logz=logz, logw_mean=lw, ess=ess)
    if timing:
        out["device_ms"] = ms
    return out


class NSRun:
    """One nested-sampling run on the GPU (wraps one ns_ctx)."""

    def __init__(self, prob: dict, m=None, k=None, p=None, width=0.0, seed=0, run_id=0,
                 precision="fp64", term_frac=1e-3, stepout_cap=10, shrink_cap=100,
                 max_iter=100000, trace=False, timing=False, inline_directions=False,
                 graph=False, stream="torch", replacement="hrss", outer="ns", ess_frac=0.5,
                 record_points=False, autotune=False, shallow_plan=False, plan8=False,
                 gp_no_wait=False, freeze_whitening=False, diagonal_metric=False):
        self.prob = prob
        self.d = int(prob["d"])
        self.m = int(m or prob["m"])
        self.k = int(k or prob["k"])
        if outer == "smc":
            self.k = self.m   # every particle moves
        self.p = int(p or prob["p"])
        pr, en, self._keep = make_structs(prob)
        cfg = make_config(self.m, self.k, self.p, width, seed, run_id, precision, term_frac,
                          stepout_cap, shrink_cap, max_iter, trace, timing, inline_directions,
                          graph, replacement, outer, ess_frac, record_points, autotune,
                          shallow_plan, plan8, gp_no_wait, freeze_whitening,
                          diagonal_metric)
        self.cfg = cfg
        s = current_stream() if stream == "torch" else stream
        st, self.ctx = ns_init(pr, en, cfg, s)
        _check(st)

    def close(self):
        if getattr(self, "ctx", None):
            ns_free(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def reset(self, seed, run_id=0):
        _check(ns_reset(self.ctx, seed, run_id), self.ctx)

    def chains_per_workgroup(self) -> int:
        return ns_chains_per_workgroup(self.ctx, 0)

    def launch_shape(self):
        """(chains per workgroup, tests planned per round) of the run's chains."""
        st, c, p = ns_launch_shape(self.ctx, 0)
        _check(st, self.ctx)
        return c, p

    def step(self) -> bool:
        st, done = ns_step(self.ctx)
        _check(st, self.ctx, ok=(NS_OK, NS_DONE))
        return bool(done)

    def run(self, max_iter=100000) -> int:
        st, it = ns_run(self.ctx, max_iter)
        _check(st, self.ctx)
        return it

    def logz(self):
        st, z, e, h = ns_logz(self.ctx)
        _check(st, self.ctx)
        return z, e, h

    def stats(self) -> dict:
        st, s = ns_stats(self.ctx)
        _check(st, self.ctx)
        return s

    def state(self) -> dict:
        return _state_of(self.ctx, 0, self.m, self.d, self.k)

    def set_state(self, x, logL, logZ, logX, M, iter_, done=0, Lsig=None):
        """ns_set_state; Lsig (d x d lower-triangular) is the factor kept by a run with
        freeze_whitening=True."""
        x = np.ascontiguousarray(x, np.float64)
        logL = np.ascontiguousarray(logL, np.float64)
        Ls = None if Lsig is None else np.ascontiguousarray(Lsig, np.float64)
        if Ls is not None and Ls.shape != (self.d, self.d):
            raise ValueError("Lsig must be d x d")
        v = ns_state_view(_ptr(x), _ptr(logL), None, None if Ls is None else _ptr(Ls), None,
                          0.0, float(logZ), float(logX), float(M), int(iter_), int(done))
        _check(load().ns_set_state(self.ctx, C.byref(v)), self.ctx)

    def dead(self) -> np.ndarray:
        n = C.c_int64(0)
        _check(load().ns_get_dead(self.ctx, None, 0, C.byref(n)), self.ctx)
        out = np.zeros(n.value)
        _check(load().ns_get_dead(self.ctx, _ptr(out), n.value, C.byref(n)), self.ctx)
        return out

    def geom(self, R=100, beta=1.0, seed=None, run_id=None, weights=True, timing=False):
        """Post-hoc geometric uncertainty (ns_geom_uncertainty): dict(logz[R], logw_mean[N],
        ess[, device_ms]); the shrinkage stream defaults to the run's (seed, run_id)."""
        return _geom(self.ctx, 0, self.cfg, R, beta, seed, run_id, weights, timing)

    def posterior_samples(self, n, R=100, beta=1.0, seed=None, run_id=None):
        """ns_posterior_samples (needs record_points=True): (x[n, d], death indices[n])."""
        seed = self.cfg.seed if seed is None else seed
        run_id = self.cfg.run_id if run_id is None else run_id
        st, x, idx = ns_posterior_samples(self.ctx, 0, R, beta, seed, run_id, n, self.d)
        _check(st, self.ctx)
        return x, idx

    def trace(self) -> np.ndarray:
        out = np.zeros((self.k, self.p, 4), np.int32)
        _check(load().ns_get_trace(self.ctx, _ptr(out, _i32)), self.ctx)
        return out

    def eval_loglik(self, x, precision="fp64") -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        out = np.zeros(x.shape[0])
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(load().ns_eval_loglik(self.ctx, _ptr(x), x.shape[0], prec, _ptr(out)), self.ctx)
        return out


class NSBatch:
    """Independent runs in one context (ns_init_batch): runs[r] = (problem dict, config kwargs
    for make_config, with m, k, p defaulting to the problem's)."""

    def __init__(self, runs, stream="torch"):
        self._keep, prs, ens, cfgs, self.shapes = [], [], [], [], []
        for prob, kw in runs:
            kw = dict(kw)
            m, k, p = (int(kw.pop(a, None) or prob[a]) for a in ("m", "k", "p"))
            pr, en, keep = make_structs(prob)
            self._keep.append(keep)
            prs.append(pr)
            ens.append(en)
            cfgs.append(make_config(m, k, p, **kw))
            self.shapes.append((m, int(prob["d"]), k))
        s = current_stream() if stream == "torch" else stream
        st, self.ctx = ns_init_batch(prs, ens, cfgs, s)
        _check(st)
        self.n = len(runs)
        self.cfgs = cfgs

    def close(self):
        if getattr(self, "ctx", None):
            ns_free(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def reset(self, seed, run_id=0):
        _check(ns_reset(self.ctx, seed, run_id), self.ctx)

    def step(self) -> bool:
        st, done = ns_step(self.ctx)
        _check(st, self.ctx, ok=(NS_OK, NS_DONE))
        return bool(done)

    def run(self, max_iter=100000) -> int:
        st, it = ns_run(self.ctx, max_iter)
        _check(st, self.ctx)
        return it

    def logz(self):
        st, z, e, h = ns_logz_batch(self.ctx)
        _check(st, self.ctx)
        return z, e, h

    def stats(self, run) -> dict:
        st, s = ns_stats_run(self.ctx, run)
        _check(st, self.ctx)
        return s

    def state(self, run) -> dict:
        m, d, k = self.shapes[run]
        return _state_of(self.ctx, run, m, d, k)

    def geom(self, run, R=100, beta=1.0, seed=None, run_id=None, weights=True, timing=False):
        """ns_geom_uncertainty for run `run`; the stream defaults to the run's own key."""
        return _geom(self.ctx, run, self.cfgs[run], R, beta, seed, run_id, weights, timing)
