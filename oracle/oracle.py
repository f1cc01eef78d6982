"""ctypes wrapper of the plain FP64 C oracle (``oracle/nss_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline
leg of the benchmark, never by the GPU library.  It takes problems as plain arrays (the
seeded generator's output) and imports nothing from the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nss_oracle.c")
LIB = os.path.join(HERE, "libnss_oracle.so")

PRIOR_BOX, PRIOR_GAUSS = 0, 1
LIK_MIXTURE, LIK_FUNNEL, LIK_GP, LIK_RG = 1, 2, 3, 4
P_INIT, P_RESAMPLE, P_DIR, P_STEP, P_SHRINK = 1, 2, 3, 4, 5

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_lp = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Plain C, no GPU code."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


NATIVE_LIB = os.path.join(HERE, "libnss_oracle_native.so")
NATIVE_FLAGS = ["-O3", "-march=native", "-ffp-contract=off"]


def use_native_build() -> str:
    """Build a copy tuned for this host (-O3 -march=native, no contraction into fused
    multiply-adds, so every result equals the portable build's) and route later calls to it.
    Used only to time the oracle on the host it runs on; must be called before the first call
    into the oracle."""
    global LIB, _lib
    if _lib is not None and LIB == NATIVE_LIB:
        return LIB
    if _lib is not None:
        raise RuntimeError("the oracle is already loaded")
    tmp = NATIVE_LIB + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", *NATIVE_FLAGS, "-std=c99", "-fPIC", "-shared", "-fopenmp",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, NATIVE_LIB)
    LIB = NATIVE_LIB
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        L.or_philox4x32_10.argtypes = [_up, _up, _up]
        L.or_uniform_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_uint32, C.c_uint32, C.c_uint32, _dp]
        L.or_problem_new.restype = C.c_void_p
        L.or_problem_new.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_int, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p]
        L.or_problem_new_gp.restype = C.c_void_p
        L.or_problem_new_gp.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.or_problem_new_rg.restype = C.c_void_p
        L.or_problem_new_rg.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double]
        L.or_problem_free.argtypes = [C.c_void_p]
        L.or_loglik.restype = C.c_double
        L.or_loglik.argtypes = [C.c_void_p, _dp]
        L.or_logprior.restype = C.c_double
        L.or_logprior.argtypes = [C.c_void_p, _dp]
        L.or_hrss_chain.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, C.c_double,
                                    C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                    C.c_uint32, C.c_uint32, _lp, C.c_void_p]
        L.or_run_new.restype = C.c_void_p
        L.or_run_new.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int,
                                 C.c_int, C.c_double, C.c_uint64, C.c_uint32]
        L.or_run_free.argtypes = [C.c_void_p]
        L.or_init.restype = C.c_int
        L.or_init.argtypes = [C.c_void_p]
        L.or_step.restype = C.c_int
        L.or_step.argtypes = [C.c_void_p, C.c_int]
        L.or_smc_new.restype = C.c_void_p
        L.or_smc_new.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                 C.c_double, C.c_uint64, C.c_uint32]
        L.or_smc_init.restype = None
        L.or_smc_init.argtypes = [C.c_void_p]
        L.or_smc_step.restype = C.c_int
        L.or_smc_step.argtypes = [C.c_void_p, C.c_int]
        L.or_hrss_chain_tempered.restype = None
        L.or_hrss_chain_tempered.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, C.c_double,
                                             C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                             C.c_uint32, C.c_uint32, _lp, C.c_void_p]
        L.or_get_dead_x.restype = C.c_int64
        L.or_get_dead_x.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.or_posterior_samples.restype = None
        L.or_posterior_samples.argtypes = [_dp, C.c_void_p, C.c_int64, _dp, C.c_void_p,
                                           C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int,
                                           C.c_double, C.c_uint64, C.c_uint32, C.c_int,
                                           C.c_void_p, C.c_void_p]
        L.or_run_set_replacement.restype = C.c_int
        L.or_run_set_replacement.argtypes = [C.c_void_p, C.c_int]
        L.or_run_set_freeze.restype = C.c_int
        L.or_run_set_freeze.argtypes = [C.c_void_p, C.c_int]
        L.or_run_set_factor.restype = C.c_int
        L.or_run_set_diag.restype = C.c_int
        L.or_run_set_diag.argtypes = [C.c_void_p, C.c_int]
        L.or_run_set_factor.argtypes = [C.c_void_p, _dp]
        L.or_rw_chain.restype = None
        L.or_rw_chain.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, C.c_double, C.c_int,
                                  C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, _lp,
                                  C.c_void_p]
        L.or_logz.argtypes = [C.c_void_p, _dp]
        L.or_get_state.argtypes = [C.c_void_p, _dp, _dp, _ip, _dp, _lp, _lp]
        L.or_set_state.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_int64]
        L.or_get_aux.argtypes = [C.c_void_p, _dp, _ip]
        L.or_geom.restype = None
        L.or_geom.argtypes = [_dp, C.c_int64, _dp, C.c_int64, C.c_int, C.c_int, C.c_int,
                              C.c_double, C.c_uint64, C.c_uint32, _dp, C.c_void_p, C.c_void_p]
        L.or_get_dead.restype = C.c_int64
        L.or_get_dead.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        _lib = L
    return _lib


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def uniform_pair(seed, run_id, purpose, index, c1, c2, c3) -> np.ndarray:
    out = np.zeros(2)
    lib().or_uniform_pair(seed, run_id, purpose, index, c1, c2, c3, out)
    return out


class Problem:
    """Prior Pi and energy E = -log L, given as the generator's arrays."""

    def __init__(self, prob: dict):
        self.prob = prob
        d = int(prob["d"])
        self.d = d
        pa = np.ascontiguousarray(prob["prior_a"], np.float64)
        pb = np.ascontiguousarray(prob["prior_b"], np.float64)
        pk = PRIOR_BOX if prob["prior"] == "box" else PRIOR_GAUSS
        if prob["lik"] == "mixture":
            K = int(prob["K"])
            self._keep = [np.ascontiguousarray(prob["logw"], np.float64),
                          np.ascontiguousarray(prob["mu"], np.float64).reshape(K, d),
                          np.ascontiguousarray(prob["cov"], np.float64).reshape(K, d, d)]
            ptrs = [a.ctypes.data for a in self._keep]
            self.h = lib().or_problem_new(d, pk, pa, pb, LIK_MIXTURE, K, *ptrs)
        elif prob["lik"] == "funnel":
            self.h = lib().or_problem_new(d, pk, pa, pb, LIK_FUNNEL, 0, None, None, None)
        elif prob["lik"] == "rastrigin":
            self.h = lib().or_problem_new_rg(d, pk, pa, pb, float(prob["alpha"]),
                                             float(prob["amp"]))
        elif prob["lik"] == "gp":
            gx = np.ascontiguousarray(prob["gp_x"], np.float64)
            gy = np.ascontiguousarray(prob["gp_y"], np.float64)
            if d != 6 or prob["prior"] != "box" or gx.shape != (len(gy), 2):
                raise ValueError("GP problem: d = 6, box prior on log theta, X of shape (n, 2)")
            self._keep = [gx, gy]
            self.h = lib().or_problem_new_gp(len(gy), gx, gy, pa, pb)
        else:
            raise ValueError(prob["lik"])
        if not self.h:
            raise ValueError("oracle rejected the problem")

    def __del__(self):
        # at interpreter shutdown the module globals may already be gone
        if getattr(self, "h", None) and _lib is not None:
            _lib.or_problem_free(self.h)
            self.h = None

    def loglik(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        return np.array([lib().or_loglik(self.h, xi) for xi in x])

    def logprior(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), np.float64)
        return np.array([lib().or_logprior(self.h, xi) for xi in x])

    def hrss_chain(self, x, logL, Lstar, Lsig, width, p, seed, run_id, it, chain,
                   stepout_cap=10, shrink_cap=100, trace=False):
        """One chain of p HRSS steps; returns (x, logL, counters[6], trace or None)."""
        x = np.array(x, np.float64, copy=True)
        lv = np.array([logL], np.float64)
        ctr = np.zeros(6, np.int64)
        tr = np.zeros((p, 4), np.int32) if trace else None
        lib().or_hrss_chain(self.h, x, lv, float(Lstar),
                            np.ascontiguousarray(Lsig, np.float64), float(width), int(p),
                            int(stepout_cap), int(shrink_cap), int(seed), int(run_id), int(it),
                            int(chain), ctr, tr.ctypes.data if trace else None)
        return x, float(lv[0]), ctr, tr

    def hrss_chain_tempered(self, x, logL, beta, Lsig, width, p, seed, run_id, it, chain,
                            stepout_cap=10, shrink_cap=100, trace=False):
        """One chain of p HRSS steps on Pi L^beta (no hard constraint); returns (x, logL,
        counters[6], trace or None)."""
        x = np.array(x, np.float64, copy=True)
        lv = np.array([logL], np.float64)
        ctr = np.zeros(6, np.int64)
        tr = np.zeros((p, 4), np.int32) if trace else None
        lib().or_hrss_chain_tempered(self.h, x, lv, float(beta),
                                     np.ascontiguousarray(Lsig, np.float64), float(width),
                                     int(p), int(stepout_cap), int(shrink_cap), int(seed),
                                     int(run_id), int(it), int(chain), ctr,
                                     tr.ctypes.data if trace else None)
        return x, float(lv[0]), ctr, tr

    def rw_chain(self, x, logL, Lstar, Lsig, scale, p, seed, run_id, it, chain, trace=False):
        """One chain of p constrained random-walk steps; returns (x, logL, counters[6],
        trace or None)."""
        x = np.array(x, np.float64, copy=True)
        lv = np.array([logL], np.float64)
        ctr = np.zeros(6, np.int64)
        tr = np.zeros((p, 4), np.int32) if trace else None
        lib().or_rw_chain(self.h, x, lv, float(Lstar), np.ascontiguousarray(Lsig, np.float64),
                          float(scale), int(p), int(seed), int(run_id), int(it), int(chain), ctr,
                          tr.ctypes.data if trace else None)
        return x, float(lv[0]), ctr, tr


class Run:
    """One NS run of the oracle: init, step until done, logz."""

    def __init__(self, problem: Problem, m, k, p, width, seed, run_id=0, term_frac=1e-3,
                 stepout_cap=10, shrink_cap=100, threads=1, replacement="hrss",
                 freeze_whitening=False, diagonal_metric=False):
        """replacement "hrss" (width = slice width) or "rw" (width = random-walk scale);
        freeze_whitening keeps the first iteration's whitening factor for the whole run;
        diagonal_metric whitens by the survivors' variances alone."""
        self.P = problem
        self.m, self.k, self.p, self.d = m, k, p, problem.d
        self.threads = threads
        self.h = lib().or_run_new(problem.h, m, k, p, float(width), stepout_cap, shrink_cap,
                                  float(term_frac), int(seed), int(run_id))
        if not self.h:
            raise ValueError("oracle rejected the run configuration")
        if lib().or_run_set_replacement(self.h, {"hrss": 0, "rw": 1}[replacement]) != 0:
            raise ValueError(replacement)
        if lib().or_run_set_freeze(self.h, 1 if freeze_whitening else 0) != 0:
            raise ValueError(freeze_whitening)
        if lib().or_run_set_diag(self.h, 1 if diagonal_metric else 0) != 0:
            raise ValueError(diagonal_metric)
        self.done = False

    def set_factor(self, L):
        """Keep the lower-triangular factor L (d x d) as the whitening for the whole run
        (runs with freeze_whitening only)."""
        L = np.ascontiguousarray(L, np.float64)
        if L.shape != (self.d, self.d) or lib().or_run_set_factor(self.h, L) != 0:
            raise ValueError("a d x d factor on a run with frozen whitening")

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_run_free(self.h)
            self.h = None

    def init(self) -> bool:
        self.done = bool(lib().or_init(self.h))
        return self.done

    def step(self) -> bool:
        r = lib().or_step(self.h, int(self.threads))
        if r < 0:
            raise RuntimeError("no survivor strictly above the threshold")
        self.done = bool(r)
        return self.done

    def run(self, max_iter=100000) -> int:
        if not self.done:
            it = 0
            while not self.done and it < max_iter:
                self.step()
                it += 1
        return self.iter

    def logz(self):
        out = np.zeros(3)
        lib().or_logz(self.h, out)
        return float(out[0]), float(out[1]), float(out[2])

    def state(self) -> dict:
        m, d = self.m, self.d
        x = np.zeros((m, d)); logL = np.zeros(m); perm = np.zeros(m, np.int32)
        sc = np.zeros(4); it = np.zeros(1, np.int64); ctr = np.zeros(6, np.int64)
        lib().or_get_state(self.h, x, logL, perm, sc, it, ctr)
        return dict(x=x, logL=logL, perm=perm, Lstar=sc[0], logZ=sc[1], logX=sc[2], M=sc[3],
                    iter=int(it[0]), evals=int(ctr[0]), tests=int(ctr[1]),
                    prior_rejects=int(ctr[2]), stepout_caps=int(ctr[3]),
                    shrink_caps=int(ctr[4]), nonfinite=int(ctr[5]))

    def set_state(self, x, logL, logZ, logX, M, iter_):
        lib().or_set_state(self.h, np.ascontiguousarray(x, np.float64),
                           np.ascontiguousarray(logL, np.float64),
                           np.array([logZ, logX, M], np.float64), int(iter_))

    def aux(self):
        Ls = np.zeros((self.d, self.d)); par = np.zeros(self.k, np.int32)
        lib().or_get_aux(self.h, Ls, par)
        return Ls, par

    def dead(self) -> np.ndarray:
        n = lib().or_get_dead(self.h, None, 0)
        out = np.zeros(n)
        lib().or_get_dead(self.h, out.ctypes.data, n)
        return out

    def dead_x(self) -> np.ndarray:
        n = lib().or_get_dead_x(self.h, None, 0)
        out = np.zeros((n, self.d))
        lib().or_get_dead_x(self.h, out.ctypes.data, n)
        return out

    @property
    def iter(self) -> int:
        return self.state()["iter"]


def posterior_samples(dead, dead_x, final_logL, final_x, m, k, R, n, beta=1.0, seed=0,
                      run_id=0):
    """Weighted posterior samples (resampling with the geometric-mean weights of geom()).
    final_logL / final_x are the survivors in ascending (logL, index) order.  Returns
    (x[n, d], idx[n])."""
    dead = np.ascontiguousarray(dead, np.float64)
    dx = np.ascontiguousarray(dead_x, np.float64)
    fl = np.ascontiguousarray(final_logL, np.float64)
    fx = np.ascontiguousarray(final_x, np.float64)
    d = fx.shape[1]
    x = np.zeros((n, d))
    idx = np.zeros(n, np.int64)
    lib().or_posterior_samples(dead, dx.ctypes.data, len(dead), fl, fx.ctypes.data, len(fl), d,
                               int(m), int(k), int(R), float(beta), int(seed), int(run_id),
                               int(n), x.ctypes.data, idx.ctypes.data)
    return x, idx


def geom(dead, final_logL, m, k, R, beta=1.0, seed=0, run_id=0, weights=True):
    """Post-hoc geometric uncertainty of an NS run (App. "Estimation of prior volumes and
    propagation of geometric uncertainty"): dead = dead-point logL in death order, final_logL =
    the final survivors' logL.  Returns (logz[R], logw_mean[N] or None, ess)."""
    dead = np.ascontiguousarray(dead, np.float64)
    fin = np.ascontiguousarray(np.sort(np.asarray(final_logL, np.float64)))
    N = len(dead) + len(fin)
    logz = np.zeros(R)
    lw = np.zeros(max(N, 1)) if weights else None
    ess = np.zeros(1)
    lib().or_geom(dead, len(dead), fin, len(fin), int(m), int(k), int(R), float(beta), int(seed),
                  int(run_id), logz, lw.ctypes.data if weights else None, ess.ctypes.data)
    return logz, (lw[:N] if weights else None), float(ess[0])


class SMC(Run):
    """Adaptive tempered SMC with the slice-sampling mutation (the oracle's or_smc_*): init(),
    step() -> True once beta = 1, run(); state()["Lstar"] holds beta, "logZ" the estimate."""

    def __init__(self, problem: Problem, m, p, width, seed, run_id=0, ess_frac=0.5,
                 stepout_cap=10, shrink_cap=100, threads=1):
        self.P = problem
        self.m, self.k, self.p, self.d = m, m, p, problem.d
        self.threads = threads
        self.h = lib().or_smc_new(problem.h, m, p, float(width), stepout_cap, shrink_cap,
                                  float(ess_frac), int(seed), int(run_id))
        if not self.h:
            raise ValueError("oracle rejected the SMC configuration")
        self.done = False

    def init(self) -> bool:
        lib().or_smc_init(self.h)
        self.done = False
        return False

    def step(self) -> bool:
        r = lib().or_smc_step(self.h, int(self.threads))
        if r < 0:
            raise RuntimeError(f"or_smc_step failed ({r})")
        self.done = bool(r)
        return self.done

    def run(self, max_iter=100000) -> int:
        n = 0
        while not self.done and n < max_iter:
            self.step()
            n += 1
        return n

    def beta(self) -> float:
        return self.state()["Lstar"]
