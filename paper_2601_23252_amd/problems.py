"""Seeded synthetic problems (prior + likelihood parameters) for Nested Slice Sampling.

This module only draws problem inputs from seeds; it holds none of the sampler's arithmetic.
Both the GPU library's callers and the CPU reference take its dictionaries as plain arrays.

A problem is a dict with
    d                   dimension
    prior               "box" (prior_a = lower, prior_b = upper) or
                        "gauss" (prior_a = mean, prior_b = standard deviation), per coordinate
    lik                 "mixture" (K, logw[K], mu[K,d], cov[K,d,d]), "funnel"
                        (v = x_0 ~ N(0, 9), x_j | v ~ N(0, e^v) for j >= 1), "gp" (gp_x, gp_y)
                        or "rastrigin" (alpha, amp)
    name, and the run shape m (live points), k (deletions per iteration), p (chain length).

Workloads (synthetic, seeded; the paper's experiments use real datasets that stand behind
these shapes, see the design notes):
    config1   d=5 isotropic Gaussian N(0, 0.01 I), uniform prior [-1,1]^5, m=200, k=50, p=5d
    config2   d=32 correlated Gaussian: mean ~ U[-1,1]^d, cov = Q diag(lam) Q^T, Q Haar,
              log10 lam uniform on [-3, 0] with both ends pinned (condition number 1e3),
              prior N(0, 4 I); m=1000, k=500, p=5d
    config3   d=64 mixture of 8 equal-weight Gaussians, means ~ U[-5,5]^d,
              cov_i = Q_i diag(s_i^2) Q_i^T with s_ij ~ U[0.05, 0.5]; uniform prior
              [-10,10]^d; m=2000, k=1000, p=5d
    gaussian20  prior N(0, I), likelihood N(x; 1, 0.01 I), d=20 (the paper's overhead example)
    funnel    prior U[-20,20]^d, Neal's funnel likelihood
    config4   GP hyperparameter marginalisation: 256 inputs ~ U[0,10]^2, targets drawn from
              a GP with a squared-exponential x periodic kernel (product over the two input
              dimensions) plus N(0, 0.1^2) noise; 6 hyperparameters
              theta = (sigma_f, l_1, l_2, l_p, P, sigma_n), log-uniform on [1e-2, 1e2]
              (a box prior on u = log theta); m=1000, k=500, p=5d=30
    config5   batched serving: 256 independent runs, d uniform on {8, 16, ..., 128}; even runs
              a correlated Gaussian drawn as config2 (prior N(0, 4 I)), odd runs the funnel
              under U[-20,20]^d; m=500, k=250, p=5d each
    rastrigin_gauss   L = alpha N-shaped f + (1 - alpha) Rastrigin-shaped g under U[-5.14,5.14]^d,
              A = 10; m=1000, k=500, p=25d
    illcond_gaussian  Gaussian N(0, C) with condition number 100 under U[-20,20]^d (the
              slice-versus-random-walk comparison); m=1000, k=500
"""
from __future__ import annotations

import numpy as np


def haar_orthogonal(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the signs of R's
    diagonal moved into Q (Mezzadri 2007)."""
    z = rng.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))[None, :]


def _sym(c):
    return 0.5 * (c + c.T)


def gaussian_problem(d, mean, cov, prior="box", prior_a=None, prior_b=None, name="gaussian",
                     m=200, k=50, p=None):
    prior_a = np.full(d, -1.0) if prior_a is None else np.broadcast_to(prior_a, (d,)).astype(np.float64)
    prior_b = np.full(d, 1.0) if prior_b is None else np.broadcast_to(prior_b, (d,)).astype(np.float64)
    return dict(name=name, d=d, prior=prior, prior_a=np.array(prior_a, np.float64),
                prior_b=np.array(prior_b, np.float64), lik="mixture", K=1,
                logw=np.zeros(1), mu=np.asarray(mean, np.float64).reshape(1, d),
                cov=np.asarray(cov, np.float64).reshape(1, d, d),
                m=m, k=k, p=5 * d if p is None else p)


def config1(seed: int = 1001):
    d = 5
    return gaussian_problem(d, np.zeros(d), 0.01 * np.eye(d), "box", -1.0, 1.0,
                            name="config1_gauss5", m=200, k=50)


def config2(seed: int = 1002, d: int = 32, m: int = 1000, k: int = 500):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, d)
    q = haar_orthogonal(rng, d)
    u = rng.uniform(0.0, 1.0, d)
    u[0], u[1] = 0.0, 1.0
    lam = 10.0 ** (-3.0 + 3.0 * u)
    cov = _sym((q * lam[None, :]) @ q.T)
    return gaussian_problem(d, mean, cov, "gauss", 0.0, 2.0, name=f"config2_corr{d}",
                            m=m, k=k)


def illcond_gaussian(d: int, seed: int = 1006, kappa: float = 100.0, m: int = 1000,
                     k: int = 500, p=None):
    """The slice-versus-random-walk comparison target: a Gaussian likelihood N(0, C) with
    C = Q diag(lam) Q^T, Q Haar, log lam uniform on [-log10 kappa, 0] with both ends pinned
    (condition number kappa = 100), under the uniform prior [-20, 20]^d (wide enough that the
    constraint, not the prior, bounds the chains)."""
    rng = np.random.default_rng(seed + d)
    q = haar_orthogonal(rng, d)
    u = rng.uniform(0.0, 1.0, d)
    u[0], u[1] = 0.0, 1.0
    lam = 10.0 ** (-np.log10(kappa) * (1.0 - u))
    cov = _sym((q * lam[None, :]) @ q.T)
    return gaussian_problem(d, np.zeros(d), cov, "box", -20.0, 20.0, name=f"illcond{d}",
                            m=m, k=k, p=d if p is None else p)


def mixture_problem(seed: int, d: int, K: int, mean_lo=-5.0, mean_hi=5.0, s_lo=0.05, s_hi=0.5,
                    box=10.0, m=2000, k=1000, p=None, name=None):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(mean_lo, mean_hi, (K, d))
    cov = np.empty((K, d, d))
    for i in range(K):
        q = haar_orthogonal(rng, d)
        s = rng.uniform(s_lo, s_hi, d)
        cov[i] = _sym((q * (s * s)[None, :]) @ q.T)
    return dict(name=name or f"mixture{K}_d{d}", d=d, prior="box",
                prior_a=np.full(d, -box), prior_b=np.full(d, box), lik="mixture", K=K,
                logw=np.full(K, -np.log(K)), mu=mu, cov=cov, m=m, k=k,
                p=5 * d if p is None else p)


def config3(seed: int = 1003):
    return mixture_problem(seed, 64, 8, name="config3_mix8_d64")


def gaussian20():
    d = 20
    return gaussian_problem(d, np.ones(d), 0.01 * np.eye(d), "gauss", 0.0, 1.0,
                            name="gauss20_overhead", m=1000, k=100, p=d)


def funnel(d: int, box: float = 20.0, m: int = 500, k: int = 250, p=None):
    return dict(name=f"funnel_d{d}", d=d, prior="box", prior_a=np.full(d, -box),
                prior_b=np.full(d, box), lik="funnel", K=0, m=m, k=k,
                p=5 * d if p is None else p)


GP_THETA_TRUE = (1.0, 2.0, 3.0, 1.0, 2.5, 0.1)


def gp_problem(seed: int = 1004, n: int = 256, m: int = 1000, k: int = 500, p=None,
               theta=GP_THETA_TRUE, lo=1e-2, hi=1e2):
    """GP regression data drawn from the model at theta (the kernel matrix is built with
    scikit-learn's kernels and factorised with numpy, so this module computes none of it
    itself)."""
    from sklearn.gaussian_process.kernels import RBF, ExpSineSquared
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 10.0, (n, 2))
    sf, l1, l2, lp, per, sn = theta
    K = (sf ** 2 * RBF([l1, l2])(X) * ExpSineSquared(lp, per)(X[:, :1])
         * ExpSineSquared(lp, per)(X[:, 1:]) + sn ** 2 * np.eye(n))
    y = np.linalg.cholesky(K) @ rng.standard_normal(n)
    d = 6
    return dict(name=f"gp_n{n}", d=d, prior="box", prior_a=np.full(d, np.log(lo)),
                prior_b=np.full(d, np.log(hi)), lik="gp", K=0, gp_x=X, gp_y=y, m=m, k=k,
                p=5 * d if p is None else p)


def rastrigin_gauss(d: int, alpha: float, r: float = 5.14, amp: float = 10.0, m: int = 1000,
                    k: int = 500, p=None):
    """The Gaussian-Rastrigin test likelihood L = alpha f + (1 - alpha) g under the uniform prior
    on [-r, r]^d (the paper's constrained-sampler evidence comparison): f a unit Gaussian, g the
    Rastrigin-shaped exp(-A d + A sum cos(2 pi x_i)) with A = amp.  d in {2, 4, 10, 30, 100}
    (the paper also uses 300), 1000 live points, and 25 d slice steps per replacement (the
    slice sampler's default number of repeats in that comparison)."""
    return dict(name=f"rastrigin_d{d}_a{alpha:g}", d=d, prior="box", prior_a=np.full(d, -r),
                prior_b=np.full(d, r), lik="rastrigin", alpha=float(alpha), amp=float(amp),
                K=0, m=m, k=k, p=25 * d if p is None else p)


def config4(seed: int = 1004):
    return gp_problem(seed)


def config5(seed: int = 1005, n_runs: int = 256, m: int = 500, k: int = 250):
    """List of n_runs problem dicts of uneven dimension (see the module docstring)."""
    rng = np.random.default_rng(seed)
    dims = 8 * rng.integers(1, 17, n_runs)
    sub = rng.integers(0, 2**31 - 1, n_runs)
    out = []
    for r in range(n_runs):
        d = int(dims[r])
        if r % 2 == 0:
            pr = config2(int(sub[r]), d=d, m=m, k=k)
            pr["name"] = f"batch_gauss{d}_{r}"
        else:
            pr = funnel(d, m=m, k=k)
            pr["name"] = f"batch_funnel{d}_{r}"
        out.append(pr)
    return out


CONFIGS = {"config1": config1, "config2": config2, "config3": config3, "config4": config4}
