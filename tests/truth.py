"""Closed-form and quadrature evidences of the synthetic problems (test-side ground truth)."""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate
from scipy.special import erf
from scipy.stats import multivariate_normal, norm


def lnz_gauss_box_isotropic(d, sigma, half_width):
    """Normalised N(0, sigma^2 I) likelihood, uniform prior on [-a, a]^d (config 1)."""
    return -d * math.log(2 * half_width) + d * math.log(erf(half_width / (sigma * math.sqrt(2))))


def lnz_gauss_gauss(mean, cov, prior_mean, prior_std):
    """Normalised N(x; mean, cov) likelihood under the prior N(prior_mean, diag(std^2)):
    Z = N(mean; prior_mean, cov + diag(std^2))."""
    d = len(mean)
    C = np.asarray(cov) + np.diag(np.broadcast_to(prior_std, (d,)) ** 2)
    return float(multivariate_normal(mean=np.broadcast_to(prior_mean, (d,)), cov=C).logpdf(mean))


def lnz_funnel_box(d, box):
    """Funnel likelihood under the uniform prior [-box, box]^d, by 1-D quadrature over v."""
    def f(v):
        s = math.exp(v / 2.0)
        return norm.pdf(v, 0.0, 3.0) * erf(box / (math.sqrt(2.0) * s)) ** (d - 1)
    val, _ = integrate.quad(f, -box, box, limit=400, epsabs=0, epsrel=1e-12)
    return -d * math.log(2 * box) + math.log(val)


def lnz_grid_2d(loglik, lo, hi, n=2001):
    """Brute-force 2-D quadrature of L(x) under a uniform prior on [lo, hi]^2 (Simpson)."""
    xs = np.linspace(lo, hi, n)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    ll = loglik(pts).reshape(n, n)
    mx = ll.max()
    inner = integrate.simpson(np.exp(ll - mx), x=xs, axis=1)
    tot = integrate.simpson(inner, x=xs)
    return mx + math.log(tot) - 2 * math.log(hi - lo)
