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


def lnz_rastrigin_gauss(d, alpha, r=5.14, amp=10.0):
    """Semi-analytic evidence of L = alpha f + (1 - alpha) g under U[-r, r]^d (the paper's
    evidence comparison of constrained samplers): the d-dimensional integrals factor into
    one-dimensional ones, int_{-r}^{r} e^{-x^2/2} dx = sqrt(2 pi) erf(r / sqrt 2) and
    int_{-r}^{r} e^{A cos 2 pi x} dx = 2 n I0(A) + 2 int_n^r e^{A cos 2 pi x} dx with n = floor(r)
    whole periods (each period integrates to the modified Bessel value I0(A))."""
    from scipy.special import i0e
    n = math.floor(r)
    tail, _ = integrate.quad(lambda x: math.exp(amp * (math.cos(2 * math.pi * x) - 1.0)), n, r,
                             epsabs=0, epsrel=1e-13)
    # log int e^{A cos} = A + log(2 n I0(A) e^{-A} + 2 tail e^{-A})
    log_ig = amp + math.log(2 * n * float(i0e(amp)) + 2 * tail)
    log_if = 0.5 * math.log(2 * math.pi) + math.log(erf(r / math.sqrt(2)))
    terms = []
    if alpha > 0:
        terms.append(math.log(alpha) + d * log_if)
    if alpha < 1:
        terms.append(math.log1p(-alpha) - amp * d + d * log_ig)
    mx = max(terms)
    return mx + math.log(sum(math.exp(t - mx) for t in terms)) - d * math.log(2 * r)
