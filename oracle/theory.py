"""Slice-width tuning theory of the paper, computed plainly (numpy / scipy quadrature).

TEST INFRASTRUCTURE ONLY (see oracle/oracle.py).

- cost of one HRSS update given the chord length l (Sec. 3.3, eq. slice-sampling cost
  formula; App. E theorem "Computational cost"): E[N_out|l] = l/w,
  E[N_shrink|l] = 1 + 2 phi(w/l), phi(u) = ((1+u) ln(1+u) - u)/u;
- optimal width for a fixed chord (App. E theorem "Optimal slice width in a fixed slice"):
  w* = u* l with u* - ln(1+u*) = 1/2, i.e. u* = -1 - W_{-1}(-e^{-3/2});
- optimal width in an ellipsoid (App. E theorem "Optimal slice width in an ellipsoid"):
  w* = 4 kappa_inf sqrt(2/(pi mu_d d)), where kappa_inf solves the fixed point
  kappa = 1/2 + E[R ln(1 + kappa/R)], R = sqrt(Q)/E[sqrt(Q)], Q ~ Gamma(3/2, scale 2);
- the ball corollary w* = 4 kappa_inf R sqrt(2/(pi d)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize, special, stats


def phi(u):
    u = np.asarray(u, np.float64)
    return ((1.0 + u) * np.log1p(u) - u) / u


def expected_stepouts(l, w):
    return l / w


def expected_shrinks(l, w):
    return 1.0 + 2.0 * phi(w / l)


def expected_cost(l, w):
    """E[N_evals | l] as the paper states it (expansions + shrink proposals)."""
    return expected_stepouts(l, w) + expected_shrinks(l, w)


def u_star() -> float:
    """Root of u - ln(1+u) = 1/2 (bracketed root finding)."""
    return optimize.brentq(lambda u: u - math.log1p(u) - 0.5, 1e-6, 10.0, xtol=1e-15)


def u_star_lambertw() -> float:
    return float(-1.0 - special.lambertw(-math.exp(-1.5), k=-1).real)


def kappa_inf(tol=1e-13, max_iter=200) -> float:
    """Fixed-point iteration kappa_{n+1} = 1/2 + f(kappa_n)."""
    eq = 2.0 * math.sqrt(2.0 / math.pi)          # E[sqrt(Q)], Q ~ Gamma(3/2, scale 2)
    dens = stats.gamma(a=1.5, scale=2.0).pdf

    def f(kap):
        g = lambda s: math.sqrt(s) * math.log1p(kap * eq / math.sqrt(s)) * dens(s) if s > 0 else 0.0
        val, _ = integrate.quad(g, 0.0, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)
        return val / eq

    k = 1.0
    for _ in range(max_iter):
        kn = 0.5 + f(k)
        if abs(kn - k) < tol:
            return kn
        k = kn
    return k


def width_ellipsoid(mu_d: float, d: int, kap: float | None = None) -> float:
    kap = kappa_inf() if kap is None else kap
    return 4.0 * kap * math.sqrt(2.0 / (math.pi * mu_d * d))


def width_ball(R: float, d: int, kap: float | None = None) -> float:
    kap = kappa_inf() if kap is None else kap
    return 4.0 * kap * R * math.sqrt(2.0 / (math.pi * d))


def width_whitened(d: int, kap: float | None = None) -> float:
    """Width in whitened coordinates: a uniform ball with unit covariance has radius
    sqrt(d+2) (its covariance is R^2/(d+2) I), so the ball rule gives this value."""
    return width_ball(math.sqrt(d + 2.0), d, kap)


def mean_chord_ellipsoid(mu_d: float, d: int) -> float:
    """Leading-order mean chord length 4 sqrt(2/(pi mu_d d)) (App. E, chord-length lemma)."""
    return 4.0 * math.sqrt(2.0 / (math.pi * mu_d * d))
