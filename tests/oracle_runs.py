"""Oracle-side runs for the GPU parity tests.

Every input the oracle receives here is drawn by the oracle itself, from the same seeds and
Philox streams as the GPU run it is compared with: the initial state, the threshold, the
whitening factor and the parents of an iteration come from the oracle's own run, never from
the GPU's outputs.  The GPU's values are only ever compared against these.
"""
from __future__ import annotations

import os

THREADS = min(os.cpu_count() or 1, 16)


def first_iteration(O, prob, m, k, p, width, seed, run_id=0, replacement="hrss"):
    """The oracle's run through its first iteration: (Problem, Run, state before, state after,
    whitening factor, parents) of iteration 1."""
    P = O.Problem(prob)
    r = O.Run(P, m, k, p, width, seed, run_id=run_id, threads=THREADS, replacement=replacement)
    r.init()
    s0 = r.state()
    r.step()
    s1 = r.state()
    Ls, par = r.aux()
    return P, r, s0, s1, Ls, par


def run_iterations(O, prob, m, k, p, width, seed, n_iter, run_id=0):
    """The oracle's run after n_iter iterations (or at termination, whichever comes first)."""
    P = O.Problem(prob)
    r = O.Run(P, m, k, p, width, seed, run_id=run_id, threads=THREADS)
    r.init()
    for _ in range(n_iter):
        if r.done:
            break
        r.step()
    return P, r


def deaths(r):
    """(dead record, survivors' logL in ascending order, their coordinates in that order)."""
    s = r.state()
    fin = s["perm"][r.k:]
    return r.dead(), s["logL"][fin], s["x"][fin]
