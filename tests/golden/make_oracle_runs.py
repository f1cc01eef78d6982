"""Writes the oracle's full-size reference runs used by the end-to-end GPU parity tests.

Calls only the FP64 CPU oracle (``oracle/``) and the seeded problem generator; nothing here
comes from the GPU library.  Run from the repository root:

    python tests/golden/make_oracle_runs.py [mixture|gp|all]

mixture: the d=64, 8-component mixture (uniform prior [-10,10]^64, n_live=2000, k=1000) at the
    chain length p = 5d, whitened-ball width, seed 0, FP64, run to termination (Alg. 1 with the
    stop rule of Sec. 2.1): iteration count, evaluation counts and ln Z, sigma, H; and per
    iteration L*, ln Z and the evaluation counts.
gp: the GP hyperparameter workload (256 inputs, n_live=1000, k=500, p=30), seed 0, FP64, over
    a fixed number of iterations: after each iteration L*, ln Z, ln X and the evaluation count.
"""
from __future__ import annotations

import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O, theory as T          # noqa: E402
from paper_2601_23252_amd import problems as G        # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = os.cpu_count() or 1
GP_ITERS = 8


def _write(name, header, rows):
    with open(os.path.join(HERE, name), "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        for r in rows:
            f.write(" ".join(str(v) for v in r) + "\n")


def mixture(seed=0):
    prob = G.config3()
    d, m, k = prob["d"], prob["m"], prob["k"]
    p = 5 * d
    w = T.width_whitened(d)
    r = O.Run(O.Problem(prob), m, k, p, w, seed, threads=THREADS)
    t0 = time.time()
    r.init()
    per_iter = []
    while True:
        st = r.state()
        per_iter.append((st["iter"], repr(float(st["Lstar"])), repr(float(st["logZ"])),
                         st["evals"], st["tests"]))
        if r.done:
            break
        r.step()
        if r.iter % 25 == 0:
            print(f"mixture iteration {r.iter}, {time.time() - t0:.0f} s", flush=True)
    z, err, H = r.logz()
    st = r.state()
    _write(f"oracle_mixture8_d64_p5d_seed{seed}_iters.txt",
           ["Per-iteration record of the run in oracle_mixture8_d64_p5d_seed0.txt (same script):",
            "iteration L* lnZ evals tests"], per_iter)
    rows = [("iterations", st["iter"]), ("evals", st["evals"]), ("tests", st["tests"]),
            ("prior_rejects", st["prior_rejects"]), ("stepout_caps", st["stepout_caps"]),
            ("shrink_caps", st["shrink_caps"]), ("logz", repr(float(z))),
            ("sigma", repr(float(err))), ("H", repr(float(H))),
            ("Lstar", repr(float(st["Lstar"]))), ("logX", repr(float(st["logX"])))]
    _write(f"oracle_mixture8_d64_p5d_seed{seed}.txt",
           ["Oracle run (FP64, written by tests/golden/make_oracle_runs.py): d=64 mixture of 8",
            f"Gaussians, n_live={m}, k={k}, p={p}, width {w!r}, seed {seed}, term_frac 1e-3,",
            f"run to termination; {time.time() - t0:.0f} s on {THREADS} threads.",
            f"ln Z truth -64 ln 20 = {-64 * math.log(20.0)!r}"], rows)


def gp(seed=0):
    prob = G.config4()
    d, m, k, p = prob["d"], prob["m"], prob["k"], prob["p"]
    w = T.width_whitened(d)
    r = O.Run(O.Problem(prob), m, k, p, w, seed, threads=THREADS)
    t0 = time.time()
    r.init()
    rows = []
    for it in range(GP_ITERS + 1):
        if it > 0:
            r.step()
        st = r.state()
        rows.append((it, repr(float(st["Lstar"])), repr(float(st["logZ"])),
                     repr(float(st["logX"])), st["evals"], st["tests"],
                     repr(float(st["logL"].sum()))))
        print(f"gp iteration {it}, {time.time() - t0:.0f} s", flush=True)
    _write(f"oracle_gp_n256_seed{seed}.txt",
           ["Oracle run (FP64, written by tests/golden/make_oracle_runs.py): GP workload, 256",
            f"inputs, n_live={m}, k={k}, p={p}, width {w!r}, seed {seed}; one row per iteration:",
            "iteration L* lnZ lnX evals tests sum(live logL)"], rows)


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    if which in ("gp", "all"):
        gp()
    if which in ("mixture", "all"):
        mixture()
