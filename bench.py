"""Benchmark: slice-step likelihood evaluations per second of Nested Slice Sampling on the
d=64, 8-component Gaussian mixture (uniform prior [-10,10]^64, n_live=2000, k=1000), mixed
precision vs FP64, with every timed run checked against the closed-form evidence
ln Z = -64 ln 20 (|d ln Z| < 3 sigma, sigma = sqrt(H / n_live)).

One step = one complete run of the hot path on the GPU: prior draws and the first delete-k,
then iterations of whitening, direction generation, k parallel HRSS chains, replacement,
delete-k and evidence accumulation until the remaining-evidence bound is below 1e-3 of Z, then
the final live-set contribution.  The problem is uploaded once, before the timed region.

The headline runs the workload's chain length p = 5d with the direction metric from the
survivors' variances (the diagonal restriction of the conditioning matrix that Sec. 3.2 suggests
for high dimensions; with the full covariance the 8-mode mixture's metric is dominated by the
spread between the modes and ln Z comes out far too high at p = 5d).  ``value`` counts only the
evaluations of runs whose ln Z passes the 3 sigma check, divided by the wall time of all timed
runs (the pass count is printed beside it, and ``rate_all_runs`` is the raw rate).  Labelled
legs run the same workload with the full-covariance metric at p = 5d and at p = 20d, and the
plain FP64 form with the headline's settings.

Prints one JSON line (see the keys below).  --gpus N > 1 is not supported (one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HBM bytes per launch of the chain kernel from the FETCH_SIZE / WRITE_SIZE counter passes, each
# scaled by the same counter on a copy of known size (FETCH x 2, WRITE x 1), keyed by
# (precision, chain length, chains per workgroup, planned tests per round), recorded for the
# kernel sources with this sha256 prefix; reported as null once the sources differ or for a
# shape the counters were not taken on.
TRAFFIC = {("fp16x3", 320, 4, 8): 196.7e6}
TRAFFIC_SOURCE_SHA = "fd6c2f8f156d9218"


# VALU lane-instructions per evaluation issued by the chain kernel (SQ_INSTS_VALU x 64 /
# evaluations of the profiled launches), keyed like TRAFFIC, for the kernel sources with this
# prefix: the instruction view of the same kernel (its chain logic runs on the vector ALU).
HRSS_VALU_PER_EVAL = {("fp16x3", 320, 4, 8): 24544.0}
HRSS_VALU_SOURCE_SHA = "fd6c2f8f156d9218"

KERNEL_SOURCES = ("nss_kernels.hip", "nss_hrss_plan.hip", "nss_tiles.hpp", "nss_internal.hpp")


def _kernel_sha():
    """sha256 prefix over the chain kernels' sources (the counters above hold for them only)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2601_23252_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _shape_key(precision, p, shape):
    return (precision, p, shape.get("chains_per_workgroup"), shape.get("tests_per_round"))


def hrss_valu_per_eval(precision, p, shape):
    if _kernel_sha() != HRSS_VALU_SOURCE_SHA:
        return None
    return HRSS_VALU_PER_EVAL.get(_shape_key(precision, p, shape))


def kernel_traffic(precision, p, shape):
    if _kernel_sha() != TRAFFIC_SOURCE_SHA:
        return None
    return TRAFFIC.get(_shape_key(precision, p, shape))


def chain_kernel_name(precision, shape):
    """The chain kernel a launch shape runs: the planned-test kernel for 8 or 16 tests per
    round, else the 4-test kernel."""
    mode = {"fp64": 0, "bf16": 1, "fp16": 2, "bf16x3": 3, "fp16x3": 4}.get(precision)
    plan = shape.get("tests_per_round")
    return ("k_hrss_plan" if plan in (8, 16) else "k_hrss") + f" (mode {mode}, {plan} tests)"


def algorithmic_flop_per_eval(K: int, d: int) -> int:
    """Triangular quadratic form per component (d(d+1) flop), residual, square and scaling
    (3d), per component: the work the likelihood must do per evaluation."""
    return K * d * (d + 1) + 3 * K * d


def run_gpu(N, prob, precision, seeds, p, warmup, timing=True, autotune=True, shape_out=None,
            diagonal_metric=False):
    """Runs len(seeds) full NS runs on one context (the launch shape tuned during the warmup
    runs, or on the first timed run without warmup); returns per-run records and totals."""
    import torch
    R = N.NSRun(prob, p=p, seed=seeds[0], precision=precision, timing=timing,
                autotune=autotune, diagonal_metric=diagonal_metric)
    for w in range(warmup):
        R.reset(10_000 + w)
        R.run()
    recs = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for s in seeds:
        t0 = time.perf_counter()
        R.reset(s)
        it = R.run()
        z, err, H = R.logz()
        dt = time.perf_counter() - t0
        st = R.stats()
        print(f"[bench] {precision} seed {s}: {it} iterations, {dt:.2f} s, {st['evals']} evals, "
              f"{st['evals'] / dt:.3e} evals/s, ln Z {z:.3f} +- {err:.3f}", file=sys.stderr,
              flush=True)
        recs.append(dict(seed=s, iters=it, wall_s=dt, evals=st["evals"], logz=z, err=err, H=H,
                         hrss_ms=st["hrss_ms"], hrss_launches=st["hrss_launches"],
                         rechecks=st["rechecks"], band_violations=st["band_violations"],
                         tests=st["tests"]))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    if shape_out is not None:
        c, plan = R.launch_shape()
        shape_out.update(chains_per_workgroup=c, tests_per_round=plan,
                         tune_launches=R.stats()["tune_launches"])
    R.close()
    return recs, total


def cpu_baseline(prob, p, seconds_budget=20.0, warm_iters=None, diagonal_metric=False):
    """The FP64 oracle on the host cores, built for this host (-O3 -march=native): iterations of
    the same workload from a mid-run live set until the time budget; evals/s over the timed
    iterations.  The mid-run state comes from the oracle itself: warm_iters iterations with a
    4-step chain (cheap), then the live set is copied into a run with the workload's chain
    length, so the timed iterations see contours from the middle of a run, not the prior."""
    from oracle import oracle as O, theory as T
    O.use_native_build()
    threads = os.cpu_count() or 1
    P = O.Problem(prob)
    m, k, d = prob["m"], prob["k"], prob["d"]
    w = T.width_whitened(d)
    warm_iters = warm_iters if warm_iters is not None else 150
    iters = ev = runs = 0
    dt = 0.0
    seed = 0
    wall0 = last = time.perf_counter()
    # the timed budget, bounded in wall time too (the warm-up iterations are untimed)
    while dt < seconds_budget and time.perf_counter() - wall0 < 4 * seconds_budget:
        run = O.Run(P, m, k, p, w, seed, threads=threads, diagonal_metric=diagonal_metric)
        if warm_iters > 0:
            warm = O.Run(P, m, k, 4, w, seed, threads=threads, diagonal_metric=diagonal_metric)
            warm.init()
            for _ in range(warm_iters):
                if warm.done:
                    break
                warm.step()
            ws = warm.state()
            del warm
            run.init()
            run.set_state(ws["x"], ws["logL"], ws["logZ"], ws["logX"], ws["M"], ws["iter"])
            e0 = run.state()["evals"]
            t0 = time.perf_counter()
        else:   # whole runs from the prior draws (short workloads)
            e0 = 0
            t0 = time.perf_counter()
            run.init()
        while dt + (time.perf_counter() - t0) < seconds_budget and not run.done:
            run.step()
            iters += 1
        dt += time.perf_counter() - t0
        ev += run.state()["evals"] - e0
        runs += 1
        seed += 1
        if time.perf_counter() - last > 5.0:
            last = time.perf_counter()
            print(f"[bench] cpu baseline: {iters} iterations, {dt:.1f} s timed", file=sys.stderr,
                  flush=True)
    how = (f"each from the live set after {warm_iters} iterations of a 4-step chain"
           if warm_iters > 0 else "whole runs from the prior draws")
    return dict(value=ev / dt, unit="evals/s", cores=threads, kind="oracle",
                sample=f"{iters} iterations over {runs} run(s) (seeds 0..{runs - 1}) of the same "
                       f"workload (p={p}), {how}, {ev} evaluations in {dt:.1f} s, OpenMP over chains "
                       "on every host thread, oracle built -O3 -march=native"
                       + (", diagonal metric" if diagonal_metric else ""), **host_info())


def host_info():
    """The host's logical CPU count and model (for the oracle timings)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def profile_run(args):
    """A short run for rocprofv3: the reference copy kernel, then a few outer iterations."""
    import torch
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    prob = G.config3()
    kw = {"tuned": dict(autotune=True), "rule": {}, "plan8": dict(plan8=True),
          "shallow": dict(shallow_plan=True),
          "inline": dict(shallow_plan=True, inline_directions=True)}[args.profile_shape]
    R = N.NSRun(prob, p=args.chain_factor * prob["d"], seed=0, precision=args.precision,
                timing=True, diagonal_metric=args.metric == "diagonal", **kw)
    t0 = time.perf_counter()
    for _ in range(args.profile_iters):
        R.step()
    torch.cuda.synchronize()
    st = R.stats()
    c, plan = R.launch_shape()
    print(json.dumps({"profile_iters": args.profile_iters, "precision": args.precision,
                      "shape": args.profile_shape, "chains_per_workgroup": c,
                      "tests_per_round": plan, "wall_s": time.perf_counter() - t0,
                      "evals": st["evals"], "hrss_ms": st["hrss_ms"],
                      "copy_bytes": 256 << 20}), flush=True)
    R.close()


def gp_flop_per_eval(n: int) -> float:
    """Cholesky n^3/3, forward solve n^2, and about 20 flops per lower-triangle entry of the
    kernel matrix."""
    return n ** 3 / 3 + n ** 2 + 20 * n * (n + 1) / 2


def run_until(R, max_seconds, chunk=4):
    """Outer iterations until termination or the time budget; returns (iterations, seconds)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    while time.perf_counter() - t0 < max_seconds:
        k = R.run(max_iter=chunk)
        it += k
        print(f"[bench] {it} iterations, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
        if k == 0:
            break
    torch.cuda.synchronize()
    return it, time.perf_counter() - t0


def bench_gp(args):
    """GP hyperparameter marginalisation: one run from the prior draws, timed until it
    terminates or the time budget ends (FP64, decisions identical to the oracle's)."""
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    prob = G.config4()
    n = len(prob["gp_y"])
    # FP32 leg first: FP32 MFMA Cholesky, FP64 refinement of the quadratic form, FP64
    # log-determinant sum; decisions near L* (and beyond n s = 2e6) in FP64
    R32 = N.NSRun(prob, seed=0, precision="fp32", timing=True)
    it32, dt32 = run_until(R32, args.max_seconds)
    st32 = R32.stats()
    z32 = R32.logz()[0]
    s32 = R32.state()
    R32.close()
    R = N.NSRun(prob, seed=0, precision="fp64", timing=True)
    it, dt = run_until(R, args.max_seconds)
    st = R.stats()
    z, err, H = R.logz()
    fpe = gp_flop_per_eval(n)
    hrss_s = st["hrss_ms"] / 1e3
    achieved = st["evals"] * fpe / hrss_s if hrss_s > 0 else 0.0
    out = {
        "metric": "slice-step likelihood evals/s (GP hyperparameter marginalisation)",
        "value": st["evals"] / dt, "unit": "evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "gp_rbfxperiodic_n256_nlive1000_k500", "n_obs": n, "d": 6,
                   "n_live": prob["m"], "k": prob["k"], "chain_len": prob["p"],
                   "iterations": it, "done": R.state()["done"]},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": "k_hrss_gp", "flop_per_eval": fpe,
                     "avg_launch_ms": st["hrss_ms"] / max(1, st["hrss_launches"])},
        "lnz": {"logz": z, "sigma": err, "H": H},
        "fp32": {"value": st32["evals"] / dt32, "unit": "evals/s", "iterations": it32,
                 "speedup_vs_fp64": (st32["evals"] / dt32) / (st["evals"] / dt),
                 "rechecks_per_eval": st32["rechecks"] / max(1, st32["evals"]),
                 "band_violations": st32["band_violations"],
                 "same_trajectory_as_fp64": bool(it32 == it and st32["evals"] == st["evals"]
                                                 and abs(z32 - z) < 1e-9),
                 "avg_launch_ms": st32["hrss_ms"] / max(1, st32["hrss_launches"]),
                 "done": s32["done"]},
    }
    if not args.no_cpu:
        # the oracle's GP likelihood (one host thread) on prior draws for the time budget
        import numpy as np
        from oracle import oracle as O
        P = O.Problem(prob)
        rng = np.random.default_rng(0)
        ev, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            P.loglik(rng.uniform(prob["prior_a"], prob["prior_b"], (64, 6)))
            ev += 64
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": ev / tc, "unit": "evals/s", "cores": 1, "kind": "oracle",
                               "sample": f"{ev} GP likelihood evaluations at prior draws in "
                                         f"{tc:.1f} s (the chains' evaluations cost the same)",
                               **host_info()}
    print(json.dumps(out), flush=True)
    R.close()


def bench_batch(args):
    """256 independent runs of uneven dimension (correlated Gaussians in BF16x3, funnels in
    FP64) in one context, timed until all terminate or the time budget ends."""
    import numpy as np
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    probs = G.config5()
    # eager iterations, the groups' chains concurrently on side streams (--graph: replays of
    # 16-iteration HIP graphs, which run the groups in sequence), no per-launch events: the
    # whole job is timed on the host clock; the launch shapes are tuned at the start
    runs = [(p, dict(seed=5, run_id=r, precision="bf16x3" if p["lik"] == "mixture" else "fp64",
                     max_iter=4000, graph=args.graph, autotune=not args.no_autotune,
                     serial_groups=args.serial_groups))
            for r, p in enumerate(probs)]
    B = N.NSBatch(runs)
    it, dt = run_until(B, args.max_seconds, chunk=64)
    cpw = {}
    for r in range(len(probs)):
        c = N.ns_chains_per_workgroup(B.ctx, r)
        cpw[str(c)] = cpw.get(str(c), 0) + 1
    stats = [B.stats(r) for r in range(len(probs))]
    evals = sum(s["evals"] for s in stats)
    fpe = [p["d"] * (p["d"] + 1) + 3 * p["d"] if p["lik"] == "mixture" else 3 * p["d"]
           for p in probs]
    flops = sum(s["evals"] * f for s, f in zip(stats, fpe))
    done = sum(B.state(r)["done"] for r in range(len(probs)))
    zs, errs, _ = B.logz()
    z_of = []
    for r, pr in enumerate(probs):
        if pr["lik"] == "mixture":
            from tests import truth as TR
            tz = TR.lnz_gauss_gauss(pr["mu"][0], pr["cov"][0], 0.0, 2.0)
        else:
            from tests import truth as TR
            tz = TR.lnz_funnel_box(pr["d"], 20.0)
        z_of.append((zs[r] - tz) / errs[r])
    out = {
        "metric": "slice-step likelihood evals/s (256 batched runs, d in {8..128})",
        "value": evals / dt, "unit": "evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "batch256_gauss_funnel_nlive500_k250_p5d", "runs": len(probs),
                   "runs_done": done, "max_iterations": it, "graphs": args.graph,
                   "concurrent_groups": not args.serial_groups,
                   "autotune": not args.no_autotune, "runs_by_chains_per_workgroup": cpw},
        "roofline": {"bound": "mfma", "achieved": flops / dt / 1e12, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": flops / dt / 2.5e15, "traffic": None,
                     "kernel": "whole job (host clock, all runs and kernels)",
                     "flop_per_eval": "d(d+1)+3d (Gaussian), 3d (funnel)"},
        "lnz": {"runs_within_3sigma": f"{sum(abs(z) < 3 for z in z_of)}/{len(z_of)}",
                "z_by_run": z_of},
    }
    if not args.no_cpu:
        # the oracle on a stratified subset: every 16th run, each for an equal share of the
        # time budget (init plus whole iterations)
        from oracle import oracle as O, theory as T
        threads = min(os.cpu_count() or 1, 16)
        ev_tot, t_tot, iters = 0, 0.0, 0
        sub = list(range(0, len(probs), 16))
        for r in sub:
            pr = probs[r]
            run = O.Run(O.Problem(pr), pr["m"], pr["k"], pr["p"], T.width_whitened(pr["d"]), 5,
                        run_id=r, threads=threads)
            run.init()
            e0 = run.state()["evals"]
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < args.cpu_seconds / len(sub) and not run.done:
                run.step()
                iters += 1
            t_tot += time.perf_counter() - t0
            ev_tot += run.state()["evals"] - e0
        out["cpu_baseline"] = {"value": ev_tot / t_tot, "unit": "evals/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"runs 0, 16, ..., 240 of the batch, {iters} iterations "
                                         f"after init in total, {ev_tot} evaluations in "
                                         f"{t_tot:.1f} s, OpenMP over chains", **host_info()}
    print(json.dumps(out), flush=True)
    B.close()


# The geometric-uncertainty kernels are bound by vector-ALU issue (Philox, FP64 log, exp and
# log1p per replica-death; no HBM stream).  VALU lane-instructions per replica-death of one
# ns_geom_uncertainty call (SQ_INSTS_VALU over its five kernels x 64 lanes / (R N)), recorded
# for the kernel source with this sha256 prefix; the peak is one lane-instruction per lane per
# cycle: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
GEOM_VALU_PER_UNIT = 455.2
GEOM_SOURCE_SHA = "ac3a36c198ebef19"
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def geom_ops():
    import hashlib
    src = os.path.join(ROOT, "paper_2601_23252_amd", "csrc", "nss_post.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return GEOM_VALU_PER_UNIT if sha == GEOM_SOURCE_SHA else None


def bench_geom(args):
    """Post-hoc geometric uncertainty of one full mixture run (the d=64 workload above, BF16x3,
    seed 0): R = 100 replicas of the shrinkage trajectory over all N deaths, log Z per replica,
    geometric-mean weights and the Kish ESS.  The run itself is set-up (untimed); each step is one
    ns_geom_uncertainty call, timed on the device with events around its launches."""
    import numpy as np
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    prob = G.config3()
    R_rep = args.replicas
    run = N.NSRun(prob, p=args.chain_factor * prob["d"], seed=0, precision="bf16x3",
                  record_points=True)
    run.run()
    print(f"[bench] setup run done: {run.stats()['n_dead']} dead points", file=sys.stderr,
          flush=True)
    for _ in range(args.warmup):
        run.geom(R=R_rep, beta=1.0, seed=1)
    ms, walls = [], []
    for i in range(args.steps):
        t0 = time.perf_counter()
        g = run.geom(R=R_rep, beta=1.0, seed=1, timing=True)
        walls.append(time.perf_counter() - t0)
        ms.append(g["device_ms"])
    n_deaths = len(g["logw_mean"])
    units = R_rep * n_deaths
    t = float(np.mean(ms)) / 1e3
    out = {
        "metric": "replica-deaths/s (post-hoc geometric uncertainty, R=100)",
        "value": units / t, "unit": "replica-deaths/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "geom_mixture8_d64_nlive2000_k1000_R100", "replicas": R_rep,
                   "deaths": n_deaths, "beta": 1.0,
                   "wall_ms_with_copies": 1e3 * float(np.mean(walls))},
        "result": {"logz_mean": float(np.mean(g["logz"])), "logz_std": float(np.std(g["logz"])),
                   "ess": g["ess"], "sigma_from_H": run.logz()[1]},
    }
    # weighted posterior samples from the same weights (10^4 draws), wall time with copies
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, _ = run.posterior_samples(10000, R=R_rep, beta=1.0, seed=1)
    out["config"]["posterior_samples_10k_wall_ms"] = 1e3 * (time.perf_counter() - t0)
    out["result"]["posterior_samples"] = int(xs.shape[0])
    ops = geom_ops()
    if ops is not None:
        achieved = ops * units / t
        out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12,
                           "peak": VALU_PEAK / 1e12, "unit": "TOP/s (VALU lane-instructions)",
                           "frac": achieved / VALU_PEAK, "traffic": None,
                           "kernel": "ns_geom_uncertainty (k_geom_weights 71%, k_geom_sums 26%)",
                           "valu_per_replica_death": ops}
    else:
        out["roofline"] = None
    if not args.no_cpu:
        from oracle import oracle as O
        # a seeded ascending record of the same length (the oracle's cost does not depend on
        # the values)
        rng = np.random.default_rng(1)
        n_dead = n_deaths - (run.m - run.k)
        Ls = np.sort(rng.normal(-300.0, 60.0, n_deaths))
        dead, fin = Ls[:n_dead], Ls[n_dead:]
        t0 = time.perf_counter()
        O.geom(dead, fin, run.m, run.k, 2, 1.0, seed=1)
        t2 = time.perf_counter() - t0
        r_cpu = max(2, min(R_rep, int(args.cpu_seconds / max(t2 / 2, 1e-6))))
        t0 = time.perf_counter()
        O.geom(dead, fin, run.m, run.k, r_cpu, 1.0, seed=1)
        tc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": r_cpu * n_deaths / tc, "unit": "replica-deaths/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{r_cpu} replicas over a seeded record of "
                                         f"{n_deaths} deaths (the run's count)"}
    print(json.dumps(out), flush=True)
    run.close()


def lnz_rastrigin_gauss(d, alpha, r=5.14, amp=10.0):
    """Semi-analytic evidence of the Gaussian-Rastrigin workload: the d-dimensional integrals
    factor into one-dimensional ones; the Rastrigin one is floor(r) whole periods, each the
    modified Bessel value I0(A), plus the remainder by quadrature."""
    from scipy import integrate
    from scipy.special import erf, i0e
    n = math.floor(r)
    tail, _ = integrate.quad(lambda x: math.exp(amp * (math.cos(2 * math.pi * x) - 1.0)), n, r,
                             epsabs=0, epsrel=1e-13)
    log_ig = amp + math.log(2 * n * float(i0e(amp)) + 2 * tail)
    log_if = 0.5 * math.log(2 * math.pi) + math.log(erf(r / math.sqrt(2)))
    terms = ([math.log(alpha) + d * log_if] if alpha > 0 else []) + \
            ([math.log1p(-alpha) - amp * d + d * log_ig] if alpha < 1 else [])
    mx = max(terms)
    return mx + math.log(sum(math.exp(t - mx) for t in terms)) - d * math.log(2 * r)


# VALU lane-instructions per likelihood evaluation of the Gaussian-Rastrigin k_hrss at d=100
# (SQ_INSTS_VALU x 64 / evaluations of the profiled launches), for the kernel source with this
# sha256 prefix.
RG_VALU_PER_EVAL = 53026.0
RG_SOURCE_SHA = "fff455ad04dd563f"


def _rastrigin_table(args):
    """Untimed full runs per (d, alpha, seed) of the table options; ln Z against the
    semi-analytic evidence."""
    from paper_2601_23252_amd import nss as N, problems as G
    table = []
    for dd in [int(v) for v in args.table_dims.split(",") if v]:
        for a in [float(v) for v in args.table_alphas.split(",") if v]:
            for sd in range(1, 1 + args.table_seeds):
                Q = N.NSRun(G.rastrigin_gauss(dd, a, k=args.table_k), seed=sd)
                t0 = time.perf_counter()
                while not Q.state()["done"]:   # in slices of 200 iterations, with progress
                    Q.run(max_iter=200)
                    print(f"[bench]   d={dd} alpha={a}: {Q.state()['iter']} iterations, "
                          f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
                z, err, _ = Q.logz()
                t = lnz_rastrigin_gauss(dd, a)
                table.append({"d": dd, "alpha": a, "k": args.table_k, "seed": sd, "logz": z,
                              "sigma": err, "truth": t, "z": (z - t) / err,
                              "seconds": time.perf_counter() - t0,
                              "evals": Q.stats()["evals"],
                              "iterations": Q.stats()["iterations"]})
                print(f"[bench] table d={dd} alpha={a} k={args.table_k} seed={sd}: "
                      f"z {(z - t) / err:.2f} ({time.perf_counter() - t0:.0f} s)",
                      file=sys.stderr, flush=True)
                Q.close()
    print(f"[bench] ln Z table done", file=sys.stderr, flush=True)
    return table


def _rastrigin_table_only(args):
    """--steps 0: the ln Z table alone (no timed runs, no throughput figure)."""
    table = _rastrigin_table(args)
    print(json.dumps({"metric": "Gaussian-Rastrigin ln Z against the semi-analytic evidence",
                      "value": None, "unit": "z-score", "n_gpus": 1, "steps": 0,
                      "warmup": 0, "higher_is_better": False, "dtype": "f64",
                      "data": "synthetic",
                      "config": {"workload": f"rastrigin_gauss_table_nlive1000_k{args.table_k}"
                                             "_p25d"},
                      "lnz": {"table": table}}), flush=True)


def bench_rastrigin(args):
    """The Gaussian-Rastrigin evidence workload: full runs at d = 100, alpha = 0.5 (n_live 1000,
    k 500, p = 25d, FP64), timed; then one untimed run per (d, alpha) in
    {2, 4, 10, 30, 100, 300} x {0, 0.5, 1} for the ln Z table against the semi-analytic
    evidence."""
    import hashlib
    import numpy as np
    import torch
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    d, alpha = 100, 0.5
    prob = G.rastrigin_gauss(d, alpha)
    if args.steps == 0:
        _rastrigin_table_only(args)
        return
    # the launch shape tuned during the warm-up run (cached for the timed runs)
    R = N.NSRun(prob, seed=0, timing=True, autotune=not args.no_autotune)
    for w in range(args.warmup):
        R.reset(10_000 + w)
        R.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = hrss_ms = launches = 0
    zs = []
    tz = lnz_rastrigin_gauss(d, alpha)
    for sd in range(args.steps):
        R.reset(sd)
        R.run()
        st = R.stats()
        evals += st["evals"]
        hrss_ms += st["hrss_ms"]
        launches += st["hrss_launches"]
        z, err, _ = R.logz()
        zs.append((z - tz) / err)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"[bench] timed runs done in {dt:.1f} s", file=sys.stderr, flush=True)
    table = [] if args.no_table else _rastrigin_table(args)
    src = os.path.join(ROOT, "paper_2601_23252_amd", "csrc", "nss_kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    roof = None
    shape = R.launch_shape()
    # the VALU count was taken at two chains per workgroup (the rule's shape for k = 500)
    if RG_VALU_PER_EVAL is not None and sha == RG_SOURCE_SHA and hrss_ms > 0 and shape[0] == 2:
        achieved = RG_VALU_PER_EVAL * evals / (hrss_ms / 1e3)
        roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
                "unit": "TOP/s (VALU lane-instructions)", "frac": achieved / VALU_PEAK,
                "traffic": None, "kernel": "k_hrss<128, FP64, Gaussian-Rastrigin>",
                "valu_per_eval": RG_VALU_PER_EVAL,
                "avg_launch_ms": hrss_ms / max(1, launches)}
    out = {
        "metric": "slice-step likelihood evals/s (Gaussian-Rastrigin, d=100, alpha=0.5)",
        "value": evals / dt, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "rastrigin_gauss_d100_alpha0.5_nlive1000_k500_p25d", "d": d,
                   "alpha": alpha, "n_live": prob["m"], "k": prob["k"], "chain_len": prob["p"],
                   "chains_per_workgroup": shape[0]},
        "roofline": roof,
        "lnz": {"truth": tz, "z_scores": zs, "table": table},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, prob["p"], args.cpu_seconds)
    print(json.dumps(out), flush=True)
    R.close()


def _step_costs(tr, rw):
    """Evaluations per step (slice: both bracket ends, the expansions and the shrink proposals)
    or, for the random walk, evaluations per accepted move (runs of steps up to and including
    an acceptance; a chain's unfinished run is dropped)."""
    import numpy as np
    if not rw:
        return (2 + tr[:, :, 0] + tr[:, :, 1] + tr[:, :, 2]).ravel().astype(float)
    cs = np.cumsum(tr[:, :, 2], axis=1)
    rows, cols = np.nonzero(tr[:, :, 3])
    if rows.size == 0:
        return np.zeros(0)
    vals = cs[rows, cols]
    prev = np.zeros_like(vals)
    same = np.r_[False, rows[1:] == rows[:-1]]
    prev[same] = vals[:-1][same[1:]]
    return (vals - prev).astype(float)


def _rw_costs(R, kind):
    """Run R to the end with traces; per-step costs (see _step_costs), and for the random walk
    its acceptance rate and the fraction of chains that never moved in their iteration."""
    import numpy as np
    from paper_2601_23252_amd import nss as N
    costs, acc, steps, stuck, chains = [], 0, 0, 0, 0
    done = False
    while not done:
        try:
            done = R.step()
        except N.NSError:   # the live set collapsed onto one point (plateau): stop there
            done = True
        tr = R.trace()
        costs.append(_step_costs(tr, kind == "rw"))
        if kind == "rw":
            acc += int(tr[:, :, 3].sum())
            steps += tr.shape[0] * tr.shape[1]
            stuck += int((tr[:, :, 3].sum(axis=1) == 0).sum())
            chains += tr.shape[0]
    c = np.concatenate(costs)
    if c.size == 0:       # no move accepted in the whole run
        c = np.array([np.nan])
    extra = {"acceptance": acc / steps, "chains_never_moved": stuck / chains} if steps else {}
    return c, extra


def bench_rw(args):
    """Slice (HRSS) against the constrained random walk on the condition-100 Gaussian at
    d = 10, 50, 100 (n_live 1000, k 500, FP64): HRSS with p = d steps, the random walk with
    p = 5d proposals at scale 2.38 / sqrt(d) of a proposal covariance that is (a) the live
    set's, recomputed every iteration, (b) the first iteration's live set's, kept for the run
    (a fixed scale), or (c) the target's own covariance, kept for the run.  Whole runs:
    per-step evaluation counts over every iteration (the paper's table of evaluations per
    step), the random walk's acceptance rate, ln Z against the closed form -d ln 40, and the
    adaptive random-walk kernel's throughput at d = 100 with its FP64 MFMA roofline."""
    import numpy as np
    import torch
    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    table = []
    timed = None
    variants = (("hrss", "hrss", None), ("rw", "rw", None), ("rw_fixed_first", "rw", "first"),
                ("rw_target_cov", "rw", "target"))
    for d in (10, 50, 100):
        prob = G.illcond_gaussian(d)
        tz = -d * math.log(40.0)
        Lt = np.linalg.cholesky(prob["cov"][0])
        row = {"d": d}
        for name, kind, fixed in variants:
            p = d if kind == "hrss" else 5 * d
            kw = dict(p=p, seed=0, replacement=kind, freeze_whitening=fixed is not None)

            def start(R):
                if fixed == "target":
                    s0 = R.state()
                    R.set_state(s0["x"], s0["logL"], s0["logZ"], s0["logX"], s0["M"],
                                s0["iter"], Lsig=Lt)
            # timed run (no trace), then the same trajectory again with traces for the costs
            R = N.NSRun(prob, timing=True, **kw)
            start(R)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            collapsed = False
            try:
                R.run()
            except N.NSError:   # every survivor a copy of one point: no strict survivor left
                collapsed = True
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = R.stats()
            z, err, _ = R.logz()
            R.close()
            R = N.NSRun(prob, trace=True, **kw)
            start(R)
            c, extra = _rw_costs(R, kind)
            row[name] = {"mean": float(c.mean()), "std": float(c.std()), "max": float(c.max()),
                         "p99": float(np.percentile(c, 99)), "p": p,
                         "iterations": st["iterations"], "evals": st["evals"],
                         "tests": st["tests"], "evals_per_s": st["evals"] / dt,
                         "kernel_ms": st["hrss_ms"] / max(1, st["hrss_launches"]),
                         "logz": z, "z": (z - tz) / err, "collapsed": collapsed, **extra}
            if d == 100 and name == "rw":
                timed = (st, dt)
            R.close()
            print(f"[bench] d={d} {name}: {row[name]['mean']:.2f} +- {row[name]['std']:.2f} "
                  f"(max {row[name]['max']:.0f}, z {row[name]['z']:.2f}, "
                  f"{st['iterations']} iterations{', collapsed' if collapsed else ''}"
                  + (f", acceptance {extra['acceptance']:.3f}" if extra else "") + ")",
                  file=sys.stderr, flush=True)
        table.append(row)
    st, dt = timed
    fpe = algorithmic_flop_per_eval(1, 100)
    hrss_s = st["hrss_ms"] / 1e3
    achieved = st["evals"] * fpe / hrss_s
    out = {
        "metric": "random-walk replacement likelihood evals/s (condition-100 Gaussian, d=100)",
        "value": st["evals"] / dt, "unit": "evals/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 * dt, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "illcond_gaussian_d100_rw_p5d_nlive1000_k500", "d": 100,
                   "kappa": 100, "replacement": "rw", "scale": 2.38 / 10.0,
                   "tests_per_s": st["tests"] / dt},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": "k_rw<128, FP64, mixture, 1>", "flop_per_eval": fpe,
                     "avg_launch_ms": st["hrss_ms"] / max(1, st["hrss_launches"])},
        "evals_per_step": table,
    }
    print(json.dumps(out), flush=True)


def bench_smc(args):
    """Adaptive tempered SMC with the slice-sampling mutation against nested sampling, same
    inner kernel and tuning (the paper's SMC-SS control): the d = 32 correlated Gaussian
    (condition number 1e3, prior N(0, 4 I)), n_live = particles = 1000, p = 5d = 160, FP64;
    NS with k = 500, SMC with ESS target 0.5.  --steps full runs of each (seeds 0..K-1), timed;
    ln Z against the closed form; the SMC runs' throughput with the FP64 MFMA roofline of the
    mutation kernel."""
    import numpy as np
    import torch
    from paper_2601_23252_amd import nss as N, problems as G
    from scipy.stats import multivariate_normal
    N.load()
    prob = G.config2()
    d = prob["d"]
    C = prob["cov"][0] + 4.0 * np.eye(d)
    tz = float(multivariate_normal(mean=np.zeros(d), cov=C).logpdf(prob["mu"][0]))
    res = {}
    for outer in ("ns", "smc"):
        R = N.NSRun(prob, p=5 * d, seed=0, timing=True, outer=outer)
        zs, errs, evals, iters, hrss_ms, launches = [], [], 0, [], 0.0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for sd in range(args.steps):
            R.reset(sd)
            R.run()
            st = R.stats()
            z, err, _ = R.logz()
            zs.append(z); errs.append(err); evals += st["evals"]; iters.append(st["iterations"])
            hrss_ms += st["hrss_ms"]; launches += st["hrss_launches"]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[outer] = {"logz": zs, "sigma": errs, "evals": evals, "iterations": iters,
                      "seconds": dt, "evals_per_s": evals / dt,
                      "hrss_ms": hrss_ms, "launches": launches}
        print(f"[bench] {outer}: ln Z {np.mean(zs):.3f} (truth {tz:.3f}), "
              f"{evals / args.steps:.3g} evals per run, {dt / args.steps:.2f} s per run",
              file=sys.stderr, flush=True)
        R.close()
    smc = res["smc"]
    fpe = algorithmic_flop_per_eval(1, d)
    achieved = smc["evals"] * fpe / (smc["hrss_ms"] / 1e3)
    zs = np.array(smc["logz"])
    out = {
        "metric": "SMC-SS likelihood evals/s (d=32 correlated Gaussian, 1000 particles)",
        "value": smc["evals_per_s"], "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 0, "ms_per_step": 1e3 * smc["seconds"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "smc_ss_corr32_particles1000_p5d_rho0.5", "d": d,
                   "particles": prob["m"], "chain_len": 5 * d, "ess_frac": 0.5},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": 78.6,
                     "unit": "TFLOP/s", "frac": achieved / 78.6e12, "traffic": None,
                     "kernel": "k_hrss<32, FP64, mixture, 1> (tempered)", "flop_per_eval": fpe,
                     "avg_launch_ms": smc["hrss_ms"] / max(1, smc["launches"])},
        "lnz": {"truth": tz, "smc": smc["logz"], "smc_mean_error": float(zs.mean() - tz),
                "smc_spread": float(zs.std()), "ns": res["ns"]["logz"],
                "ns_z": [(z - tz) / e for z, e in zip(res["ns"]["logz"], res["ns"]["sigma"])]},
        "ns_vs_smc": {k: {"evals_per_run": v["evals"] / args.steps,
                          "seconds_per_run": v["seconds"] / args.steps,
                          "iterations": v["iterations"]} for k, v in res.items()},
    }
    print(json.dumps(out), flush=True)


def bench_small(args, which):
    """The two small Gaussian configurations as benchmark lines: config 1 (d = 5, n_live 200,
    k 50, p = 25, FP64; evals/s only, RNG and control dominate) or config 2 (the d = 32
    correlated Gaussian under N(0, 4I), n_live 1000, k 500, p = 160) in BF16x3 and FP64, with
    ln Z against the closed form; --steps seeds each."""
    import numpy as np
    from paper_2601_23252_amd import nss as N, problems as G
    from scipy.stats import multivariate_normal
    from scipy.special import erf
    N.load()
    if which == "gauss5":
        prob, precs = G.config1(), ["fp64"]
        truth = -5 * math.log(2.0) + 5 * math.log(erf(1.0 / (0.1 * math.sqrt(2.0))))
        fpe, workload = 3 * 5 + 2, "gauss5_box1_nlive200_k50_p25"
    else:
        prob, precs = G.config2(), ["bf16x3", "fp64"]
        d = prob["d"]
        truth = float(multivariate_normal(mean=np.zeros(d), cov=prob["cov"][0] + 4 * np.eye(d))
                      .logpdf(prob["mu"][0]))
        fpe, workload = algorithmic_flop_per_eval(1, d), "corr32_cond1e3_prior4_nlive1000_k500_p160"
    seeds = list(range(args.steps))
    res = {}
    for prec in precs:
        recs, total = run_gpu(N, prob, prec, seeds, prob["p"], args.warmup)
        evals = sum(r["evals"] for r in recs)
        hrss_s = sum(r["hrss_ms"] for r in recs) / 1e3
        res[prec] = dict(recs=recs, total=total, evals=evals, hrss_s=hrss_s,
                         launches=sum(r["hrss_launches"] for r in recs))
    main_prec = precs[0]
    r0 = res[main_prec]
    mixed = main_prec != "fp64"
    peak = 2.5e15 if mixed else 78.6e12
    achieved = r0["evals"] * fpe / r0["hrss_s"] if r0["hrss_s"] > 0 else 0.0
    rates = [r["evals"] / r["wall_s"] for r in r0["recs"]]
    out = {
        "metric": f"slice-step likelihood evals/s ({which})", "value": r0["evals"] / r0["total"],
        "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * r0["total"] / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "d": prob["d"], "n_live": prob["m"], "k": prob["k"],
                   "chain_len": prob["p"], "precision": main_prec, "seeds": seeds},
        "roofline": {"bound": "mfma" if which == "corr32" else "alu", "achieved": achieved / 1e12,
                     "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None, "kernel": "k_hrss", "flop_per_eval": fpe,
                     "avg_launch_ms": 1e3 * r0["hrss_s"] / max(1, r0["launches"])},
        "per_seed_evals_per_s": {"median": statistics.median(rates),
                                 "range": [min(rates), max(rates)]},
        "lnz": {"truth": truth, prec_key(main_prec): [(r["logz"] - truth) / r["err"]
                                                      for r in r0["recs"]]},
    }
    for prec in precs[1:]:
        r1 = res[prec]
        out[prec] = {"value": r1["evals"] / r1["total"], "unit": "evals/s",
                     "z_scores": [(r["logz"] - truth) / r["err"] for r in r1["recs"]],
                     "frac_of_fp64_peak": r1["evals"] * fpe / max(r1["hrss_s"], 1e-12) / 78.6e12}
    if not args.no_cpu:
        # a mid-run live set about a third of the way through these short runs
        out["cpu_baseline"] = cpu_baseline(prob, prob["p"], args.cpu_seconds, warm_iters=0)
    print(json.dumps(out), flush=True)


def prec_key(p):
    return f"z_scores_{p}"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed full runs (seeds 0..K-1)")
    ap.add_argument("--metric", default="diagonal", choices=["diagonal", "full"],
                    help="headline direction metric: the survivors' variances (the diagonal "
                         "restriction of Sec. 3.2) or their full covariance")
    ap.add_argument("--other-metric-steps", type=int, default=5,
                    help="runs of the labelled line with the other direction metric (0 = skip)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp16x3",
                    choices=["bf16", "fp16", "bf16x3", "fp16x3", "fp64"])
    ap.add_argument("--chain-factor", type=int, default=5,
                    help="chain length p = factor * d of the headline (the workload's 5d)")
    ap.add_argument("--fp64-steps", type=int, default=3, help="FP64 comparison runs (0 = skip)")
    ap.add_argument("--long-chain-factor", type=int, default=20,
                    help="chain length factor of the labelled long-chain line")
    ap.add_argument("--long-chain-steps", type=int, default=5,
                    help="runs of the long-chain line (full-covariance metric; 0 = skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the launch-shape rule (4 chains per workgroup, 16 planned tests "
                         "for 16-bit mixture chains) instead of timing the candidates")
    ap.add_argument("--profile-shape", default="tuned",
                    choices=["tuned", "rule", "plan8", "shallow", "inline"],
                    help="profiling run: the chains' launch shape (tuned, the rule, 8 planned "
                         "tests per round, the 4-test kernel, or the 4-test kernel drawing its "
                         "directions inline)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--workload", default="mixture8_d64",
                    choices=["mixture8_d64", "gp_n256", "batch256", "geom", "rastrigin",
                             "rw", "smc", "gauss5", "corr32"],
                    help="mixture8_d64: the benchmark above; gp_n256: GP hyperparameter "
                         "marginalisation (n=256, n_live=1000, k=500, p=30), FP64; batch256: "
                         "256 independent runs of uneven d in one context; geom: post-hoc "
                         "geometric uncertainty of a full mixture run; rastrigin: the "
                         "Gaussian-Rastrigin evidence workload at d = 100; rw: slice against "
                         "random-walk replacement on a condition-100 Gaussian; smc: "
                         "tempered SMC with the slice mutation against nested sampling; "
                         "gauss5 / corr32: the small Gaussian configurations")
    ap.add_argument("--replicas", type=int, default=100, help="geom: shrinkage replicas")
    ap.add_argument("--graph", action="store_true",
                    help="batch256: replay 16-iteration HIP graphs (the groups' chains then run "
                         "in sequence) instead of eager iterations with the groups concurrent")
    ap.add_argument("--serial-groups", action="store_true",
                    help="batch256: launch the kernel groups' chains one after the other "
                         "instead of concurrently on side streams")
    ap.add_argument("--no-table", action="store_true",
                    help="rastrigin: skip the untimed ln Z table over (d, alpha)")
    ap.add_argument("--table-k", type=int, default=500,
                    help="rastrigin: deletions per iteration of the table's runs (n_live 1000)")
    ap.add_argument("--table-dims", default="2,4,10,30,100,300",
                    help="rastrigin: the table's dimensions")
    ap.add_argument("--table-alphas", default="0,0.5,1", help="rastrigin: the table's alphas")
    ap.add_argument("--table-seeds", type=int, default=1,
                    help="rastrigin: runs per table cell (seeds 1..)")
    ap.add_argument("--max-seconds", type=float, default=120.0,
                    help="gp_n256 / batch256: stop the timed run after about this long")
    ap.add_argument("--profile-iters", type=int, default=0,
                    help="profiling run: a 256 MiB device copy (the counters' reference), then "
                         "this many outer iterations of one run; prints their timing only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.profile_iters > 0:
        profile_run(args)
        return
    if args.workload == "gp_n256":
        bench_gp(args)
        return
    if args.workload == "batch256":
        bench_batch(args)
        return
    if args.workload == "geom":
        bench_geom(args)
        return
    if args.workload == "rastrigin":
        bench_rastrigin(args)
        return
    if args.workload == "rw":
        bench_rw(args)
        return
    if args.workload == "smc":
        bench_smc(args)
        return
    if args.workload in ("gauss5", "corr32"):
        bench_small(args, args.workload)
        return

    from paper_2601_23252_amd import nss as N, problems as G
    N.load()
    prob = G.config3()
    d, K = prob["d"], prob["K"]
    p = args.chain_factor * d
    truth = -d * math.log(20.0)
    fpe = algorithmic_flop_per_eval(K, d)
    mixed = args.precision != "fp64"

    def summary(recs, total):
        """Rates of one timed leg.  value counts only the evaluations of runs whose ln Z lies
        within 3 sigma of the closed form, over the wall time of every timed run."""
        z = [(r["logz"] - truth) / r["err"] for r in recs]
        ok = [abs(v) < 3.0 for v in z]
        ev_all = sum(r["evals"] for r in recs)
        ev_ok = sum(r["evals"] for r, good in zip(recs, ok) if good)
        return dict(value=ev_ok / total, rate_all_runs=ev_all / total,
                    runs_within_3sigma=f"{sum(ok)}/{len(ok)}", z_scores=z,
                    z_mean=statistics.fmean(z), z_sd=statistics.stdev(z) if len(z) > 1 else None,
                    logz=[r["logz"] for r in recs], sigma=[r["err"] for r in recs],
                    iterations=[r["iters"] for r in recs],
                    per_seed_evals_per_s=[r["evals"] / r["wall_s"] for r in recs])

    seeds = list(range(args.steps))
    shape = {}
    diag = args.metric == "diagonal"
    recs, total = run_gpu(N, prob, args.precision, seeds, p, args.warmup,
                          autotune=not args.no_autotune, shape_out=shape, diagonal_metric=diag)
    head = summary(recs, total)
    evals = sum(r["evals"] for r in recs)
    hrss_s = sum(r["hrss_ms"] for r in recs) / 1e3
    launches = sum(r["hrss_launches"] for r in recs)
    peak = 2.5e15 if mixed else 78.6e12
    achieved = evals * fpe / hrss_s if hrss_s > 0 else 0.0

    out = {
        "metric": "slice-step likelihood evals/s (d=64 mixture), mixed vs FP64, at |dlogZ|<3sigma",
        "value": head["value"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "bf16x3": "bf16", "fp16": "fp16", "fp16x3": "fp16",
                  "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "mixture8_d64_uniform10_nlive2000_k1000", "d": d, "n_comp": K,
                   "n_live": prob["m"], "k": prob["k"], "chain_len": p,
                   "precision": args.precision, "term_frac": 1e-3, "seeds": seeds,
                   "direction_metric": "survivor variances (diagonal)" if diag
                   else "survivor covariance (full)"},
        "value_rule": "evaluations of the runs with |ln Z + 64 ln 20| < 3 sqrt(H/n_live), "
                      "divided by the wall time of all timed runs",
        "runs_within_3sigma": head["runs_within_3sigma"],
        "rate_all_runs": head["rate_all_runs"],
        "launch_shape": shape,
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": kernel_traffic(args.precision, p, shape),
                     "kernel": chain_kernel_name(args.precision, shape), "flop_per_eval": fpe,
                     "avg_launch_ms": 1e3 * hrss_s / max(1, launches)},
        "lnz": {"truth": truth, "z_scores": head["z_scores"], "z_mean": head["z_mean"],
                "z_sd": head["z_sd"], "logz": head["logz"], "sigma": head["sigma"]},
        "per_seed_evals_per_s": {"values": head["per_seed_evals_per_s"],
                                 "median": statistics.median(head["per_seed_evals_per_s"]),
                                 "range": [min(head["per_seed_evals_per_s"]),
                                           max(head["per_seed_evals_per_s"])]},
        "valu_issue": None,
        "rechecks_per_eval": sum(r["rechecks"] for r in recs) / max(1, evals),
        "band_violations": sum(r["band_violations"] for r in recs),
        "iterations": head["iterations"],
    }
    vpe = hrss_valu_per_eval(args.precision, p, shape)
    if vpe is not None and hrss_s > 0:
        a = vpe * evals / hrss_s
        out["valu_issue"] = {"kernel": chain_kernel_name(args.precision, shape),
                             "lane_instr_per_eval": vpe,
                             "achieved": a / 1e12, "peak": VALU_PEAK / 1e12,
                             "unit": "T lane-instr/s", "frac": a / VALU_PEAK}
    if args.fp64_steps > 0 and mixed:
        r64, t64 = run_gpu(N, prob, "fp64", list(range(args.fp64_steps)), p, 1,
                           autotune=not args.no_autotune, diagonal_metric=diag)
        s64 = summary(r64, t64)
        ev64 = sum(r["evals"] for r in r64)
        out["fp64"] = {"value": s64["value"], "rate_all_runs": s64["rate_all_runs"],
                       "unit": "evals/s", "seeds": list(range(args.fp64_steps)),
                       "runs_within_3sigma": s64["runs_within_3sigma"],
                       "z_scores": s64["z_scores"],
                       "same_trajectory_as_mixed": [
                           a["iters"] == b["iters"] and a["evals"] == b["evals"]
                           and abs(a["logz"] - b["logz"]) < 1e-9 for a, b in zip(r64, recs)],
                       "hrss_frac_of_fp64_peak": ev64 * fpe / (sum(r["hrss_ms"] for r in r64) / 1e3) / 78.6e12}
        out["speedup_vs_fp64"] = head["rate_all_runs"] / s64["rate_all_runs"]
    if args.other_metric_steps > 0:
        # the same workload and chain length with the other direction metric
        ro, to = run_gpu(N, prob, args.precision, list(range(args.other_metric_steps)), p, 0,
                         autotune=not args.no_autotune, diagonal_metric=not diag)
        so = summary(ro, to)
        out["other_metric"] = {
            "label": "the same workload at p = 5d with the direction metric from the survivors' "
                     + ("full covariance (the paper's default)" if diag
                        else "variances alone (diagonal)"),
            "value": so["value"], "rate_all_runs": so["rate_all_runs"], "unit": "evals/s",
            "runs_within_3sigma": so["runs_within_3sigma"], "z_scores": so["z_scores"],
            "z_mean": so["z_mean"], "z_sd": so["z_sd"]}
    if args.long_chain_steps > 0:
        pl = args.long_chain_factor * d
        rl, tl = run_gpu(N, prob, args.precision, list(range(args.long_chain_steps)), pl, 0,
                         autotune=not args.no_autotune, diagonal_metric=False)
        sl = summary(rl, tl)
        out["long_chain"] = {"label": f"the same workload at chain length p = "
                                      f"{args.long_chain_factor}d = {pl} (not the configured "
                                      "5d), full-covariance metric",
                             "chain_len": pl, "value": sl["value"],
                             "rate_all_runs": sl["rate_all_runs"], "unit": "evals/s",
                             "runs_within_3sigma": sl["runs_within_3sigma"],
                             "z_scores": sl["z_scores"], "z_mean": sl["z_mean"],
                             "z_sd": sl["z_sd"], "iterations": sl["iterations"]}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, p, args.cpu_seconds, diagonal_metric=diag)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
