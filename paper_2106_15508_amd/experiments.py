"""The paper's comparison of the two step-size methods (§IV-A, Fig. 6) on
synthetic observations, run with the HIP library.

For each number of simulations per run (the batch size: 10 ... 100000) and
each trial seed, both the eq. 16 Beta step sizes (BDSS) and the MCMC-tuned
single step size (eqs. 12-15, adapted during the first 10% of the run
budget) collect N = 1000 particles per stage; the process stops at the
stage in which the cumulative number of runs reaches 1000 (or after 60
stages, the limit of eq. 16's integer shape 2i <= 128).  Each stage records
(cumulative runs, tolerance eps^i).  The summary reports, per method and
batch size, the tolerance reached at the end, its spread over trials and
the runs needed to come within 10% of the method's final tolerance.

    python -m paper_2106_15508_amd.experiments fig6 [--trials 10] [--out results/fig6_synthetic.json]
    python -m paper_2106_15508_amd.experiments fig7 [--out results/fig7_synthetic.json]

The observations are the synthetic series of the headline model (P = 1e7,
120 days, THETA_TRUE); the paper's own data set is not used.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from typing import Dict, List

import numpy as np

from . import abcsmc as A
from . import workloads as W

BATCHES = (10, 100, 1000, 10000, 100000)
RUN_BUDGET = 1000
MAX_STAGES = 60


def trace(w: W.Workload, obs, run_budget: int = RUN_BUDGET, max_stages: int = MAX_STAGES) -> Dict:
    """Stages of one run until the cumulative batch count reaches run_budget."""
    runs, eps, sims = [], [], []
    total_runs = total_sims = 0
    with A.Context(w, obs, flags=A.F_EARLY_EXIT) as ctx:
        for _ in range(max_stages):
            try:
                info = ctx.round()
            except A.AbcsmcError as e:
                if e.code == A.EBUDGET:
                    break
                raise
            total_runs += info["batches"]
            total_sims += info["simulated"]
            runs.append(total_runs)
            eps.append(info["eps_next"])
            sims.append(total_sims)
            if total_runs >= run_budget:
                break
    return {"runs": runs, "eps": eps, "sims": sims}


def fig6(trials: int = 10, batches=BATCHES, n_particles: int = 1000, mcmc_s0: float = 0.1) -> Dict:
    base = W.C2.with_(n_particles=n_particles, n_rounds=MAX_STAGES)
    obs = A.observations(base)
    out = {"config": {"population": base.population, "n_days": base.n_days, "n_particles": n_particles,
                      "run_budget": RUN_BUDGET, "max_stages": MAX_STAGES, "trials": trials,
                      "mcmc_s0": mcmc_s0, "mcmc_tune": RUN_BUDGET // 10},
           "results": []}
    for B in batches:
        for method in ("bdss", "mcmc"):
            for t in range(trials):
                # a stage may use at most twice the whole run budget
                w = base.with_(batch=B, seed=100 + t, max_proposals=2 * RUN_BUDGET * B)
                if method == "mcmc":
                    w = w.with_(step_schedule=W.STEP_MCMC, mcmc_s0=mcmc_s0, mcmc_tune=RUN_BUDGET // 10)
                t0 = time.perf_counter()
                tr = trace(w, obs)
                tr.update(batch=B, method=method, trial=t, seconds=time.perf_counter() - t0)
                out["results"].append(tr)
                print(f"batch {B:6d} {method} trial {t}: stages {len(tr['eps'])} runs {tr['runs'][-1]} "
                      f"eps {tr['eps'][-1]:.4g} ({tr['seconds']:.2f} s)", flush=True)
    return out


def summarise(res: Dict) -> str:
    rows = ["| sims per run | method | final eps (median) | final eps (min .. max) | run-to-run std | "
            "runs to within 10% of final (median) |", "|---|---|---|---|---|---|"]
    by = {}
    for r in res["results"]:
        by.setdefault((r["batch"], r["method"]), []).append(r)
    for (B, m), rs in sorted(by.items()):
        fin = np.array([r["eps"][-1] for r in rs])
        reach = []
        for r in rs:
            e = np.array(r["eps"])
            k = int(np.argmax(e <= 1.1 * e[-1]))
            reach.append(r["runs"][k])
        rows.append(f"| {B} | {m} | {np.median(fin):.4g} | {fin.min():.4g} .. {fin.max():.4g} | "
                    f"{fin.std():.3g} | {int(np.median(reach))} |")
    return "\n".join(rows)


def fig7(batch: int = 100000, n_particles: int = 1000, t_train: int = 120, t_test: int = 30,
         early_runs: int = 10, mcmc_s0: float = 0.1, seed: int = 100) -> Dict:
    """Predictive check (§IV-B, Fig. 7): fit the first t_train days of a
    synthetic series observed for t_train + t_test days, then simulate the
    population of the stage that reached early_runs runs and of the last
    stage (run budget or stage limit) over all days; report the band
    (0.5%, 50%, 99.5% per day) against the held-out days."""
    full = W.C2.with_(n_days=t_train + t_test)
    obs_full = A.observations(full)
    w = W.C2.with_(n_particles=n_particles, n_rounds=MAX_STAGES, batch=batch, seed=seed,
                   max_proposals=2 * RUN_BUDGET * batch)
    obs = obs_full[: t_train + 1]
    q = (0.005, 0.5, 0.995)
    out = {"config": {"batch": batch, "n_particles": n_particles, "t_train": t_train, "t_test": t_test,
                      "early_runs": early_runs, "quantiles": q, "seed": seed}, "obs": obs_full.tolist(),
           "results": []}
    for method in ("bdss", "mcmc"):
        wm = w if method == "bdss" else w.with_(step_schedule=W.STEP_MCMC, mcmc_s0=mcmc_s0, mcmc_tune=RUN_BUDGET // 10)
        runs = 0
        snaps = {}
        with A.Context(wm, obs, flags=A.F_EARLY_EXIT) as ctx:
            for st in range(MAX_STAGES):
                try:
                    info = ctx.round()
                except A.AbcsmcError as e:
                    if e.code == A.EBUDGET:
                        break
                    raise
                runs += info["batches"]
                if "early" not in snaps and runs >= early_runs:
                    snaps["early"] = (st, runs, info["eps_next"], ctx.predict(t_train + t_test, seed=7, quantiles=q))
                last = (st, runs, info["eps_next"])
                if runs >= RUN_BUDGET:
                    break
            snaps["late"] = last + (ctx.predict(t_train + t_test, seed=7, quantiles=q),)
        for tag, (st, r, eps, bands) in snaps.items():
            held = obs_full[t_train + 1:].astype(np.float64)          # days t_train+1 .. end
            b = bands[t_train + 1:]
            inside = (held >= b[:, :, 0]) & (held <= b[:, :, 2])
            rel = np.abs(b[:, :, 1] - held) / np.maximum(held, 1.0)
            out["results"].append({
                "method": method, "snapshot": tag, "stage": st, "runs": r, "eps": eps,
                "coverage_test": inside.mean(axis=0).tolist(),
                "median_rel_err_test": np.median(rel, axis=0).tolist(),
                "band_rel_width_test": np.median((b[:, :, 2] - b[:, :, 0]) / np.maximum(held, 1.0), axis=0).tolist(),
                "bands": bands.tolist()})
            print(f"{method} {tag}: stage {st} runs {r} eps {eps:.4g} coverage(A,R,D) "
                  f"{np.round(inside.mean(axis=0), 2).tolist()} median rel err {np.round(np.median(rel, axis=0), 3).tolist()}",
                  flush=True)
    return out


def summarise7(res: Dict) -> str:
    rows = ["| method | snapshot | stage | runs | eps | held-out coverage of the 99% band (A, R, D) | "
            "median relative error of the median (A, R, D) | median relative band width (A, R, D) |",
            "|---|---|---|---|---|---|---|---|"]
    for r in res["results"]:
        f = lambda v: ", ".join(f"{x:.3g}" for x in v)
        rows.append(f"| {r['method']} | {r['snapshot']} | {r['stage']} | {r['runs']} | {r['eps']:.4g} | "
                    f"{f(r['coverage_test'])} | {f(r['median_rel_err_test'])} | {f(r['band_rel_width_test'])} |")
    return "\n".join(rows)


def main(argv: List[str] = None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("what", choices=["fig6", "fig7"])
    ap.add_argument("--trials", type=int, default=10)
    ap.add_argument("--batches", type=str, default=",".join(map(str, BATCHES)))
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    if args.what == "fig7":
        res = fig7()
        table = summarise7(res)
    else:
        res = fig6(trials=args.trials, batches=[int(b) for b in args.batches.split(",")])
        table = summarise(res)
    print(table, flush=True)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        with open(args.out, "w") as f:
            json.dump(res, f)
        with open(os.path.splitext(args.out)[0] + ".md", "w") as f:
            f.write(table + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
