#!/usr/bin/env python3
"""Throughput of the ABC-SMC BDSS hot path on one MI355X.

One step is one complete ABC-SMC run of the headline workload (population
1e7, 120 days, N = 131072 particles, 10 stages: the prior stage plus nine
stages with eq. 16 step sizes): resampling, Beta-step perturbation,
simulation, distance, acceptance with ordered compaction, importance
weights and the next tolerance, all in the HIP library.  The observations
and the workspace are resident in HBM before the timed region; each step
restarts the context at stage 0 (abcsmc_reset), so every step does the same
work.

Prints one JSON line: accepted particles/s (value), simulations/s, the
roofline of the dominant kernel (device time from HIP events recorded on the
library's stream around each launch), and the CPU oracle timed on a bounded
sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

# FP64 flops of one importance-weight term as the kernel evaluates it (every
# FP64 instruction counted, fma = 2): 8 differences, 8 fma for the squared
# distance, exponent scaling 1, table exp 11 (rounding to an integer 1, reduced argument 1,
# integer conversion 1, 3 fma 6, table product 1, 2^k 1), weight times term
# fused into the running sum 2.
FLOPS_PER_PAIR = 8 + 16 + 1 + 11 + 2

# HBM bytes per launch of the dominant kernel measured with rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE on this workload, scaled by the counters' reading
# for a 256 MiB device copy (FETCH 0.5x, WRITE 1.0x of the bytes moved).  Keyed
# by the SHA-256 of the kernel sources and the build flags: a changed kernel
# reports null.
TRAFFIC_SOURCES = ("paper_2106_15508_amd/csrc/smc.hip", "paper_2106_15508_amd/csrc/dmath.h",
                   "paper_2106_15508_amd/csrc/kernels.h", "paper_2106_15508_amd/csrc/wterm.h",
                   "paper_2106_15508_amd/csrc/sim.hip", "paper_2106_15508_amd/csrc/propose.h",
                   "paper_2106_15508_amd/build.py")
TRAFFIC_MEASURED = {
    # c2, per launch: FETCH_SIZE KiB x 2 + WRITE_SIZE KiB x 1
    ("e6370fa24c3b5b22", "c2", "weights_kernel"): 559541 * 1024 * 2 + 26916 * 1024,
    ("e6370fa24c3b5b22", "c2", "propose_kernel"): 15984 * 1024 * 2 + 15874 * 1024,
}
# FP64 flops of one simulated proposal-day with all five transitions in the
# normal branch of the binomial draw: state sums 2, g (log 34, exp 33, 4) 71,
# rate 2, p_SI (expm1) 29, five draws 5 x 93, chain sources 2, update 10,
# distance 9.
FLOPS_PER_DAY = 2 + 71 + 2 + 29 + 5 * 93 + 2 + 10 + 9


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c4: 96 uneven runs in the batched mode, compared with the same runs one at a time")
    ap.add_argument("--runs", type=int, default=96, help="c4: number of runs")
    ap.add_argument("--early-exit", type=int, default=1, help="stop simulating a proposal once its "
                    "partial distance exceeds eps (acceptances unchanged)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first run one device-to-device copy of BYTES (the plain copy kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_baseline(w, infos, budget_s: float):
    """Oracle (single thread, as it stands) on a bounded sample of the same
    workload: (a) simulate proposals of stage 0 at full size until half the
    budget is spent, (b) importance-weight rows against a synthetic previous
    population of the stage's survivor count until the other half is spent;
    the per-unit costs are scaled by the stage's own proposal and pair counts
    (identical in the oracle, whose runs match the GPU bit for bit)."""
    import numpy as np
    from oracle import ref

    obs = ref.observations(w)
    t0 = time.perf_counter()
    n_sim = 0
    while time.perf_counter() - t0 < budget_s / 2:
        u = ref.prior_draw(w, n_sim)
        ref.sim_distance(w, obs, u, 0, n_sim)
        n_sim += 1
    t_sim = (time.perf_counter() - t0) / n_sim
    rng = np.random.default_rng(0)
    M = int(np.median([i["survivors"] for i in infos[1:]])) if len(infos) > 1 else w.n_particles // 2
    u_prev = rng.uniform(size=(M, 8))
    q = rng.integers(1, 2**40, M).astype(np.uint64)
    t0 = time.perf_counter()
    n_rows = 0
    while time.perf_counter() - t0 < budget_s / 2:
        ref.log_weight(rng.uniform(size=8), 0.05, u_prev, q)
        n_rows += 1
    t_pair = (time.perf_counter() - t0) / (n_rows * M)
    sims = sum(i["simulated"] for i in infos)
    pairs = sum(i["weight_pairs"] for i in infos)
    t_run = sims * t_sim + pairs * t_pair
    acc = w.n_particles * len(infos)
    return {
        "value": acc / t_run, "unit": "accepted particles/s", "cores": 1, "kind": "oracle",
        "sample": (f"{n_sim} stage-0 proposals simulated ({w.n_days} days, P={w.population:.0e}) and "
                   f"{n_rows} weight rows x {M} columns on 1 core; per-proposal and per-pair costs scaled "
                   f"by the run's {sims} simulated proposals and {pairs} weight terms"),
        "sec_per_sim": t_sim, "sec_per_pair": t_pair, "extrapolated_run_s": t_run,
    }


def bench_batched(args):
    """96 independent runs (populations log-uniform in [1e5, 3e8], 40-150
    days, N in {2^11..2^16}) advanced together by the batched mode (one graph
    replay per stage), against the same runs one after another."""
    import torch

    from paper_2106_15508_amd import abcsmc as A
    from paper_2106_15508_amd import workloads as W

    runs = W.batched_runs(n_runs=args.runs, seed=4, n_rounds=10)
    R = runs[0].n_rounds
    obs = [A.observations(w) for w in runs]
    flags = A.F_EARLY_EXIT if args.early_exit else 0
    stream = torch.cuda.Stream()
    nbytes = A.Batch.workspace_size(runs, flags=flags)
    ws_tensor = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ws = ((ws_tensor.data_ptr() + 255) // 256 * 256, nbytes)
    b = A.Batch(runs, obs, stream=stream.cuda_stream, workspace=ws, flags=flags)
    t0 = time.perf_counter()
    sched = b.autotune(stages=1)
    tune_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        b.reset()
        b.run(R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.reset()
        infos = b.run(R)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    accepted = sum(w.n_particles for w in runs) * R
    simulated = sum(i["simulated"] for st in infos for i in st)
    terms = sum(i["weight_terms"] for st in infos for i in st)
    pairs = sum(i["weight_pairs"] for st in infos for i in st)
    days = sum(i["sim_days"] for st in infos for i in st)
    failed = [r for r in range(len(runs)) if b.status(r) != A.OK]
    b.close()
    # the same runs one at a time through the single-run path (contexts created
    # and warmed up before the clock starts; library-chosen batches, same flags)
    ctxs = [A.Context(w, o, flags=flags) for w, o in zip(runs, obs)]
    for ctx in ctxs:
        ctx.run(R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ctx in ctxs:
        ctx.reset()
        ctx.run(R)
    torch.cuda.synchronize()
    sec_plain = time.perf_counter() - t0
    for ctx in ctxs:
        ctx.close()
    # whole-stage FP64 work over the graph replays: evaluated weight terms and
    # simulated proposal-days at the flop counts above
    achieved = (terms * FLOPS_PER_PAIR + days * FLOPS_PER_DAY) / sec / 1e12
    out = {
        "metric": "accepted particles/s", "value": accepted / sec, "unit": "accepted particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"c4: {len(runs)} independent runs, P log-uniform in [1e5, 3e8], T in [40, 150], "
                               f"N in {{2^11..2^16}} (sum N = {sum(w.n_particles for w in runs)}), {R} stages, "
                               "batched mode (one graph replay per stage)",
                   "early_exit": bool(args.early_exit), "schedule": sched, "autotune_s": round(tune_s, 2)},
        "simulations_per_s": simulated / sec,
        "plain_sequential_value": accepted / sec_plain,
        "speedup_vs_plain": sec_plain / sec,
        "failed_runs": failed,
        "weight_terms": {"defined": pairs, "evaluated": terms},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel": "whole batched stage (graph replay; bweights_kernel and propose_persistent_kernel "
                               f"dominate), evaluated weight terms x {FLOPS_PER_PAIR} + proposal-days x "
                               f"{FLOPS_PER_DAY} flops",
                     "avg_launch_ms": round(sec * 1e3 / R, 3), "launches": R},
    }
    del ws_tensor
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """The headline workload with the learned screen: per step, stage 0, the
    network's initial fit on 2^22 prior simulations (2 passes, minibatch
    8192, included in the step), then nine screened stages (keep 10% of each
    stage's first batch by score, audit rho = 1%, screening kept on in every
    stage).  The same steps of the plain form run beside it for the
    comparison of throughput and posterior moments."""
    import numpy as np
    import torch

    from paper_2106_15508_amd import abcsmc as A
    from paper_2106_15508_amd import workloads as W

    w = W.C2
    R = w.n_rounds
    obs = A.observations(w)
    stream = torch.cuda.current_stream()
    flags = A.F_EARLY_EXIT if args.early_exit else 0
    sur = dict(n_train=1 << 22, epochs=2, batch=8192, keep_frac=0.1, audit_rho=0.01, fn_max=1.0, seed=11)

    def one(ctx, screened):
        ctx.reset()
        infos = [ctx.round()]
        if screened:
            ctx.surrogate_enable(**sur)
        sinfo = []
        for _ in range(R - 1):
            infos.append(ctx.round())
            if screened:
                sinfo.append(ctx.surrogate_info())
        return infos, sinfo

    def moments(ctx):
        th, _, wt = ctx.weights()
        mu = (wt[:, None] * th).sum(0)
        var = (wt[:, None] * (th - mu) ** 2).sum(0)
        return dict(mu=mu, var=var, mu_u=th.mean(0), var_u=th.var(0))

    def rel(a, b):
        return [round(float(v), 4) for v in np.abs(a - b) / np.maximum(np.abs(b), 1e-300)]

    res = {}
    sched = ()
    for screened in (False, True):
        # the screened form replays the plain form's tolerances, so that both
        # sample the same sequence of ABC targets
        ctx = A.Context(w.with_(eps_schedule=sched), obs, stream=stream.cuda_stream, flags=flags)
        for _ in range(args.warmup):
            one(ctx, screened)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [one(ctx, screened) for _ in range(args.steps)]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / args.steps
        res[screened] = dict(sec=sec, runs=runs, sinfo=None if not screened else ctx.surrogate_info(),
                             **moments(ctx))
        ctx.close()
        if not screened:
            sched = tuple(i["eps"] for i in runs[-1][0][1:])
    # Monte Carlo reference: the plain form with another seed at the same schedule
    with A.Context(w.with_(eps_schedule=sched, seed=w.seed + 1), obs, stream=stream.cuda_stream,
                   flags=flags) as ctx:
        ref_infos, _ = one(ctx, False)
        noise = moments(ctx)
    N = w.n_particles
    plain, scr = res[False], res[True]
    last_i, last_s = scr["runs"][-1]
    si0 = scr["sinfo"]
    train_flops = si0["train_flops"]
    ms_train = si0["ms_train"]
    achieved = train_flops / (ms_train * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_BF16_TFLOPS, 5), "traffic": None,
                "kernel": "network initial fit (gemm_bf16_kernel and its epilogue kernels)",
                "avg_launch_ms": None, "phase_ms": round(ms_train, 3), "flops": train_flops}
    out = {
        "metric": "accepted particles/s", "value": N * R / scr["sec"], "unit": "accepted particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": scr["sec"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+bf16",
        "data": "synthetic",
        "config": {"workload": f"C5: C2 (P={w.population}, T={w.n_days}, N={N}, stages={R}) with the learned "
                               "screen: fit on 2^22 prior simulations x 2 passes, keep 10%, audit 1%",
                   "early_exit": bool(args.early_exit)},
        "plain_value": N * R / plain["sec"],
        "speedup_vs_plain": plain["sec"] / scr["sec"],
        "surrogate": {
            "ms_data": si0["ms_data"], "ms_train": si0["ms_train"], "loss_first": si0["loss_first"],
            "loss_last": si0["loss_last"],
            "enrichment": [round(s["enrichment"], 3) for s in last_s],
            "fn_mass": [round(s["fn_mass"], 4) for s in last_s],
            "ms_score": [round(s["ms_score"], 2) for s in last_s],
            "ms_tune": [round(s["ms_tune"], 2) for s in last_s],
            "proposals": [i["proposals"] for i in last_i[1:]],
            "plain_proposals": [i["proposals"] for i in plain["runs"][-1][0][1:]],
        },
        "posterior": {
            "schedule": "screened stages replay the plain run's tolerances (eps_schedule)",
            "weighted_mean_rel_diff_vs_plain": rel(scr["mu"], plain["mu"]),
            "weighted_var_rel_diff_vs_plain": rel(scr["var"], plain["var"]),
            "population_mean_rel_diff_vs_plain": rel(scr["mu_u"], plain["mu_u"]),
            "population_var_rel_diff_vs_plain": rel(scr["var_u"], plain["var_u"]),
            "mc_reference_plain_other_seed": {
                "weighted_mean_rel_diff": rel(noise["mu"], plain["mu"]),
                "population_mean_rel_diff": rel(noise["mu_u"], plain["mu_u"]),
                "population_var_rel_diff": rel(noise["var_u"], plain["var_u"])},
            "ess_final": [round(plain["runs"][-1][0][-1]["ess"], 1), round(last_i[-1]["ess"], 1),
                          round(ref_infos[-1]["ess"], 1)]},
        "roofline": roofline,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the ABC-SMC path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2106_15508_amd import abcsmc as A
    from paper_2106_15508_amd import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "c4":
        return bench_batched(args)
    if args.workload == "c5":
        return bench_surrogate(args)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = W.WORKLOADS[args.workload]
    R = w.n_rounds
    obs = A.observations(w)                       # synthetic series from THETA_TRUE (on the GPU)
    ws_tensor, ws = A.torch_workspace(w)          # workspace: device memory owned by torch
    stream = torch.cuda.current_stream()
    flags = A.F_EARLY_EXIT if args.early_exit else 0
    ctx = A.Context(w, obs, stream=stream.cuda_stream, workspace=ws, flags=flags)

    for _ in range(args.warmup):
        ctx.reset()
        ctx.run(R)
        ctx.weights()                             # the copy-out path's one-time set-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = []
    for _ in range(args.steps):
        ctx.reset()
        steps.append(ctx.run(R))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = (t1 - t0) / args.steps
    last = steps[-1]
    # PCIe-inclusive: the final population (theta, d, W) copied to host memory
    # through the C ABI after the run (pinned staging allocated during the
    # warm-up); the observations go in once at init
    tc = time.perf_counter()
    ctx.weights()
    sec_copy = time.perf_counter() - tc
    N = w.n_particles
    accepted = N * R
    simulated = sum(i["simulated"] for i in last)
    proposals = sum(i["proposals"] for i in last)
    sim_days = sum(i["sim_days"] for i in last)

    # dominant kernel over the timed steps
    ms_prop = sum(i["ms_k_propose"] for s in steps for i in s)
    n_prop = sum(i["n_k_propose"] for s in steps for i in s)
    ms_w = sum(i["ms_k_weights"] for s in steps for i in s)
    n_w = sum(1 for s in steps for i in s if i["round"] > 0)
    sha = kernel_sources_sha()

    def alu_roofline(kernel, flops, ms_total, launches):
        avg_ms = ms_total / launches
        achieved = flops / launches / (avg_ms * 1e-3) / 1e12
        return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": TRAFFIC_MEASURED.get((sha, args.workload, kernel)),
                "kernel": kernel, "avg_launch_ms": round(avg_ms, 4), "launches": launches,
                "flops_per_launch": flops / launches, "kernel_sources_sha": sha}

    # flops of the weight terms the kernel evaluates (the others lie outside
    # every row's window and cannot change a sum; reported beside), and of the
    # simulated proposal-days
    rl_w = alu_roofline("weights_kernel", sum(i["weight_terms"] for s in steps for i in s) * FLOPS_PER_PAIR,
                        ms_w, n_w) if n_w else None
    rl_p = alu_roofline("propose_kernel", sum(i["sim_days"] for s in steps for i in s) * FLOPS_PER_DAY,
                        ms_prop, n_prop)
    roofline = rl_w if (rl_w and ms_w >= ms_prop) else rl_p
    other = rl_p if roofline is rl_w else rl_w

    out = {
        "metric": "accepted particles/s", "value": accepted / sec, "unit": "accepted particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: P={w.population}, T={w.n_days}, N={N}, stages={R}, "
                               "eq.16 Beta step sizes, chain-binomial simulator, synthetic observations "
                               "of theta_true",
                   "early_exit": bool(args.early_exit)},
        "pcie_inclusive_value": accepted / (sec + sec_copy),
        "ms_copy_out": round(sec_copy * 1e3, 3),
        "simulations_per_s": simulated / sec,
        "useful_simulations_per_s": proposals / sec,
        "particle_days_per_s": sim_days / sec,
        "eps_final": last[-1]["eps_next"],
        "phase_ms": {k: round(sum(i[k] for i in last), 3)
                     for k in ("ms_resample", "ms_simulate", "ms_weights", "ms_select", "ms_total")},
        "kernel_ms": {"propose": round(ms_prop / args.steps, 3), "weights": round(ms_w / args.steps, 3)},
        "weight_terms": {"defined": sum(i["weight_pairs"] for i in last),
                         "evaluated": sum(i["weight_terms"] for i in last)},
        "roofline": roofline,
        "roofline_other_kernel": other,
    }
    if args.verbose:
        for i in last:
            print(json.dumps(i), file=sys.stderr)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(w, last, args.cpu_seconds)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / cb["value"]
    ctx.close()
    del ws_tensor
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
