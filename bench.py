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
library's stream around each launch; algorithmic flops from the op-counting
build of the oracle), the CPU oracle timed on a bounded sample of the same
workload on one core and on all cores, and sub-objects for the large single
run (c3), the batched mode (c4) and the learned screen (c5).

    python bench.py [--steps K] [--warmup W] [--workload c2|c3|c4|c5] [--no-extra]
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

# Algorithmic FP64 flops (fma = 2) counted by the op-counting build of the
# oracle on its own branch decisions (python -m oracle.opcount c2 / c3; the
# output is kept in profiles/opcount_c2_c3.md):
#   PAIR: one importance-weight term whose exponential is evaluated (8
#         differences, 8 squares, 8 additions, the scaling division, the
#         exponential 31, the weight product and the addition into the sum);
#   day:  one simulated day (eqs. 3-5 and the day's three squared
#         differences), per stage (the binomial branches taken change as the
#         populations concentrate);
#   prop: per simulated proposal outside the day loop (parameters from the
#         unit cube, initial state, the four fixed rates, the final sqrt);
#   att:  per perturbation attempt (categorical draw, Beta step size with b
#         logarithms, eight normals, the support check); stage 0: the prior
#         draw.
PAIR_FLOPS = 58.0
OPCOUNT = {
    "c2": dict(day=[393.4, 443.8, 498.9, 527.1, 533.5, 533.8, 533.3, 532.9, 533.2, 533.4],
               prop=[142.8, 142.8, 142.1, 140.8, 138.5, 136.3, 136.0, 136.0, 136.0, 136.0],
               att=[16.0, 441.5, 516.4, 591.2, 665.9, 740.8, 815.7, 890.4, 965.3, 1040.0]),
    "c3": dict(day=[373.1, 393.0, 452.5, 508.7, 531.9, 535.4, 535.9, 536.5, 536.8, 536.8, 536.8, 536.8],
               prop=[142.8, 142.3, 141.9, 140.8, 139.7, 138.7, 136.5, 136.0, 136.0, 136.0, 136.0, 136.0],
               att=[16.0, 441.5, 516.3, 591.1, 665.9, 740.8, 815.7, 890.4, 965.4, 1040.0, 1114.9, 1189.7]),
}

# HBM bytes per launch of a kernel measured with rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE on a workload, scaled by the counters' reading for a 256 MiB
# device copy (FETCH 0.5x, WRITE 1.0x of the bytes moved).  Keyed by the
# SHA-256 of the kernel sources and the build flags: a changed kernel reports
# null.
TRAFFIC_SOURCES = ("paper_2106_15508_amd/csrc/smc.hip", "paper_2106_15508_amd/csrc/dmath.h",
                   "paper_2106_15508_amd/csrc/kernels.h", "paper_2106_15508_amd/csrc/wterm.h",
                   "paper_2106_15508_amd/csrc/sim.hip", "paper_2106_15508_amd/csrc/propose.h",
                   "paper_2106_15508_amd/build.py")
TRAFFIC_MEASURED = {
    # (sources, workload, kernel): (FETCH_SIZE KiB x 2 + WRITE_SIZE KiB x 1) x 1024 bytes per launch,
    # averaged over the launches of one run (commands and raw values in profiles/)
    ("dddc6a4450cfe0f7", "c2", "weights_kernel"): 1.1746e9,
    ("dddc6a4450cfe0f7", "c2", "propose_kernel"): 4.8978e7,
    ("dddc6a4450cfe0f7", "c3", "weights_kernel"): 8.9099e10,
    ("dddc6a4450cfe0f7", "c3", "propose_kernel"): 8.7435e8,
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5"],
                    help="c4: 96 uneven runs in the batched mode, compared with the same runs one at a time; "
                         "c5: the headline workload with the learned screen")
    ap.add_argument("--runs", type=int, default=96, help="c4: number of runs")
    ap.add_argument("--early-exit", type=int, default=1, help="stop simulating a proposal once its "
                    "partial distance exceeds eps (acceptances unchanged)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="budget of the one-core oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline line without the c3/c4/c5 sub-objects")
    ap.add_argument("--no-peaks", action="store_true", help="skip the FP64 fma and copy microbenchmarks")
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


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------------- CPU oracle

def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_unit_costs(w, budget_s: float, workers: int):
    """The oracle (as it stands, one process per core) timed on per-stage
    samples of the same work: a reference run of workload w's model with
    N = 1024 supplies each stage's previous population; per stage, proposals
    are perturbed, simulated in full and measured, and importance-weight rows
    of the stage are summed against the previous population.  Returns
    per-stage seconds per examined proposal and per defined weight term."""
    from oracle import parallel
    wr, obs, run = parallel.reference_run(w, 1024)
    # size the sample to the budget from a short calibration on one core
    cal, _ = parallel.time_stages(wr, obs, run, 8, 2, 1)
    t_prop = sum(c[2] for c in cal) / 8
    t_row = sum(c[5] for c in cal) / 2
    n_prop = max(16, int(0.5 * budget_s / max(t_prop, 1e-6)))
    n_rows = max(4, int(0.5 * budget_s / max(t_row, 1e-6)))
    tot, wall = parallel.time_stages(wr, obs, run, n_prop, n_rows, workers)
    s_prop = [c[2] / c[0] for c in tot]
    s_term = [c[5] / c[4] if c[4] else 0.0 for c in tot]
    return dict(s_prop=s_prop, s_term=s_term, n_prop=n_prop * workers, n_rows=n_rows * workers, wall=wall,
                workers=workers, n_stages=wr.n_rounds)


def cpu_baseline(w, infos, units_1, units_all):
    """Accepted particles/s of the oracle at the GPU run's own per-stage
    counts: examined proposals (the oracle stops at the N-th acceptance and
    simulates every day) and defined weight terms (N x survivors)."""
    def run_seconds(u):
        t = 0.0
        for i, inf in enumerate(infos):
            k = min(i, u["n_stages"] - 1)
            t += inf["proposals"] * u["s_prop"][k] + inf["weight_pairs"] * u["s_term"][k]
        return t
    acc = w.n_particles * len(infos)
    t1 = run_seconds(units_1)
    out = {
        "value": acc / t1, "unit": "accepted particles/s", "cores": 1, "kind": "oracle",
        "sample": (f"per stage of a reference run of the same model (N=1024): {units_1['n_prop']} proposals "
                   f"perturbed and simulated in full and {units_1['n_rows']} importance-weight rows on one core "
                   f"({units_1['wall']:.1f} s); per-proposal and per-term seconds scaled by this run's examined "
                   f"proposals ({sum(i['proposals'] for i in infos)}) and defined weight terms "
                   f"({sum(i['weight_pairs'] for i in infos)}) per stage"),
        "extrapolated_run_s": round(t1, 1), "cpu_model": cpu_model(),
    }
    if units_all:
        ta = run_seconds(units_all) / units_all["workers"]
        out["all_cores"] = {
            "value": acc / ta, "unit": "accepted particles/s", "cores": units_all["workers"], "kind": "oracle",
            "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
            "sample": (f"the same per-stage sample on {units_all['workers']} processes at once (one per core, "
                       f"{units_all['n_prop']} proposals and {units_all['n_rows']} rows per stage in all, "
                       f"{units_all['wall']:.1f} s wall); seconds per unit measured under that load, divided "
                       f"by the process count"),
            "extrapolated_run_s": round(ta, 2),
        }
    return out


# ----------------------------------------------------------------- rooflines

def propose_flops(infos, table):
    """Algorithmic flops of a run's proposal launches: simulated days, the
    per-proposal work outside the day loop and the perturbation attempts,
    each at its stage's op count."""
    f = 0.0
    for i, inf in enumerate(infos):
        k = min(i, len(table["day"]) - 1)
        f += inf["sim_days"] * table["day"][k]
        f += (inf["simulated"] - inf["invalid"]) * table["prop"][k]
        f += inf["attempts"] * table["att"][k]
    return f


def alu_roofline(kernel, flops, ms_total, launches, traffic, units):
    avg_ms = ms_total / launches
    achieved = flops / launches / (avg_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic, "kernel": kernel,
            "avg_launch_ms": round(avg_ms, 4), "launches": launches, "flops_per_launch": flops / launches,
            "units": units}


def run_single(w, steps, warmup, flags, sha, key):
    """Time `steps` complete runs of workload w (after `warmup`) on a torch
    workspace and stream; returns the timing, the stage infos of every step
    and both kernels' rooflines."""
    import torch

    from paper_2106_15508_amd import abcsmc as A
    R = w.n_rounds
    obs = A.observations(w)                       # synthetic series from THETA_TRUE (on the GPU)
    ws_tensor, ws = A.torch_workspace(w)          # workspace: device memory owned by torch
    stream = torch.cuda.current_stream()
    ctx = A.Context(w, obs, stream=stream.cuda_stream, workspace=ws, flags=flags)
    for _ in range(warmup):
        ctx.reset()
        ctx.run(R)
        ctx.weights()                             # the copy-out path's one-time set-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps_infos = []
    for _ in range(steps):
        ctx.reset()
        steps_infos.append(ctx.run(R))
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    # PCIe-inclusive: the final population (theta, d, W) copied to host memory
    # through the C ABI after the run (pinned staging allocated during the
    # warm-up); the observations go in once at init
    tc = time.perf_counter()
    ctx.weights()
    sec_copy = time.perf_counter() - tc
    ctx.close()
    del ws_tensor
    allinf = [i for s in steps_infos for i in s]
    ms_p = sum(i["ms_k_propose"] for i in allinf)
    n_p = sum(i["n_k_propose"] for i in allinf)
    ms_w = sum(i["ms_k_weights"] for i in allinf)
    n_w = sum(1 for i in allinf if i["round"] > 0)
    table = OPCOUNT.get(key, OPCOUNT["c2"])
    wterms = sum(i["weight_window_terms"] for i in allinf)
    eterms = sum(i["weight_terms"] for i in allinf)
    rl_w = None
    if n_w:
        rl_w = alu_roofline("weights_kernel", wterms * PAIR_FLOPS, ms_w, n_w,
                            TRAFFIC_MEASURED.get((sha, key, "weights_kernel")),
                            f"terms inside the rows' own windows x {PAIR_FLOPS:g} flops")
        ev = eterms * PAIR_FLOPS / (ms_w * 1e-3) / 1e12
        rl_w["achieved_on_evaluated_terms"] = round(ev, 3)
        rl_w["frac_on_evaluated_terms"] = round(ev / PEAK_FP64_TFLOPS, 4)
    rl_p = alu_roofline("propose_kernel", propose_flops([i for s in steps_infos for i in s], table), ms_p, n_p,
                        TRAFFIC_MEASURED.get((sha, key, "propose_kernel")),
                        "simulated days, proposals and perturbation attempts x their per-stage op counts")
    return dict(sec=sec, sec_copy=sec_copy, infos=steps_infos, last=steps_infos[-1], rl_w=rl_w, rl_p=rl_p,
                ms_p=ms_p / steps, ms_w=ms_w / steps, wterms=wterms / steps, eterms=eterms / steps)


def single_summary(w, r, args):
    last = r["last"]
    N, R = w.n_particles, w.n_rounds
    sec = r["sec"]
    roofline = r["rl_w"] if (r["rl_w"] and r["ms_w"] >= r["ms_p"]) else r["rl_p"]
    other = r["rl_p"] if roofline is r["rl_w"] else r["rl_w"]
    return {
        "value": N * R / sec,
        "ms_per_step": sec * 1e3,
        "pcie_inclusive_value": N * R / (sec + r["sec_copy"]),
        "ms_copy_out": round(r["sec_copy"] * 1e3, 3),
        "simulations_per_s": sum(i["simulated"] for i in last) / sec,
        "useful_simulations_per_s": sum(i["proposals"] for i in last) / sec,
        "particle_days_per_s": sum(i["sim_days"] for i in last) / sec,
        "eps_final": last[-1]["eps_next"],
        "phase_ms": {k: round(sum(i[k] for i in last), 3)
                     for k in ("ms_resample", "ms_simulate", "ms_weights", "ms_select", "ms_total")},
        "kernel_ms": {"propose": round(r["ms_p"], 3), "weights": round(r["ms_w"], 3)},
        "weight_terms": {"defined": sum(i["weight_pairs"] for i in last),
                         "in_window": sum(i["weight_window_terms"] for i in last),
                         "evaluated": sum(i["weight_terms"] for i in last)},
        "roofline": roofline,
        "roofline_other_kernel": other,
    }


def workload_text(w):
    return (f"{w.name}: P={w.population}, T={w.n_days}, N={w.n_particles}, stages={w.n_rounds}, "
            "eq.16 Beta step sizes, chain-binomial simulator, synthetic observations of theta_true")


# ----------------------------------------------------------------- batched (c4)

def bench_batched(args, steps, warmup):
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
    for _ in range(warmup):
        b.reset()
        b.run(R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.reset()
        infos = b.run(R)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / steps
    accepted = sum(w.n_particles for w in runs) * R
    simulated = sum(i["simulated"] for st in infos for i in st)
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
    del ws_tensor
    return {
        "value": accepted / sec, "unit": "accepted particles/s", "steps": steps, "ms_per_step": sec * 1e3,
        "workload": (f"c4: {len(runs)} independent runs, P log-uniform in [1e5, 3e8], T in [40, 150], "
                     f"N in {{2^11..2^16}} (sum N = {sum(w.n_particles for w in runs)}), {R} stages, "
                     "batched mode (one graph replay per stage)"),
        "simulations_per_s": simulated / sec,
        "plain_sequential_value": accepted / sec_plain,
        "speedup_vs_plain": sec_plain / sec,
        "failed_runs": failed, "schedule": sched, "autotune_s": round(tune_s, 2),
        "weight_terms": {"defined": sum(i["weight_pairs"] for st in infos for i in st),
                         "in_window": sum(i["weight_window_terms"] for st in infos for i in st),
                         "evaluated": sum(i["weight_terms"] for st in infos for i in st)},
    }


# ----------------------------------------------------------------- screened (c5)

def bench_surrogate(args, steps, warmup):
    """The headline workload with the learned screen: per step, stage 0, the
    network's initial fit on 2^22 prior simulations (2 passes, minibatch
    32768, Adam step 5e-3, included in the step), then nine screened stages
    (keep 10% of each stage's first batch by score, audit rho = 1%,
    screening kept on in every stage).  The same steps of the plain form run
    beside it for the comparison of throughput and posterior moments."""
    import numpy as np
    import torch

    from paper_2106_15508_amd import abcsmc as A
    from paper_2106_15508_amd import workloads as W

    w = W.C2
    R = w.n_rounds
    obs = A.observations(w)
    stream = torch.cuda.current_stream()
    flags = A.F_EARLY_EXIT if args.early_exit else 0
    sur = dict(n_train=1 << 22, epochs=2, batch=32768, lr=5e-3, keep_frac=0.1, audit_rho=0.01, fn_max=1.0, seed=11)

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
        for _ in range(warmup):
            one(ctx, screened)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runs = [one(ctx, screened) for _ in range(steps)]
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
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
    return {
        "value": N * R / scr["sec"], "unit": "accepted particles/s", "steps": steps, "ms_per_step": scr["sec"] * 1e3,
        "workload": (f"c5: c2 (P={w.population}, T={w.n_days}, N={N}, stages={R}) with the learned screen: fit "
                     "on 2^22 prior simulations x 2 passes of minibatch 32768, keep 10%, audit 1%"),
        "plain_value": N * R / plain["sec"],
        "speedup_vs_plain": plain["sec"] / scr["sec"],
        "fn_mass": [round(s["fn_mass"], 4) for s in last_s],
        "surrogate": {
            "ms_data": si0["ms_data"], "ms_train": si0["ms_train"], "loss_first": si0["loss_first"],
            "loss_last": si0["loss_last"],
            "enrichment": [round(s["enrichment"], 3) for s in last_s],
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
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_TFLOPS, 5), "traffic": None,
                     "kernel": "network initial fit (matrix products and their epilogues)",
                     "phase_ms": round(ms_train, 3), "flops": train_flops},
    }


# ----------------------------------------------------------------- main

def envelope(args, steps, warmup, value, ms, workload, dtype="f64", extra=None):
    out = {"metric": "accepted particles/s", "value": value, "unit": "accepted particles/s", "n_gpus": 1,
           "steps": steps, "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": workload, "early_exit": bool(args.early_exit)}}
    out.update(extra or {})
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the ABC-SMC path here runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    from paper_2106_15508_amd import workloads as W

    # the CPU legs first, before anything touches the GPU (their worker
    # processes are started fresh)
    units_1 = units_all = None
    if not args.no_cpu_baseline and args.workload in ("c1", "c2", "c3"):
        w = W.WORKLOADS[args.workload]
        log("oracle on one core ...")
        units_1 = cpu_unit_costs(w, args.cpu_seconds, 1)
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
        if workers > 1:
            log(f"oracle on {workers} cores ...")
            units_all = cpu_unit_costs(w, args.cpu_seconds / 2, workers)
    units_c3 = None
    if not args.no_cpu_baseline and args.workload == "c2" and not args.no_extra:
        log("oracle on one core, c3 sample ...")
        units_c3 = cpu_unit_costs(W.C3, args.cpu_seconds / 2, 1)

    import torch

    from paper_2106_15508_amd import abcsmc as A
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    flags = A.F_EARLY_EXIT if args.early_exit else 0
    sha = kernel_sources_sha()

    if args.workload == "c4":
        r = bench_batched(args, args.steps, args.warmup)
        print(json.dumps(envelope(args, args.steps, args.warmup, r["value"], r["ms_per_step"], r["workload"],
                                  extra={"c4": r})), flush=True)
        return
    if args.workload == "c5":
        r = bench_surrogate(args, args.steps, args.warmup)
        print(json.dumps(envelope(args, args.steps, args.warmup, r["value"], r["ms_per_step"], r["workload"],
                                  dtype="f64+bf16", extra={"c5": r, "roofline": r["roofline"]})), flush=True)
        return

    w = W.WORKLOADS[args.workload]
    log(f"{w.name}: {args.steps} steps after {args.warmup} warm-up")
    r = run_single(w, args.steps, args.warmup, flags, sha, args.workload)
    s = single_summary(w, r, args)
    out = envelope(args, args.steps, args.warmup, s.pop("value"), s.pop("ms_per_step"), workload_text(w),
                   extra=s)
    if args.verbose:
        for i in r["last"]:
            print(json.dumps(i), file=sys.stderr)
    if not args.no_peaks:
        # context for the fractions above (which stay against the published
        # peaks): what this device sustains on a plain FP64 fma loop and a copy
        pk = A.measure_peaks(5)
        out["measured_peaks"] = {"fp64_fma_tflops": round(pk["fp64_tflops"], 2),
                                 "clock_mhz_during_fma": round(pk["clock_mhz"]),
                                 "copy_gbs": round(pk["copy_gbs"], 1)}
        for key in ("roofline", "roofline_other_kernel"):
            if key in out and pk["fp64_tflops"] > 0:
                out[key]["frac_of_measured_fp64"] = round(out[key]["achieved"] / pk["fp64_tflops"], 4)
    if units_1:
        out["cpu_baseline"] = cpu_baseline(w, r["last"], units_1, units_all)
        out["cpu_baseline"]["gpu_over_cpu"] = out["value"] / out["cpu_baseline"]["value"]
    if args.workload == "c2" and not args.no_extra:
        w3 = W.C3
        log("c3: 2 steps after 1 warm-up")
        r3 = run_single(w3, 2, 1, flags, sha, "c3")
        s3 = single_summary(w3, r3, args)
        out["c3"] = {"value": s3["value"], "unit": "accepted particles/s", "steps": 2,
                     "ms_per_step": s3["ms_per_step"], "workload": workload_text(w3),
                     "simulations_per_s": s3["simulations_per_s"], "particle_days_per_s": s3["particle_days_per_s"],
                     "kernel_ms": s3["kernel_ms"], "weight_terms": s3["weight_terms"],
                     "roofline": s3["roofline"], "roofline_other_kernel": s3["roofline_other_kernel"]}
        if units_c3:
            out["c3"]["cpu_baseline"] = cpu_baseline(w3, r3["last"], units_c3, None)
            out["c3"]["cpu_baseline"]["gpu_over_cpu"] = s3["value"] / out["c3"]["cpu_baseline"]["value"]
        log("c4: batched mode, 3 steps after 1 warm-up, then the runs one at a time")
        out["c4"] = bench_batched(args, min(args.steps, 3), 1)
        log("c5: learned screen, 1 step after 1 warm-up, beside the plain form")
        out["c5"] = bench_surrogate(args, 1, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
