"""Process-parallel driver of the CPU oracle for full-size parity checks.

TEST INFRASTRUCTURE ONLY.  Proposals of a stage are independent given the
previous population, so the oracle's per-proposal functions are mapped over
index ranges in worker processes (started with "spawn": they never touch a
GPU).  The arithmetic is the oracle's, unchanged.
"""
from __future__ import annotations

import multiprocessing as mp
from typing import List, Sequence

import numpy as np


def _stage0(args):
    from oracle import ref
    w, obs, j0, j1 = args
    u = np.zeros((j1 - j0, 8))
    d = np.zeros(j1 - j0)
    for j in range(j0, j1):
        u[j - j0] = ref.prior_draw(w, j)
        d[j - j0] = ref.sim_distance(w, obs, u[j - j0], 0, j)
    return u, d


def _stage(args):
    from oracle import ref
    w, obs, rnd, u_prev, cdf, beta_a, beta_b, js = args
    out = []
    for j in js:
        a, u, s, par = ref.perturb(w, rnd, int(j), u_prev, cdf, beta_a, beta_b)
        d = ref.sim_distance(w, obs, u, rnd, int(j)) if a > 0 else float("inf")
        out.append((int(j), a, u, s, par, d))
    return out


def _pool(workers: int):
    return mp.get_context("spawn").Pool(workers)


def stage0(w, obs, n: int, workers: int = 8, chunk: int = 4096):
    """Stage-0 (prior) particles 0..n-1: unit-cube coordinates and distances."""
    jobs = [(w, obs, j, min(n, j + chunk)) for j in range(0, n, chunk)]
    with _pool(workers) as p:
        parts = p.map(_stage0, jobs)
    return np.concatenate([u for u, _ in parts]), np.concatenate([d for _, d in parts])


def stage(w, obs, rnd: int, u_prev, cdf, beta_a: float, beta_b: int, js: Sequence[int],
          workers: int = 8, chunk: int = 2048) -> List[tuple]:
    """(index, attempts, u, sigma, parent, d) of proposals js of stage rnd >= 1."""
    js = list(js)
    jobs = [(w, obs, rnd, u_prev, cdf, beta_a, beta_b, js[i:i + chunk]) for i in range(0, len(js), chunk)]
    with _pool(workers) as p:
        parts = p.map(_stage, jobs)
    return [r for part in parts for r in part]


# ------------------------------------------------------------------ timing
# The CPU-baseline leg of the benchmark times the oracle, as it stands, on
# per-stage samples of the same work: proposals of stage i (perturbation
# attempts, full simulation, distance) and importance-weight rows of stage i
# against stage i-1.

def reference_run(w, n_ref: int):
    """A run of workload w's model with N = n_ref: the populations whose
    proposals and weight rows are timed."""
    from oracle import ref
    wr = w.with_(n_particles=n_ref)
    obs = ref.observations(wr)
    run = ref.run(wr, obs)
    if run.rc != 0:
        raise RuntimeError(f"reference run failed: {run.rc}")
    return wr, obs, run


def _time_stages(args):
    """Seconds spent on proposals j0 .. j0+n_prop-1 of every stage and on
    weight rows r0 .. r0+n_rows-1 of every stage >= 1; returns per-stage
    (proposals, simulated, seconds) and (rows, terms, seconds)."""
    import time
    from oracle import ref
    wr, obs, run, j0, n_prop, r0, n_rows = args
    out = []
    for i in range(wr.n_rounds):
        if i > 0:
            q, Cc, _ = ref.resample_weights(run.dist[i - 1], run.eps[i])
        t0 = time.perf_counter()
        sim = 0
        for j in range(j0, j0 + n_prop):
            if i == 0:
                u, a = ref.prior_draw(wr, j), 1
            else:
                a, u, _, _ = ref.perturb(wr, i, j, run.u[i - 1], Cc, run.beta_a[i], int(run.beta_b[i]))
            if a > 0:
                ref.sim_distance(wr, obs, u, i, j)
                sim += 1
        t_sim = time.perf_counter() - t0
        rows = terms = 0
        t_w = 0.0
        if i > 0:
            # the previous population repeated 32 times: the same distances per
            # term, with the per-call overhead spread over 32x more columns
            N = len(run.sigma[i])
            up = np.ascontiguousarray(np.tile(run.u[i - 1], (32, 1)))
            qq = np.ascontiguousarray(np.tile(q, 32))
            t0 = time.perf_counter()
            for k in range(r0, r0 + n_rows):
                ref.log_weight(run.u[i][k % N], run.sigma[i][k % N], up, qq)
            t_w = time.perf_counter() - t0
            rows = n_rows
            terms = n_rows * int(np.count_nonzero(qq))
        out.append((n_prop, sim, t_sim, rows, terms, t_w))
    return out


def time_stages(wr, obs, run, n_prop: int, n_rows: int, workers: int = 1):
    """Per-stage oracle timing on `workers` processes, each on its own
    proposal indices and weight rows.  Returns (per-stage totals summed over
    the workers, wall seconds)."""
    import time
    jobs = [(wr, obs, run, 10_000_000 + k * n_prop, n_prop, k * n_rows, n_rows) for k in range(workers)]
    t0 = time.perf_counter()
    if workers == 1:
        parts = [_time_stages(jobs[0])]
    else:
        with _pool(workers) as p:
            parts = p.map(_time_stages, jobs)
    wall = time.perf_counter() - t0
    tot = [tuple(sum(p[i][k] for p in parts) for k in range(6)) for i in range(wr.n_rounds)]
    return tot, wall
