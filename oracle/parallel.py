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
