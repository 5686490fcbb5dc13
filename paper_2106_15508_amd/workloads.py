"""Synthetic workloads: prior boxes, generating parameters and run sizes.

This module holds configuration only (numbers and seeded draws of sizes),
none of the method's arithmetic, so that the HIP library, the CPU oracle and
the benchmark all start from the same inputs.

The paper fits the model to 120 days of one country's confirmed case series
(§IV-A); that dataset is not available here.  Each workload instead observes
a trajectory simulated from a known generating vector ``THETA_TRUE`` with a
fixed observation seed, which gives the same structure (three integer series,
R and D cumulative, A rising then falling, counts reaching a sizeable share of
the population) and, unlike real data, a known answer for posterior-recovery
checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

#: Parameter order of eq. (1): [alpha0, alpha, n, beta, gamma, delta, eta, kappa]
PARAM_NAMES = ("alpha0", "alpha", "n", "beta", "gamma", "delta", "eta", "kappa")

#: Uniform prior box of eq. (2): U(0, [1, 100, 2, 1, 1, 1, 1, 2]).
PAPER_LO = (0.0,) * 8
PAPER_HI = (1.0, 100.0, 2.0, 1.0, 1.0, 1.0, 1.0, 2.0)

#: Prior box of the benchmark workloads (same parameters, narrower ranges:
#: alpha0 in [0,1], alpha in [1,100], n in [0,1], beta in [0,1],
#: gamma, delta, eta in [0,0.5], kappa in [0,2]).
BENCH_LO = (0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
BENCH_HI = (1.0, 100.0, 1.0, 1.0, 0.5, 0.5, 0.5, 2.0)

#: Generating parameters of the synthetic observations (inside both boxes).
THETA_TRUE = (0.3, 2.0, 0.5, 0.05, 0.1, 0.005, 0.2, 1.0)

#: Round index used for the observation stream (distinct from every SMC round).
OBS_ROUND = 0xFFFF

STEP_PAPER = 0   # eq. (16): Beta(eps_i / eps_1, 2 i)
STEP_FIXED = 1   # Beta(beta_a, beta_b) in every round
STEP_MCMC = 2    # one MCMC-tuned step size s per batch (eqs. 12-15); batch > 0
STEP_MEANVAR = 3   # Beta by mean (eps_i/eps_1)/3 and variance mu(1-mu)/(3i+1)
STEP_MODECONC = 4  # Beta by mode (eps_i/eps_1)/4 and concentration 2i+2
SAMPLER_BINOMIAL = 0
SAMPLER_NORMAL_FLOOR = 1


@dataclass(frozen=True)
class Workload:
    name: str
    population: int
    n_days: int
    n_particles: int
    n_rounds: int
    lo: Sequence[float] = BENCH_LO
    hi: Sequence[float] = BENCH_HI
    surv_ratio: float = 0.5
    step_schedule: int = STEP_PAPER
    beta_a: float = 0.0
    beta_b: int = 0
    step_is_variance: bool = False
    sampler: int = SAMPLER_BINOMIAL
    max_attempts: int = 256
    seed: int = 1
    obs_seed: int = 210615508
    batch: int = 0            # proposals per batch, 0 = library default
    max_proposals: int = 0    # per-round budget, 0 = 4096 * N
    theta_true: Sequence[float] = THETA_TRUE
    mcmc_s0: float = 0.1      # STEP_MCMC: initial step size
    mcmc_tune: int = 100      # STEP_MCMC: tuned batches (the first 10% of a 1000-run budget)
    eps_schedule: Sequence[float] = ()  # tolerances replayed in stages 1.. (eq. 8 afterwards)

    @property
    def a0(self) -> int:
        """Initial active confirmed cases: max(10, floor(1e-5 P)); R0 = D0 = 0."""
        return max(10, int(math.floor(1e-5 * self.population)))

    @property
    def obs0(self):
        return (self.a0, 0, 0)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


#: Smallest instance (parity-sized): P 1e5, 50 days, N 1024, 4 rounds,
#: fixed Beta(2,5) step sizes.
C1 = Workload("c1", population=100_000, n_days=50, n_particles=1024, n_rounds=4,
              step_schedule=STEP_FIXED, beta_a=2.0, beta_b=5, obs_seed=210615508 + 1)

#: Headline single-GPU instance: P 1e7, 120 days, N 131072, 10 rounds,
#: eq. (16) schedule.
C2 = Workload("c2", population=10_000_000, n_days=120, n_particles=131072, n_rounds=10,
              obs_seed=210615508 + 2)

#: Large single run: P 3e8, 180 days, N 1048576, 12 rounds.
C3 = Workload("c3", population=300_000_000, n_days=180, n_particles=1_048_576, n_rounds=12,
              obs_seed=210615508 + 3)

WORKLOADS = {"c1": C1, "c2": C2, "c3": C3}


def batched_runs(n_runs: int = 96, seed: int = 4, n_rounds: int = 10) -> List[Workload]:
    """The uneven multi-run workload: populations log-uniform in [1e5, 3e8],
    horizons uniform in {40..150} days, particle counts uniform on
    {2^11, ..., 2^16}, run seeds 1000 + r, own observation seeds."""
    rng = np.random.default_rng(seed)
    runs = []
    for r in range(n_runs):
        pop = int(round(math.exp(rng.uniform(math.log(1e5), math.log(3e8)))))
        days = int(rng.integers(40, 151))
        n = 1 << int(rng.integers(11, 17))
        runs.append(Workload(f"c4_{r}", population=pop, n_days=days, n_particles=n,
                             n_rounds=n_rounds, seed=1000 + r, obs_seed=210615508 + 400 + r))
    return runs


def tiny(**kw) -> Workload:
    """A small instance that spans several GPU tiles and a ragged tail."""
    base = Workload("tiny", population=20_000, n_days=30, n_particles=300, n_rounds=4,
                    obs_seed=210615508 + 9, seed=7)
    return base.with_(**kw)
