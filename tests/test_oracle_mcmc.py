"""Pins of the MCMC-tuned step variant (the paper's baseline, eqs. 12-15) in
the oracle: the adaptation's closed forms and the run's invariants."""
import numpy as np
import pytest

from paper_2106_15508_amd import workloads as W

A_T = 0.234


@pytest.mark.parametrize("n", [0, 1, 7, 1000])
def test_update_closed_forms(oracle, n):
    s = 0.37
    # A = A_T: no change
    assert oracle.mcmc_update(s, 234, 1000, n) == pytest.approx(s, rel=1e-15)
    # A = 1: s (n + 2) / (n + 1)
    assert oracle.mcmc_update(s, 50, 50, n) == pytest.approx(s * (n + 2) / (n + 1), rel=1e-15)
    # A = 0 (and no valid proposal): s (1 - A_T / ((1 - A_T)(n + 1)))
    for acc, valid in ((0, 40), (0, 0)):
        assert oracle.mcmc_update(s, acc, valid, n) == pytest.approx(
            s * (1 - A_T / ((1 - A_T) * (n + 1))), rel=1e-15)


def test_update_direction_and_gain(oracle):
    s = 0.2
    assert oracle.mcmc_update(s, 90, 100, 5) > s > oracle.mcmc_update(s, 10, 100, 5)
    # the gain shrinks as 1 / (n_acc + 1)
    assert abs(oracle.mcmc_update(s, 90, 100, 1000) - s) < abs(oracle.mcmc_update(s, 90, 100, 10) - s)
    # the step never changes sign
    assert oracle.mcmc_update(s, 0, 100, 0) > 0


def _mcmc(**kw):
    base = dict(step_schedule=W.STEP_MCMC, batch=256, mcmc_s0=0.1, mcmc_tune=5)
    base.update(kw)
    return W.tiny(**base)


def test_untuned_run_uses_the_initial_step(oracle):
    w = _mcmc(mcmc_tune=0, mcmc_s0=0.05)
    obs = oracle.observations(w)
    r = oracle.run(w, obs)
    assert r.rc == 0
    assert np.all(r.mcmc_s == 0.05)
    for i in range(1, w.n_rounds):
        assert np.all(r.sigma[i] == 0.05)


def test_tuned_run_one_step_per_batch(oracle):
    w = _mcmc()
    obs = oracle.observations(w)
    r = oracle.run(w, obs)
    assert r.rc == 0
    # every particle of a batch carries that batch's step size
    for i in range(1, w.n_rounds):
        b = r.index[i] // w.batch
        for k in np.unique(b):
            assert len(np.unique(r.sigma[i][b == k])) == 1
        # whole batches are simulated and the N-th acceptance lies in the last one
        assert r.simulated[i] % w.batch == 0
        assert r.simulated[i] - w.batch < r.proposals[i] <= r.simulated[i]
    # acceptance well above A_T here, so every tuned step grows s
    assert np.all(np.diff(r.mcmc_s) >= 0) and r.mcmc_s[-1] > w.mcmc_s0
    # the step of stage 1's first batch is the initial one
    assert np.all(r.sigma[1][r.index[1] < w.batch] == w.mcmc_s0)


def test_step_as_variance(oracle):
    w = _mcmc(mcmc_tune=0, mcmc_s0=0.0025, step_is_variance=True)
    obs = oracle.observations(w)
    r = oracle.run(w, obs)
    assert np.all(r.sigma[1] == 0.05)
