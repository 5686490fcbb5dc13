"""GPU parity of the whole hot path against the oracle.

Trajectories, distances, acceptances (population membership and order),
parents, step sizes, attempts and tolerances are compared bit for bit; the
importance weights to 1e-12 relative (the GPU sums the N x M terms in tile
order, the oracle with compensation)."""
import numpy as np
import pytest

from paper_2106_15508_amd import abcsmc as A
from paper_2106_15508_amd import workloads as W

pytestmark = pytest.mark.gpu

W_RTOL = 1e-12


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


@pytest.mark.parametrize("sampler", [W.SAMPLER_BINOMIAL, W.SAMPLER_NORMAL_FLOOR])
def test_trajectories_bitwise(oracle, sampler):
    w = W.C1.with_(sampler=sampler)
    rng = np.random.default_rng(10 + sampler)
    n = 700  # several workgroups and a ragged tail
    u = rng.uniform(size=(n, 8))
    theta = np.asarray(w.lo) + u * (np.asarray(w.hi) - np.asarray(w.lo))
    got = A.simulate(w, theta, seed=99, rnd=3, index0=5)
    for k in range(n):
        want = oracle.simulate(w, theta[k], 99, 3, 5 + k)
        assert np.array_equal(got[k], want), k


def test_trajectories_large_population(oracle):
    w = W.C3.with_(n_days=180)
    rng = np.random.default_rng(12)
    n = 300
    u = rng.uniform(size=(n, 8))
    theta = np.asarray(w.lo) + u * (np.asarray(w.hi) - np.asarray(w.lo))
    got = A.simulate(w, theta, seed=5, rnd=1, index0=0)
    for k in range(0, n, 7):
        assert np.array_equal(got[k], oracle.simulate(w, theta[k], 5, 1, k)), k


def test_observations_match_oracle(oracle):
    for w in (W.C1, W.C2, W.C3):
        assert np.array_equal(A.observations(w), oracle.observations(w))


def _compare_run(oracle, w, ref, ctx_rounds, pops, rounds):
    N = w.n_particles
    for i in range(rounds):
        info, pop = ctx_rounds[i], pops[i]
        assert info["eps"] == ref.eps[i] or (np.isinf(info["eps"]) and np.isinf(ref.eps[i]))
        assert _bits([info["eps_next"]])[0] == _bits([ref.eps_next[i]])[0], i
        assert info["proposals"] == ref.proposals[i], i
        assert np.array_equal(pop["index"], ref.index[i]), i
        assert np.array_equal(_bits(pop["u"]), _bits(ref.u[i])), i
        assert np.array_equal(_bits(pop["d"]), _bits(ref.dist[i])), i
        assert np.array_equal(_bits(pop["sigma"]), _bits(ref.sigma[i])), i
        assert np.array_equal(pop["parent"], ref.parent[i]), i
        assert np.array_equal(pop["attempts"], ref.attempts[i]), i
        if i > 0:
            assert info["beta_a"] == ref.beta_a[i] and info["beta_b"] == ref.beta_b[i]
            np.testing.assert_allclose(pop["W"], ref.W[i], rtol=W_RTOL, atol=0)
            # unnormalised log-weights agree up to the dropped constant log Q
            np.testing.assert_allclose(pop["logw"], ref.logw[i], rtol=1e-13, atol=1e-11)
        else:
            assert np.all(pop["W"] == 1.0 / N)


def _gpu_run(w, obs, rounds, **kw):
    infos, pops = [], []
    with A.Context(w, obs, **kw) as ctx:
        for _ in range(rounds):
            infos.append(ctx.round())
            p = ctx.population()
            th, d, wt = ctx.weights()
            p["d"], p["W"], p["theta"] = d, wt, th
            pops.append(p)
    return infos, pops


@pytest.mark.parametrize("wl", [
    W.tiny(),
    W.tiny(step_schedule=W.STEP_FIXED, beta_a=2.0, beta_b=5, seed=8),
    W.C1,
])
def test_run_bitwise(oracle, wl):
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0
    infos, pops = _gpu_run(wl, obs, wl.n_rounds)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)


def test_run_paper_schedule_many_rounds(oracle):
    wl = W.C1.with_(n_rounds=8, step_schedule=W.STEP_PAPER, seed=3)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    infos, pops = _gpu_run(wl, obs, wl.n_rounds)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)


@pytest.mark.parametrize("batch", [256, 1000, 4096])
def test_batch_size_does_not_change_results(oracle, batch):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    a_infos, a = _gpu_run(wl, obs, 3)
    b_infos, b = _gpu_run(wl.with_(batch=batch), obs, 3)
    for i in range(3):
        assert a_infos[i]["eps_next"] == b_infos[i]["eps_next"]
        assert np.array_equal(a[i]["index"], b[i]["index"])
        assert np.array_equal(_bits(a[i]["u"]), _bits(b[i]["u"]))
        assert np.array_equal(_bits(a[i]["W"]), _bits(b[i]["W"]))


def test_short_first_batch_completed_and_weights_redone(oracle):
    """A later stage's first batch is sized from the previous stage's
    acceptance rate and its counters come back only with the tolerance; when
    the replayed tolerance of stage 2 drops far below the one stage 1 accepted
    against, that batch falls short of N, the stage runs further batches and
    forms its weights and tolerance again.  Every stage equals the oracle's
    run under the same schedule."""
    base = W.C1.with_(n_rounds=4, seed=5)
    obs = oracle.observations(base)
    pilot = oracle.run(base.with_(n_rounds=2), obs)
    d1 = np.sort(pilot.dist[1])
    sched = (float(pilot.eps_next[0]), float(d1[len(d1) // 50]))
    wl = base.with_(eps_schedule=sched)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0
    infos, pops = _gpu_run(wl, obs, wl.n_rounds)
    assert infos[2]["batches"] >= 2, infos[2]
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)
    # the terms counted are those of the one weight pass that stands
    assert infos[2]["weight_terms"] <= wl.n_particles * infos[2]["survivors"]


def _random_workload(k):
    """Seeded draw of a small configuration: population, horizon, particle
    count (ragged against the 256-lane workgroups), survival ratio and seeds
    drawn; step law, sampler, the variance reading of the step and early
    exit cycled so that the six draws cover each of them."""
    rng = np.random.default_rng(9000 + k)
    step = (W.STEP_PAPER, W.STEP_FIXED, W.STEP_MEANVAR, W.STEP_PAPER, W.STEP_MODECONC, W.STEP_FIXED)[k]
    kw = dict(population=int(np.exp(rng.uniform(np.log(2e4), np.log(5e6)))), n_days=int(rng.integers(20, 91)),
              n_particles=int(rng.choice([300, 517, 1024, 1500, 2048])), n_rounds=3,
              surv_ratio=float(rng.choice([0.3, 0.5, 0.7])), sampler=k % 2, step_schedule=step,
              seed=int(rng.integers(1, 1 << 30)), obs_seed=int(rng.integers(1, 1 << 30)),
              step_is_variance=(k // 2) % 2 == 1)
    if step == W.STEP_FIXED:
        kw.update(beta_a=float(rng.uniform(0.5, 4.0)), beta_b=int(rng.integers(1, 9)))
    return W.tiny(**kw), (A.F_EARLY_EXIT if k % 3 else 0)


@pytest.mark.parametrize("k", range(6))
def test_random_configurations_bitwise(oracle, k):
    wl, flags = _random_workload(k)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0, wl
    infos, pops = _gpu_run(wl, obs, wl.n_rounds, flags=flags)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)


def test_early_exit_keeps_acceptances(oracle):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    infos, pops = _gpu_run(wl, obs, 3, flags=A.F_EARLY_EXIT)
    _compare_run(oracle, wl, ref, infos, pops, 3)


def test_step_is_variance_and_normal_floor(oracle):
    wl = W.tiny(n_rounds=3, step_is_variance=True, sampler=W.SAMPLER_NORMAL_FLOOR, seed=11)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    infos, pops = _gpu_run(wl, obs, 3)
    _compare_run(oracle, wl, ref, infos, pops, 3)


def test_resampling_law_matches(oracle):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    with A.Context(wl, obs) as ctx:
        ctx.run(3)
        q, cdf = ctx.resampling()
    q_ref, c_ref, _ = oracle.resample_weights(ref.dist[1], ref.eps[2])
    assert np.array_equal(q, q_ref) and np.array_equal(cdf, c_ref)


def test_abcsmc_run_entry_point(oracle):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    th, d, wt, infos = A.run(wl, obs)
    assert np.array_equal(_bits(d), _bits(ref.dist[-1]))
    assert np.array_equal(_bits(th), _bits(ref.theta(wl)[-1]))
    np.testing.assert_allclose(wt, ref.W[-1], rtol=W_RTOL)
    assert [i["proposals"] for i in infos] == list(ref.proposals)


def test_budget_error_leaves_context_usable(oracle):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    with A.Context(wl, obs, max_proposals=wl.n_particles + 10, batch=256) as ctx:
        ctx.round()
        with pytest.raises(A.AbcsmcError) as e:
            ctx.round()
        assert e.value.code == A.EBUDGET
        assert ctx.rounds_done() == 1
        th, d, wt = ctx.weights()
        assert np.all(wt == 1.0 / wl.n_particles)


def test_weights_before_round_is_state_error(oracle):
    wl = W.tiny()
    obs = oracle.observations(wl)
    with A.Context(wl, obs) as ctx:
        with pytest.raises(A.AbcsmcError) as e:
            ctx.weights()
        assert e.value.code == A.ESTATE


@pytest.mark.parametrize("wl", [
    W.tiny(step_schedule=W.STEP_MCMC, batch=256, mcmc_s0=0.1, mcmc_tune=5),
    W.tiny(step_schedule=W.STEP_MCMC, batch=1000, mcmc_s0=0.003, mcmc_tune=100, step_is_variance=True, seed=5),
    W.C1.with_(step_schedule=W.STEP_MCMC, batch=1024, mcmc_s0=0.05, mcmc_tune=3),
])
def test_mcmc_variant_bitwise(oracle, wl):
    """The paper's baseline (one tuned step size per batch, eqs. 12-15):
    every stage, the step size after every tuned batch and the whole-batch
    counts agree with the oracle bit for bit."""
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0
    infos, pops = _gpu_run(wl, obs, wl.n_rounds, flags=A.F_EARLY_EXIT)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)
    for i in range(1, wl.n_rounds):
        assert _bits([infos[i]["mcmc_s"]])[0] == _bits([ref.mcmc_s[i]])[0], i
        assert infos[i]["simulated"] == ref.simulated[i], i
        assert infos[i]["invalid"] == ref.invalid[i], i


@pytest.mark.parametrize("wl,days", [(W.tiny(n_rounds=3), 45), (W.C1.with_(n_rounds=2), 80)])
def test_predictive_bands_bitwise(oracle, wl, days):
    """Posterior predictive bands (Fig. 7) past the fitted horizon: the
    oracle's own run and predictive simulations against the GPU's."""
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    q = (0.005, 0.25, 0.5, 0.75, 0.995, 0.0, 1.0)
    want = oracle.predict(wl, obs, ref.u[-1], days, seed=77, quantiles=q)
    with A.Context(wl, obs) as ctx:
        ctx.run(wl.n_rounds)
        got = ctx.predict(days, seed=77, quantiles=q)
    assert np.array_equal(_bits(got), _bits(want))
    # day 0 is the observed initial state for every particle
    assert np.all(got[0, :, :] == np.asarray(obs[0], dtype=np.float64)[:, None])


@pytest.mark.parametrize("wl", [
    W.tiny(step_schedule=W.STEP_MEANVAR),
    W.tiny(step_schedule=W.STEP_MODECONC, seed=12),
    W.C1.with_(step_schedule=W.STEP_MEANVAR, n_rounds=5),
])
def test_alternative_beta_parameterisations_bitwise(oracle, wl):
    """Mean-variance and mode-concentration step-size Betas (real shapes,
    gamma-ratio sampler): runs match the oracle bit for bit."""
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0
    infos, pops = _gpu_run(wl, obs, wl.n_rounds)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)
    for i in range(1, wl.n_rounds):
        assert _bits([infos[i]["beta_b_real"]])[0] == _bits([ref.beta_b_real[i]])[0], i


@pytest.mark.parametrize("wl", [
    # smallest population of particles, one simulated day
    W.tiny(n_particles=2, n_days=1, n_rounds=4, seed=21),
    # degenerate prior box: three parameters fixed (lo = hi)
    W.tiny(lo=(0.3, 1.0, 0.5, 0.0, 0.1, 0.0, 0.2, 0.0), hi=(0.3, 100.0, 0.5, 1.0, 0.1, 0.5, 0.2, 2.0),
           n_rounds=3, seed=22),
    # tiny survival ratio (eq. 8 at the 2nd order statistic) and N not a multiple of a wave
    W.tiny(n_particles=97, surv_ratio=0.01, n_rounds=4, seed=23),
    # the longest horizon the library accepts (4096 days)
    W.tiny(n_particles=64, n_days=4096, n_rounds=3, seed=24),
    # a population of 2^52: counts near the top of the exact-integer range of doubles
    W.tiny(population=1 << 52, n_days=40, n_rounds=3, seed=25),
])
def test_edge_configurations_bitwise(oracle, wl):
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    assert ref.rc == 0
    infos, pops = _gpu_run(wl, obs, wl.n_rounds, flags=A.F_EARLY_EXIT)
    _compare_run(oracle, wl, ref, infos, pops, wl.n_rounds)


def test_predict_shorter_than_fitted_horizon(oracle):
    wl = W.tiny(n_rounds=2)
    obs = oracle.observations(wl)
    ref = oracle.run(wl, obs)
    want = oracle.predict(wl, obs, ref.u[-1], 5, seed=3, quantiles=(0.5,))
    with A.Context(wl, obs) as ctx:
        ctx.run(2)
        got = ctx.predict(5, seed=3, quantiles=(0.5,))
        with pytest.raises(A.AbcsmcError):
            ctx.predict(0, seed=3, quantiles=(0.5,))
        with pytest.raises(A.AbcsmcError):
            ctx.predict(5, seed=3, quantiles=(1.5,))
    assert np.array_equal(_bits(got), _bits(want))


def test_mcmc_budget_error_leaves_context_usable(oracle):
    """A stage that cannot reach N acceptances within max_proposals returns
    EBUDGET and leaves the last completed stage in place.  The oracle, run
    on the same configuration, says which stage runs out (here stage 1: its
    five 64-proposal batches hold fewer than 300 acceptances)."""
    wl = W.tiny(step_schedule=W.STEP_MCMC, batch=64, mcmc_s0=0.1, mcmc_tune=3, max_proposals=320, seed=24)
    obs = oracle.observations(wl)
    want = oracle.run(wl, obs, n_rounds=6)
    assert want.rc == -4
    completed = int(np.count_nonzero(want.proposals))
    assert completed == 1
    with A.Context(wl, obs) as ctx:
        for i in range(completed):
            info = ctx.round()
            assert info["eps_next"] == want.eps_next[i]
        before = ctx.population()
        with pytest.raises(A.AbcsmcError) as e:
            ctx.round()
        assert e.value.code == A.EBUDGET
        assert ctx.rounds_done() == completed
        after = ctx.population()
        assert np.array_equal(after["index"], before["index"])
        assert np.array_equal(_bits(after["u"]), _bits(before["u"]))
        assert np.array_equal(_bits(after["u"]), _bits(want.u[completed - 1]))
        _, d, wt = ctx.weights()
        assert np.array_equal(_bits(d), _bits(want.dist[completed - 1]))
