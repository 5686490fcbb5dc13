"""Checkpoint/resume, replayed tolerance schedules and weight-free runs on
the GPU.

A run continued from abcsmc_snapshot / abcsmc_restore must be the same run
bit for bit; a replayed schedule is checked against the oracle running the
same schedule (the oracle's own pins show that replaying its eq. 8 values
changes nothing); ABCSMC_F_SKIP_WEIGHTS leaves every trajectory, acceptance
and tolerance untouched."""
import numpy as np
import pytest

from paper_2106_15508_amd import abcsmc as A
from paper_2106_15508_amd import workloads as W
from test_gpu_parity import _bits, _compare_run, _gpu_run

pytestmark = pytest.mark.gpu


def _state(ctx):
    p = ctx.population()
    th, d, wt = ctx.weights()
    return p, d, wt


def _same(a, b):
    (pa, da, wa), (pb, db, wb) = a, b
    assert np.array_equal(_bits(pa["u"]), _bits(pb["u"]))
    assert np.array_equal(_bits(da), _bits(db))
    assert np.array_equal(_bits(pa["sigma"]), _bits(pb["sigma"]))
    assert np.array_equal(pa["parent"], pb["parent"]) and np.array_equal(pa["index"], pb["index"])
    assert np.array_equal(_bits(wa), _bits(wb))


@pytest.mark.parametrize("wl", [
    W.tiny(n_rounds=5),
    W.tiny(n_rounds=5, step_schedule=W.STEP_MCMC, batch=512, mcmc_tune=3, seed=4),
    W.tiny(n_rounds=5, step_schedule=W.STEP_MEANVAR, seed=6),
])
def test_snapshot_restore_continues_bitwise(oracle, wl):
    obs = oracle.observations(wl)
    with A.Context(wl, obs, flags=A.F_EARLY_EXIT) as ctx:
        ctx.run(2)
        snap = ctx.snapshot()
        cont = ctx.run(3)
        end = _state(ctx)
    with A.Context(wl, obs, flags=A.F_EARLY_EXIT, snapshot=snap) as ctx:
        assert ctx.rounds_done() == 2
        again = ctx.run(3)
        end2 = _state(ctx)
        # the restored context still knows its own start
        ctx.reset()
        assert ctx.rounds_done() == 0
    for a, b in zip(cont, again):
        for k in ("round", "eps", "eps_next", "proposals", "simulated", "beta_a", "beta_b", "mcmc_s"):
            assert a[k] == b[k], k
    _same(end, end2)


def test_restore_rejects_other_config(oracle):
    wl = W.tiny(n_rounds=2)
    obs = oracle.observations(wl)
    with A.Context(wl, obs) as ctx:
        ctx.run(2)
        snap = ctx.snapshot()
    with pytest.raises(A.AbcsmcError) as e:
        A.Context(wl.with_(seed=wl.seed + 1), obs, snapshot=snap)
    assert e.value.code == A.EINVAL
    obs2 = obs.copy()
    obs2[-1, 0] += 1
    with pytest.raises(A.AbcsmcError) as e:
        A.Context(wl, obs2, snapshot=snap)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AbcsmcError) as e:
        A.Context(wl, obs, snapshot=snap[:-8])
    assert e.value.code == A.EINVAL


def test_snapshot_needs_a_completed_stage(oracle):
    wl = W.tiny(n_rounds=2)
    with A.Context(wl, oracle.observations(wl)) as ctx:
        with pytest.raises(A.AbcsmcError) as e:
            ctx.snapshot()
        assert e.value.code == A.ESTATE


def test_snapshot_refused_with_the_learned_screen(oracle):
    wl = W.tiny(n_rounds=2)
    with A.Context(wl, oracle.observations(wl)) as ctx:
        ctx.round()
        ctx.surrogate_enable(n_train=4096, epochs=1, batch=256, seed=1)
        with pytest.raises(A.AbcsmcError) as e:
            ctx.snapshot()
        assert e.value.code == A.ESTATE
        ctx.surrogate_disable()
        assert len(ctx.snapshot()) > 0


def test_replayed_schedule_matches_oracle(oracle):
    wl = W.tiny(n_rounds=4)
    obs = oracle.observations(wl)
    plain = oracle.run(wl, obs)
    sched = (0.9 * plain.eps_next[0], 1.1 * plain.eps_next[1])
    ws = wl.with_(eps_schedule=sched)
    ref = oracle.run(ws, obs)
    assert ref.rc == 0
    assert ref.eps[1] == sched[0] and ref.eps[2] == sched[1] and ref.eps[3] == ref.eps_next[2]
    infos, pops = _gpu_run(ws, obs, 4)
    _compare_run(oracle, ws, ref, infos, pops, 4)


def test_skip_weights_changes_nothing_else(oracle):
    wl = W.tiny(n_rounds=3)
    obs = oracle.observations(wl)
    a_infos, a = _gpu_run(wl, obs, 3)
    b_infos, b = _gpu_run(wl, obs, 3, flags=A.F_SKIP_WEIGHTS)
    N = wl.n_particles
    for i in range(3):
        assert a_infos[i]["eps_next"] == b_infos[i]["eps_next"]
        assert np.array_equal(_bits(a[i]["u"]), _bits(b[i]["u"]))
        assert np.array_equal(_bits(a[i]["d"]), _bits(b[i]["d"]))
        assert np.all(b[i]["W"] == 1.0 / N) and np.all(b[i]["logw"] == 0.0)
        assert b_infos[i]["ess"] == N and b_infos[i]["weight_terms"] == 0
