"""Parity at the benchmark's sizes and launch configuration (torch
workspace and stream, early exit on, library-chosen batches).

C2 (P=1e7, T=120, N=131072): stages 0 and 1 are recomputed completely by the
oracle (process pool) and compared bit for bit, including eps^1 and eps^2;
importance weights on sampled rows of stages 1, 5 and 9 within 1e-12.  C3
(P=3e8, T=180, N=2^20): sampled stage-0 particles bit for bit, invariants of
stage 1, sampled weights of stages 1 and 11.  The largest population the
library accepts (N=2^22): sampled stage-0 particles, invariants of stage 1.  C5
(C2 with the learned screen at the benchmark's settings): sampled
acceptances of the first screened stage against the oracle."""
import numpy as np
import pytest

from paper_2106_15508_amd import abcsmc as A
from paper_2106_15508_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bits(x):
    return np.ascontiguousarray(x, dtype=np.float64).view(np.uint64)


def _gpu_stages(w, obs, stages, keep=None):
    """Run `stages` stages at the benchmark's launch configuration; return
    the populations of the stages in `keep` (all if None), each with its
    distances, weights, round info and (stage >= 1) resampling law."""
    import torch
    ws_tensor, ws = A.torch_workspace(w)
    stream = torch.cuda.current_stream()
    out = {}
    with A.Context(w, obs, stream=stream.cuda_stream, workspace=ws, flags=A.F_EARLY_EXIT) as ctx:
        for i in range(stages):
            info = ctx.round()
            if keep is not None and i not in keep:
                continue
            pop = ctx.population()
            _, d, wt = ctx.weights()
            pop["d"], pop["W"], pop["info"] = d, wt, info
            if i >= 1:
                pop["q"], pop["cdf"] = ctx.resampling()
            out[i] = pop
    torch.cuda.synchronize()
    del ws_tensor
    return out


def _check_weights_sampled(oracle, g, i, n_rows, seed, n_floor=64):
    """Log-weights of stage i on sampled rows -- the first and last particle,
    the largest and smallest step size, up to n_floor rows whose step size
    sits at the 1e-8 floor (the narrowest windows), and n_rows random rows --
    against the oracle's sum over the stage's own previous population and
    quantised weights q, to 1e-12 absolute (so the weights themselves agree
    to 1e-12 relative); the normalised weights are the softmax of the
    log-weights to 1e-12 relative."""
    st, u_prev = g[i], g[i - 1]["u"]
    q, sig = st["q"], st["sigma"]
    N = len(sig)
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(N, n_rows, replace=False).tolist()) | {0, N - 1, int(np.argmax(sig)), int(np.argmin(sig))}
    floor = np.flatnonzero(sig == 1e-8)
    rows |= set(rng.permutation(floor)[:n_floor].tolist())
    rows = np.array(sorted(rows))
    want = np.array([oracle.log_weight(st["u"][k], sig[k], u_prev, q) for k in rows])
    dl = np.abs(st["logw"][rows] - want)
    assert dl.max() <= 1e-12, (i, int(rows[np.argmax(dl)]), float(dl.max()))
    l = st["logw"]
    e = np.exp(l - l.max())
    np.testing.assert_allclose(st["W"], e / e.sum(), rtol=1e-12, atol=1e-300)
    return len(floor)


def test_c2_stages_0_1_bitwise(oracle):
    from oracle import parallel
    w = W.C2
    N = w.n_particles
    obs = oracle.observations(w)
    g = _gpu_stages(w, obs, 2)

    # stage 0: all N particles
    u0, d0 = parallel.stage0(w, obs, N)
    assert np.array_equal(g[0]["index"], np.arange(N))
    assert np.array_equal(_bits(g[0]["u"]), _bits(u0))
    assert np.array_equal(_bits(g[0]["d"]), _bits(d0))
    eps1 = oracle.quantile(d0, w.surv_ratio)
    assert _bits([g[0]["info"]["eps_next"]])[0] == _bits([eps1])[0]

    # stage 1: every proposal up to the N-th acceptance
    q, cdf, _ = oracle.resample_weights(d0, eps1)
    assert np.array_equal(g[1]["q"], q) and np.array_equal(g[1]["cdf"], cdf)
    n_prop = g[1]["info"]["proposals"]
    res = parallel.stage(w, obs, 1, u0, cdf, 1.0, 2, range(n_prop))
    acc = [r for r in res if r[1] > 0 and r[5] <= eps1]
    assert len(acc) == N                      # the N-th acceptance is the last proposal
    assert acc[-1][0] == n_prop - 1
    idx = np.array([r[0] for r in acc])
    assert np.array_equal(g[1]["index"], idx)
    assert np.array_equal(_bits(g[1]["u"]), _bits(np.stack([r[2] for r in acc])))
    assert np.array_equal(_bits(g[1]["sigma"]), _bits(np.array([r[3] for r in acc])))
    assert np.array_equal(g[1]["parent"], np.array([r[4] for r in acc]))
    assert np.array_equal(g[1]["attempts"], np.array([r[1] for r in acc]))
    d1 = np.array([r[5] for r in acc])
    assert np.array_equal(_bits(g[1]["d"]), _bits(d1))
    eps2 = oracle.quantile(d1, w.surv_ratio)
    assert _bits([g[1]["info"]["eps_next"]])[0] == _bits([eps2])[0]

    # importance weights on sampled rows: the oracle's own particles k (bit-equal
    # to the GPU's, as checked above) summed against the oracle's stage 0
    rows = np.unique(np.concatenate([[0, N - 1], np.random.default_rng(1).integers(0, N, 254)]))
    for k in rows:
        want = oracle.log_weight(acc[k][2], acc[k][3], u0, q)
        assert abs(g[1]["logw"][k] - want) <= 1e-12, k
    assert abs(g[1]["W"].sum() - 1.0) < 1e-12
    assert np.all(g[1]["W"] >= 0)


def test_c2_weights_late_stages(oracle):
    """Importance weights of the benchmark run (C2, ten stages) at stages 1,
    5 and 9, where eq. 16 has pushed many step sizes to the 1e-8 floor and the
    per-row windows are narrowest."""
    w = W.C2
    obs = oracle.observations(w)
    g = _gpu_stages(w, obs, 10, keep={0, 1, 4, 5, 8, 9})
    n_floor = {i: _check_weights_sampled(oracle, g, i, 256, 20 + i) for i in (1, 5, 9)}
    assert n_floor[9] > 0


def _check_stage0_sampled(oracle, w, obs, g, seed, n_sample):
    N = w.n_particles
    rng = np.random.default_rng(seed)
    for j in np.unique(np.concatenate([[0, 1, N - 1], rng.integers(0, N, n_sample)])):
        u = oracle.prior_draw(w, int(j))
        assert np.array_equal(_bits(g[0]["u"][j]), _bits(u)), j
        assert _bits([g[0]["d"][j]])[0] == _bits([oracle.sim_distance(w, obs, u, 0, int(j))])[0], j
    # eps^1 is the linear-interpolation median of the stage-0 distances (numpy)
    assert g[0]["info"]["eps_next"] == np.quantile(g[0]["d"], w.surv_ratio, method="linear")


def _check_stage1_invariants(w, g):
    st = g[1]
    eps1 = st["info"]["eps"]
    assert np.all(st["d"] <= eps1)
    assert np.all(np.diff(st["index"]) > 0)
    assert st["index"][-1] == st["info"]["proposals"] - 1
    assert np.all((st["u"] >= 0) & (st["u"] <= 1))
    assert np.all(st["W"] >= 0) and np.all(np.isfinite(st["logw"]))
    assert abs(st["W"].sum() - 1.0) < 1e-12
    assert st["info"]["eps_next"] == np.quantile(st["d"], w.surv_ratio, method="linear")
    # the integer CDF is the running sum of the quantised eq. 10 weights: zero
    # outside the prior set d < eps^1, largest weight exactly 2^40
    q, cdf = st["q"], st["cdf"]
    d0 = g[0]["d"]
    assert np.all(q[d0 >= eps1] == 0) and np.all(q[d0 < eps1] <= 2**40)
    assert q.max() == 2**40 and q[np.argmin(d0)] == 2**40
    assert np.array_equal(cdf, np.cumsum(q.astype(object)).astype(np.uint64))
    assert st["info"]["survivors"] == int(np.count_nonzero(q))
    # every parent drawn is a survivor of stage 0 (eq. 11 has no mass elsewhere)
    assert np.all(q[st["parent"]] > 0)


def test_c3_sampled_and_invariants(oracle):
    """C3 (P = 3e8, 180 days, N = 2^20, twelve stages): sampled stage-0
    particles bit for bit, stage-1 invariants, and sampled log-weights of
    stages 1 and 11 against the oracle."""
    w = W.C3
    obs = oracle.observations(w)
    g = _gpu_stages(w, obs, 12, keep={0, 1, 10, 11})
    _check_stage0_sampled(oracle, w, obs, g, 3, 200)
    _check_stage1_invariants(w, g)
    for i in (1, 11):
        _check_weights_sampled(oracle, g, i, 96, 30 + i, n_floor=32)


def test_largest_population_sampled_and_invariants(oracle):
    """N = 2^22, the largest population the library accepts (the integer CDF
    of eq. 10 weights, at most 2^40 each, then still fits 64 bits): sampled
    stage-0 particles bit for bit against the oracle, invariants of stage 1
    (its importance weights over 2^22 x survivors terms included)."""
    w = W.C2.with_(n_particles=1 << 22, population=1_000_000, n_days=40, n_rounds=2)
    obs = oracle.observations(w)
    g = _gpu_stages(w, obs, 2)
    assert len(g[0]["d"]) == len(g[1]["d"]) == 1 << 22
    _check_stage0_sampled(oracle, w, obs, g, 4, 100)
    _check_stage1_invariants(w, g)


def test_c5_screened_stage_sampled(oracle):
    """The learned screen at the benchmark's configuration (fit on 2^22
    prior simulations, keep 10%, audit 1%): sampled acceptances of the first
    screened stage are the oracle's own perturbations and simulations, within
    eps, with the oracle's log-weight (minus log rho when kept by the audit);
    no acceptable proposal that the audit kept is missing."""
    import math

    from oracle import mlp_ref as M
    w = W.C2
    obs = A.observations(w)
    sur = dict(n_train=1 << 22, epochs=2, batch=32768, lr=5e-3, keep_frac=0.1, audit_rho=0.01, fn_max=1.0, seed=11)
    with A.Context(w, obs, flags=A.F_EARLY_EXIT) as ctx:
        ctx.round()
        p0 = ctx.population()
        _, d0, _ = ctx.weights()
        ctx.surrogate_enable(**sur)
        info = ctx.round()
        pop = ctx.population()
        _, d1, _ = ctx.weights()
        audit = ctx.surrogate_audit()
    eps = info["eps"]
    q, Cc, _ = oracle.resample_weights(d0, eps)
    idx = pop["index"]
    rng = np.random.default_rng(5)
    for k in rng.choice(w.n_particles, 24, replace=False):
        j = int(idx[k])
        a, u, s, par = oracle.perturb(w, 1, j, p0["u"], Cc, 1.0, 2)
        assert a > 0 and np.array_equal(pop["u"][k], u) and pop["sigma"][k] == s and pop["parent"][k] == par, j
        dj = oracle.sim_distance(w, obs, u, 1, j)
        assert dj == d1[k] and dj <= eps, j
        if audit[k]:
            assert M.audit_u(w.seed, 1, j) < sur["audit_rho"], j
        lo = oracle.log_weight(u, s, p0["u"], q) - (math.log(sur["audit_rho"]) if audit[k] else 0.0)
        assert abs(pop["logw"][k] - lo) <= 1e-12 * max(1.0, abs(lo)), j
    accepted = set(idx.tolist())
    for j in rng.choice(int(idx[-1]) + 1, 300, replace=False):
        j = int(j)
        if j in accepted or M.audit_u(w.seed, 1, j) >= sur["audit_rho"]:
            continue
        a, u, _, _ = oracle.perturb(w, 1, j, p0["u"], Cc, 1.0, 2)
        assert a < 0 or oracle.sim_distance(w, obs, u, 1, j) > eps, j
