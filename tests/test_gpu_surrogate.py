"""GPU tests of the learned surrogate screen: the network kernels against the
BF16-emulating oracle, its training, the training data against the oracle's
simulations, and the screened stage's output checked index by index against
the oracle's own perturbations, simulations and audit draws."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2106_15508_amd import abcsmc as A
from paper_2106_15508_amd import workloads as W

pytestmark = pytest.mark.gpu


def _params(seed):
    """Oracle initialisation plus non-zero biases (so the bias path is exercised)."""
    p = M.init(seed).copy()
    rng = np.random.default_rng(seed)
    for b in ("b1", "b2", "b3", "b4"):
        a0, a1 = M.offsets()[b]
        p[a0:a1] = rng.normal(0, 0.1, a1 - a0).astype(np.float32)
    return p


def _smooth_targets(x):
    return np.stack([np.sin(2 * x[:, 0]) + x[:, 1] ** 2, x[:, 2] * x[:, 3] - x[:, 7],
                     np.abs(x[:, 4]) + 0.5 * x[:, 5]], axis=1).astype(np.float32)


def test_param_count():
    assert A.mlp_param_count() == M.N_PARAMS


def test_init_matches_oracle():
    assert np.array_equal(A.mlp_init(3), M.init(3))


@pytest.mark.parametrize("n", [1, 63, 300])
def test_forward_matches_bf16_oracle(n):
    p = _params(5)
    x = np.random.default_rng(n).uniform(-1, 1, (n, 8)).astype(np.float32)
    got = A.mlp_forward(p, x)
    emu, _ = M.forward_bf16(p, x)
    scale = max(1.0, float(np.max(np.abs(emu))))
    assert np.max(np.abs(got - emu)) <= 2e-3 * scale
    o64, _ = M.forward(p.astype(np.float64), x.astype(np.float64))
    assert np.max(np.abs(got - o64)) <= 3e-2 * scale


@pytest.mark.parametrize("n", [7, 200])
def test_gradients_match_bf16_oracle(n):
    p = _params(6)
    rng = np.random.default_rng(100 + n)
    x = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    y = _smooth_targets(x)
    g, loss = A.mlp_gradients(p, x, y)
    lo, go = M.loss_grad_bf16(p, x, y)
    assert abs(loss - lo) <= 1e-4 * lo
    for name, (a, b) in M.offsets().items():
        rel = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        # element-wise: no single entry off by more than 1e-3 of the tensor's scale
        # (measured: at most 1e-4 at n = 200)
        el = np.max(np.abs(g[a:b] - go[a:b])) / np.max(np.abs(go[a:b]))
        print(f"gradient {name}: relative norm error {rel:.2e}, largest element error {el:.2e}", flush=True)
        assert rel <= 1e-3, (name, rel)
        assert el <= 1e-3, (name, el)


def test_gradients_match_bf16_oracle_wide_blocks():
    """A minibatch large enough for the pass kernel's 64-row workgroups
    (16448 rows: 257 of them, the last padded to the 64-row K step), whose
    per-block sums carry the bias, W1 and W4 gradients: element by element
    against the emulating oracle, as at small sizes."""
    n = 16448
    p = _params(9)
    rng = np.random.default_rng(900)
    x = rng.uniform(-1, 1, (n, 8)).astype(np.float32)
    y = _smooth_targets(x)
    g, loss = A.mlp_gradients(p, x, y)
    lo, go = M.loss_grad_bf16(p, x, y)
    assert abs(loss - lo) <= 1e-4 * lo
    for name, (a, b) in M.offsets().items():
        rel = np.linalg.norm(g[a:b] - go[a:b]) / np.linalg.norm(go[a:b])
        el = np.max(np.abs(g[a:b] - go[a:b])) / np.max(np.abs(go[a:b]))
        print(f"gradient {name}: relative norm error {rel:.2e}, largest element error {el:.2e}", flush=True)
        assert rel <= 1e-3, (name, rel)
        assert el <= 1e-3, (name, el)


def test_training_tracks_bf16_oracle():
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (1000, 8)).astype(np.float32)
    y = _smooth_targets(x)
    p0 = _params(8)
    pg, lg = A.mlp_train(p0, x, y, 256, 3, 1e-3)
    po, lo = M.train(p0, x, y, 256, 3, 1e-3, emulate=True)
    assert lg[-1] < lg[0]
    assert np.all(np.abs(lg - lo) <= 2e-2 * lo), (lg, lo)
    dg, do = pg.astype(np.float64) - p0, po - p0
    cos = float(dg @ do / (np.linalg.norm(dg) * np.linalg.norm(do)))
    assert cos >= 0.95, cos


@pytest.fixture(scope="module")
def tiny_obs(oracle):
    return oracle.observations(W.tiny())


def test_training_data_matches_oracle(tiny_obs):
    w = W.tiny()
    with A.Context(w, tiny_obs) as ctx:
        info = ctx.surrogate_enable(n_train=4096, epochs=3, batch=256, seed=1)
        x, y = ctx.surrogate_data(40)
    for j in range(40):
        xo, yo, _ = M.train_row(w, tiny_obs, j)
        assert np.array_equal(x[j], xo), j
        np.testing.assert_array_max_ulp(y[j], yo, maxulp=1)
    assert info["loss_last"] < info["loss_first"]
    assert info["train_steps"] == 3 * 16


def _oracle_stage1(oracle, w, obs):
    """The oracle's stage 0 and the resampling law of stage 1."""
    r = oracle.run(w, obs, n_rounds=1)
    eps = float(r.eps_next[0])
    q, Cc, _ = oracle.resample_weights(r.dist[0], eps)
    return r, eps, q, Cc


@pytest.mark.parametrize("keep_frac,rho", [(0.3, 0.2), (1.0, 0.5)])
def test_screened_stage_against_oracle(oracle, tiny_obs, keep_frac, rho):
    w = W.tiny()
    N = w.n_particles
    with A.Context(w, tiny_obs, batch=1024) as ctx:
        ctx.round()
        ctx.surrogate_enable(n_train=4096, epochs=2, batch=256, keep_frac=keep_frac, audit_rho=rho,
                             pool=1024, tune_rows=256, seed=2)
        info = ctx.round()
        pop = ctx.population()
        _, d, Wt = ctx.weights()
        audit = ctx.surrogate_audit()
        si = ctx.surrogate_info()
    r0, eps, q, Cc = _oracle_stage1(oracle, w, tiny_obs)
    assert info["eps"] == eps
    idx = pop["index"]
    assert np.all(np.diff(idx) > 0) and len(idx) == N
    J = int(idx[-1]) + 1
    assert info["proposals"] == J
    accepted = set(idx.tolist())
    u_prev = r0.u[0]
    lw_gpu = pop["logw"]
    n_audit_acc = 0
    for j in range(J):
        a, u, s, par = oracle.perturb(w, 1, j, u_prev, Cc, 1.0, 2)
        if a < 0:
            assert j not in accepted
            continue
        dj = oracle.sim_distance(w, tiny_obs, u, 1, j)
        au = M.audit_u(w.seed, 1, j)
        if j in accepted:
            k = int(np.searchsorted(idx, j))
            assert dj <= eps, j
            assert np.array_equal(pop["u"][k], u) and pop["sigma"][k] == s and pop["parent"][k] == par, j
            assert pop["attempts"][k] == a and d[k] == dj, j
            if audit[k]:
                assert au < rho, j
                n_audit_acc += 1
            lo = oracle.log_weight(u, s, u_prev, q) - (math.log(rho) if audit[k] else 0.0)
            assert abs(lw_gpu[k] - lo) <= 1e-12 * max(1.0, abs(lo)), j
        else:
            # an acceptable proposal the audit kept is never dropped
            assert not (dj <= eps and au < rho), j
    if keep_frac == 1.0:
        assert n_audit_acc == 0 and si["kept_audit"] == 0
    assert abs(Wt.sum() - 1.0) <= 1e-12
    assert si["round"] == 1 and si["accepted_audit"] >= n_audit_acc


def test_screened_run_reset_repeats(tiny_obs):
    w = W.tiny()
    with A.Context(w, tiny_obs) as ctx:
        ctx.round()
        ctx.surrogate_enable(n_train=8192, epochs=2, keep_frac=0.5, audit_rho=0.1, pool=4096, seed=4)
        first = [ctx.round() for _ in range(3)]
        pop1 = ctx.population()
        ctx.reset()
        ctx.round()
        again = [ctx.round() for _ in range(3)]
        pop2 = ctx.population()
    for a, b in zip(first, again):
        assert a["eps"] == b["eps"] and a["proposals"] == b["proposals"]
    for k in pop1:
        assert np.array_equal(pop1[k], pop2[k]), k


def test_trained_network_enriches_more_than_random():
    """A survival ratio of 0.1 makes stage 1 selective enough for the screen
    to matter: the fitted network keeps proposals whose acceptance rate is
    well above the pool's, an untrained one does not."""
    w = W.tiny(surv_ratio=0.1)
    obs = A.observations(w)
    res = {}
    for name, epochs in (("trained", 6), ("random", -1)):
        with A.Context(w, obs) as ctx:
            ctx.round()
            ctx.surrogate_enable(n_train=32768, epochs=epochs, batch=512, keep_frac=0.2, audit_rho=0.1, pool=8192,
                                 tune_rows=-1, fn_max=1.0, seed=5)
            ctx.round()
            res[name] = ctx.surrogate_info()
    assert res["trained"]["enrichment"] > 1.2, res
    assert res["trained"]["enrichment"] > res["random"]["enrichment"] + 0.3, res
    assert res["trained"]["fn_mass"] < res["random"]["fn_mass"], res
