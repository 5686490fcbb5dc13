"""Pins of the surrogate-network oracle against library routines, finite
differences and exact arithmetic (CPU only)."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_ref as M
from oracle import ref
from paper_2106_15508_amd import workloads as W


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(M.N_PARAMS)
    for name, (a, b) in M.offsets().items():
        fan = {"W1": 8, "W2": 256, "W3": 256, "W4": 256}.get(name)
        p[a:b] = rng.normal(0.0, scale / math.sqrt(fan), b - a) if fan else rng.normal(0.0, 0.1, b - a)
    return p


def _torch_net(p):
    P = M.unpack(np.asarray(p, dtype=np.float64))
    layers = []
    for i, (fi, fo) in enumerate([(8, 256), (256, 256), (256, 256), (256, 3)], start=1):
        lin = torch.nn.Linear(fi, fo, dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(P[f"W{i}"].copy()))
            lin.bias.copy_(torch.from_numpy(P[f"b{i}"].copy()))
        layers.append(lin)
        if i < 4:
            layers.append(torch.nn.GELU(approximate="tanh"))
    return torch.nn.Sequential(*layers)


def test_param_count():
    assert M.N_PARAMS == 134659


def test_gelu_matches_torch_tanh_form():
    x = np.linspace(-8, 8, 4001)
    ref_ = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    assert np.max(np.abs(M.gelu(x) - ref_)) <= 1e-15 * 8


def test_gelu_grad_matches_autograd():
    x = torch.linspace(-8, 8, 2001, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(x, approximate="tanh").sum().backward()
    assert np.max(np.abs(M.gelu_grad(x.detach().numpy()) - x.grad.numpy())) <= 1e-14


def test_forward_matches_torch_modules():
    p = _params(1)
    x = np.random.default_rng(2).uniform(-1, 1, (37, 8))
    out, _ = M.forward(p, x)
    ref_ = _torch_net(p)(torch.from_numpy(x)).detach().numpy()
    assert np.max(np.abs(out - ref_)) <= 1e-12


def test_gradient_matches_autograd():
    p = _params(3)
    rng = np.random.default_rng(4)
    x, y = rng.uniform(-1, 1, (29, 8)), rng.normal(0, 1, (29, 3))
    loss, g = M.loss_grad(p, x, y)
    net = _torch_net(p)
    out = net(torch.from_numpy(x))
    L = torch.mean((out - torch.from_numpy(y)) ** 2)
    L.backward()
    tg = np.concatenate([t.grad.numpy().ravel() for t in net.parameters()])
    assert abs(loss - L.item()) <= 1e-14 * max(1.0, abs(loss))
    assert np.max(np.abs(g - tg)) <= 1e-12 * max(1.0, np.max(np.abs(tg)))


def test_gradient_central_finite_differences():
    p = _params(5)
    rng = np.random.default_rng(6)
    x, y = rng.uniform(-1, 1, (6, 8)), rng.normal(0, 1, (6, 3))
    _, g = M.loss_grad(p, x, y)
    h = 1e-6
    for name, (a, b) in M.offsets().items():
        for i in rng.choice(np.arange(a, b), size=min(6, b - a), replace=False):
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (M.loss_grad(pp, x, y)[0] - M.loss_grad(pm, x, y)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (name, i)


def test_adam_matches_torch():
    rng = np.random.default_rng(7)
    w = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(4)]
    t = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for s, g in enumerate(grads, start=1):
        w, m, v = M.adam_step(w, g, m, v, s, 1e-2)
        opt.zero_grad()
        t.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(w - t.detach().numpy())) <= 1e-14


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(8)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.uniform(-1e-30, 1e-30, 100)]).astype(np.float32)
    # exact ties: low 16 bits 0x8000 with even and odd upper halves
    ties = (np.arange(200, dtype=np.uint32) << 16 | 0x8000) + np.uint32(0x3F800000)
    x = np.concatenate([x, ties.view(np.float32)])
    ref_ = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(M.bf16(x), ref_)


def test_matmul_bf16_exact_on_representable_operands():
    rng = np.random.default_rng(9)
    A = (rng.integers(-16, 17, (33, 70)) / 8.0).astype(np.float32)
    B = (rng.integers(-16, 17, (70, 19)) / 4.0).astype(np.float32)
    assert np.array_equal(M.matmul_bf16(A, B).astype(np.float64), A.astype(np.float64) @ B.astype(np.float64))


def test_matmul_bf16_within_float32_bound():
    rng = np.random.default_rng(10)
    A = rng.normal(size=(20, 256)).astype(np.float32)
    B = rng.normal(size=(256, 7)).astype(np.float32)
    a, b = M.bf16(A).astype(np.float64), M.bf16(B).astype(np.float64)
    exact = a @ b
    bound = 256 * 2.0 ** -24 * (np.abs(a) @ np.abs(b))
    assert np.all(np.abs(M.matmul_bf16(A, B) - exact) <= bound)
    # and bf16 operand rounding is relative 2^-9 per operand
    assert np.all(np.abs(exact - A.astype(np.float64) @ B.astype(np.float64))
                  <= 2 * 2.0 ** -8 * (np.abs(A) @ np.abs(B)) + 1e-30)


def test_f16_rounding_bitwise():
    """The float16 rounding point of the emulation against the binary16
    format written out: 11 significant bits, ties to even, subnormals in
    steps of 2^-24, and the range GELU' takes."""
    cases = {
        1.0 + 2.0 ** -11: 1.0,                         # tie -> even (1.0)
        1.0 + 3 * 2.0 ** -11: 1.0 + 2 * 2.0 ** -10,    # tie -> even (the larger)
        1.0 + 2.0 ** -11 + 2.0 ** -20: 1.0 + 2.0 ** -10,  # above the tie
        -1.128: -(1.0 + 131 * 2.0 ** -10),             # nearest of the grid of [1, 2)
        3 * 2.0 ** -25: 2.0 ** -23,                    # subnormal tie (1.5 steps) -> even (2 steps)
        2.0 ** -26: 0.0,                               # below half a subnormal step
    }
    for x, want in cases.items():
        assert M.f16(np.float32(x)) == np.float32(want), x
    # every value of [-0.2, 1.2]: the result lies on the binary16 grid of its
    # binade and is the nearest grid point
    xs = np.linspace(-0.2, 1.2, 20001, dtype=np.float32)
    r = M.f16(xs).astype(np.float64)
    for x, y in zip(xs.astype(np.float64), r):
        if x == 0.0:
            assert y == 0.0
            continue
        e = max(math.floor(math.log2(abs(x))), -14)
        step = 2.0 ** (e - 10)
        assert abs(y / step - round(y / step)) == 0.0
        assert abs(y - x) <= step / 2


def test_bf16_forward_and_gradient_close_to_fp64():
    p = _params(11)
    rng = np.random.default_rng(12)
    x, y = rng.uniform(-1, 1, (40, 8)), rng.normal(0, 1, (40, 3))
    o64, _ = M.forward(p, x)
    o16, _ = M.forward_bf16(p.astype(np.float32), x.astype(np.float32))
    assert np.max(np.abs(o16 - o64)) <= 0.03 * max(1.0, np.max(np.abs(o64)))
    _, g64 = M.loss_grad(p, x, y)
    _, g16 = M.loss_grad_bf16(p.astype(np.float32), x.astype(np.float32), y.astype(np.float32))
    for name, (a, b) in M.offsets().items():
        rel = np.linalg.norm(g16[a:b] - g64[a:b]) / np.linalg.norm(g64[a:b])
        assert rel <= 0.05, (name, rel)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(13)
    x = rng.uniform(-1, 1, (512, 8))
    y = np.stack([np.sin(x[:, 0]) + x[:, 1] ** 2, x[:, 2] * x[:, 3], np.abs(x[:, 4])], axis=1)
    p = M.init(1).astype(np.float64)
    _, losses = M.train(p, x, y, 128, 4, 1e-3, emulate=False)
    assert losses[-1] < 0.5 * losses[0]


def test_init_statistics_and_zero_biases():
    p = M.init(3)
    P = M.unpack(p)
    for b in ("b1", "b2", "b3", "b4"):
        assert not P[b].any()
    for name, fan in (("W1", 8), ("W2", 256), ("W3", 256)):
        w = P[name].astype(np.float64).ravel()
        assert abs(w.mean()) < 4 * (1 / math.sqrt(fan)) / math.sqrt(w.size)
        assert abs(w.std() * math.sqrt(fan) - 1.0) < 0.05 if w.size > 10000 else abs(w.std() * math.sqrt(fan) - 1.0) < 0.15
    # weight 0 is the first Box-Muller normal of word 0 of its stream over sqrt(8)
    z = ref.box_muller(ref.words(3, 0, 0, M.MLP, 0, 1))[0, 0]
    assert P["W1"][0, 0] == np.float32(z / math.sqrt(8))


def test_u01_is_centred_grid():
    w = np.array([0, (1 << 64) - 1, 1 << 12], dtype=np.uint64)
    assert np.array_equal(M.u01(w), np.array([0.5, (2.0 ** 52 - 0.5), 1.5]) * 2.0 ** -52)


def test_train_rows_score_recovers_squared_distance():
    w = W.tiny()
    obs = ref.observations(w)
    for j in (0, 1, 17):
        x, y, S = M.train_row(w, obs, j)
        u = ref.prior_draw(w, j)
        d = ref.sim_distance(w, obs, u, 0, j)
        assert np.array_equal(x, (2.0 * u - 1.0).astype(np.float32))
        # the three per-series sums add up to the distance's sum of squares
        assert abs(S.sum() - d * d) <= 1e-12 * d * d
        assert abs(M.score(y.astype(np.float64)) - d * d) <= 1e-5 * d * d
