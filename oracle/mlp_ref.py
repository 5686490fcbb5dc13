"""CPU oracle of the learned surrogate screen (test infrastructure only: used
by the tests and nothing else; it shares no code with the HIP path).

Network: 8 -> 256 -> 256 -> 256 -> 3 multilayer perceptron, y = W h + b per
layer, tanh-form GELU (Hendrycks & Gimpel) after the three hidden layers,
mean-squared-error loss over the n x 3 outputs, Adam (Kingma & Ba) with
(beta1, beta2, eps) = (0.9, 0.999, 1e-8).  Flat parameter layout:
W1[256][8] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[3][256] b4[3].

Two arithmetic modes:
  * FP64 (``forward``, ``loss_grad``): the definition, in float64.
  * BF16-emulating (``forward_bf16``, ``loss_grad_bf16``): every matrix
    product rounds both operands to bfloat16 (round to nearest even) and
    accumulates in float32 in increasing k order; GELU'(a) is rounded to
    float16 (nearest even) between the forward and the backward pass, where
    the kernels keep it; everything else (bias, activation, loss, bias sums)
    is float32.  This is the arithmetic the matrix-core kernels perform, up
    to the order of the float32 sums.

Inputs of the screen: x = 2u - 1 of a proposal's unit-cube coordinates;
targets y_c = log1p(sqrt(S_c)) for the per-series sums of squares S_A, S_R,
S_D whose total is the squared distance of §II-C; score = sum_c expm1(y_c)^2.
Audit draw: U = u01(word 0 of the proposal's AUDIT stream, purpose 4).
Initialisation: weight i = z / sqrt(fan_in), z the first Box-Muller normal of
word 0 of stream (index i, round 0, purpose 5); biases 0.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

from . import ref

K_IN, K_H, K_OUT = 8, 256, 3
SHAPES = [("W1", (K_H, K_IN)), ("b1", (K_H,)), ("W2", (K_H, K_H)), ("b2", (K_H,)),
          ("W3", (K_H, K_H)), ("b3", (K_H,)), ("W4", (K_OUT, K_H)), ("b4", (K_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 134659
AUDIT, MLP = 4, 5
ADAM = (0.9, 0.999, 1e-8)
C_GELU = math.sqrt(2.0 / math.pi)
A_GELU = 0.044715


def unpack(p: np.ndarray) -> Dict[str, np.ndarray]:
    """Views of the flat parameter vector by tensor name."""
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def offsets() -> Dict[str, Tuple[int, int]]:
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = (o, o + k)
        o += k
    return out


# ------------------------------------------------------------------ FP64

def gelu(x):
    """0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(C_GELU * (x + A_GELU * x ** 3)))


def gelu_grad(x):
    """d/dx of gelu: 0.5 (1 + t) + 0.5 x (1 - t^2) sqrt(2/pi) (1 + 3 * 0.044715 x^2)."""
    t = np.tanh(C_GELU * (x + A_GELU * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * C_GELU * (1.0 + 3.0 * A_GELU * x * x)


def forward(p, x):
    """FP64 forward: returns (out n x 3, cache of pre-activations and activations)."""
    P = unpack(np.asarray(p, dtype=np.float64))
    h0 = np.asarray(x, dtype=np.float64)
    a1 = h0 @ P["W1"].T + P["b1"]
    h1 = gelu(a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(a2)
    a3 = h2 @ P["W3"].T + P["b3"]
    h3 = gelu(a3)
    out = h3 @ P["W4"].T + P["b4"]
    return out, dict(h0=h0, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3)


def loss_grad(p, x, y):
    """FP64 loss = mean over n x 3 of (out - y)^2 and its gradient (flat)."""
    P = unpack(np.asarray(p, dtype=np.float64))
    out, c = forward(p, x)
    n = out.shape[0]
    r = out - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    g4 = 2.0 * r / (3.0 * n)                      # dL/dout
    G = {"W4": g4.T @ c["h3"], "b4": g4.sum(0)}
    g3 = (g4 @ P["W4"]) * gelu_grad(c["a3"])     # dL/da3
    G["W3"], G["b3"] = g3.T @ c["h2"], g3.sum(0)
    g2 = (g3 @ P["W3"]) * gelu_grad(c["a2"])
    G["W2"], G["b2"] = g2.T @ c["h1"], g2.sum(0)
    g1 = (g2 @ P["W2"]) * gelu_grad(c["a1"])
    G["W1"], G["b1"] = g1.T @ c["h0"], g1.sum(0)
    grad = np.concatenate([G[name].ravel() for name, _ in SHAPES])
    return loss, grad


def adam_step(w, g, m, v, step: int, lr: float):
    """One Adam update (FP64): m, v moments, bias corrections 1 - beta^step."""
    b1, b2, eps = ADAM
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ BF16 emulation

def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).reshape(f.shape)


def f16(x) -> np.ndarray:
    """Round float32 values to IEEE binary16 (nearest, ties to even,
    subnormals kept), returned as float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def matmul_bf16(A, B) -> np.ndarray:
    """A (M x K) times B (K x N): bfloat16 operands, float32 sum in k order."""
    a, b = bf16(A), bf16(B)
    acc = np.zeros((a.shape[0], b.shape[1]), dtype=np.float32)
    for k in range(a.shape[1]):
        acc = acc + np.outer(a[:, k], b[k, :]).astype(np.float32)  # bf16 x bf16 is exact in float32
    return acc


def _gelu32(x):
    x = np.asarray(x, dtype=np.float32)
    c, a = np.float32(C_GELU), np.float32(A_GELU)
    t = np.tanh(c * (x + a * x * x * x))
    return np.float32(0.5) * x * (np.float32(1.0) + t)


def _gelu_grad32(x):
    x = np.asarray(x, dtype=np.float32)
    c, a = np.float32(C_GELU), np.float32(A_GELU)
    x2 = x * x
    t = np.tanh(c * (x + a * x2 * x))
    one, half = np.float32(1.0), np.float32(0.5)
    return half * (one + t) + half * x * (one - t * t) * c * (one + np.float32(3.0) * a * x2)


def _colsum32(X):
    acc = np.zeros(X.shape[1], dtype=np.float32)
    for m in range(X.shape[0]):
        acc = acc + X[m]
    return acc


def forward_bf16(p, x):
    P = unpack(np.asarray(p, dtype=np.float32))
    h0 = np.asarray(x, dtype=np.float32)
    a1 = matmul_bf16(h0, P["W1"].T) + P["b1"]
    h1 = _gelu32(a1)
    a2 = matmul_bf16(h1, P["W2"].T) + P["b2"]
    h2 = _gelu32(a2)
    a3 = matmul_bf16(h2, P["W3"].T) + P["b3"]
    h3 = _gelu32(a3)
    out = matmul_bf16(h3, P["W4"].T) + P["b4"]
    return out, dict(h0=h0, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3)


def loss_grad_bf16(p, x, y):
    P = unpack(np.asarray(p, dtype=np.float32))
    out, c = forward_bf16(p, x)
    n = out.shape[0]
    r = out - np.asarray(y, dtype=np.float32)
    loss = float(np.sum(r.astype(np.float64) ** 2) / (3.0 * n))
    g4 = (np.float32(2.0) * r) / np.float32(3.0 * n)
    G = {"W4": matmul_bf16(g4.T, c["h3"]), "b4": _colsum32(g4)}
    g3 = matmul_bf16(g4, P["W4"]) * f16(_gelu_grad32(c["a3"]))
    G["W3"], G["b3"] = matmul_bf16(g3.T, c["h2"]), _colsum32(g3)
    g2 = matmul_bf16(g3, P["W3"]) * f16(_gelu_grad32(c["a2"]))
    G["W2"], G["b2"] = matmul_bf16(g2.T, c["h1"]), _colsum32(g2)
    g1 = matmul_bf16(g2, P["W2"]) * f16(_gelu_grad32(c["a1"]))
    G["W1"], G["b1"] = matmul_bf16(g1.T, c["h0"]), _colsum32(g1)
    grad = np.concatenate([G[name].ravel() for name, _ in SHAPES]).astype(np.float32)
    return loss, grad


def train(p, x, y, batch: int, epochs: int, lr: float, emulate: bool = True):
    """Minibatch Adam in row order (the last minibatch of a pass may be short);
    returns (params, per-pass mean loss before each step)."""
    w = np.asarray(p, dtype=np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    n = x.shape[0]
    step = 0
    losses: List[float] = []
    for _ in range(epochs):
        tot = 0.0
        for o in range(0, n, batch):
            xb, yb = x[o:o + batch], y[o:o + batch]
            if emulate:
                l, g = loss_grad_bf16(w.astype(np.float32), xb, yb)
            else:
                l, g = loss_grad(w, xb, yb)
            tot += l * xb.shape[0]
            step += 1
            w, m, v = adam_step(w, g.astype(np.float64), m, v, step, lr)
            if emulate:
                w = w.astype(np.float32).astype(np.float64)
        losses.append(tot / n)
    return w, np.array(losses)


# ------------------------------------------------------------------ data, screen, init

def u01(w) -> np.ndarray:
    """((w >> 12) + 0.5) 2^-52: a uniform draw in (0, 1) from a 64-bit word."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52


def audit_u(seed: int, rnd: int, index: int) -> float:
    return float(u01(ref.words(seed, index, rnd, AUDIT, 0, 1))[0])


def init(seed: int) -> np.ndarray:
    """Weights N(0, 1/fan_in) from the MLP stream, biases 0 (float32)."""
    p = np.zeros(N_PARAMS, dtype=np.float32)
    fans = {"W1": K_IN, "W2": K_H, "W3": K_H, "W4": K_H}
    for name, (a, b) in offsets().items():
        if name not in fans:
            continue
        idx = np.arange(a, b)
        w0 = np.array([ref.words(seed, int(i), 0, MLP, 0, 1)[0] for i in idx], dtype=np.uint64)
        z = ref.box_muller(w0)[:, 0]
        p[a:b] = (z / math.sqrt(fans[name])).astype(np.float32)
    return p


def split_sums(traj, obs) -> np.ndarray:
    """S_A, S_R, S_D: per-series sums over days 1..T of squared differences,
    each summed in day order."""
    traj = np.asarray(traj, dtype=np.int64)
    obs = np.asarray(obs, dtype=np.int64)
    S = [0.0, 0.0, 0.0]
    for t in range(1, traj.shape[0]):
        for c, col in enumerate((2, 3, 4)):
            d = float(traj[t, col] - obs[t, c])
            S[c] = S[c] + d * d
    return np.array(S)


def train_row(w, obs, j: int):
    """Training row j: the stage-0 proposal of index j, simulated."""
    u = ref.prior_draw(w, j)
    theta = np.asarray(w.lo) + u * (np.asarray(w.hi) - np.asarray(w.lo))
    traj = ref.simulate(w, theta, w.seed, 0, j, obs0=obs[0])
    S = split_sums(traj, obs)
    x = (2.0 * u - 1.0).astype(np.float32)
    y = np.log1p(np.sqrt(S)).astype(np.float32)
    return x, y, S


def score(out) -> np.ndarray:
    """Predicted squared distance sum_c expm1(y_c)^2 (FP64)."""
    e = np.expm1(np.asarray(out, dtype=np.float64))
    return np.sum(e * e, axis=-1)
