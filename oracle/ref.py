"""ctypes binding of the CPU oracle ``libabcsmc_ref.so`` (built from
``abcsmc_ref.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  It never touches the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "abcsmc_ref.c")
LIB = os.path.join(HERE, "libabcsmc_ref.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]

PRIOR, PERTURB, SIM = 1, 2, 3
FN = {"exp": 0, "expm1": 1, "log": 2, "log1p": 3, "cos2pi": 4, "sin2pi": 5}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Config(C.Structure):
    _fields_ = [
        ("lo", C.c_double * 8), ("hi", C.c_double * 8),
        ("population", C.c_int64), ("n_days", C.c_int32), ("n_particles", C.c_int64),
        ("surv_ratio", C.c_double), ("step_schedule", C.c_int32), ("beta_a", C.c_double),
        ("beta_b", C.c_int32), ("step_is_variance", C.c_int32), ("sampler", C.c_int32),
        ("max_attempts", C.c_int32), ("seed", C.c_uint64), ("max_proposals", C.c_int64),
        ("batch", C.c_int64), ("mcmc_s0", C.c_double), ("mcmc_tune", C.c_int32),
        ("beta_b_real", C.c_double), ("n_eps_schedule", C.c_int32), ("eps_schedule", C.c_void_p),
    ]


class Result(C.Structure):
    _fields_ = [
        ("u", C.c_void_p), ("dist", C.c_void_p), ("sigma", C.c_void_p), ("parent", C.c_void_p),
        ("index", C.c_void_p), ("attempts", C.c_void_p), ("logw", C.c_void_p), ("W", C.c_void_p),
        ("eps", C.c_void_p), ("eps_next", C.c_void_p), ("beta_a", C.c_void_p), ("beta_b", C.c_void_p),
        ("proposals", C.c_void_p), ("invalid", C.c_void_p), ("attempts_total", C.c_void_p),
        ("ess", C.c_void_p), ("mcmc_s", C.c_void_p), ("beta_b_real", C.c_void_p), ("simulated", C.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = bind(C.CDLL(LIB, mode=os.RTLD_LOCAL))
    return _lib


def bind(L):
    """Set the argument and result types of the oracle's exported functions
    on a loaded library (this one, or the op-counting build of the same
    source)."""
    d, i64, u64, i32, u32, vp = C.c_double, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32, C.c_void_p
    sig = {
        "ref_philox4x32_10": (None, [vp, vp, vp]),
        "ref_word": (u64, [u64, u32, u32, u32, u32, u32]),
        "ref_words": (None, [u64, u32, u32, u32, u32, u32, vp]),
        "ref_u01": (d, [u64]),
        "ref_exp": (d, [d]), "ref_expm1": (d, [d]), "ref_log": (d, [d]), "ref_log1p": (d, [d]),
        "ref_map": (None, [i32, vp, vp, i64]),
        "ref_box_muller_many": (None, [vp, vp, i64]),
        "ref_binomial": (i64, [i64, d, u64]),
        "ref_binomial_many": (None, [vp, vp, vp, vp, i64]),
        "ref_normal_floor": (i64, [i64, d, u64]),
        "ref_beta_int": (d, [d, i32, vp]),
        "ref_beta_many": (None, [d, i32, vp, vp, i64]),
        "ref_simulate": (None, [vp, vp, vp, u64, u32, u32, vp]),
        "ref_distance": (d, [i32, vp, vp]),
        "ref_quantile": (d, [vp, i64, d]),
        "ref_resample_weights": (i64, [vp, i64, d, vp, vp]),
        "ref_parent": (i64, [vp, i64, u64]),
        "ref_perturb": (i32, [vp, u32, u32, vp, vp, i64, d, i32, vp, vp, vp]),
        "ref_prior_draw": (None, [vp, u32, vp]),
        "ref_sim_distance": (d, [vp, vp, vp, u32, u32, vp]),
        "ref_log_weight": (d, [vp, d, vp, vp, i64]),
        "ref_normalise": (d, [vp, i64, vp]),
        "ref_run": (i32, [vp, vp, i32, vp]),
        "ref_mcmc_update": (d, [d, i64, i64, i64]),
        "ref_beta_general_many": (None, [d, d, u64, u32, u32, u32, vp, i64]),
        "ref_gamma_many": (None, [d, u64, u32, u32, u32, vp, i64]),
        "ref_beta_shape_real": (None, [vp, i32, d, d, vp, vp]),
        "ref_accept_count": (i64, [vp, vp, vp, d, u32, u32, i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def make_config(w, **over) -> Config:
    """ref_config from a workloads.Workload (plus field overrides)."""
    w = w.with_(**over) if over else w
    c = Config()
    c.lo[:] = list(w.lo)
    c.hi[:] = list(w.hi)
    c.population = w.population
    c.n_days = w.n_days
    c.n_particles = w.n_particles
    c.surv_ratio = w.surv_ratio
    c.step_schedule = w.step_schedule
    c.beta_a = w.beta_a
    c.beta_b = w.beta_b
    c.step_is_variance = int(w.step_is_variance)
    c.sampler = w.sampler
    c.max_attempts = w.max_attempts
    c.seed = w.seed
    c.max_proposals = w.max_proposals or 4096 * w.n_particles
    c.batch = w.batch
    c.mcmc_s0 = w.mcmc_s0
    c.mcmc_tune = w.mcmc_tune
    sched = np.ascontiguousarray(getattr(w, "eps_schedule", ()), dtype=np.float64)
    c._eps_keep = sched                     # alive as long as the config
    c.n_eps_schedule = len(sched)
    c.eps_schedule = sched.ctypes.data if len(sched) else None
    return c


# ---------------------------------------------------------------- primitives

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def words(seed, index, rnd, purpose, sub, n) -> np.ndarray:
    o = np.zeros(n, dtype=np.uint64)
    lib().ref_words(seed, index, rnd, purpose, sub, n, _p(o))
    return o


def fmap(name: str, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().ref_map(FN[name], _p(x), _p(y), x.size)
    return y


def box_muller(w) -> np.ndarray:
    w = np.ascontiguousarray(w, dtype=np.uint64)
    z = np.empty(2 * w.size, dtype=np.float64)
    lib().ref_box_muller_many(_p(w), _p(z), w.size)
    return z.reshape(-1, 2)


def binomial(n, p, w) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.int64)
    p = np.ascontiguousarray(np.broadcast_to(p, n.shape), dtype=np.float64)
    w = np.ascontiguousarray(np.broadcast_to(w, n.shape), dtype=np.uint64)
    o = np.empty_like(n)
    lib().ref_binomial_many(_p(n), _p(p), _p(w), _p(o), n.size)
    return o


def beta_int(a: float, b: int, w) -> np.ndarray:
    """One Beta(a, b) draw per row of w (shape (cnt, b))."""
    w = np.ascontiguousarray(w, dtype=np.uint64).reshape(-1, b)
    o = np.empty(w.shape[0], dtype=np.float64)
    lib().ref_beta_many(a, b, _p(w), _p(o), w.shape[0])
    return o


def simulate(w, theta, seed: int, rnd: int, index: int, obs0=None, **over) -> np.ndarray:
    """(T+1) x 6 trajectory [S, I, A, R, D, Ru]."""
    cfg = make_config(w, **over)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    o0 = np.ascontiguousarray(obs0 if obs0 is not None else w.obs0, dtype=np.int64)
    traj = np.zeros((cfg.n_days + 1, 6), dtype=np.int64)
    lib().ref_simulate(C.byref(cfg), _p(th), _p(o0), seed, rnd, index, _p(traj))
    return traj


def observations(w, **over) -> np.ndarray:
    """Synthetic observed series: (T+1) x 3 (A, R, D) of the trajectory of
    THETA_TRUE under the observation seed."""
    from paper_2106_15508_amd.workloads import OBS_ROUND
    traj = simulate(w, w.theta_true, w.obs_seed, OBS_ROUND, 0, **over)
    return np.ascontiguousarray(traj[:, 2:5])


def distance(traj, obs) -> float:
    traj = np.ascontiguousarray(traj, dtype=np.int64)
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    return lib().ref_distance(traj.shape[0] - 1, _p(traj), _p(obs))


def quantile(x, alpha: float) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().ref_quantile(_p(x), x.size, alpha)


def resample_weights(d, eps: float):
    d = np.ascontiguousarray(d, dtype=np.float64)
    q = np.zeros(d.size, dtype=np.uint64)
    Cc = np.zeros(d.size, dtype=np.uint64)
    ns = lib().ref_resample_weights(_p(d), d.size, eps, _p(q), _p(Cc))
    return q, Cc, ns


def parent(Cc, R: int) -> int:
    Cc = np.ascontiguousarray(Cc, dtype=np.uint64)
    return lib().ref_parent(_p(Cc), Cc.size, R)


def log_weight(u_j, sigma_j, u_prev, q) -> float:
    u_j = np.ascontiguousarray(u_j, dtype=np.float64)
    u_prev = np.ascontiguousarray(u_prev, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.uint64)
    return lib().ref_log_weight(_p(u_j), sigma_j, _p(u_prev), _p(q), q.size)


def normalise(l):
    l = np.ascontiguousarray(l, dtype=np.float64)
    W = np.empty_like(l)
    ess = lib().ref_normalise(_p(l), l.size, _p(W))
    return W, ess


def prior_draw(w, index: int, **over) -> np.ndarray:
    cfg = make_config(w, **over)
    u = np.zeros(8)
    lib().ref_prior_draw(C.byref(cfg), index, _p(u))
    return u


def sim_distance(w, obs, u, rnd: int, index: int, **over) -> float:
    cfg = make_config(w, **over)
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    traj = np.zeros((cfg.n_days + 1, 6), dtype=np.int64)
    return lib().ref_sim_distance(C.byref(cfg), _p(obs), _p(u), rnd, index, _p(traj))


def accept_count(w, obs, u, eps: float, rnd: int, index0: int, n: int, **over) -> int:
    """How many of n simulations of u (streams index0.. of stage rnd) have
    distance <= eps."""
    cfg = make_config(w, **over)
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    return lib().ref_accept_count(C.byref(cfg), _p(obs), _p(u), eps, rnd, index0, n)


def beta_general(a: float, b: float, seed: int, index0: int, rnd: int, sub: int, n: int) -> np.ndarray:
    """n real-shape Beta(a, b) draws (gamma ratio, Marsaglia-Tsang), draw i on
    stream (seed, index0 + i, rnd, PERTURB, sub)."""
    out = np.zeros(n)
    lib().ref_beta_general_many(a, b, seed, index0, rnd, sub, _p(out), n)
    return out


def gamma_mt(k: float, seed: int, index0: int, rnd: int, sub: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    lib().ref_gamma_many(k, seed, index0, rnd, sub, _p(out), n)
    return out


def beta_shape_real(w, rnd: int, eps_i: float, eps_1: float):
    """(a, b) of the alternative parameterisations (schedules 3, 4)."""
    cfg = make_config(w)
    a, b = C.c_double(), C.c_double()
    lib().ref_beta_shape_real(C.byref(cfg), rnd, eps_i, eps_1, C.byref(a), C.byref(b))
    return a.value, b.value


PREDICT_ROUND = 0xFFFE


def predict(w, obs, u_pop, n_days: int, seed: int, quantiles) -> np.ndarray:
    """Posterior predictive bands (§IV-B): each particle simulated for n_days
    from the observed day-0 state with stream (seed, j, PREDICT_ROUND); per
    day and series (A, R, D) the type-7 quantiles over the particles."""
    wp = w.with_(n_days=n_days)
    lo, hi = np.asarray(w.lo), np.asarray(w.hi)
    series = np.zeros((n_days + 1, 3, len(u_pop)))
    for j, u in enumerate(u_pop):
        theta = lo + u * (hi - lo)
        traj = simulate(wp, theta, seed, PREDICT_ROUND, j, obs0=obs[0])
        series[:, :, j] = traj[:, 2:5]
    out = np.zeros((n_days + 1, 3, len(quantiles)))
    for t in range(n_days + 1):
        for c in range(3):
            for k, a in enumerate(quantiles):
                out[t, c, k] = quantile(series[t, c], a)
    return out


def mcmc_update(s: float, acc: int, valid: int, n_acc: int) -> float:
    """Step size after a tuned batch of the MCMC variant (eqs. 14-15 reading)."""
    return lib().ref_mcmc_update(s, acc, valid, n_acc)


def perturb(w, rnd: int, index: int, u_prev, Cc, beta_a: float, beta_b: int, **over):
    """Returns (attempts, u, sigma, parent); attempts < 0 marks a void proposal."""
    cfg = make_config(w, **over)
    u_prev = np.ascontiguousarray(u_prev, dtype=np.float64)
    Cc = np.ascontiguousarray(Cc, dtype=np.uint64)
    u = np.zeros(8)
    s = C.c_double()
    par = C.c_int64()
    a = lib().ref_perturb(C.byref(cfg), rnd, index, _p(u_prev), _p(Cc), Cc.size, beta_a, beta_b,
                          _p(u), C.byref(s), C.byref(par))
    return a, u, s.value, par.value


@dataclass
class RunResult:
    rc: int
    u: np.ndarray
    dist: np.ndarray
    sigma: np.ndarray
    parent: np.ndarray
    index: np.ndarray
    attempts: np.ndarray
    logw: np.ndarray
    W: np.ndarray
    eps: np.ndarray
    eps_next: np.ndarray
    beta_a: np.ndarray
    beta_b: np.ndarray
    proposals: np.ndarray
    invalid: np.ndarray
    attempts_total: np.ndarray
    ess: np.ndarray
    mcmc_s: np.ndarray
    beta_b_real: np.ndarray
    simulated: np.ndarray

    def theta(self, w) -> np.ndarray:
        lo = np.asarray(w.lo)
        hi = np.asarray(w.hi)
        return lo + self.u * (hi - lo)


def run(w, obs, n_rounds: Optional[int] = None, **over) -> RunResult:
    """Whole ABC-SMC run (stage 0 plus n_rounds-1 BDSS stages)."""
    cfg = make_config(w, **over)
    R = n_rounds or w.n_rounds
    N = cfg.n_particles
    arrs = dict(
        u=np.zeros((R, N, 8)), dist=np.zeros((R, N)), sigma=np.zeros((R, N)),
        parent=np.zeros((R, N), np.int64), index=np.zeros((R, N), np.int64),
        attempts=np.zeros((R, N), np.int32), logw=np.zeros((R, N)), W=np.zeros((R, N)),
        eps=np.zeros(R), eps_next=np.zeros(R), beta_a=np.zeros(R), beta_b=np.zeros(R, np.int32),
        proposals=np.zeros(R, np.int64), invalid=np.zeros(R, np.int64),
        attempts_total=np.zeros(R, np.int64), ess=np.zeros(R), mcmc_s=np.zeros(R),
        beta_b_real=np.zeros(R), simulated=np.zeros(R, np.int64),
    )
    res = Result(**{k: v.ctypes.data for k, v in arrs.items()})
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    rc = lib().ref_run(C.byref(cfg), _p(obs), R, C.byref(res))
    return RunResult(rc=rc, **arrs)
