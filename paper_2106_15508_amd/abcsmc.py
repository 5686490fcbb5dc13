"""Python binding of the HIP library (``libabcsmc_hip.so``, C ABI in
``include/abcsmc.h``).

Argument marshalling only: every step of the method runs in the library's
kernels.  PyTorch, when used, supplies device memory (a workspace tensor) and
the stream; it is optional.  Loading fails loudly when the library is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabcsmc_hip.so")

ABI_VERSION = 4
OK, EINVAL, ENOMEM, EDEVICE, EBUDGET, ESTATE, EDEGENERATE = 0, -1, -2, -3, -4, -5, -6
F_EARLY_EXIT = 1
F_STEP_IS_VARIANCE = 2
F_SKIP_WEIGHTS = 4

#: every function the header declares
EXPORTS = (
    "abcsmc_workspace_size", "abcsmc_init", "abcsmc_round", "abcsmc_weights", "abcsmc_population",
    "abcsmc_resampling", "abcsmc_reset", "abcsmc_rounds_done", "abcsmc_snapshot", "abcsmc_restore",
    "abcsmc_run", "abcsmc_simulate", "abcsmc_debug_eval", "abcsmc_measure_peaks",
    "abcsmc_free", "abcsmc_strerror", "abcsmc_last_error", "abcsmc_abi_version",
    "abcsmc_batch_workspace_size", "abcsmc_batch_init", "abcsmc_batch_set_schedule",
    "abcsmc_batch_get_schedule", "abcsmc_batch_autotune", "abcsmc_batch_round", "abcsmc_batch_run",
    "abcsmc_batch_reset", "abcsmc_batch_status", "abcsmc_batch_rounds_done", "abcsmc_batch_population",
    "abcsmc_batch_free", "abcsmc_batch_last_error",
    "abcsmc_surrogate_enable", "abcsmc_surrogate_disable", "abcsmc_surrogate_info_get", "abcsmc_surrogate_params",
    "abcsmc_surrogate_data", "abcsmc_surrogate_audit", "abcsmc_mlp_param_count", "abcsmc_mlp_init",
    "abcsmc_mlp_forward", "abcsmc_mlp_forward_noalloc", "abcsmc_mlp_gradients", "abcsmc_mlp_train", "abcsmc_predict",
)


class AbcsmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"abcsmc error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("n_params", C.c_int32),
        ("prior_lo", C.c_double * 8), ("prior_hi", C.c_double * 8),
        ("population", C.c_int64), ("n_days", C.c_int32), ("n_particles", C.c_int64),
        ("batch", C.c_int64), ("surv_ratio", C.c_double), ("step_schedule", C.c_int32),
        ("beta_a", C.c_double), ("beta_b", C.c_int32), ("sampler", C.c_int32),
        ("flags", C.c_int32), ("max_attempts", C.c_int32), ("seed", C.c_uint64),
        ("max_proposals", C.c_int64), ("stream", C.c_void_p), ("workspace", C.c_void_p),
        ("workspace_bytes", C.c_size_t), ("mcmc_s0", C.c_double), ("mcmc_tune", C.c_int32),
        ("n_eps_schedule", C.c_int32), ("eps_schedule", C.c_void_p),
    ]


class Schedule(C.Structure):
    _fields_ = [("propose_blocks", C.c_int32), ("run_order", C.c_int32), ("weight_cols", C.c_int32),
                ("issue_margin", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RoundInfo(C.Structure):
    _fields_ = [
        ("round", C.c_int32), ("beta_b", C.c_int32), ("eps", C.c_double), ("eps_next", C.c_double),
        ("beta_a", C.c_double), ("ess", C.c_double), ("proposals", C.c_int64),
        ("simulated", C.c_int64), ("invalid", C.c_int64), ("attempts", C.c_int64),
        ("survivors", C.c_int64), ("batches", C.c_int64), ("ms_resample", C.c_double),
        ("ms_simulate", C.c_double), ("ms_weights", C.c_double), ("ms_select", C.c_double),
        ("ms_total", C.c_double), ("ms_k_propose", C.c_double), ("ms_k_weights", C.c_double),
        ("n_k_propose", C.c_int64), ("sim_days", C.c_int64), ("weight_pairs", C.c_int64),
        ("weight_terms", C.c_int64), ("mcmc_s", C.c_double), ("beta_b_real", C.c_double),
        ("weight_window_terms", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SurrogateConfig(C.Structure):
    _fields_ = [
        ("n_train", C.c_int64), ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
        ("keep_frac", C.c_double), ("audit_rho", C.c_double), ("pool", C.c_int64), ("tune_rows", C.c_int64),
        ("tune_epochs", C.c_int32), ("fn_max", C.c_double), ("seed", C.c_uint64),
    ]


class SurrogateInfo(C.Structure):
    _fields_ = [
        ("loss_first", C.c_double), ("loss_last", C.c_double), ("train_steps", C.c_int64),
        ("ms_train", C.c_double), ("active", C.c_int32), ("round", C.c_int32), ("tau", C.c_double),
        ("kept_screen", C.c_int64), ("kept_audit", C.c_int64), ("accepted_screen", C.c_int64),
        ("accepted_audit", C.c_int64), ("enrichment", C.c_double), ("fn_mass", C.c_double),
        ("ms_score", C.c_double), ("ms_tune", C.c_double), ("ms_data", C.c_double), ("train_flops", C.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: Optional[str] = None):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run python -m paper_2106_15508_amd.build)")
    # One HIP runtime per process: when PyTorch is installed its bundled
    # runtime must be the one loaded first (same soname), otherwise torch
    # cannot initialise the device later in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path, mode=os.RTLD_LOCAL)
    vp, i32, i64, u32, u64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
    sig = {
        "abcsmc_workspace_size": (C.c_int, [vp, vp]),
        "abcsmc_init": (C.c_int, [vp, vp, vp]),
        "abcsmc_round": (C.c_int, [vp, vp]),
        "abcsmc_weights": (C.c_int, [vp, vp, vp, vp]),
        "abcsmc_population": (C.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "abcsmc_resampling": (C.c_int, [vp, vp, vp]),
        "abcsmc_reset": (C.c_int, [vp]),
        "abcsmc_rounds_done": (C.c_int, [vp]),
        "abcsmc_run": (C.c_int, [vp, vp, i32, vp, vp, vp, vp]),
        "abcsmc_simulate": (C.c_int, [vp, i64, vp, vp, u64, u32, u32, vp]),
        "abcsmc_debug_eval": (C.c_int, [i32, i64, vp, vp, d, i32]),
        "abcsmc_measure_peaks": (C.c_int, [i32, vp, vp, vp]),
        "abcsmc_free": (None, [vp]),
        "abcsmc_strerror": (C.c_char_p, [C.c_int]),
        "abcsmc_last_error": (C.c_char_p, [vp]),
        "abcsmc_abi_version": (C.c_int, []),
        "abcsmc_batch_workspace_size": (C.c_int, [vp, i32, vp]),
        "abcsmc_batch_init": (C.c_int, [vp, i32, vp, vp]),
        "abcsmc_batch_set_schedule": (C.c_int, [vp, vp]),
        "abcsmc_batch_get_schedule": (C.c_int, [vp, vp]),
        "abcsmc_batch_autotune": (C.c_int, [vp, i32, C.c_char_p, vp]),
        "abcsmc_batch_round": (C.c_int, [vp, vp]),
        "abcsmc_batch_run": (C.c_int, [vp, i32, vp]),
        "abcsmc_batch_reset": (C.c_int, [vp]),
        "abcsmc_batch_status": (C.c_int, [vp, i32]),
        "abcsmc_batch_rounds_done": (C.c_int, [vp, i32]),
        "abcsmc_batch_population": (C.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "abcsmc_batch_free": (None, [vp]),
        "abcsmc_batch_last_error": (C.c_char_p, [vp]),
        "abcsmc_surrogate_enable": (C.c_int, [vp, vp]),
        "abcsmc_surrogate_disable": (C.c_int, [vp]),
        "abcsmc_surrogate_info_get": (C.c_int, [vp, vp]),
        "abcsmc_surrogate_params": (C.c_int, [vp, vp]),
        "abcsmc_surrogate_data": (C.c_int, [vp, i64, vp, vp]),
        "abcsmc_surrogate_audit": (C.c_int, [vp, vp]),
        "abcsmc_mlp_param_count": (i64, []),
        "abcsmc_mlp_init": (C.c_int, [u64, vp]),
        "abcsmc_mlp_forward": (C.c_int, [vp, i64, vp, vp]),
        "abcsmc_mlp_forward_noalloc": (C.c_int, [vp, i64, vp, vp, vp]),
        "abcsmc_mlp_gradients": (C.c_int, [vp, i64, vp, vp, vp, vp]),
        "abcsmc_mlp_train": (C.c_int, [vp, i64, vp, vp, i32, i32, d, vp]),
        "abcsmc_predict": (C.c_int, [vp, i32, u64, i32, vp, vp]),
        "abcsmc_snapshot": (C.c_int, [vp, vp, vp]),
        "abcsmc_restore": (C.c_int, [vp, vp, vp, C.c_size_t, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.abcsmc_abi_version() != ABI_VERSION:
        raise RuntimeError("ABI version mismatch")
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc: int, ctx=None):
    if rc != OK:
        L = load()
        msg = L.abcsmc_last_error(ctx).decode()
        raise AbcsmcError(rc, msg or L.abcsmc_strerror(rc).decode())


def make_config(w: W.Workload, *, stream=None, workspace=None, flags: int = 0, **over) -> Config:
    """abcsmc_config of a workload (plus field overrides)."""
    w = w.with_(**over) if over else w
    c = Config()
    c.abi_version = ABI_VERSION
    c.n_params = 8
    c.prior_lo[:] = list(w.lo)
    c.prior_hi[:] = list(w.hi)
    c.population = w.population
    c.n_days = w.n_days
    c.n_particles = w.n_particles
    c.batch = w.batch
    c.surv_ratio = w.surv_ratio
    c.step_schedule = w.step_schedule
    c.beta_a = w.beta_a
    c.beta_b = w.beta_b
    c.sampler = w.sampler
    c.flags = flags | (F_STEP_IS_VARIANCE if w.step_is_variance else 0)
    c.max_attempts = w.max_attempts
    c.seed = w.seed
    c.max_proposals = w.max_proposals
    c.mcmc_s0 = w.mcmc_s0
    c.mcmc_tune = w.mcmc_tune
    sched = np.ascontiguousarray(w.eps_schedule, dtype=np.float64)
    c._eps_keep = sched                     # the library copies it at init
    c.n_eps_schedule = len(sched)
    c.eps_schedule = sched.ctypes.data if len(sched) else None
    c.stream = stream
    if workspace is not None:
        ptr, nbytes = workspace
        c.workspace = ptr
        c.workspace_bytes = nbytes
    return c


def workspace_size(w: W.Workload, **kw) -> int:
    c = make_config(w, **kw)
    n = C.c_size_t()
    _check(load().abcsmc_workspace_size(C.byref(c), C.byref(n)))
    return n.value


def simulate(w: W.Workload, theta, seed: int, rnd: int, index0: int = 0, obs0=None, **over) -> np.ndarray:
    """Trajectories (n, T+1, 6) of parameter vectors theta (n, 8) on the GPU."""
    c = make_config(w, **over)
    th = np.ascontiguousarray(np.atleast_2d(theta), dtype=np.float64)
    n = th.shape[0]
    o0 = np.ascontiguousarray(obs0 if obs0 is not None else w.obs0, dtype=np.int64)
    traj = np.zeros((n, c.n_days + 1, 6), dtype=np.int64)
    _check(load().abcsmc_simulate(C.byref(c), n, _p(th), _p(o0), seed, rnd, index0, _p(traj)))
    return traj


def observations(w: W.Workload, **over) -> np.ndarray:
    """Synthetic observed series (T+1, 3) from the generating vector, on the GPU."""
    traj = simulate(w, np.asarray(w.theta_true)[None], w.obs_seed, W.OBS_ROUND, 0, **over)
    return np.ascontiguousarray(traj[0, :, 2:5])


def debug_eval(fn: int, inp: np.ndarray, n: int, out: np.ndarray, pa: float = 0.0, pb: int = 0) -> np.ndarray:
    inp = np.ascontiguousarray(inp)
    _check(load().abcsmc_debug_eval(fn, n, _p(inp), _p(out), pa, pb))
    return out


def measure_peaks(repeats: int = 3) -> dict:
    """abcsmc_measure_peaks: what the current device sustains (FP64 fma
    TFLOP/s, the shader clock in MHz during that launch, copy GB/s)."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(load().abcsmc_measure_peaks(repeats, C.byref(a), C.byref(b), C.byref(c)))
    return dict(fp64_tflops=a.value, clock_mhz=b.value, copy_gbs=c.value)


class Context:
    """One ABC-SMC run on the GPU (abcsmc_init ... abcsmc_free)."""

    def __init__(self, w: W.Workload, obs, *, stream=None, workspace=None, flags: int = 0,
                 snapshot: Optional[bytes] = None, **over):
        self.w = w.with_(**over) if over else w
        self.cfg = make_config(self.w, stream=stream, workspace=workspace, flags=flags)
        self.obs = np.ascontiguousarray(obs, dtype=np.int64)
        self._h = C.c_void_p()
        self.L = load()
        if snapshot is None:
            _check(self.L.abcsmc_init(C.byref(self.cfg), _p(self.obs), C.byref(self._h)))
        else:
            buf = C.create_string_buffer(bytes(snapshot), len(snapshot))
            _check(self.L.abcsmc_restore(C.byref(self.cfg), _p(self.obs), buf, len(snapshot), C.byref(self._h)))
        self.infos: List[dict] = []

    def snapshot(self) -> bytes:
        """Checkpoint after the last completed stage (abcsmc_snapshot); pass it
        as Context(..., snapshot=...) with the same workload and observations
        to continue the run."""
        n = C.c_size_t(0)
        _check(self.L.abcsmc_snapshot(self._h, None, C.byref(n)), self._h)
        buf = C.create_string_buffer(n.value)
        _check(self.L.abcsmc_snapshot(self._h, buf, C.byref(n)), self._h)
        return buf.raw[: n.value]

    @property
    def N(self) -> int:
        return self.w.n_particles

    def round(self) -> dict:
        info = RoundInfo()
        _check(self.L.abcsmc_round(self._h, C.byref(info)), self._h)
        d = info.as_dict()
        self.infos.append(d)
        return d

    def run(self, n_rounds: int) -> List[dict]:
        return [self.round() for _ in range(n_rounds)]

    def reset(self):
        """Restart at stage 0 (same config and seed; workspace stays resident)."""
        _check(self.L.abcsmc_reset(self._h), self._h)
        self.infos = []

    def rounds_done(self) -> int:
        return self.L.abcsmc_rounds_done(self._h)

    def weights(self):
        N = self.N
        th, d, wt = np.zeros((N, 8)), np.zeros(N), np.zeros(N)
        _check(self.L.abcsmc_weights(self._h, _p(th), _p(d), _p(wt)), self._h)
        return th, d, wt

    def population(self):
        N = self.N
        out = dict(u=np.zeros((N, 8)), sigma=np.zeros(N), parent=np.zeros(N, np.int64),
                   index=np.zeros(N, np.int64), attempts=np.zeros(N, np.int32), logw=np.zeros(N))
        _check(self.L.abcsmc_population(self._h, *(_p(out[k]) for k in
                                                    ("u", "sigma", "parent", "index", "attempts", "logw"))),
               self._h)
        return out

    def resampling(self):
        N = self.N
        q, cdf = np.zeros(N, np.uint64), np.zeros(N, np.uint64)
        _check(self.L.abcsmc_resampling(self._h, _p(q), _p(cdf)), self._h)
        return q, cdf

    def predict(self, n_days: int, seed: int, quantiles=(0.005, 0.5, 0.995)) -> np.ndarray:
        """abcsmc_predict: (n_days+1) x 3 (A, R, D) x len(quantiles) bands."""
        q = np.ascontiguousarray(quantiles, dtype=np.float64)
        out = np.zeros((n_days + 1, 3, q.size))
        _check(self.L.abcsmc_predict(self._h, n_days, seed, q.size, _p(q), _p(out)), self._h)
        return out

    # -- learned surrogate screen
    def surrogate_enable(self, **kw) -> dict:
        """abcsmc_surrogate_enable with SurrogateConfig fields as keywords
        (unset = library default); returns the surrogate info."""
        sc = SurrogateConfig(**kw)
        _check(self.L.abcsmc_surrogate_enable(self._h, C.byref(sc)), self._h)
        return self.surrogate_info()

    def surrogate_disable(self):
        _check(self.L.abcsmc_surrogate_disable(self._h), self._h)

    def surrogate_info(self) -> dict:
        i = SurrogateInfo()
        _check(self.L.abcsmc_surrogate_info_get(self._h, C.byref(i)), self._h)
        return i.as_dict()

    def surrogate_params(self) -> np.ndarray:
        p = np.zeros(mlp_param_count(), np.float32)
        _check(self.L.abcsmc_surrogate_params(self._h, _p(p)), self._h)
        return p

    def surrogate_data(self, n: int):
        x, y = np.zeros((n, 8), np.float32), np.zeros((n, 3), np.float32)
        _check(self.L.abcsmc_surrogate_data(self._h, n, _p(x), _p(y)), self._h)
        return x, y

    def surrogate_audit(self) -> np.ndarray:
        a = np.zeros(self.N, np.uint8)
        _check(self.L.abcsmc_surrogate_audit(self._h, _p(a)), self._h)
        return a

    def close(self):
        if self._h:
            self.L.abcsmc_free(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- network hooks (host arrays in, host arrays out)
def mlp_param_count() -> int:
    return int(load().abcsmc_mlp_param_count())


def mlp_init(seed: int) -> np.ndarray:
    p = np.zeros(mlp_param_count(), np.float32)
    _check(load().abcsmc_mlp_init(seed, _p(p)))
    return p


def _f32(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float32)
    if shape is not None:
        a = a.reshape(shape)
    return a


def mlp_forward(params, x) -> np.ndarray:
    params, x = _f32(params), _f32(x)
    n = x.shape[0]
    out = np.zeros((n, 3), np.float32)
    _check(load().abcsmc_mlp_forward(_p(params), n, _p(x), _p(out)))
    return out


def mlp_forward_noalloc(params_ptr: int, n: int, x_ptr: int, out_ptr: int, stream: int = 0) -> None:
    """abcsmc_mlp_forward_noalloc on caller device memory (raw device
    addresses, e.g. torch tensors' data_ptr()); enqueued on `stream`."""
    _check(load().abcsmc_mlp_forward_noalloc(C.c_void_p(params_ptr), n, C.c_void_p(x_ptr), C.c_void_p(out_ptr),
                                             C.c_void_p(stream or None)))


def mlp_gradients(params, x, y):
    params, x, y = _f32(params), _f32(x), _f32(y)
    g = np.zeros_like(params)
    loss = C.c_double()
    _check(load().abcsmc_mlp_gradients(_p(params), x.shape[0], _p(x), _p(y), _p(g), C.byref(loss)))
    return g, loss.value


def mlp_train(params, x, y, batch: int, epochs: int, lr: float):
    p, x, y = _f32(params).copy(), _f32(x), _f32(y)
    losses = np.zeros(max(epochs, 1))
    _check(load().abcsmc_mlp_train(_p(p), x.shape[0], _p(x), _p(y), batch, epochs, lr, _p(losses)))
    return p, losses[:epochs]


def run(w: W.Workload, obs, n_rounds: Optional[int] = None, **over):
    """abcsmc_run: returns (theta, dist, weight, infos)."""
    c = make_config(w, **over)
    R = n_rounds or w.n_rounds
    N = c.n_particles
    obs = np.ascontiguousarray(obs, dtype=np.int64)
    th, d, wt = np.zeros((N, 8)), np.zeros(N), np.zeros(N)
    infos = (RoundInfo * R)()
    _check(load().abcsmc_run(C.byref(c), _p(obs), R, _p(th), _p(d), _p(wt), infos))
    return th, d, wt, [i.as_dict() for i in infos]


def torch_workspace(w: W.Workload, device: str = "cuda", **kw):
    """A torch uint8 tensor big enough for the context's workspace, plus the
    (pointer, bytes) pair the config takes."""
    import torch
    nbytes = workspace_size(w, **kw)
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    ptr = (t.data_ptr() + 255) // 256 * 256
    return t, (ptr, nbytes)


def _bcheck(rc: int, b=None):
    if rc != OK:
        L = load()
        msg = L.abcsmc_batch_last_error(b).decode()
        raise AbcsmcError(rc, msg or L.abcsmc_strerror(rc).decode())


class Batch:
    """Many independent runs advanced together (abcsmc_batch_*)."""

    def __init__(self, workloads: Sequence[W.Workload], obs_list, *, stream=None, workspace=None,
                 flags: int = 0):
        self.ws = list(workloads)
        self.R = len(self.ws)
        cfgs = (Config * self.R)()
        made = [make_config(w, stream=stream if r == 0 else None, workspace=workspace if r == 0 else None,
                            flags=flags) for r, w in enumerate(self.ws)]
        for r, c in enumerate(made):
            cfgs[r] = c
        self._cfgs, self._made = cfgs, made  # keep any schedule arrays alive
        self._obs = [np.ascontiguousarray(o, dtype=np.int64) for o in obs_list]
        ptrs = (C.c_void_p * self.R)(*[o.ctypes.data for o in self._obs])
        self._h = C.c_void_p()
        self.L = load()
        _bcheck(self.L.abcsmc_batch_init(cfgs, self.R, ptrs, C.byref(self._h)))

    @staticmethod
    def workspace_size(workloads, flags: int = 0) -> int:
        R = len(workloads)
        cfgs = (Config * R)()
        made = [make_config(w, flags=flags) for w in workloads]  # alive for the call
        for r, c in enumerate(made):
            cfgs[r] = c
        n = C.c_size_t()
        _bcheck(load().abcsmc_batch_workspace_size(cfgs, R, C.byref(n)))
        return n.value

    def set_schedule(self, propose_blocks=0, run_order=1, weight_cols=0, issue_margin=0.0):
        s = Schedule(propose_blocks, run_order, weight_cols, issue_margin)
        _bcheck(self.L.abcsmc_batch_set_schedule(self._h, C.byref(s)), self._h)

    def schedule(self) -> dict:
        s = Schedule()
        _bcheck(self.L.abcsmc_batch_get_schedule(self._h, C.byref(s)), self._h)
        return s.as_dict()

    def autotune(self, stages: int = 2, cache_path: Optional[str] = None) -> dict:
        s = Schedule()
        cp = cache_path.encode() if cache_path else None
        _bcheck(self.L.abcsmc_batch_autotune(self._h, stages, cp, C.byref(s)), self._h)
        return s.as_dict()

    def round(self) -> List[dict]:
        infos = (RoundInfo * self.R)()
        _bcheck(self.L.abcsmc_batch_round(self._h, infos), self._h)
        return [i.as_dict() for i in infos]

    def run(self, n_rounds: int) -> List[List[dict]]:
        return [self.round() for _ in range(n_rounds)]

    def reset(self):
        _bcheck(self.L.abcsmc_batch_reset(self._h), self._h)

    def status(self, r: int) -> int:
        return self.L.abcsmc_batch_status(self._h, r)

    def rounds_done(self, r: int) -> int:
        return self.L.abcsmc_batch_rounds_done(self._h, r)

    def population(self, r: int) -> dict:
        N = self.ws[r].n_particles
        out = dict(u=np.zeros((N, 8)), sigma=np.zeros(N), parent=np.zeros(N, np.int64),
                   index=np.zeros(N, np.int64), attempts=np.zeros(N, np.int32), logw=np.zeros(N),
                   d=np.zeros(N), W=np.zeros(N))
        _bcheck(self.L.abcsmc_batch_population(self._h, r, *(_p(out[k]) for k in
                ("u", "sigma", "parent", "index", "attempts", "logw", "d", "W"))), self._h)
        return out

    def close(self):
        if self._h:
            self.L.abcsmc_batch_free(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
