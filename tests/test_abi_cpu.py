"""Host-side checks of the C ABI: the library loads, exports every function
include/abcsmc.h declares, and rejects bad configurations before touching a
device (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2106_15508_amd import abcsmc as A
from paper_2106_15508_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "abcsmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(abcsmc_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert sorted(A.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = A.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.abcsmc_abi_version() == A.ABI_VERSION


def test_strerror_codes():
    L = A.load()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.abcsmc_strerror(code).decode()


@pytest.mark.parametrize("field,value", [
    ("n_particles", 1), ("n_particles", (1 << 22) + 1), ("n_days", 0), ("n_days", 5000),
    ("population", 0), ("surv_ratio", 0.0), ("surv_ratio", 1.0), ("step_schedule", 7),
    ("sampler", 3), ("flags", 64), ("max_attempts", -1), ("batch", -5), ("n_params", 7),
    ("abi_version", 99),
])
def test_invalid_config_rejected(field, value):
    c = A.make_config(W.C1)
    setattr(c, field, value)
    n = C.c_size_t()
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL
    assert A.load().abcsmc_last_error(None)


def test_invalid_prior_and_fixed_beta_rejected():
    c = A.make_config(W.C1)
    c.prior_lo[3] = 2.0  # lo > hi
    n = C.c_size_t()
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL
    c = A.make_config(W.C1, step_schedule=W.STEP_FIXED, beta_a=2.0, beta_b=0)
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL


@pytest.mark.parametrize("sched", [(1.0, float("nan")), (-1.0,), (float("inf"),)])
def test_invalid_eps_schedule_rejected(sched):
    c = A.make_config(W.C1, eps_schedule=sched)
    n = C.c_size_t()
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL
    c = A.make_config(W.C1)
    c.n_eps_schedule = 2  # no array
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL
    c.n_eps_schedule = 5000
    assert A.load().abcsmc_workspace_size(C.byref(c), C.byref(n)) == A.EINVAL


@pytest.mark.parametrize("over,flags", [(dict(eps_schedule=(5.0,)), 0), ({}, A.F_SKIP_WEIGHTS),
                                        (dict(step_schedule=W.STEP_MEANVAR), 0)])
def test_batch_rejects_unsupported_options(over, flags):
    runs = [W.tiny(seed=3), W.tiny(seed=4, **over)]
    with pytest.raises(A.AbcsmcError) as e:
        A.Batch.workspace_size(runs, flags=flags)
    assert e.value.code == A.EINVAL


def test_restore_rejects_malformed_snapshots():
    # checked before any device work
    L = A.load()
    c = A.make_config(W.C1)
    obs = np.zeros((W.C1.n_days + 1, 3), np.int64)
    h = C.c_void_p()
    for buf in (b"", b"x" * 16, b"ABCSMCK1" + b"\0" * 200):
        b = C.create_string_buffer(buf, max(len(buf), 1))
        assert L.abcsmc_restore(C.byref(c), obs.ctypes.data_as(C.c_void_p), b, len(buf), C.byref(h)) == A.EINVAL
        assert not h.value


def test_init_rejects_bad_observations():
    L = A.load()
    c = A.make_config(W.C1)
    obs = np.zeros((W.C1.n_days + 1, 3), np.int64)
    obs[3, 1] = -4
    h = C.c_void_p()
    assert L.abcsmc_init(C.byref(c), obs.ctypes.data_as(C.c_void_p), C.byref(h)) == A.EINVAL
    assert not h.value
    obs[3, 1] = W.C1.population + 1
    assert L.abcsmc_init(C.byref(c), obs.ctypes.data_as(C.c_void_p), C.byref(h)) == A.EINVAL


def test_workspace_size_grows_with_n():
    a = A.workspace_size(W.C1)
    b = A.workspace_size(W.C2)
    assert 0 < a < b
    # C2 needs: two populations, staging for 4N proposals, columns; all well under 1 GiB
    assert b < (1 << 30)


def test_null_arguments():
    L = A.load()
    assert L.abcsmc_round(None, None) == A.EINVAL
    assert L.abcsmc_weights(None, None, None, None) == A.EINVAL
    L.abcsmc_free(None)


def test_measure_peaks_rejects_bad_arguments():
    L = A.load()
    x = C.c_double()
    assert L.abcsmc_measure_peaks(0, C.byref(x), C.byref(x), C.byref(x)) == A.EINVAL
    assert L.abcsmc_measure_peaks(101, C.byref(x), C.byref(x), C.byref(x)) == A.EINVAL
    assert L.abcsmc_measure_peaks(3, None, C.byref(x), C.byref(x)) == A.EINVAL
    assert b"measure_peaks" in L.abcsmc_last_error(None)


def test_c_example_compiles_against_the_header(tmp_path):
    """The plain-C example builds with -std=c99 -Wall -Wextra -Werror against
    include/abcsmc.h and links against the library (no GPU needed)."""
    import subprocess
    from paper_2106_15508_amd import build as B
    out = tmp_path / "demo"
    cmd = ["cc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), B.DEMO_SRC,
           "-L", B.HERE, "-labcsmc_hip", "-lm", "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=120)
    assert out.exists()
