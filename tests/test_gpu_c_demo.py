"""The C ABI from a plain C99 program (paper_2106_15508_amd/examples/
abcsmc_demo.c, built with the library): its stages equal the oracle's run
of the same configuration bit for bit."""
import os
import subprocess

import numpy as np
import pytest

from paper_2106_15508_amd import build as B
from paper_2106_15508_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_c_program_run_equals_oracle(oracle):
    assert os.path.exists(B.DEMO), "build the library first (python -m paper_2106_15508_amd.build)"
    w = W.C1.with_(step_schedule=W.STEP_PAPER, beta_a=0.0, beta_b=0, seed=17)
    args = [str(v) for v in (w.n_particles, w.n_days, w.population, w.n_rounds, w.seed, w.obs_seed)]
    p = subprocess.run([B.DEMO, *args], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, p.stderr
    lines = [l.split() for l in p.stdout.splitlines() if l.startswith("stage ")]
    assert len(lines) == w.n_rounds
    ref = oracle.run(w, oracle.observations(w))
    assert ref.rc == 0
    for i, f in enumerate(lines):
        assert int(f[1]) == i
        eps, eps_next, props = float.fromhex(f[3]), float.fromhex(f[5]), int(f[7])
        assert eps == ref.eps[i] or (np.isinf(eps) and np.isinf(ref.eps[i])), i
        assert eps_next == ref.eps_next[i], i
        assert props == ref.proposals[i], i
    mean = [float(v) for v in p.stdout.splitlines()[-1].split()[2:]]
    want = (np.asarray(ref.W[-1])[:, None] * (np.asarray(w.lo) + ref.u[-1] * (np.asarray(w.hi) - np.asarray(w.lo)))).sum(0)
    np.testing.assert_allclose(mean, want, rtol=1e-5)
