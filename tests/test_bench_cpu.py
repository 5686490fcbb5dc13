"""Host logic of bench.py (CPU only): the one-GPU refusal, the JSON line's
contract fields, and the roofline arithmetic behind `roofline.frac`."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e, capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_envelope_carries_the_contract_fields():
    args = SimpleNamespace(early_exit=1)
    out = bench.envelope(args, 3, 1, 3.0e7, 43.1, "c2: ...", extra={"roofline": {"frac": 0.6}})
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config"):
        assert k in out, k
    assert out["n_gpus"] == 1 and out["steps"] == 3 and out["warmup"] == 1
    assert out["metric"] == out["unit"] == "accepted particles/s"
    assert out["higher_is_better"] is True and out["vs_baseline"] is None
    assert out["dtype"] == "f64" and out["data"] == "synthetic"
    assert out["config"]["workload"] == "c2: ..." and "model" not in out["config"]
    assert out["roofline"] == {"frac": 0.6}


def test_alu_roofline_arithmetic():
    # 10 launches taking 30 ms in all, 3e12 flops: 3e11 flops per 3 ms launch = 100 TFLOP/s
    r = bench.alu_roofline("k", 3.0e12, 30.0, 10, None, "units")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.PEAK_FP64_TFLOPS == 78.6
    assert r["avg_launch_ms"] == pytest.approx(3.0)
    assert r["flops_per_launch"] == pytest.approx(3.0e11)
    assert r["achieved"] == pytest.approx(100.0, abs=1e-3)
    assert r["frac"] == pytest.approx(100.0 / 78.6, abs=1e-4)
    assert r["traffic"] is None


def test_propose_flops_counts_each_stage_at_its_own_rates():
    table = dict(day=[10.0, 20.0], prop=[100.0, 200.0], att=[1.0, 2.0])
    infos = [dict(sim_days=5, simulated=3, invalid=1, attempts=4),
             dict(sim_days=7, simulated=6, invalid=2, attempts=9),
             dict(sim_days=1, simulated=1, invalid=0, attempts=1)]  # past the table: its last column
    want = (5 * 10 + 2 * 100 + 4 * 1) + (7 * 20 + 4 * 200 + 9 * 2) + (1 * 20 + 1 * 200 + 1 * 2)
    assert bench.propose_flops(infos, table) == want


def test_opcount_tables_cover_their_workloads():
    from paper_2106_15508_amd import workloads as W
    for key in ("c2", "c3"):
        t = bench.OPCOUNT[key]
        n = W.WORKLOADS[key].n_rounds
        assert len(t["day"]) == len(t["prop"]) == len(t["att"]) == n
        assert all(v > 0 for col in t.values() for v in col)


def test_pair_flops_is_the_op_counted_term(oracle):
    """The 58 flops per weight term used for `roofline.achieved` is what the
    op-counting build of the oracle counts for one evaluated term."""
    import numpy as np
    from oracle import opcount
    opcount.lib()
    rng = np.random.default_rng(3)
    uj = rng.uniform(0.3, 0.7, 8)
    cols = np.clip(uj + 0.05 * rng.normal(0, 1, (32, 8)), 0, 1)
    c = opcount.pair_counts(uj[None, :], [0.05], cols, np.ones(32, dtype=np.uint64))
    assert opcount.flops(c) == pytest.approx(bench.PAIR_FLOPS, abs=0.05)


def test_kernel_sources_sha_is_stable():
    a, b = bench.kernel_sources_sha(), bench.kernel_sources_sha()
    assert a == b and len(a) == 16 and int(a, 16) >= 0
