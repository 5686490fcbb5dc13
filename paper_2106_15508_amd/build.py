"""Build the HIP library ``libabcsmc_hip.so`` for gfx950 with hipcc.

    python -m paper_2106_15508_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libabcsmc_hip.so")
SOURCES = ["sim.hip", "smc.hip", "sort.hip", "runtime.hip", "batch.hip", "batch_rt.hip", "mlp.hip", "train.hip", "screen.hip",
           "surrogate_rt.hip", "predict.hip", "checkpoint.hip", "peak.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # every rounding is the one written: no contraction, no fast-math
    "-ffp-contract=off",
    "-fno-fast-math",
    # packed FP32 instructions are not emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP64 fma as the three-operand v_fma_f64 only: with the two-operand
    # v_fmac_f64 every Horner step whose addend is a loop-invariant
    # coefficient held in a VGPR costs an extra v_mov_b64 (same results)
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_demo(verbose)
    return LIB


DEMO_SRC = os.path.join(HERE, "examples", "abcsmc_demo.c")
DEMO = os.path.join(HERE, "examples", "abcsmc_demo")


def build_demo(verbose: bool = False) -> str:
    """The plain-C example program, linked against the library built above
    (found next to it at run time)."""
    cc = shutil.which("cc") or shutil.which("gcc")
    if cc is None:
        raise RuntimeError("no C compiler for the example program")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), DEMO_SRC,
           "-L", HERE, "-labcsmc_hip", "-Wl,-rpath,$ORIGIN/..", "-lm", "-o", DEMO]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return DEMO


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
