"""Pins of the oracle's random-number and elementary-function layer.

Philox4x32-10 is pinned to the published known-answer vectors and, where a
HIP compiler is present, to rocRAND's independent host implementation.  The
elementary functions are pinned to mpmath at 40 digits.
"""
import os
import shutil
import subprocess
import tempfile
import zlib
from fractions import Fraction

import mpmath

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle):
    for ctr, key, out in _kat():
        assert list(oracle.philox(ctr, key)) == out


def test_philox_matches_rocrand_host_engine(oracle, tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc to build the rocRAND host engine")
    src = tmp_path / "p.cpp"
    src.write_text(
        "#include <cstdio>\n#include <rocrand/rocrand_philox4x32_10.h>\n"
        "int main(){unsigned c0,c1,c2,c3,k0,k1;\n"
        "while(scanf(\"%x %x %x %x %x %x\",&c0,&c1,&c2,&c3,&k0,&k1)==6){\n"
        "unsigned long long s=((unsigned long long)k1<<32)|k0;\n"
        "unsigned long long sub=((unsigned long long)c3<<32)|c2;\n"
        "unsigned long long off=4ull*(((unsigned long long)c1<<32)|c0);\n"
        "rocrand_device::philox4x32_10_engine e(s,sub,off); uint4 r=e.next4();\n"
        "printf(\"%08x %08x %08x %08x\\n\",r.x,r.y,r.z,r.w);}}\n")
    exe = tmp_path / "p"
    r = subprocess.run([hipcc, "-O1", "-o", str(exe), str(src)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("rocRAND host engine did not build: " + r.stderr[-300:])
    rng = np.random.default_rng(11)
    lines, want = [], []
    for _ in range(300):
        c = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)),
             int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        k = [int(rng.integers(0, 2**32)), int(rng.integers(0, 2**32))]
        lines.append(" ".join("%x" % v for v in c + k))
        want.append(" ".join("%08x" % v for v in oracle.philox(c, k)))
    out = subprocess.run([str(exe)], input="\n".join(lines) + "\n", capture_output=True,
                         text=True, timeout=60).stdout.split("\n")
    assert out[:len(want)] == want


def test_word_layout(oracle):
    """Word w of a stream is half w%2 of block w/2 of the counter
    (index, round, purpose<<24|sub, block)."""
    seed = 0x0123456789ABCDEF
    ws = oracle.words(seed, 7, 3, 2, 5, 6)
    for w in range(6):
        o = oracle.philox([7, 3, (2 << 24) | 5, w // 2], [seed & 0xFFFFFFFF, seed >> 32])
        lo, hi = (o[0], o[1]) if w % 2 == 0 else (o[2], o[3])
        assert int(ws[w]) == (int(hi) << 32) | int(lo)


def test_u01_exact_open_interval(oracle):
    L = oracle.lib()
    for w in [0, 1, 4095, 4096, 2**63, 2**64 - 1, 0xDEADBEEFCAFEBABE]:
        u = L.ref_u01(w)
        assert Fraction(u) == (Fraction(w >> 12) + Fraction(1, 2)) / 2**52
        assert 0.0 < u < 1.0
        assert Fraction(1.0 - u) == 1 - Fraction(u)  # 1-u exact


mpmath.mp.dps = 40


def _max_ulp(got, x, f):
    worst = 0.0
    for g, xv in zip(got, x):
        t = f(mpmath.mpf(float(xv)))
        tf = float(t)
        if tf == 0.0:
            assert g == 0.0
            continue
        worst = max(worst, float(abs(mpmath.mpf(float(g)) - t) / np.spacing(abs(tf))))
    return worst


@pytest.mark.parametrize("name,lo,hi,f,bound", [
    ("exp", -708.0, 709.0, mpmath.exp, 1.0),
    ("exp", -1.0, 1.0, mpmath.exp, 1.0),
    # series branch (|x| <= ln2/2): close to correctly rounded
    ("expm1", -0.34657359027997264, 0.34657359027997264, mpmath.expm1, 1.0),
    # exp(x) - 1 beyond it: exp's error is up to 4 ulps of the result just above ln2/2
    ("expm1", 0.34657359027997264, 0.41, mpmath.expm1, 4.0),
    ("expm1", -40.0, 5.0, mpmath.expm1, 4.0),
    ("log1p", -0.999, 4.0, mpmath.log1p, 2.0),
])
def test_elementary_uniform_ranges(oracle, name, lo, hi, f, bound):
    x = np.random.default_rng(zlib.crc32(f"{name} {lo} {hi}".encode())).uniform(lo, hi, 2500)
    assert _max_ulp(oracle.fmap(name, x), x, f) <= bound


def test_log_wide_range(oracle):
    rng = np.random.default_rng(5)
    x = np.concatenate([10 ** rng.uniform(-300, 300, 2500), rng.uniform(0.5, 2.0, 2500),
                        [np.nextafter(1.0, 0), 1.0, np.nextafter(1.0, 2), 2.0 ** -1074]])
    assert _max_ulp(oracle.fmap("log", x), x, mpmath.log) <= 2.0


def test_log1p_tiny_and_edges(oracle):
    rng = np.random.default_rng(6)
    x = np.concatenate([10 ** rng.uniform(-300, -1, 1000), -(10 ** rng.uniform(-300, -1, 1000)),
                        [0.41421356237309515, -0.29289321881345243, 0.5, -0.5]])
    assert _max_ulp(oracle.fmap("log1p", x), x, mpmath.log1p) <= 2.0
    assert oracle.fmap("log1p", [0.0])[0] == 0.0


def test_exp_special_values(oracle):
    y = oracle.fmap("exp", [0.0, 710.0, -708.5, -1e9, np.inf, -np.inf])
    assert y[0] == 1.0 and np.isinf(y[1]) and y[2] == 0.0 and y[3] == 0.0
    assert np.isinf(y[4]) and y[5] == 0.0


def test_sincos2pi_against_mpmath(oracle):
    rng = np.random.default_rng(8)
    t = (rng.integers(0, 2**32, 3000) + 0.5) / 2**32
    err = 0.0
    for name, f in (("cos2pi", mpmath.cos), ("sin2pi", mpmath.sin)):
        got = oracle.fmap(name, t)
        for g, tv in zip(got, t):
            err = max(err, abs(float(mpmath.mpf(float(g)) - f(2 * mpmath.pi * mpmath.mpf(float(tv))))))
    assert err < 4e-16
