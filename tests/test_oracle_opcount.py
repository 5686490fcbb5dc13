"""The op-counting build of the oracle (oracle/opcount.cpp: the oracle's
source with a counting double) computes exactly what the oracle computes,
and counts operations as its source performs them."""
import numpy as np
import pytest

from paper_2106_15508_amd import workloads as W


@pytest.fixture(scope="module")
def opc(oracle):
    from oracle import opcount
    opcount.lib()
    return opcount


def test_counting_build_is_bit_identical(oracle, opc):
    w = W.tiny(n_rounds=3)
    obs = oracle.observations(w)
    plain = oracle.run(w, obs)
    with opc.counting():
        counted = oracle.run(w, obs)
    for k in ("u", "dist", "sigma", "W", "logw", "eps_next"):
        a, b = getattr(plain, k), getattr(counted, k)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), k
    assert np.array_equal(plain.index, counted.index)
    assert np.array_equal(plain.parent, counted.parent)


def test_counts_of_the_exponential(oracle, opc):
    """ref_exp as written: three comparisons (NaN, overflow, underflow), then
    k = rint(x log2 e) (1 mul, 1 rounding), t = x - k ln2_hi (1 mul, 1 add),
    r = fma(-k, ln2_lo, t), thirteen Horner fma, the int conversion of k and
    one ldexp: 31 flops.  Below e^-708 only the three comparisons."""
    L = opc.lib()
    opc.reset()
    L.ref_exp(1.0)
    c = opc.read()
    assert c == dict(add=1, mul=2, div=0, sqrt=0, fma=14, cmp=3, cvt=1, rnd=1, scale=1, abs=0)
    assert opc.flops(c) == 31
    opc.reset()
    assert L.ref_exp(-800.0) == 0.0
    assert opc.read() == dict(add=0, mul=0, div=0, sqrt=0, fma=0, cmp=3, cvt=0, rnd=0, scale=0, abs=0)


def test_counts_of_a_weight_term(oracle, opc):
    """One term of the importance-weight row sum whose exponential is
    evaluated: 8 differences, 8 squares, 8 additions into the squared
    distance, its division by 2 sigma^2, the exponential (31), the product
    with q_k and the addition into the sum: 58 flops."""
    rng = np.random.default_rng(1)
    uj = rng.uniform(0.3, 0.7, 8)
    near = np.clip(uj + 0.05 * rng.normal(0, 1, (64, 8)), 0, 1)
    c = opc.pair_counts(uj[None, :], [0.05], near, np.ones(64, dtype=np.uint64))
    assert abs(opc.flops(c) - 58.0) < 0.05
