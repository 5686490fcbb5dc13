"""Pins of the oracle's samplers: Box-Muller normals, the one-word binomial
draw, and the integer-b Beta step-size law of eq. (16)."""
import math
import os

import mpmath
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


def _words(n, seed=0):
    return np.random.default_rng(seed).integers(0, 2**64, n, dtype=np.uint64)


def test_box_muller_matches_numpy_formula(oracle):
    w = _words(20000, 1)
    z = oracle.box_muller(w)
    u1 = ((w & np.uint64(0xFFFFFFFF)).astype(np.float64) + 0.5) * 2.0**-32
    u2 = ((w >> np.uint64(32)).astype(np.float64) + 0.5) * 2.0**-32
    rho = np.sqrt(-2.0 * np.log(u1))
    np.testing.assert_allclose(z[:, 0], rho * np.cos(2 * np.pi * u2), rtol=0, atol=2e-14)
    np.testing.assert_allclose(z[:, 1], rho * np.sin(2 * np.pi * u2), rtol=0, atol=2e-14)


def test_box_muller_is_standard_normal(oracle):
    z = oracle.box_muller(_words(50000, 2))
    for col in (0, 1):
        assert stats.kstest(z[:, col], "norm").pvalue > 1e-3
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.02


def _word_for_u(k):
    """word whose u01 is (k + 1/2) 2^-52"""
    return np.uint64(k) << np.uint64(12)


def _exact_cdf(n, q, kmax=200):
    """CDF of Bin(n, q) at k = 0..min(n, kmax), to 60 digits (mpmath), for
    q equal to the double q exactly."""
    mpmath.mp.dps = 60
    qm = mpmath.mpf(Fraction(q).numerator) / Fraction(q).denominator
    F, out = mpmath.mpf(0), []
    for k in range(min(n, kmax) + 1):
        F += mpmath.binomial(n, k) * qm**k * (1 - qm) ** (n - k)
        out.append(F)
    return out


@pytest.mark.parametrize("n,p", [(7, 0.3), (40, 0.05), (3, 0.45), (1000, 0.004), (12, 0.8), (5, 0.999)])
def test_binv_branch_is_exact_inversion(oracle, n, p):
    """For m = n min(p,1-p) < 10 the draw is the inverse CDF of Bin(n, p) at
    u, up to u within 1e-12 of a CDF step (exact rational CDF)."""
    flip = p > 0.5
    q = 1.0 - p if flip else p
    cdf = _exact_cdf(n, q)
    ks = np.random.default_rng(n).integers(0, 2**52, 3000)
    w = np.array([_word_for_u(k) for k in ks], dtype=np.uint64)
    got = oracle.binomial(np.full(w.size, n), np.full(w.size, p), w)
    checked = 0
    for k, g in zip(ks, got):
        u = (mpmath.mpf(int(k)) + mpmath.mpf(0.5)) / mpmath.mpf(2) ** 52
        if any(abs(u - F) < 1e-12 for F in cdf):
            continue
        if u > cdf[-1]:
            continue
        want = next(j for j, F in enumerate(cdf) if u <= F)
        want = n - want if flip else want
        assert g == want
        checked += 1
    assert checked > 2900


def test_binomial_special_cases(oracle):
    w = _words(50, 3)
    assert np.all(oracle.binomial(np.zeros(50, np.int64), 0.3, w) == 0)
    assert np.all(oracle.binomial(np.full(50, 17), 0.0, w) == 0)
    assert np.all(oracle.binomial(np.full(50, 17), 1.0, w) == 17)
    # the draw never leaves [0, n]
    n = np.random.default_rng(4).integers(0, 10**8, 20000)
    p = np.random.default_rng(5).uniform(0, 1, 20000)
    x = oracle.binomial(n, p, _words(20000, 6))
    assert np.all((x >= 0) & (x <= n))


@pytest.mark.parametrize("n,p", [(1000, 0.3), (10**7, 2e-5), (3 * 10**8, 0.7), (200, 0.06)])
def test_normal_branch_moments(oracle, n, p):
    """m >= 10: floor(m + 1/2 + sqrt(m(1-q)) z) has mean n p and variance
    n p (1-p) (+1/12 from rounding) to Monte-Carlo accuracy."""
    cnt = 40000
    x = oracle.binomial(np.full(cnt, n), p, _words(cnt, n % 97)).astype(np.float64)
    mean, var = n * p, n * p * (1 - p)
    assert abs(x.mean() - mean) < 5 * math.sqrt(var / cnt) + 0.05
    assert abs(x.var() / (var + 1 / 12) - 1) < 0.05


def test_binomial_distribution_small_mean(oracle):
    """chi-square of BINV draws against scipy.stats.binom."""
    n, p, cnt = 60, 0.07, 60000
    x = oracle.binomial(np.full(cnt, n), p, _words(cnt, 9))
    obs = np.bincount(x, minlength=n + 1)
    exp = stats.binom.pmf(np.arange(n + 1), n, p) * cnt
    keep = exp > 5
    obs_k = np.append(obs[keep], obs[~keep].sum())
    exp_k = np.append(exp[keep], exp[~keep].sum())
    assert stats.chisquare(obs_k, exp_k * obs_k.sum() / exp_k.sum()).pvalue > 1e-3


def _fig3_shapes():
    rows = []
    with open(os.path.join(HERE, "golden", "beta_shapes_fig3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split()
            rows.append((float(a), int(b)))
    return rows


@pytest.mark.parametrize("a,b", _fig3_shapes() + [(2.0, 5), (1.0, 1), (0.02, 18)])
def test_beta_integer_b_law(oracle, a, b):
    cnt = 20000
    s = oracle.beta_int(a, b, _words(cnt * b, int(a * 100) + b).reshape(cnt, b))
    assert np.all((s >= 0) & (s <= 1))
    assert stats.kstest(s, stats.beta(a, b).cdf).pvalue > 1e-3
    mean = a / (a + b)
    var = a * b / ((a + b) ** 2 * (a + b + 1))
    assert abs(s.mean() - mean) < 5 * math.sqrt(var / cnt)


def test_beta_b1_is_power_of_uniform(oracle):
    """b = 1: Beta(a, 1) = U^(1/a) (inversion), checked against numpy."""
    w = _words(5000, 12)
    u = ((w >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    for a in (0.3, 1.0, 2.5):
        s = oracle.beta_int(a, 1, w.reshape(-1, 1))
        np.testing.assert_allclose(s, u ** (1.0 / a), rtol=1e-14)


# ---------------------------------------------------------------- real-shape Beta (alternative parameterisations)

@pytest.mark.parametrize("a,b", [(0.3, 2.7), (1.5, 2.5), (0.05, 14.9), (2.2, 0.6), (7.0, 31.5)])
def test_general_beta_matches_scipy(oracle, a, b):
    x = oracle.beta_general(a, b, seed=7, index0=0, rnd=3, sub=0, n=20000)
    assert np.all((x >= 0) & (x <= 1))
    assert stats.kstest(x, "beta", args=(a, b)).pvalue > 1e-3


@pytest.mark.parametrize("k", [0.4, 1.0, 3.7, 25.0])
def test_gamma_marsaglia_tsang_matches_scipy(oracle, k):
    g = oracle.gamma_mt(k, seed=9, index0=0, rnd=1, sub=0, n=20000)
    assert stats.kstest(g, "gamma", args=(k,)).pvalue > 1e-3


@pytest.mark.parametrize("stage,ratio", [(1, 1.0), (2, 0.43), (5, 0.05), (9, 0.002)])
def test_alternative_parameterisations_closed_forms(oracle, stage, ratio):
    from paper_2106_15508_amd import workloads as W
    a, b = oracle.beta_shape_real(W.tiny(step_schedule=W.STEP_MEANVAR), stage, ratio, 1.0)
    mu = ratio / 3
    assert stats.beta(a, b).mean() == pytest.approx(mu, rel=1e-12)
    assert stats.beta(a, b).var() == pytest.approx(mu * (1 - mu) / (3 * stage + 1), rel=1e-12)
    a, b = oracle.beta_shape_real(W.tiny(step_schedule=W.STEP_MODECONC), stage, ratio, 1.0)
    assert (a - 1) / (a + b - 2) == pytest.approx(ratio / 4, rel=1e-12)
    assert a + b == pytest.approx(2 * stage + 2, rel=1e-12)
