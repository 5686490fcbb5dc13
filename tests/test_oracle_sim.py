"""Pins of the oracle's epidemic simulator (§II-B, eqs. 3-5) and distance."""
import math
from collections import Counter
from itertools import product

import numpy as np
import pytest
from scipy import stats

from paper_2106_15508_amd import workloads as W


def test_conservation_monotonicity_nonnegative(oracle):
    """S+I+A+R+D+Ru = P every day; R, D, Ru never decrease, S never
    increases; A+R+D never decreases; no count is negative."""
    w = W.C1
    rng = np.random.default_rng(0)
    for i in range(40):
        u = rng.uniform(size=8)
        theta = np.asarray(w.lo) + u * (np.asarray(w.hi) - np.asarray(w.lo))
        tr = oracle.simulate(w, theta, 99, 1, i)
        assert np.all(tr.sum(1) == w.population)
        assert np.all(tr >= 0)
        for c in (3, 4, 5):
            assert np.all(np.diff(tr[:, c]) >= 0)
        assert np.all(np.diff(tr[:, 0]) <= 0)
        assert np.all(np.diff(tr[:, 2] + tr[:, 3] + tr[:, 4]) >= 0)


def test_initial_state(oracle):
    """Ru = 0, I0 = floor(kappa A0), S = P - (A0+R0+D0+I0)."""
    w = W.C1.with_(n_days=1)
    th = list(W.THETA_TRUE)
    th[7] = 1.37
    tr = oracle.simulate(w, th, 5, 0, 0, obs0=(123, 45, 6))
    assert list(tr[0]) == [100000 - (123 + 45 + 6 + 168), 168, 123, 45, 6, 0]


def test_zero_rates_constant_trajectory(oracle):
    """alpha0 = alpha = beta = gamma = delta = 0: every hazard of eq. 5 is 0,
    so the state never changes."""
    w = W.C1
    tr = oracle.simulate(w, [0, 0, 0.5, 0, 0, 0, 0.3, 1.0], 1, 1, 1)
    assert np.all(tr == tr[0])


def test_observations_reproduce_and_distance_zero(oracle):
    """Re-simulating the generating vector with the observation seed gives
    the observed series exactly, so its distance is 0."""
    w = W.C1
    obs = oracle.observations(w)
    tr = oracle.simulate(w, w.theta_true, w.obs_seed, W.OBS_ROUND, 0)
    assert np.array_equal(tr[:, 2:5], obs)
    assert oracle.distance(tr, obs) == 0.0


def test_distance_is_euclidean(oracle):
    w = W.C1
    obs = oracle.observations(w)
    for i in range(10):
        tr = oracle.simulate(w, W.THETA_TRUE, 1234, 2, i)
        want = np.linalg.norm((tr[1:, 2:5] - obs[1:]).astype(np.float64).ravel())
        assert abs(oracle.distance(tr, obs) - want) <= 1e-14 * want


def test_obs_shape_like_epidemic(oracle):
    """Synthetic observations: R and D cumulative, A rises then falls."""
    for w in (W.C1, W.C2.with_(n_days=120)):
        obs = oracle.observations(w)
        assert np.all(np.diff(obs[:, 1]) >= 0) and np.all(np.diff(obs[:, 2]) >= 0)
        peak = int(np.argmax(obs[:, 0]))
        assert 0 < peak < w.n_days
        assert obs[peak, 0] > 100 * obs[0, 0]


# -------------------------------------------------------------- brute force

def _binom_pmf(n, p):
    return [math.comb(n, k) * p**k * (1 - p) ** (n - k) for k in range(n + 1)]


def _exact_final_state_law(theta, P, T, obs0):
    """Exact law of the day-T state by enumerating every transition count
    of every day (P is tiny), with the model written out from §II-B:
    g = alpha0 + alpha/(1+(A+R+D)^n), per-day probabilities 1-exp(-rate) for
    S->I (rate g I/P), I->A (gamma), A->R (beta), A->D (delta, from A left
    after A->R), I->Ru (beta eta, from I left after I->A)."""
    a0, al, n, be, ga, de, et, ka = theta
    A, R, D = obs0
    I = min(math.floor(ka * A), P - (A + R + D))
    S = P - (A + R + D + I)
    law = {(S, I, A, R, D, 0): 1.0}
    pIA, pAR, pAD, pIRu = (1 - math.exp(-ga), 1 - math.exp(-be), 1 - math.exp(-de),
                           1 - math.exp(-be * et))
    for _ in range(T):
        nxt = Counter()
        for (S, I, A, R, D, Ru), pr in law.items():
            Cn = A + R + D
            g = a0 + al / (1 + (Cn ** n if Cn > 0 else (1.0 if n == 0 else 0.0)))
            pSI = 1 - math.exp(-g * I / P)
            for n1, p1 in enumerate(_binom_pmf(S, pSI)):
                for n2, p2 in enumerate(_binom_pmf(I, pIA)):
                    for n3, p3 in enumerate(_binom_pmf(A, pAR)):
                        for n4, p4 in enumerate(_binom_pmf(A - n3, pAD)):
                            for n5, p5 in enumerate(_binom_pmf(I - n2, pIRu)):
                                st = (S - n1, I + n1 - n2 - n5, A + n2 - n3 - n4, R + n3, D + n4, Ru + n5)
                                nxt[st] += pr * p1 * p2 * p3 * p4 * p5
        law = nxt
    return law


@pytest.mark.parametrize("theta", [
    (0.8, 5.0, 1.0, 0.3, 0.4, 0.2, 0.5, 1.0),
    (0.5, 20.0, 0.5, 0.6, 0.7, 0.1, 0.9, 2.0),
])
def test_brute_force_tiny_population(oracle, theta):
    """P = 5, T = 3: every draw is in the exact-inversion branch; the
    empirical law of the day-3 state over 60000 independent streams matches
    exact enumeration (chi-square)."""
    P, T, obs0 = 5, 3, (1, 0, 0)
    w = W.C1.with_(population=P, n_days=T)
    law = _exact_final_state_law(theta, P, T, obs0)
    cnt = 60000
    emp = Counter()
    for i in range(cnt):
        tr = oracle.simulate(w, theta, 77, 1, i, obs0=obs0)
        emp[tuple(int(v) for v in tr[T])] += 1
    assert set(emp) <= set(law)
    keys = sorted(law)
    exp = np.array([law[k] * cnt for k in keys])
    obs = np.array([emp.get(k, 0) for k in keys], dtype=np.float64)
    big = exp >= 5
    obs_k = np.append(obs[big], obs[~big].sum())
    exp_k = np.append(exp[big], exp[~big].sum())
    assert stats.chisquare(obs_k, exp_k * obs_k.sum() / exp_k.sum()).pvalue > 1e-4


def test_one_day_conditional_means(oracle):
    """At P = 1e7 the one-day transition counts have the binomial means
    S pSI, I pIA, A pAR, ... to Monte-Carlo accuracy."""
    P, A0 = 10_000_000, 50_000
    w = W.C2.with_(n_days=1)
    th = (0.3, 2.0, 0.5, 0.05, 0.1, 0.005, 0.2, 1.0)
    cnt = 3000
    trs = np.stack([oracle.simulate(w, th, 3, 1, i, obs0=(A0, 0, 0))[1] for i in range(cnt)])
    S0, I0 = P - 2 * A0, A0
    g = th[0] + th[1] / (1 + A0 ** th[2])
    pSI = 1 - math.exp(-g * I0 / P)
    n1 = S0 - trs[:, 0]
    assert abs(n1.mean() - S0 * pSI) < 5 * math.sqrt(S0 * pSI * (1 - pSI) / cnt) + 0.5
    n3 = trs[:, 3]
    pAR = 1 - math.exp(-th[3])
    assert abs(n3.mean() - A0 * pAR) < 5 * math.sqrt(A0 * pAR * (1 - pAR) / cnt) + 0.5
    n5 = trs[:, 5]
    pIA = 1 - math.exp(-th[4])
    mean5 = I0 * (1 - pIA) * (1 - math.exp(-th[3] * th[6]))
    assert abs(n5.mean() - mean5) < 5 * math.sqrt(mean5 / cnt) + 0.5


def test_normal_floor_trajectory_properties(oracle):
    """The paper's own transition sampler in the simulator: conservation,
    no negative count, R never decreasing."""
    w = W.C2.with_(n_days=30, sampler=W.SAMPLER_NORMAL_FLOOR)
    for i in range(20):
        tr = oracle.simulate(w, W.THETA_TRUE, 8, 1, i, obs0=(1000, 0, 0))
        assert np.all(tr.sum(1) == w.population) and np.all(tr >= 0)
        assert np.all(np.diff(tr[:, 3]) >= 0)


def _floor_normal_draws(oracle, n, h, cnt, index):
    """cnt floor-normal draws for (n, h), one Philox word each (stream of
    particle `index`, a purpose no run uses)."""
    ws = oracle.words(77, index, 5, 9, 0, cnt)
    return np.array([oracle.lib().ref_normal_floor(n, h, int(x)) for x in ws], dtype=np.int64)


@pytest.mark.parametrize("h", [12.5, 1e3, 1e6])
def test_normal_floor_moments(oracle, h):
    """Section II-B draws a transition count as the floor of a normal with
    mean h and spread sqrt(h), read as the standard deviation (reading R3:
    the Poisson(h) it stands in for has variance h).  With the source
    count far above h the floor of N(h, h) has mean h - 1/2 and variance
    h + 1/12 (a uniform rounding error independent of the normal, Sheppard).
    Reading sqrt(h) as the variance instead gives variance sqrt(h); rounding
    instead of flooring moves the mean by 1/2 (28 standard errors at h = 12.5)."""
    cnt = 40000
    x = _floor_normal_draws(oracle, 10**12, h, cnt, int(h) % 1000).astype(np.float64)
    se = math.sqrt((h + 1.0 / 12.0) / cnt)
    assert abs(x.mean() - (h - 0.5)) < 5 * se, (x.mean(), h - 0.5, se)
    var = x.var(ddof=1)
    assert abs(var / (h + 1.0 / 12.0) - 1.0) < 0.05, (var, h)


@pytest.mark.parametrize("h", [3.0, 12.5])
def test_normal_floor_exact_law(oracle, h):
    """The clamped law is P(X = 0) = Phi((1 - h)/sqrt h), P(X = k) =
    Phi((k + 1 - h)/sqrt h) - Phi((k - h)/sqrt h) for 0 < k: chi-square
    of 60000 draws against it."""
    cnt = 60000
    x = _floor_normal_draws(oracle, 10**9, h, cnt, 500 + int(h))
    assert x.min() >= 0
    sd = math.sqrt(h)
    kmax = int(h + 7 * sd) + 1
    edges = np.arange(0, kmax + 1, dtype=np.float64)
    cdf = stats.norm.cdf((edges + 1.0 - h) / sd)
    p = np.diff(np.concatenate([[0.0], cdf]))
    p[-1] += 1.0 - cdf[-1]
    obs = np.bincount(np.minimum(x, kmax), minlength=kmax + 1).astype(np.float64)
    big = p * cnt >= 5
    obs_k = np.append(obs[big], obs[~big].sum())
    exp_k = np.append(p[big], p[~big].sum()) * cnt
    assert stats.chisquare(obs_k, exp_k).pvalue > 1e-4


def test_normal_floor_clamps(oracle):
    """Clamped to [0, n]: at h = 0.5 three quarters of the draws are 0
    (Phi(1/sqrt 2) = 0.760); with n = h = 100 half of them are n; h <= 0 or
    n <= 0 gives 0."""
    cnt = 20000
    x = _floor_normal_draws(oracle, 10**6, 0.5, cnt, 1)
    assert x.min() == 0
    p0 = stats.norm.cdf(0.5 / math.sqrt(0.5))
    assert abs((x == 0).mean() - p0) < 5 * math.sqrt(p0 * (1 - p0) / cnt)
    y = _floor_normal_draws(oracle, 100, 100.0, cnt, 2)
    assert y.max() == 100 and y.min() >= 0
    assert abs((y == 100).mean() - 0.5) < 5 * math.sqrt(0.25 / cnt)
    for n, h in ((0, 5.0), (-3, 5.0), (10, 0.0), (10, -1.0)):
        assert oracle.lib().ref_normal_floor(n, h, 12345) == 0


def test_normal_floor_one_day_counts(oracle):
    """In the simulator every transition of a day is floor(N(h, sqrt h))
    with the eq. 5 hazard h of the start-of-day state: at P = 1e7 with 50000
    active cases the S->I, A->R and A->D counts have means h - 1/2 and
    variances h + 1/12, and counts drawn from different words are
    uncorrelated."""
    P, A0 = 10_000_000, 50_000
    w = W.C2.with_(n_days=1, sampler=W.SAMPLER_NORMAL_FLOOR)
    th = (0.3, 2.0, 0.5, 0.05, 0.1, 0.005, 0.2, 1.0)
    cnt = 4000
    tr = np.stack([oracle.simulate(w, th, 6, 1, i, obs0=(A0, 0, 0)) for i in range(cnt)]).astype(np.float64)
    S0, I0 = float(P - 2 * A0), float(A0)
    g = th[0] + th[1] / (1 + A0 ** th[2])
    n1 = S0 - tr[:, 1, 0]
    n3, n4 = tr[:, 1, 3], tr[:, 1, 4]
    for x, h in ((n1, g * I0 / P * S0), (n3, th[3] * A0), (n4, th[5] * A0)):
        se = math.sqrt((h + 1.0 / 12.0) / cnt)
        assert abs(x.mean() - (h - 0.5)) < 5 * se, (x.mean(), h)
        assert abs(x.var(ddof=1) / (h + 1.0 / 12.0) - 1.0) < 0.1
    lim = 4.0 / math.sqrt(cnt)
    assert abs(np.corrcoef(n1, n3)[0, 1]) < lim
    assert abs(np.corrcoef(n3, n4)[0, 1]) < lim


def test_paired_normal_draws_are_uncorrelated(oracle):
    """Draws 0 and 1 (and 2 and 3) of a day take the cosine and sine deviates
    of one Box-Muller pair: in the normal branch their counts must still be
    independent (reusing one deviate, or a sign-flipped copy, gives a
    correlation of +-1)."""
    P, A0 = 10_000_000, 50_000
    w = W.C2.with_(n_days=1)
    th = (0.3, 2.0, 0.5, 0.05, 0.1, 0.005, 0.2, 1.0)
    cnt = 4000
    tr = np.stack([oracle.simulate(w, th, 5, 2, i, obs0=(A0, 0, 0)) for i in range(cnt)]).astype(np.float64)
    S0, I0 = tr[0, 0, 0], tr[0, 0, 1]
    n1 = S0 - tr[:, 1, 0]
    n3, n4, n5 = tr[:, 1, 3], tr[:, 1, 4], tr[:, 1, 5]
    n2 = tr[:, 1, 2] - A0 + n3 + n4
    assert np.all(tr[:, 1, 1] == I0 + n1 - n2 - n5)
    lim = 4.0 / math.sqrt(cnt)
    assert abs(np.corrcoef(n1, n2)[0, 1]) < lim
    # n4 ~ Bin(A - n3, p_AD): its mean moves with n3 by -p_AD (a correlation of about -0.02)
    assert abs(np.corrcoef(n3, n4)[0, 1]) < lim
    for x in (n1, n2, n3, n4):
        assert x.std() > 5.0   # all four in the normal branch
