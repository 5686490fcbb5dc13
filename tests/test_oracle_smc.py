"""Pins of the oracle's SMC stage machinery: tolerance (eq. 8), prior set
and resampling weights (eqs. 9-10), categorical draw (eq. 11), importance
weights, and end-to-end behaviour of a run."""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

from paper_2106_15508_amd import workloads as W


@pytest.mark.parametrize("n", [2, 3, 4, 5, 64, 1000, 1023, 4096])
@pytest.mark.parametrize("alpha", [0.5, 0.1, 0.25, 0.9, 0.3333])
def test_quantile_bitwise_numpy_linear(oracle, n, alpha):
    rng = np.random.default_rng(n * 7 + int(alpha * 1000))
    for x in (rng.exponential(1e5, n), np.round(rng.uniform(0, 50, n)), rng.uniform(size=n)):
        want = np.quantile(x, alpha, method="linear")
        assert oracle.quantile(x, alpha) == want


def test_resample_weights_properties(oracle):
    rng = np.random.default_rng(3)
    d = rng.exponential(1.0, 500)
    eps = float(np.median(d))
    q, Cc, ns = oracle.resample_weights(d, eps)
    surv = d < eps
    assert ns == surv.sum()
    assert np.all(q[~surv] == 0)
    w = eps - d
    wmax = w[surv].max()
    # q_k = floor(2^40 w_k / w_max): within one unit of the exact scaled weight
    exact = w[surv] / wmax * 2.0**40
    assert np.all(np.abs(q[surv].astype(np.float64) - exact) < 1.0 + 1e-3)
    assert q.max() == 2**40
    assert np.array_equal(Cc, np.cumsum(q.astype(object)).astype(np.uint64))


def test_resample_weights_fallbacks(oracle):
    d = np.array([3.0, 3.0, 5.0, 3.0])
    q, Cc, ns = oracle.resample_weights(d, 3.0)   # nothing strictly below: use <=
    assert ns == 3
    assert list(q) == [1, 1, 0, 1]          # all survivors at w = 0: equal weights
    assert list(Cc) == [1, 2, 2, 3]


def test_parent_draw_boundaries(oracle):
    """r = floor(R Q / 2^64); parent = first k with C_k > r.  Words that
    land exactly on r = C_{k-1} and r = C_k - 1 select particle k."""
    q = np.array([5, 0, 3, 1, 0, 7, 2**40, 0, 9], dtype=np.uint64)
    Cc = np.cumsum(q).astype(np.uint64)
    Q = int(Cc[-1])
    prev = 0
    for k, ck in enumerate(Cc):
        ck = int(ck)
        if q[k] == 0:
            continue
        for r in (prev, ck - 1):
            R = -(-(r << 64) // Q)  # smallest R with floor(R Q / 2^64) = r
            assert (R * Q) >> 64 == r
            assert oracle.parent(Cc, R) == k
        prev = ck


def test_parent_frequencies(oracle):
    rng = np.random.default_rng(4)
    q = rng.integers(0, 1000, 40).astype(np.uint64)
    q[::7] = 0
    Cc = np.cumsum(q).astype(np.uint64)
    cnt = 100000
    Rs = rng.integers(0, 2**64, cnt, dtype=np.uint64)
    ks = np.array([oracle.parent(Cc, int(R)) for R in Rs])
    obs = np.bincount(ks, minlength=q.size)
    assert np.all(obs[q == 0] == 0)
    p = q.astype(np.float64) / q.sum()
    keep = q > 0
    assert stats.chisquare(obs[keep], p[keep] * cnt).pvalue > 1e-3


def _mp_log_weight(u_j, s, u_prev, q):
    mpmath.mp.dps = 50
    L = mpmath.mpf(0)
    for k in range(len(q)):
        if q[k] == 0:
            continue
        D = sum((mpmath.mpf(float(u_j[d])) - mpmath.mpf(float(u_prev[k][d]))) ** 2 for d in range(8))
        L += int(q[k]) * mpmath.exp(-D / (2 * mpmath.mpf(float(s)) ** 2))
    return 8 * mpmath.log(mpmath.mpf(float(s))) - mpmath.log(L)


def test_log_weight_brute_force(oracle):
    """Row sum of the importance weight against 50-digit arithmetic, N <= 8."""
    rng = np.random.default_rng(5)
    for trial in range(20):
        M = int(rng.integers(1, 9))
        u_prev = rng.uniform(size=(M, 8))
        q = rng.integers(0, 2**40, M).astype(np.uint64)
        q[0] = max(int(q[0]), 1)
        if M > 2:
            q[1] = 0
        s = float(10 ** rng.uniform(-3, -0.3))
        u_j = np.clip(u_prev[0] + s * rng.standard_normal(8), 0, 1)
        got = oracle.log_weight(u_j, s, u_prev, q)
        want = _mp_log_weight(u_j, s, u_prev, q)
        assert abs(got - float(want)) <= 1e-13 * max(1.0, abs(float(want)))


def test_log_weight_is_gaussian_mixture_density(oracle):
    """With equal q_k the weight is the reciprocal of an equal-weight
    Gaussian mixture density (scipy.stats.multivariate_normal)."""
    rng = np.random.default_rng(6)
    M, s = 6, 0.2
    u_prev = rng.uniform(size=(M, 8))
    q = np.full(M, 1000, dtype=np.uint64)
    for _ in range(5):
        u_j = rng.uniform(size=8)
        dens = np.mean([stats.multivariate_normal(u_prev[k], s * s * np.eye(8)).pdf(u_j) for k in range(M)])
        # l = 8 log s - log sum_k q exp(...) = -log(dens) - 4 log(2 pi) - log(q M)
        want = -math.log(dens) - 4 * math.log(2 * math.pi) - math.log(1000 * M)
        assert abs(oracle.log_weight(u_j, s, u_prev, q) - want) < 1e-9 * abs(want) + 1e-9


def test_normalise(oracle):
    rng = np.random.default_rng(7)
    l = rng.normal(0, 30, 5000)
    Wn, ess = oracle.normalise(l)
    assert abs(Wn.sum() - 1) < 1e-14
    assert np.all(Wn >= 0)
    want = np.exp(l - l.max()) / np.exp(l - l.max()).sum()
    np.testing.assert_allclose(Wn, want, rtol=1e-12, atol=1e-300)
    assert abs(ess - 1 / np.sum(want**2)) < 1e-9 * ess


# ----------------------------------------------------------------- runs

@pytest.fixture(scope="module")
def c1_run(oracle):
    w = W.C1.with_(n_rounds=10, step_schedule=W.STEP_PAPER)
    obs = oracle.observations(w)
    return w, obs, oracle.run(w, obs)


def test_run_invariants(oracle, c1_run):
    w, obs, r = c1_run
    assert r.rc == 0
    N = w.n_particles
    assert np.all(np.diff(r.eps_next) <= 0)            # eq. 8: non-increasing
    for i in range(1, w.n_rounds):
        assert np.all(r.dist[i] <= r.eps[i])            # accepted only if d <= eps
        assert np.all(np.diff(r.index[i]) > 0)          # first N in proposal order
        assert r.proposals[i] == r.index[i][-1] + 1
        assert np.all((r.u[i] >= 0) & (r.u[i] <= 1))
        assert abs(r.W[i].sum() - 1) < 1e-13
        assert r.beta_b[i] == 2 * i and r.beta_a[i] == r.eps[i] / r.eps[1]   # eq. 16
        assert np.all(r.sigma[i] >= 1e-8)
    assert r.beta_a[1] == 1.0 and r.beta_b[1] == 2   # Beta(1,2) in the first stage
    assert np.all(r.W[0] == 1.0 / N)
    # the accepted particles re-simulate to the same distance
    for i in (0, 3, 9):
        for k in (0, N // 2, N - 1):
            d = oracle.sim_distance(w, obs, r.u[i][k], i, int(r.index[i][k]))
            assert d == r.dist[i][k]


def test_run_reproduces_proposals(oracle, c1_run):
    """Each accepted particle of stage i is the proposal its index draws
    from the stage's own resampling law (eqs. 9-11, 16-17)."""
    w, obs, r = c1_run
    for i in (1, 5):
        q, Cc, _ = oracle.resample_weights(r.dist[i - 1], r.eps[i])
        for k in (0, 7, w.n_particles - 1):
            a, u, s, par = oracle.perturb(w, i, int(r.index[i][k]), r.u[i - 1], Cc,
                                          r.beta_a[i], int(r.beta_b[i]))
            assert a == r.attempts[i][k] and s == r.sigma[i][k] and par == r.parent[i][k]
            assert np.array_equal(u, r.u[i][k])


def test_posterior_recovery(oracle, c1_run):
    """After 10 stages the population concentrates around the generating
    values of the identifiable parameters alpha0, beta, gamma, delta, eta."""
    w, obs, r = c1_run
    th = r.theta(w)[-1]
    width = np.asarray(w.hi) - np.asarray(w.lo)
    for p in (0, 3, 4, 5, 6):
        med = np.median(th[:, p])
        assert abs(med - W.THETA_TRUE[p]) < 0.05 * width[p], (W.PARAM_NAMES[p], med)
        wm = float((r.W[-1] * th[:, p]).sum())
        assert abs(wm - W.THETA_TRUE[p]) < 0.08 * width[p], (W.PARAM_NAMES[p], wm)
    assert r.eps_next[-1] < 0.2 * r.eps_next[0]


def test_bdss_beats_fixed_step(oracle):
    """The eq. 16 schedule reaches a lower tolerance than a fixed Beta(2,5)
    step law in the same number of stages (the paper's central claim,
    §IV-A, on the synthetic series)."""
    w = W.C1.with_(n_rounds=7)
    obs = oracle.observations(w)
    paper = oracle.run(w.with_(step_schedule=W.STEP_PAPER), obs)
    fixed = oracle.run(w.with_(step_schedule=W.STEP_FIXED), obs)
    assert paper.eps_next[-1] < fixed.eps_next[-1]


def test_replaying_own_schedule_is_identity(oracle):
    # a run fed its own eq. 8 tolerances is the same run; a changed entry
    # changes exactly the stage that uses it (and what follows from it)
    wl = W.tiny(n_rounds=4)
    obs = oracle.observations(wl)
    a = oracle.run(wl, obs)
    b = oracle.run(wl.with_(eps_schedule=tuple(a.eps_next[:3])), obs)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.dist, b.dist)
    assert np.array_equal(a.eps, b.eps) and np.array_equal(a.W, b.W)
    c = oracle.run(wl.with_(eps_schedule=(a.eps_next[0], 0.8 * a.eps_next[1])), obs)
    assert np.array_equal(a.u[:2], c.u[:2]) and c.eps[2] == 0.8 * a.eps_next[1]
    assert np.all(c.dist[2] <= c.eps[2]) and not np.array_equal(a.u[2], c.u[2])


# ----------------------------------------------------- perturbation law (eq. 17)

def _perturb_many(oracle, w, rnd, u_prev, q, beta_a, beta_b, cnt, **over):
    """cnt proposals (indices 0..cnt-1) of stage rnd from the oracle's
    perturbation: arrays of attempts, u, sigma, parent."""
    Cc = np.cumsum(np.asarray(q, dtype=np.uint64)).astype(np.uint64)
    out = [oracle.perturb(w, rnd, j, u_prev, Cc, beta_a, beta_b, **over) for j in range(cnt)]
    a = np.array([o[0] for o in out])
    u = np.array([o[1] for o in out])
    s = np.array([o[2] for o in out])
    par = np.array([o[3] for o in out])
    return a, u, s, par


@pytest.mark.parametrize("variance", [False, True])
def test_perturbation_offsets_are_iid_standard_normal(oracle, variance):
    """Eq. 17 in the unit cube: u = u_parent + sigma z with z ~ N(0, I_8).
    With a fixed step size (the MCMC variant's s) and every parent at least
    40 sigma inside the cube no proposal is redrawn, so the eight
    standardised offsets (u - u_parent)/sigma must each be N(0, 1) (KS) and
    pairwise uncorrelated (|r| < 4/sqrt(n)); sigma is s, or sqrt(s) when s
    is read as a variance (eq. 12).  A deviate reused across two
    coordinates, sigma^2 in place of sigma, or a wrong scale fails this."""
    rng = np.random.default_rng(11)
    M, cnt, sig = 16, 20000, 0.01
    u_prev = rng.uniform(0.4, 0.6, size=(M, 8))
    q = rng.integers(1, 1000, M)
    s = sig * sig if variance else sig
    w = W.tiny(step_schedule=W.STEP_MCMC, step_is_variance=variance)
    a, u, sg, par = _perturb_many(oracle, w, 3, u_prev, q, s, 0, cnt)
    assert np.all(a == 1)
    assert np.all(sg == (math.sqrt(s) if variance else s))
    z = (u - u_prev[par]) / sig
    for d in range(8):
        assert stats.kstest(z[:, d], "norm").pvalue > 1e-4, d
    r = np.corrcoef(z.T)
    lim = 4.0 / math.sqrt(cnt)
    assert np.all(np.abs(r[np.triu_indices(8, 1)]) < lim)
    # the parents follow the categorical law of eq. 11
    obs = np.bincount(par, minlength=M)
    assert stats.chisquare(obs, q / q.sum() * cnt).pvalue > 1e-4


def test_perturbation_redraws_the_whole_triple(oracle):
    """A proposal outside [0,1]^8 is redrawn with a new parent, step size
    and normal vector (reading R10), so each attempt lands inside with
    probability p = sum_k P_k Pr(inside | k): the attempt count is
    geometric(p), and the accepted parent is k with probability
    P_k Pr(inside | k) / p.  Two parents with q = (1, 3): one deep inside,
    one with its first coordinate sigma/2 from the face u = 0 (inside with
    probability Phi(1/2)).  Keeping the parent and redrawing only z would
    give the second parent probability 3/4 instead of 0.675; its accepted
    offsets are N(0, 1) truncated below at -1/2."""
    sig, cnt = 0.05, 20000
    u_prev = np.full((2, 8), 0.5)
    u_prev[1, 0] = 0.5 * sig
    q = np.array([1, 3])
    w = W.tiny(step_schedule=W.STEP_MCMC)
    a, u, sg, par = _perturb_many(oracle, w, 2, u_prev, q, sig, 0, cnt)
    assert np.all(a >= 1) and np.all((u >= 0) & (u <= 1))
    pin = stats.norm.cdf(0.5)
    p = 0.25 + 0.75 * pin
    pb = 0.75 * pin / p
    nb = int((par == 1).sum())
    assert abs(nb / cnt - pb) < 5 * math.sqrt(pb * (1 - pb) / cnt), (nb / cnt, pb)
    kmax = 6
    obs = np.array([(a == k).sum() for k in range(1, kmax)] + [(a >= kmax).sum()], dtype=np.float64)
    exp = np.array([(1 - p) ** (k - 1) * p for k in range(1, kmax)] + [(1 - p) ** (kmax - 1)]) * cnt
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    z0 = (u[par == 1, 0] - u_prev[1, 0]) / sig
    assert stats.kstest(z0, stats.truncnorm(-0.5, np.inf).cdf).pvalue > 1e-4


def test_perturbation_step_size_redrawn_with_the_triple(oracle):
    """With the eq. 16 law s ~ Beta(1, 2) and one parent at the centre of
    the cube, an attempt lands inside with probability
    g(s) = (2 Phi(1/(2 s)) - 1)^8, so the accepted step sizes have density
    proportional to f(s) g(s) (f the Beta(1, 2) density) and the attempts
    are geometric with p = integral of f g.  Keeping s across the redraws
    would leave the accepted step sizes close to f itself."""
    from scipy import integrate
    cnt = 20000
    u_prev = np.full((1, 8), 0.5)
    w = W.tiny()
    a, u, sg, par = _perturb_many(oracle, w, 1, u_prev, [1], 1.0, 2, cnt)
    assert np.all(a > 0) and np.all(par == 0)

    def f(s):
        return 2.0 * (1.0 - s)

    def g(s):
        return (2.0 * stats.norm.cdf(0.5 / s) - 1.0) ** 8

    p = integrate.quad(lambda s: f(s) * g(s), 0, 1, epsabs=1e-13)[0]
    grid = np.linspace(0.0, 1.0, 4001)
    dens = np.array([f(s) * g(s) if s > 0 else 2.0 for s in grid])
    cdf = np.concatenate([[0.0], np.cumsum((dens[1:] + dens[:-1]) * 0.5 * np.diff(grid))])
    cdf /= cdf[-1]
    assert stats.kstest(sg, lambda x: np.interp(x, grid, cdf)).pvalue > 1e-4
    kmax = 8
    obs = np.array([(a == k).sum() for k in range(1, kmax)] + [(a >= kmax).sum()], dtype=np.float64)
    exp = np.array([(1 - p) ** (k - 1) * p for k in range(1, kmax)] + [(1 - p) ** (kmax - 1)]) * cnt
    assert stats.chisquare(obs, exp).pvalue > 1e-4


# ------------------------------------------------- full SMC against a grid posterior

def test_weighted_population_is_the_abc_posterior(oracle):
    """The importance weights (reading R17) make each stage's population a
    sample of the ABC posterior pi(theta) Pr(d <= eps_i | theta) (§II-C,
    §II-D).  Toy: every prior interval but beta's is a single point
    (lo = hi = the generating value), P = 60, 6 days, so the posterior of
    the one free parameter is known on a grid from the acceptance
    probability, estimated by 3000 simulations per grid point on streams no
    run uses.  Twelve runs (seeds 1..12, N = 1000, eq. 16 step sizes, the
    same replayed tolerances) give W-weighted means and standard deviations
    that must agree with the grid posterior's within 4 standard errors of
    the seed-to-seed spread, at stages 1, 2 and 3.  The unweighted
    population is biased (more than 30 standard errors at every stage), so
    the agreement is the weights' doing."""
    th = list(W.THETA_TRUE)
    free = 3
    lo, hi = list(th), list(th)
    lo[free], hi[free] = 0.0, 0.5
    w = W.Workload("toy", population=60, n_days=6, n_particles=1000, n_rounds=4, lo=tuple(lo), hi=tuple(hi),
                   obs_seed=4242, seed=1)
    obs = oracle.observations(w)
    sched = tuple(oracle.run(w, obs).eps_next[:3])
    M, S, U = [], [], []
    for seed in range(1, 13):
        r = oracle.run(w.with_(seed=seed, eps_schedule=sched), obs)
        assert r.rc == 0 and np.array_equal(r.eps[1:], sched)
        x = r.theta(w)[:, :, free]
        m = [float((r.W[i] * x[i]).sum()) for i in (1, 2, 3)]
        # weighted standard deviation with the 1 / (1 - sum W^2) bias correction
        s = [math.sqrt(float((r.W[i] * (x[i] - m[i - 1]) ** 2).sum()) / (1.0 - float((r.W[i] ** 2).sum())))
             for i in (1, 2, 3)]
        M.append(m)
        S.append(s)
        U.append([float(x[i].mean()) for i in (1, 2, 3)])
    M, S, U = np.array(M), np.array(S), np.array(U)
    G, n = 80, 3000
    grid_u = (np.arange(G) + 0.5) / G
    grid_th = lo[free] + grid_u * (hi[free] - lo[free])
    for i in (1, 2, 3):
        p = np.zeros(G)
        for g in range(G):
            u = np.full(8, 0.5)
            u[free] = grid_u[g]
            p[g] = oracle.accept_count(w, obs, u, sched[i - 1], 0xABC, g * n, n) / n
        gm = float((p * grid_th).sum() / p.sum())
        gs = math.sqrt(float((p * (grid_th - gm) ** 2).sum() / p.sum()))
        k = i - 1
        se_m = M[:, k].std(ddof=1) / math.sqrt(len(M))
        se_s = S[:, k].std(ddof=1) / math.sqrt(len(S))
        se_u = U[:, k].std(ddof=1) / math.sqrt(len(U))
        assert abs(M[:, k].mean() - gm) < 4 * se_m + 1e-3 * gs, (i, M[:, k].mean(), gm, se_m)
        assert abs(S[:, k].mean() - gs) < 4 * se_s + 1e-3 * gs, (i, S[:, k].mean(), gs, se_s)
        assert abs(U[:, k].mean() - gm) > 30 * se_u, (i, U[:, k].mean(), gm, se_u)
