"""GPU parity of the device primitives against the oracle: IEEE division
and square root, the series-based elementary functions, Philox, the normal
pair, the binomial, Beta and floor-normal draws.  All bit-exact."""
import numpy as np
import pytest

from paper_2106_15508_amd import abcsmc as A

pytestmark = pytest.mark.gpu


def _ev(fn, inp, n, out_dtype, out_shape, pa=0.0, pb=0):
    out = np.zeros(out_shape, dtype=out_dtype)
    return A.debug_eval(fn, inp, n, out, pa, pb)


def _same(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.dtype == np.float64:
        return np.array_equal(a.view(np.uint64), b.view(np.uint64))
    return np.array_equal(a, b)


def _inputs():
    rng = np.random.default_rng(2106)
    return {
        "exp": np.concatenate([rng.uniform(-708, 709.7, 20000), rng.uniform(-1, 1, 20000),
                               [0.0, -0.0, -708.0, -707.99, 709.78, 1e-300, -1e-300]]),
        "expm1": np.concatenate([rng.uniform(-0.35, 0.35, 20000), rng.uniform(-50, 5, 20000),
                                 -(10 ** rng.uniform(-300, 2, 5000)), [0.0, -0.34657359027997264]]),
        "log": np.concatenate([10 ** rng.uniform(-300, 300, 20000), rng.uniform(0.5, 2, 20000),
                               [1.0, 2.0 ** -1074, np.nextafter(1, 0), np.nextafter(1, 2)]]),
        "log1p": np.concatenate([rng.uniform(-0.999, 4, 20000), -(10 ** rng.uniform(-300, -0.01, 5000)),
                                 10 ** rng.uniform(-300, 8, 5000), [0.0, -0.5, 0.41421356237309515]]),
        "cos2pi": (rng.integers(0, 2**32, 30000) + 0.5) / 2**32,
        "sin2pi": (rng.integers(0, 2**32, 30000) + 0.5) / 2**32,
    }


@pytest.mark.parametrize("name,fn", [("exp", 0), ("expm1", 1), ("log", 2), ("log1p", 3),
                                     ("cos2pi", 4), ("sin2pi", 5)])
def test_elementary_bitwise(oracle, name, fn):
    x = _inputs()[name]
    got = _ev(fn, x, x.size, np.float64, x.size)
    want = oracle.fmap(name, x)
    bad = np.flatnonzero(got.view(np.uint64) != want.view(np.uint64))
    assert bad.size == 0, (name, x[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_sqrt_and_division_correctly_rounded():
    """gfx950 FP64 sqrt and division are IEEE correctly rounded (numpy on
    the host is the reference)."""
    rng = np.random.default_rng(3)
    x = np.concatenate([10 ** rng.uniform(-300, 300, 50000), rng.uniform(0, 4, 50000),
                        (rng.integers(0, 2**52, 20000) + 0.5) * 2.0**-52 * 1e17])
    got = _ev(6, x, x.size, np.float64, x.size)
    assert _same(got, np.sqrt(x))
    a = rng.uniform(-1e6, 1e6, 60000) * 10 ** rng.uniform(-100, 100, 60000)
    b = rng.uniform(0.1, 10, 60000) * 10 ** rng.uniform(-100, 100, 60000)
    pairs = np.stack([a, b], 1).ravel()
    got = _ev(7, pairs, a.size, np.float64, a.size)
    assert _same(got, a / b)


def test_philox_bitwise(oracle):
    rng = np.random.default_rng(4)
    n = 4000
    ck = rng.integers(0, 2**32, (n, 6), dtype=np.uint64).astype(np.uint32)
    got = _ev(8, ck, n, np.uint32, (n, 4))
    for i in range(0, n, 97):
        assert np.array_equal(got[i], oracle.philox(ck[i, :4], ck[i, 4:]))


def test_box_muller_bitwise(oracle):
    w = np.random.default_rng(5).integers(0, 2**64, 30000, dtype=np.uint64)
    got = _ev(9, w, w.size, np.float64, (w.size, 2))
    assert _same(got, oracle.box_muller(w))


def _draw_inputs(seed, cnt):
    rng = np.random.default_rng(seed)
    n = np.concatenate([rng.integers(0, 20, cnt // 4), rng.integers(0, 2000, cnt // 4),
                        rng.integers(0, 10**6, cnt // 4), rng.integers(0, 3 * 10**8, cnt - 3 * (cnt // 4))])
    p = np.concatenate([rng.uniform(0, 1, cnt // 2), 10 ** rng.uniform(-9, 0, cnt - cnt // 2)])
    p[::17] = 0.0
    p[::19] = 1.0
    p[::23] = 0.5
    w = rng.integers(0, 2**64, cnt, dtype=np.uint64)
    rec = np.zeros((cnt, 3), dtype=np.uint64)
    rec[:, 0] = n.astype(np.int64).view(np.uint64)
    rec[:, 1] = p.view(np.uint64)
    rec[:, 2] = w
    return n.astype(np.int64), p, w, rec


def test_binomial_bitwise(oracle):
    n, p, w, rec = _draw_inputs(6, 40000)
    got = _ev(10, rec, n.size, np.int64, n.size)
    want = oracle.binomial(n, p, w)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (n[bad[:5]], p[bad[:5]], got[bad[:5]], want[bad[:5]])


def test_normal_floor_bitwise(oracle):
    n, p, w, rec = _draw_inputs(7, 20000)
    h = p * n  # use n p as the hazard
    rec[:, 1] = h.view(np.uint64)
    got = _ev(12, rec, n.size, np.int64, n.size)
    L = oracle.lib()
    want = np.array([L.ref_normal_floor(int(a), float(b), int(c)) for a, b, c in zip(n, h, w)])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("a,b", [(1.0, 2), (0.5, 5), (0.1, 15), (2.0, 5), (0.003, 24), (1.0, 1)])
def test_beta_bitwise(oracle, a, b):
    cnt = 5000
    w = np.random.default_rng(int(a * 1000) + b).integers(0, 2**64, (cnt, b), dtype=np.uint64)
    got = _ev(11, w, cnt, np.float64, cnt, a, b)
    assert _same(got, oracle.beta_int(a, b, w))


@pytest.mark.parametrize("a,b,seed,rnd", [(0.3, 2.7, 7, 3), (1.5, 2.5, 11, 1), (0.05, 14.9, 5, 9),
                                           (2.2, 0.6, 1, 2), (7.0, 31.5, 3, 4)])
def test_general_beta_bitwise(oracle, a, b, seed, rnd):
    n = 5000
    got = np.zeros(n)
    A.debug_eval(13, np.array([a, b]), n, got, float(seed), rnd)
    want = oracle.beta_general(a, b, seed, 0, rnd, 0, n)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_weight_term_against_oracle(oracle):
    """One importance-weight term q_k exp(-|u_j - u_k|^2 / (2 sigma_j^2)) as
    the weight kernels evaluate it (table exponential) against the oracle's
    term: within 1.5e-15 + 2.5e-15 x relative, x = |u_j - u_k|^2 / (2 sigma_j^2)
    (the cubic's truncation r^4/24 < 5.6e-16 and a few roundings, plus the
    exponent's own rounding, which scales with x: the squared distance is
    summed with fused multiply-adds on one side and separate roundings on
    the other, at most 16 roundings of 1.1e-16 between them, and the scaling
    adds four more), where the oracle's term is at least 1e-300;
    exactly 0 where the exponent is below -2^31 in units of ln2/1024 (a
    sigma at the 1e-8 floor and a column 0.01 or more away: the integer
    conversion saturates instead of being undefined); below 1e-300 wherever
    the oracle's term is 0."""
    rng = np.random.default_rng(14)
    n = 30000
    uj = rng.uniform(size=(n, 8))
    sig = 10 ** rng.uniform(-3, -0.3, n)
    uk = np.clip(uj + sig[:, None] * rng.normal(0, 1, (n, 8)) * rng.uniform(0.1, 8, (n, 1)), 0, 1)
    far = n - 4000
    sig[far:] = 1e-8                                   # floor: t = -D 1024/(2e-16 ln 2) ~ -1e18 .. -1e20
    uk[far:] = np.clip(uj[far:] + rng.choice([-1, 1], (4000, 8)) * rng.uniform(0.01, 0.5, (4000, 8)), 0, 1)
    q = rng.integers(1, 2**40, n).astype(np.float64)
    rec = np.concatenate([uj, sig[:, None], uk, q[:, None]], axis=1)
    got = _ev(14, np.ascontiguousarray(rec), n, np.float64, n)
    want = np.array([q[i] * oracle.fmap("exp", [-(float(((uj[i] - uk[i]) ** 2).sum()) / (2.0 * (sig[i] * sig[i])))])[0]
                     for i in range(n)])
    D = ((uj - uk) ** 2).sum(1)
    t = -D * (1024 / np.log(2)) / (2 * sig * sig)
    assert np.all(t[far:] < -2.0**31)
    assert np.all(got[far:] == 0.0)
    big = want >= 1e-300
    assert big.sum() > 10000
    rel = np.abs(got[big] - want[big]) / want[big]
    x = D[big] / (2 * sig[big] * sig[big])
    ratio = rel / (1.5e-15 + 2.5e-15 * x)
    w = int(np.argmax(ratio))
    print("weight term: largest relative error %.2e (x = %.1f); worst against the bound: %.2e at x = %.2f"
          % (rel.max(), x[np.argmax(rel)], rel[w], x[w]), flush=True)
    assert ratio.max() <= 1.0, (rel[w], x[w])
    assert np.all(got[~big] < 1e-300) and np.all(got >= 0)


def test_measured_peaks_are_plausible():
    """The measurement helper behind bench.py's `measured_peaks`: an FP64 fma
    loop cannot beat the published 78.6 TFLOP/s (at most 2.4 GHz), the clock
    it reports lies in the device's range, and a copy cannot beat 8 TB/s."""
    pk = A.measure_peaks(2)
    assert 30.0 < pk["fp64_tflops"] <= 78.6 * 1.02
    assert 1000.0 < pk["clock_mhz"] <= 2500.0
    # the fma rate follows from the clock: 256 CUs x 64 lanes x 2 flops per cycle
    assert pk["fp64_tflops"] <= 256 * 64 * 2 * pk["clock_mhz"] * 1e6 / 1e12 * 1.05
    assert 1000.0 < pk["copy_gbs"] <= 8000.0 * 1.02
