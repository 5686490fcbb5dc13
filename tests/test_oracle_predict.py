"""Pins of the oracle's posterior predictive bands (§IV-B, Fig. 7)."""
import numpy as np

from paper_2106_15508_amd import workloads as W


def test_bands_are_numpy_quantiles_of_the_trajectories(oracle):
    w = W.tiny(n_rounds=2)
    obs = oracle.observations(w)
    r = oracle.run(w, obs)
    u = r.u[-1][:40]
    days = 37
    q = (0.0, 0.1, 0.5, 0.9, 1.0)
    bands = oracle.predict(w, obs, u, days, seed=5, quantiles=q)
    lo, hi = np.asarray(w.lo), np.asarray(w.hi)
    series = np.stack([oracle.simulate(w.with_(n_days=days), lo + uj * (hi - lo), 5, oracle.PREDICT_ROUND, j,
                                       obs0=obs[0])[:, 2:5] for j, uj in enumerate(u)], axis=-1)
    want = np.quantile(series.astype(np.float64), q, axis=-1, method="linear").transpose(1, 2, 0)
    assert np.array_equal(bands, want)
    # quantile levels are ordered, day 0 is the observed state, R and D never fall
    assert np.all(np.diff(bands, axis=-1) >= 0)
    assert np.all(bands[0] == np.asarray(obs[0])[:, None])
    assert np.all(np.diff(bands[:, 1:, -1], axis=0) >= 0)


def test_fitted_days_use_a_fresh_stream(oracle):
    """The predictive stream (round 0xFFFE) is not the observation stream:
    even theta_true does not reproduce the observed series exactly."""
    w = W.tiny()
    obs = oracle.observations(w)
    u_true = (np.asarray(w.theta_true) - np.asarray(w.lo)) / (np.asarray(w.hi) - np.asarray(w.lo))
    bands = oracle.predict(w, obs, u_true[None, :], w.n_days, seed=w.obs_seed, quantiles=(0.5,))
    assert not np.array_equal(bands[:, :, 0], obs.astype(np.float64))
