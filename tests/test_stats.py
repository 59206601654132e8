"""Pins for the host-side ESS estimator (closed forms)."""
import numpy as np

from paper_2104_07097_amd.stats import ess, ks_distance, ks_two_sample


def test_ess_iid():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((8, 4000))
    e = ess(x)
    assert 0.85 * x.size < e < 1.15 * x.size


def test_ess_ar1():
    # AR(1) x_t = rho x_{t-1} + e_t has integrated autocorrelation time (1+rho)/(1-rho)
    rng = np.random.default_rng(1)
    rho, c, t = 0.9, 8, 20000
    x = np.zeros((c, t))
    x[:, 0] = rng.standard_normal(c) / np.sqrt(1 - rho**2)
    e = rng.standard_normal((c, t))
    for i in range(1, t):
        x[:, i] = rho * x[:, i - 1] + e[:, i]
    want = c * t * (1 - rho) / (1 + rho)
    assert 0.85 * want < ess(x) < 1.15 * want


def test_ks_helpers():
    rng = np.random.default_rng(2)
    u = rng.uniform(size=5000)
    assert ks_distance(u, lambda v: v) < 0.03
    assert ks_distance(u, lambda v: v**2) > 0.2
    assert ks_two_sample(u, rng.uniform(size=5000)) < 0.04
