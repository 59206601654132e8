"""Pins for the host-side statistics: the ESS estimator against closed forms,
the Friedman-Rafsky statistic against its null distribution (simulation) and
against clearly different laws."""
import numpy as np

from paper_2104_07097_amd.stats import (ess, friedman_rafsky, ks_distance, ks_two_sample,
                                        split_rhat)


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


def test_friedman_rafsky_null_is_standard_normal():
    # equal laws: z over 200 independent replicates has mean ~0 and sd ~1
    rng = np.random.default_rng(5)
    zs = [friedman_rafsky(rng.uniform(-1, 1, (60, 3)), rng.uniform(-1, 1, (80, 3)))[1]
          for _ in range(200)]
    assert abs(np.mean(zs)) < 0.25
    assert 0.75 < np.std(zs) < 1.25


def test_friedman_rafsky_detects_different_laws():
    rng = np.random.default_rng(6)
    x = rng.uniform(-1, 1, (300, 5))
    shifted = rng.uniform(-1, 1, (300, 5)) + np.array([0.8, 0, 0, 0, 0])
    squeezed = rng.uniform(-0.7, 0.7, (300, 5))
    assert friedman_rafsky(x, shifted)[1] < -4.0
    assert friedman_rafsky(x, squeezed)[1] < -4.0


def test_friedman_rafsky_runs_by_hand():
    # 1-D points: the MST is the sorted chain, so R - 1 counts label changes
    x = np.array([[0.0], [1.0], [2.0]])
    y = np.array([[0.5], [5.0]])
    R, _ = friedman_rafsky(x, y)
    assert R == 1 + 3   # order 0(x) .5(y) 1(x) 2(x) 5(y): changes x-y, y-x, x-y


def test_split_rhat():
    rng = np.random.default_rng(9)
    # i.i.d. chains: R-hat within sampling error of 1
    assert abs(split_rhat(rng.standard_normal((8, 4000))) - 1.0) < 0.01
    # chains stuck at different levels: between-half variance dominates
    stuck = rng.standard_normal((8, 4000)) * 0.1 + np.arange(8)[:, None]
    assert split_rhat(stuck) > 5.0
    # a trend within each chain shows up through the split halves
    trend = rng.standard_normal((8, 4000)) * 0.1 + np.linspace(0, 3, 4000)[None, :]
    assert split_rhat(trend) > 2.0
    # closed form for two halves of constant levels a, b with within variance s^2:
    # W = s^2, B/n = var(levels, ddof=1) -> R = sqrt(((n-1)/n s^2 + B/n) / s^2)
    x = np.concatenate([np.full(1000, 0.0), np.full(1000, 1.0)])[None, :]
    x = x + np.tile([-0.5, 0.5], 1000)[None, :]   # within-half variance 0.25 (ddof=1: 0.25025)
    w = np.var(np.tile([-0.5, 0.5], 500), ddof=1)
    want = np.sqrt((999.0 / 1000.0 * w + 0.5) / w)
    assert abs(split_rhat(x) - want) < 1e-12
