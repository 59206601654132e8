"""Statistical pins for the oracle's MHAR iteration (Alg. 2): the target law.

Fixed from outside the oracle by closed-form uniform laws:
  * stationarity: chains started at exact uniform draws (cube: U(-1,1)^n;
    simplex: Dirichlet(1)) stay uniform after k steps;
  * hypercube n = 10 (16 chains from the origin, 10,000 steps): thinned
    marginals are U(-1, 1);
  * simplex from its centre: marginals are Beta(1, n-1);
  * 2-D triangle: two-sample KS against rejection sampling from its box;
  * every iterate feasible (A x <= b, |A_E x - b_E| <= 1e-9), flags clear.
Seeds are fixed, so every check is deterministic."""
import numpy as np
import pytest
from scipy import stats

from paper_2104_07097_amd import instances as inst


def _proj(oracle, p):
    if p.A_eq is None:
        return None
    rc, P = oracle.projection(p.n, p.A_eq)
    assert rc == 0
    return P


def _assert_feasible(p, X):
    assert np.all(X @ p.A.T <= p.b + 1e-12 * np.maximum(1.0, np.abs(p.b)))
    if p.A_eq is not None:
        assert np.abs(X @ p.A_eq.T - p.b_eq).max() <= 1e-9


def test_cube_stationary_from_exact_start(oracle):
    rng = np.random.default_rng(20)
    n, z = 5, 3000
    p = inst.hypercube(n, z, inst.exact_cube(rng, z, n))
    X, st, _ = oracle.run(p.A, p.b, p.X0, 25, seed=4)
    assert not st.any()
    _assert_feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.uniform(-1, 2).cdf).pvalue > 1e-3


def test_simplex_stationary_from_exact_start(oracle):
    rng = np.random.default_rng(21)
    n, z = 7, 3000
    p = inst.simplex(n, z, inst.exact_simplex(rng, z, n))
    X, st, _ = oracle.run(p.A, p.b, p.X0, 25, seed=5, P=_proj(oracle, p))
    assert not st.any()
    _assert_feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.beta(1, n - 1).cdf).pvalue > 1e-3


def test_cube10_marginals(oracle):
    p = inst.cube10(16)
    X, st, rec = oracle.run(p.A, p.b, p.X0, 10000, seed=0, rec_stride=50, rec_chains=16)
    assert not st.any()
    _assert_feasible(p, X)
    samples = rec[20:].reshape(-1, 10)  # drop 1000 burn-in steps
    _assert_feasible(p, samples)
    for j in range(10):
        # thinned HAR draws are mildly correlated: bound the KS distance
        d = stats.kstest(samples[:, j], stats.uniform(-1, 2).cdf).statistic
        assert d < 0.06, (j, d)


@pytest.mark.parametrize("n", [5, 10])
def test_simplex_from_centre(oracle, n):
    z = 2000
    p = inst.simplex(n, z)
    X, st, _ = oracle.run(p.A, p.b, p.X0, 400, seed=6, P=_proj(oracle, p))
    assert not st.any()
    _assert_feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.beta(1, n - 1).cdf).pvalue > 1e-3


def test_triangle_vs_rejection(oracle):
    z = 4000
    p = inst.triangle(z)
    X, st, _ = oracle.run(p.A, p.b, p.X0, 200, seed=8)
    assert not st.any()
    _assert_feasible(p, X)
    ref = inst.exact_by_rejection(np.random.default_rng(9), p.A, p.b, [0, 0], [2, 1], z)
    dirs = [np.array([1.0, 0.0]), np.array([0.0, 1.0]), np.array([0.6, 0.8]),
            np.array([0.8, -0.6]), np.array([-0.28, 0.96])]
    for v in dirs:
        assert stats.ks_2samp(X @ v, ref @ v).pvalue > 1e-3


def test_simplex_cut_small_feasible(oracle):
    # a reduced copy of the non-full-dimensional workload: all iterates stay feasible
    p = inst.simplex_cut(n=30, m_extra=200, m_eq_extra=3, z=64)
    assert oracle.check_interior(p.A, p.b, p.X0, p.A_eq, p.b_eq) == 0
    X, st, rec = oracle.run(p.A, p.b, p.X0, 300, seed=1, P=_proj(oracle, p), rec_stride=1,
                            rec_chains=64)
    assert not st.any()
    _assert_feasible(p, rec.reshape(-1, p.n))


def test_interior_check(oracle):
    p = inst.hypercube(3, 2)
    assert oracle.check_interior(p.A, p.b, p.X0) == 0
    X = p.X0.copy()
    X[1, 2] = 1.0  # on a facet
    assert oracle.check_interior(p.A, p.b, X) == -4
    q = inst.simplex(4, 1)
    bad = np.array([[0.2, 0.2, 0.2, 0.3]])  # sum != 1
    assert oracle.check_interior(q.A, q.b, bad, q.A_eq, q.b_eq) == -4


def test_chain_offset_and_resume(oracle):
    p = inst.randpoly(n=8, m=40, z=6, seed=3)
    full, _, _ = oracle.run(p.A, p.b, p.X0, 30, seed=2)
    a, _, _ = oracle.run(p.A, p.b, p.X0[:3], 30, seed=2)
    b, _, _ = oracle.run(p.A, p.b, p.X0[3:], 30, seed=2, chain_offset=3)
    assert np.array_equal(full, np.vstack([a, b]))
    half, _, _ = oracle.run(p.A, p.b, p.X0, 12, seed=2)
    rest, _, _ = oracle.run(p.A, p.b, half, 18, seed=2, step0=12)
    assert np.array_equal(full, rest)
