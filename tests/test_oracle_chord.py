"""Pins for the oracle's line sets and sample choice (paper S4.4 Lemma 4.2,
S4.5 Lemma 4.3).

Fixed from outside the oracle by:
  * the n = 1 worked example: on [l, u] one step lands at l + U (u - l) when
    d > 0 and at u - U (u - l) when d < 0, whatever the start;
  * the hypercube closed form lambda_max = min_j (sgn d_j - x_j)/d_j,
    lambda_min = max_j (-sgn d_j - x_j)/d_j;
  * brute force: the chord ends found by bisection on feasibility of x + t d
    for random small polytopes;
  * the UNBOUNDED flag on an open polyhedron."""
import numpy as np
import pytest

from oracle import CHAIN_UNBOUNDED, TAG_DIR, TAG_THETA


@pytest.mark.parametrize("l,u,x0", [(-1.0, 1.0, 0.0), (2.0, 7.5, 6.9), (-3.0, -2.0, -2.999)])
def test_interval_worked_example(oracle, l, u, x0):
    A = np.array([[1.0], [-1.0]])
    b = np.array([u, -l])
    seed = 9
    for step in range(200):
        X, status, _ = oracle.run(A, b, np.array([[x0]]), 1, seed=seed, step0=step)
        d = oracle.gauss(seed, TAG_DIR, 0, step, 0)
        U = oracle.uniform(seed, TAG_THETA, 0, step, 0, 0)
        want = l + U * (u - l) if d > 0 else u - U * (u - l)
        assert status[0] == 0
        assert abs(X[0, 0] - want) <= 4e-16 * (abs(l) + abs(u) + abs(x0)) + 1e-300


def test_hypercube_closed_form(oracle):
    rng = np.random.default_rng(1)
    for n in (1, 2, 7, 30):
        A = np.vstack([np.eye(n), -np.eye(n)])
        b = np.ones(2 * n)
        for _ in range(50):
            x = rng.uniform(-1, 1, n)
            d = rng.standard_normal(n)
            lo, hi, fl = oracle.chord(A, b, x, d)
            assert fl == 0
            want_hi = np.min((np.sign(d) - x) / d)
            want_lo = np.max((-np.sign(d) - x) / d)
            assert abs(hi - want_hi) <= 1e-15 * max(1, abs(want_hi))
            assert abs(lo - want_lo) <= 1e-15 * max(1, abs(want_lo))


def _feasible(A, b, y):
    return np.all(A @ y <= b)


def _bisect_end(A, b, x, d, sign):
    t_in, t_out = 0.0, 1.0
    while _feasible(A, b, x + sign * t_out * d):
        t_out *= 2.0
    for _ in range(200):
        mid = 0.5 * (t_in + t_out)
        if _feasible(A, b, x + sign * mid * d):
            t_in = mid
        else:
            t_out = mid
    return sign * t_in


def test_bisection_brute_force(oracle):
    rng = np.random.default_rng(2)
    for trial in range(60):
        n = int(rng.integers(1, 6))
        m_extra = int(rng.integers(1, 10))
        A = np.vstack([np.eye(n), -np.eye(n), rng.standard_normal((m_extra, n))])
        b = np.concatenate([np.full(2 * n, 2.0), rng.uniform(0.5, 2.0, m_extra)])
        x = rng.uniform(-0.1, 0.1, n)
        assert _feasible(A, b, x)
        d = rng.standard_normal(n)
        lo, hi, fl = oracle.chord(A, b, x, d)
        assert fl == 0
        assert abs(hi - _bisect_end(A, b, x, d, +1.0)) <= 1e-12 * max(1.0, abs(hi))
        assert abs(lo - _bisect_end(A, b, x, d, -1.0)) <= 1e-12 * max(1.0, abs(lo))


def test_unbounded_flag(oracle):
    # x <= 1 only: no row bounds the walk from below along +d
    A = np.array([[1.0, 0.0], [0.0, 1.0]])
    b = np.array([1.0, 1.0])
    lo, hi, fl = oracle.chord(A, b, np.zeros(2), np.array([1.0, 0.5]))
    assert fl & CHAIN_UNBOUNDED
    # half-line x <= 1 in one dimension: every direction leaves one side open
    X, status, _ = oracle.run(np.array([[1.0]]), np.array([1.0]), np.zeros((3, 1)), 5)
    assert np.all(status & CHAIN_UNBOUNDED)
    assert np.all(X == 0.0)
