"""The Chebyshev-centre start (the paper's Model CCHC) against closed forms."""
import math

import numpy as np
import pytest

from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd.start import chebyshev_center, start_points


def test_hypercube_centre_and_radius():
    p = inst.hypercube(7, 1)
    x, r = chebyshev_center(p.A, p.b)
    assert np.abs(x).max() <= 1e-9 and abs(r - 1.0) <= 1e-9


def test_shifted_scaled_box():
    # box [lo, hi] with one short side: the radius is half the shortest side
    lo, hi = np.array([0.0, 2.0, -1.0]), np.array([4.0, 2.5, 3.0])
    A = np.vstack([np.eye(3), -np.eye(3)])
    b = np.concatenate([hi, -lo])
    x, r = chebyshev_center(A, b)
    assert abs(r - 0.25) <= 1e-9
    assert abs(x[1] - 2.25) <= 1e-9
    assert np.all(x >= lo + r - 1e-9) and np.all(x <= hi - r + 1e-9)


def test_simplex_with_equality():
    # the paper's model on {x >= 0, sum x = 1}: x_i >= r and sum x = 1 give
    # x = 1/n, r = 1/n
    n = 6
    p = inst.simplex(n, 1)
    x, r = chebyshev_center(p.A, p.b, p.A_eq, p.b_eq)
    assert np.abs(x - 1.0 / n).max() <= 1e-9 and abs(r - 1.0 / n) <= 1e-9


def test_triangle_incircle():
    # incentre = (a A + b B + c C) / (a + b + c) with a, b, c the side lengths
    # opposite the vertices; inradius = area / semiperimeter
    P = np.array([[0.0, 0.0], [2.0, 0.0], [2.0 / 7.0, 8.0 / 7.0]])
    a = np.linalg.norm(P[1] - P[2])
    b = np.linalg.norm(P[0] - P[2])
    c = np.linalg.norm(P[0] - P[1])
    centre = (a * P[0] + b * P[1] + c * P[2]) / (a + b + c)
    u, v = P[1] - P[0], P[2] - P[0]
    area = 0.5 * abs(u[0] * v[1] - u[1] * v[0])
    t = inst.triangle(1)
    x, r = chebyshev_center(t.A, t.b)
    assert np.abs(x - centre).max() <= 1e-9
    assert abs(r - area / ((a + b + c) / 2)) <= 1e-9


def test_errors_and_start_points():
    with pytest.raises(ValueError):
        chebyshev_center(np.array([[1.0, 0.0]]), np.array([1.0]))        # unbounded
    with pytest.raises(ValueError):
        chebyshev_center(np.array([[1.0], [-1.0]]), np.array([0.0, 0.0]))  # a single point
    X = start_points(*(lambda p: (p.A, p.b))(inst.hypercube(3, 1)), z=5)
    assert X.shape == (5, 3) and np.abs(X).max() <= 1e-9
    assert math.isfinite(chebyshev_center(inst.randpoly(n=20, m=80, z=1, seed=3).A, np.ones(80))[1])
