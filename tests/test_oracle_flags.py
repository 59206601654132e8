"""Pins for the oracle's boundary and failure branches, from what the line-set
definition (S4.4, Lemma 4.2) and the readings of the silent points fix:

  * a walk on a facet (slack exactly 0): the chord end on that side is 0, the
    walk moves only inwards, no flag;
  * rounding below a facet (slack in [-1e-12, 0)): clamped to 0, no flag;
  * a walk past a facet (slack below -1e-12 max(1, |b_i|)): INFEASIBLE, the
    slack clamped to 0 for the chord;
  * a walk at a vertex with a direction leaving through two facets: both
    chord ends are 0 (lambda_max <= lambda_min), DEGENERATE, the walk stays;
  * a NaN coordinate: every slack b_i - a_i x is NaN (0 x NaN is NaN in
    IEEE arithmetic), NaN ratios bound nothing, so the walk is UNBOUNDED
    with theta = 0 and NONFINITE, and stays where it is."""
import numpy as np

from oracle import (CHAIN_DEGENERATE, CHAIN_INFEASIBLE, CHAIN_NONFINITE, CHAIN_UNBOUNDED,
                    TAG_DIR)


def _cube(n=3):
    return np.vstack([np.eye(n), -np.eye(n)]), np.ones(2 * n)


def test_facet_chord_end_is_zero(oracle):
    A, b = _cube()
    x = np.array([1.0, 0.2, -0.3])
    lo, hi, fl = oracle.chord(A, b, x, np.array([0.5, 0.1, 0.2]))
    assert fl == 0 and hi == 0.0 and lo < 0.0
    # leaving the facet inwards: that side's end is 2 / 0.5 away, the facet is behind
    lo, hi, fl = oracle.chord(A, b, x, np.array([-0.5, 0.1, 0.2]))
    assert fl == 0 and lo == 0.0 and hi > 0.0 and abs(hi - min(2.0 / 0.5, 0.8 / 0.1, 1.3 / 0.2)) < 1e-15


def test_rounding_below_facet_is_clamped(oracle):
    A, b = _cube()
    x = np.array([1.0 + 1e-13, 0.0, 0.0])
    lo, hi, fl = oracle.chord(A, b, x, np.array([1.0, 0.3, -0.2]))
    assert fl == 0 and hi == 0.0


def test_past_facet_is_infeasible_and_clamped(oracle):
    A, b = _cube()
    x = np.array([1.0 + 1e-9, 0.0, 0.0])
    lo, hi, fl = oracle.chord(A, b, x, np.array([1.0, 0.3, -0.2]))
    assert fl == CHAIN_INFEASIBLE and hi == 0.0
    # the tolerance is relative to |b_i| above 1
    A1, b1 = np.array([[1.0], [-1.0]]), np.array([1e4, 1e4])
    _, _, fl = oracle.chord(A1, b1, np.array([1e4 + 5e-9]), np.array([1.0]))
    assert fl == 0
    _, _, fl = oracle.chord(A1, b1, np.array([1e4 + 2e-8]), np.array([1.0]))
    assert fl == CHAIN_INFEASIBLE


def test_vertex_leaving_through_two_facets_is_degenerate(oracle):
    A, b = _cube()
    x = np.ones(3)
    lo, hi, fl = oracle.chord(A, b, x, np.array([1.0, -1.0, 0.5]))
    assert fl == 0 and hi == 0.0 and lo == 0.0
    # one step of the sampler from the vertex: walks whose direction has
    # mixed signs are DEGENERATE and stay; the others move inwards
    z = 12
    X, st, _ = oracle.run(A, b, np.tile(x, (z, 1)), 1, seed=3)
    for k in range(z):
        d = np.array([oracle.gauss(3, TAG_DIR, k, 0, j) for j in range(3)])
        if (d > 0).any() and (d < 0).any():
            assert st[k] == CHAIN_DEGENERATE and np.array_equal(X[k], x)
        else:
            assert st[k] == 0 and np.all(X[k] < 1.0)


def test_nan_coordinate_is_nonfinite(oracle):
    A, b = _cube()
    X = np.array([[np.nan, 0.0, 0.0], [0.1, 0.2, 0.3]])
    Xn, st, _ = oracle.run(A, b, X, 1, seed=0)
    assert st[0] == CHAIN_NONFINITE | CHAIN_UNBOUNDED
    assert np.isnan(Xn[0, 0]) and np.array_equal(Xn[0, 1:], X[0, 1:])
    lo, hi, fl = oracle.chord(A, b, X[0], np.array([0.3, 0.2, -0.1]))
    assert (lo, hi, fl) == (-np.inf, np.inf, CHAIN_UNBOUNDED)
    assert st[1] == 0 and np.isfinite(Xn[1]).all()
