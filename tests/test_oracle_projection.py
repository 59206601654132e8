"""Pins for the oracle's projection onto null(A_E)  (paper S3.2, Lemma 3.1).

Fixed from outside the oracle by: the closed form for the simplex
(P = I - 1 1^T / n), the defining invariants of an orthogonal projector onto
null(A_E) (symmetric, idempotent, A_E P = 0, trace n - m_E), agreement with
numpy's SVD-based pseudo-inverse projector I - pinv(A_E) A_E, and the
rank-deficiency error for dependent equality rows."""
import numpy as np
import pytest

from oracle import E_RANK_DEFICIENT, OK


def test_simplex_closed_form(oracle):
    for n in (3, 10, 57):
        rc, P = oracle.projection(n, np.ones((1, n)))
        assert rc == OK
        assert np.abs(P - (np.eye(n) - np.ones((n, n)) / n)).max() <= 1e-15


@pytest.mark.parametrize("n,m_eq,seed", [(6, 2, 0), (40, 5, 1), (120, 7, 2)])
def test_projector_invariants(oracle, n, m_eq, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m_eq, n))
    rc, P = oracle.projection(n, A)
    assert rc == OK
    assert np.abs(P - P.T).max() <= 1e-14
    assert np.abs(P @ P - P).max() <= 1e-13
    assert np.abs(A @ P).max() <= 1e-13 * np.abs(A).max() * n
    assert abs(np.trace(P) - (n - m_eq)) <= 1e-12
    ref = np.eye(n) - np.linalg.pinv(A) @ A
    assert np.abs(P - ref).max() <= 1e-13


def test_rank_deficient_rows(oracle):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((3, 8))
    A = np.vstack([A, A[1] * 2.0 - A[0]])  # dependent fourth row
    rc, _ = oracle.projection(8, A)
    assert rc == E_RANK_DEFICIENT


def test_no_equalities_is_identity(oracle):
    rc, P = oracle.projection(5, None)
    assert rc == OK and np.array_equal(P, np.eye(5))
