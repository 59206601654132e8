"""Pins for the oracle's direction-covariance fit to the Dikin ellipsoid.

The fit targets the log-barrier Hessian H at the mean walk state; its
objective K = 1/2 tr(H Sigma) - 1/2 log det Sigma is the Kullback-Leibler
divergence of N(0, Sigma) from N(0, H^{-1}) up to a constant.  Fixed from
outside the oracle by: second differences of the log-barrier (H), the
closed-form minimum K(H^{-1}) = n/2 + 1/2 log det H with the determinant
from numpy and Gibbs' inequality around it, central finite differences of K
(gradient), the axis box at its centre (H = diag(8/l^2) in closed form), and
for a rotated box the closed-form optimum of K over U given the diagonal,
from numpy's symmetric eigensolver."""
import numpy as np
import pytest

from oracle import E_NOT_INTERIOR, OK


def _randpoly(n=5, m=14, seed=0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A, np.ones(m)


def _barrier(A, b, x):
    return -np.sum(np.log(b - A @ x))


def test_hessian_is_barrier_second_difference(oracle):
    A, b = _randpoly()
    rng = np.random.default_rng(1)
    X = 0.2 * rng.standard_normal((7, A.shape[1]))
    rc, xbar, H = oracle.dikin_hessian(A, b, X)
    assert rc == OK
    assert np.abs(xbar - X.mean(axis=0)).max() <= 1e-15
    n, h = A.shape[1], 1e-4
    E = np.eye(n) * h
    fd = np.empty((n, n))
    for p in range(n):
        for q in range(n):
            fd[p, q] = (_barrier(A, b, xbar + E[p] + E[q]) - _barrier(A, b, xbar + E[p] - E[q])
                        - _barrier(A, b, xbar - E[p] + E[q]) + _barrier(A, b, xbar - E[p] - E[q])) / (4 * h * h)
    assert np.abs(fd - H).max() <= 1e-5 * np.abs(H).max()


def test_hessian_rejects_mean_outside(oracle):
    A = np.vstack([np.eye(2), -np.eye(2)])
    b = np.ones(4)
    X = np.array([[1.5, 0.0], [0.9, 0.0]])   # mean (1.2, 0) violates x_0 <= 1
    rc, _, _ = oracle.dikin_hessian(A, b, X)
    assert rc == E_NOT_INTERIOR


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    return M @ M.T + n * np.eye(n)


def test_objective_minimum_is_closed_form(oracle):
    n = 5
    H = _spd(n, 2)
    target = np.linalg.inv(H)
    d = 0.1 * np.linalg.eigvalsh(target).min()
    ls = np.full(n, 0.5 * np.log(d))
    U = np.linalg.cholesky(target - d * np.eye(n))      # U U^T + d I = H^{-1}, rank n
    K, gU, gl = oracle.dikin_objective(U, ls, H)
    want = 0.5 * n + 0.5 * np.linalg.slogdet(H)[1]
    assert abs(K - want) <= 1e-12 * max(1.0, abs(want))
    assert np.abs(gU).max() <= 1e-10 and np.abs(gl).max() <= 1e-10
    # Gibbs: any other Sigma of the family lies above the minimum
    rng = np.random.default_rng(3)
    for _ in range(5):
        U2 = U + 0.05 * rng.standard_normal(U.shape)
        ls2 = ls + 0.1 * rng.standard_normal(n)
        assert oracle.dikin_objective(U2, ls2, H)[0] > want


def test_objective_gradient_finite_differences(oracle):
    n, r = 6, 2
    H = _spd(n, 4)
    rng = np.random.default_rng(5)
    U = 0.3 * rng.standard_normal((n, r))
    ls = 0.2 * rng.standard_normal(n)
    _, gU, gl = oracle.dikin_objective(U, ls, H)
    h = 1e-6
    for (i, a) in [(0, 0), (3, 1), (5, 0), (2, 1)]:
        Up, Um = U.copy(), U.copy()
        Up[i, a] += h
        Um[i, a] -= h
        fd = (oracle.dikin_objective(Up, ls, H)[0] - oracle.dikin_objective(Um, ls, H)[0]) / (2 * h)
        assert abs(fd - gU[i, a]) <= 1e-6 * max(1.0, abs(fd))
    for i in range(n):
        lp, lm = ls.copy(), ls.copy()
        lp[i] += h
        lm[i] -= h
        fd = (oracle.dikin_objective(U, lp, H)[0] - oracle.dikin_objective(U, lm, H)[0]) / (2 * h)
        assert abs(fd - gl[i]) <= 1e-6 * max(1.0, abs(fd))


def test_train_step_axis_box_closed_form(oracle):
    # box |x_i| <= l_i / 2 at its centre: H = diag(8 / l^2) exactly, the
    # Jacobi-scaled Hessian is the identity (lam = 1), and the inscribed
    # diagonal is the Dikin ellipsoid itself: exp(2 l_i) = l_i^2 / 8
    sides = np.array([0.1, 1.0, 3.0, 0.02])
    n = sides.size
    A = np.vstack([np.eye(n), -np.eye(n)])
    b = np.concatenate([sides / 2, sides / 2])
    X = np.zeros((3, n))
    rc, _, H = oracle.dikin_hessian(A, b, X)
    assert rc == OK and np.allclose(H, np.diag(8 / sides**2), rtol=1e-15, atol=0)
    U = 0.01 * np.random.default_rng(6).standard_normal((n, 2))
    v = np.ones(n)
    U1, ls, v1, lam = oracle.dikin_train_step(A, b, X, U, v, k_pow=3)
    assert abs(lam - 1.0) <= 1e-14
    assert np.abs(np.exp(2 * ls) - sides**2 / 8).max() <= 1e-15 * (sides**2).max()
    # with Sigma's diagonal already the whole Dikin ellipsoid, the optimum of U
    # is 0: every step lowers K and shrinks U
    K_prev = oracle.dikin_objective(U, ls, H)[0]
    prev = np.abs(U).sum()
    for _ in range(5):
        K_now = oracle.dikin_objective(U1, ls, H)[0]
        assert K_now < K_prev and np.abs(U1).sum() < prev
        K_prev, prev = K_now, np.abs(U1).sum()
        U1, ls, v1, lam = oracle.dikin_train_step(A, b, X, U1, v1, k_pow=3)


def _rotated_box(n, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    Q = Q * np.sign(np.diag(R))
    sides = np.exp(rng.uniform(np.log(1e-2), 0.0, n))
    A = np.vstack([Q.T, -Q.T])
    b = np.concatenate([sides / 2, sides / 2])
    return A, b, Q, sides


@pytest.mark.parametrize("n,r,kappa", [(8, 2, 1.0), (10, 3, 0.3)])
def test_train_step_reaches_closed_form_optimum(oracle, n, r, kappa):
    A, b, Q, sides = _rotated_box(n, 7 + n)
    X = np.zeros((4, n))
    rc, _, H = oracle.dikin_hessian(A, b, X)
    assert rc == OK
    U = 0.01 * np.random.default_rng(8).standard_normal((n, r))
    v = np.random.default_rng(9).standard_normal(n)
    for _ in range(200):
        U, ls, v, lam = oracle.dikin_train_step(A, b, X, U, v, k_pow=4, kappa=kappa)
    Dh = np.sqrt(np.diag(H))
    J = H / np.outer(Dh, Dh)
    lam_max = np.linalg.eigvalsh(J)[-1]
    assert abs(lam - lam_max) <= 1e-9 * lam_max
    D = np.exp(2 * ls)
    assert np.abs(D - kappa**2 / (lam_max * np.diag(H))).max() <= 1e-9 * D.max()
    # the diagonal part is inside the Dikin ellipsoid: D^1/2 H D^1/2 <= kappa^2 I
    Ht = np.sqrt(D)[:, None] * H * np.sqrt(D)[None, :]
    nu, V = np.linalg.eigh(Ht)
    assert nu[-1] <= kappa**2 * (1 + 1e-9)
    # optimum of K over U given D: in D^{-1/2} coordinates the columns span the
    # r eigenvectors of D^1/2 H D^1/2 with the least eigenvalues nu, squared
    # norms 1/nu - 1
    Ut = V[:, :r] * np.sqrt(1.0 / nu[:r] - 1.0)
    want = np.sqrt(D)[:, None] * (Ut @ Ut.T) * np.sqrt(D)[None, :]
    assert np.abs(U @ U.T - want).max() <= 1e-8 * np.abs(want).max()
