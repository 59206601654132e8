"""Pins for the oracle's direction-covariance fit (learned preconditioner).

Fixed from outside the oracle by: scipy's multivariate normal log-density
(NLL = -mean log N(x_k; mean, Sigma) - n/2 log 2 pi), the diagonal closed
form when U = 0, central finite differences of the NLL for the gradient,
and the closed-form first two Adam steps.  The burn-in update in the
scale-free coordinates V = diag(exp(-l)) U is pinned by finite differences of
NLL(diag(exp(l)) V, l) and by its equivariance under a rescaling of the
states."""
import math

import numpy as np
from scipy import stats


def _problem(n=6, r=2, z=9, seed=0):
    rng = np.random.default_rng(seed)
    U = 0.3 * rng.standard_normal((n, r))
    ls = 0.2 * rng.standard_normal(n)
    X = rng.standard_normal((z, n)) * rng.uniform(0.5, 2.0, n)
    return U, ls, X


def test_nll_matches_scipy(oracle):
    U, ls, X = _problem()
    nll, _, _ = oracle.precond_nll(U, ls, X)
    Sig = U @ U.T + np.diag(np.exp(2 * ls))
    lp = stats.multivariate_normal(X.mean(axis=0), Sig).logpdf(X).mean()
    n = X.shape[1]
    assert abs(nll - (-lp - 0.5 * n * math.log(2 * math.pi))) <= 1e-12 * max(1, abs(nll))


def test_nll_diagonal_closed_form(oracle):
    _, ls, X = _problem()
    U = np.zeros((X.shape[1], 1))
    nll, gU, gl = oracle.precond_nll(U, ls, X)
    S = np.cov(X.T, bias=True)
    want = ls.sum() + 0.5 * np.sum(np.diag(S) * np.exp(-2 * ls))
    assert abs(nll - want) <= 1e-12 * abs(want)
    # d/dl_i [l_i + S_ii e^{-2 l_i}/2] = 1 - S_ii e^{-2 l_i}
    assert np.abs(gl - (1 - np.diag(S) * np.exp(-2 * ls))).max() <= 1e-12


def test_gradient_finite_differences(oracle):
    U, ls, X = _problem(n=6, r=2, z=5, seed=3)
    _, gU, gl = oracle.precond_nll(U, ls, X)
    h = 1e-6
    for (i, a) in [(0, 0), (3, 1), (5, 0), (2, 1)]:
        Up, Um = U.copy(), U.copy()
        Up[i, a] += h
        Um[i, a] -= h
        fd = (oracle.precond_nll(Up, ls, X)[0] - oracle.precond_nll(Um, ls, X)[0]) / (2 * h)
        assert abs(fd - gU[i, a]) <= 1e-7 * max(1, abs(fd))
    for i in range(6):
        lp, lm = ls.copy(), ls.copy()
        lp[i] += h
        lm[i] -= h
        fd = (oracle.precond_nll(U, lp, X)[0] - oracle.precond_nll(U, lm, X)[0]) / (2 * h)
        assert abs(fd - gl[i]) <= 1e-7 * max(1, abs(fd))


def test_adam_closed_form(oracle):
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m1 = np.zeros(3)
    m2 = np.zeros(3)
    lr, eps = 0.01, 1e-8
    p1, m1, m2 = oracle.adam(p, g, m1, m2, 1, lr, eps=eps)
    # step 1: bias-corrected moments are g and g^2
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    g2 = np.array([-0.1, 1.0, 2e-3])
    p2, _, _ = oracle.adam(p1, g2, m1, m2, 2, lr, eps=eps)
    mm = (0.9 * 0.1 * g + 0.1 * g2) / (1 - 0.81)
    vv = (0.999 * 0.001 * g * g + 0.001 * g2 * g2) / (1 - 0.999**2)
    assert np.allclose(p2, p1 - lr * mm / (np.sqrt(vv) + eps), rtol=0, atol=1e-14)


def test_direction_covariance(oracle):
    # preconditioned directions are N(0, U U^T + diag(exp(2 l))), projected by P
    rng = np.random.default_rng(4)
    n, r = 4, 2
    U = rng.standard_normal((n, r))
    ls = rng.uniform(-1, 0.5, n)
    Sig = U @ U.T + np.diag(np.exp(2 * ls))
    D = np.array([oracle.direction(n, 3, k, t, U=U, log_sigma=ls)
                  for k in range(100) for t in range(200)])
    C = D.T @ D / D.shape[0]
    assert np.abs(C - Sig).max() <= 0.04 * np.abs(Sig).max()
    rc, P = oracle.projection(n, np.ones((1, n)))
    Dp = np.array([oracle.direction(n, 3, k, t, P=P, U=U, log_sigma=ls)
                   for k in range(100) for t in range(200)])
    assert np.allclose(Dp, D @ P.T, rtol=0, atol=1e-13)
    # plain directions are N(0, I)
    H = np.array([oracle.direction(n, 5, k, t) for k in range(100) for t in range(200)])
    assert np.abs(H.T @ H / H.shape[0] - np.eye(n)).max() <= 0.04


def _grad_from_step(oracle, V, ls, X):
    """(V, l) gradient read off one Adam step with fresh moments: at t = 1 with
    eps = lr = 1e9 the step is g / (1 + |g| 1e-9), i.e. g to ~1e-9 relative."""
    z0 = (np.zeros_like(V), np.zeros_like(V), np.zeros_like(ls), np.zeros_like(ls))
    V1, l1, _, U1 = oracle.precond_train_step(V, ls, z0, X, 1, 1e9, eps=1e9)
    return V - V1, ls - l1, V1, l1, U1


def test_train_step_gradient_finite_differences(oracle):
    U, ls, X = _problem(n=6, r=2, z=7, seed=5)
    V = U * np.exp(-ls)[:, None]
    gV, gl, V1, l1, U1 = _grad_from_step(oracle, V, ls, X)

    def f(V_, l_):
        return oracle.precond_nll(V_ * np.exp(l_)[:, None], l_, X)[0]
    h = 1e-6
    for (i, a) in [(0, 0), (2, 1), (5, 1), (3, 0)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[i, a] += h
        Vm[i, a] -= h
        fd = (f(Vp, ls) - f(Vm, ls)) / (2 * h)
        assert abs(fd - gV[i, a]) <= 1e-6 * max(1, abs(fd))
    for i in range(6):
        lp, lm = ls.copy(), ls.copy()
        lp[i] += h
        lm[i] -= h
        fd = (f(V, lp) - f(V, lm)) / (2 * h)
        assert abs(fd - gl[i]) <= 1e-6 * max(1, abs(fd))
    # the returned factor is the one the new coordinates define
    assert np.abs(U1 - V1 * np.exp(l1)[:, None]).max() <= 1e-15 * np.abs(U1).max()


def test_train_step_scale_equivariance(oracle):
    # Sigma -> c^2 Sigma for states c X shifts the NLL by a constant, so in the
    # scale-free coordinates the update moves V identically and l by log c.
    U, ls, X = _problem(n=5, r=3, z=8, seed=6)
    V = U * np.exp(-ls)[:, None]
    mom = tuple(0.1 * np.abs(np.random.default_rng(7).standard_normal(a.shape))
                for a in (V, V, ls, ls))
    c = 37.0
    Va, la, ma, _ = oracle.precond_train_step(V, ls, mom, X, 3, 0.05)
    Vb, lb, mb, _ = oracle.precond_train_step(V, ls + math.log(c), mom, c * X, 3, 0.05)
    assert np.abs(Va - Vb).max() <= 1e-12
    assert np.abs((lb - la) - math.log(c)).max() <= 1e-12
    for x, y in zip(ma, mb):
        assert np.abs(x - y).max() <= 1e-12 * max(1.0, np.abs(x).max())
