"""The direction covariance fitted to the Dikin ellipsoid, on the GPU, against
the FP64 oracle (itself pinned in test_oracle_dikin.py).

  * objective K and its gradient at shared states and (U, l), ranks up to 64;
  * the burn-in loop (MHAR step with the current covariance, then one fit
    step: Hessian, power iterations, inscribed diagonal, preconditioned U
    step) against the same loop driven through the oracle;
  * a non-interior mean state is reported by mhar_sync and leaves the
    covariance unchanged;
  * gain on a scaled-down ill-conditioned rotated box: the fitted covariance
    puts its trace on the long axes, and the frozen covariance gives better
    marginals (KS distance to exact samples) and a higher min-marginal ESS
    than isotropic directions for the same number of steps."""
import numpy as np
import pytest
import torch

from oracle import TAG_TRAIN, Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar
from paper_2104_07097_amd.stats import ks_two_sample, min_marginal_ess

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _random_cov(n, r, seed):
    rng = np.random.default_rng(seed)
    return 0.05 * rng.standard_normal((n, r)), np.log(0.05) + 0.2 * rng.standard_normal(n)


@pytest.mark.parametrize("n,r,z,prec", [(12, 3, 40, "fp32"), (70, 16, 300, "bf16x3"),
                                        (100, 64, 64, "fp64"), (150, 13, 200, "fp32")])
def test_objective_and_gradient_parity(orc, n, r, z, prec):
    p = inst.rotbox(n=n, m_extra=4 * n, z=z, seed=31)[0]
    gu.announce("dikin loss", n, r, z, prec)
    _, ch = gu.make(p, prec)
    ch.step(30)
    X, _ = gu.state(ch)
    ch.precond_create(r, "dikin")
    U, ls = _random_cov(n, r, 3)
    dev = gu.device()
    ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    K, gU, gl = ch.precond_loss()
    torch.cuda.synchronize()
    rc, _, H = orc.dikin_hessian(p.A, p.b, X)
    assert rc == 0
    want_K, want_gU, want_gl = orc.dikin_objective(U, ls, H)
    assert abs(K.item() - want_K) <= 1e-9 * max(1.0, abs(want_K))
    assert np.abs(gU.cpu().numpy() - want_gU).max() <= 1e-9 * max(1.0, np.abs(want_gU).max())
    assert np.abs(gl.cpu().numpy() - want_gl).max() <= 1e-9 * max(1.0, np.abs(want_gl).max())
    assert ch.sync() == 0


def _initial_fit(orc, n, r, seed):
    U = np.array([[0.01 * orc.gauss(seed, TAG_TRAIN, j, 0, q) for q in range(r)] for j in range(n)])
    v = np.array([orc.gauss(seed, TAG_TRAIN, j, 1, 0) for j in range(n)])
    return U, v


@pytest.mark.parametrize("n,r,z,prec,path,m_extra,kappa", [(20, 4, 33, "fp32", "general", 60, 1.0),
                                                            (64, 8, 70, "bf16x3", "tiled", 300, 0.1),
                                                            (130, 64, 40, "fp64", "general", 200, 0.3),
                                                            (200, 64, 130, "fp32", "tiled", 800, 0.1)])
def test_training_loop_parity(orc, n, r, z, prec, path, m_extra, kappa):
    p = inst.rotbox(n=n, m_extra=m_extra, z=z, seed=32, side_lo=1e-2)[0]
    steps, eta, seed = 6, 0.5, 0
    gu.announce("dikin train", n, r, z, prec, path, kappa)
    _, ch = gu.make(p, prec, path=path, recompute_every=4, seed=seed)
    ch.precond_create(r, "dikin")
    ch.precond_set_complement(kappa)
    ch.precond_train(steps, eta)
    X_gpu, st = gu.state(ch)
    U_gpu, ls_gpu = (a.cpu().numpy() for a in ch.precond_get())
    assert ch.sync() == 0 and not st.any()
    U, v = _initial_fit(orc, n, r, seed)
    ls = np.zeros(n)
    X = p.X0.copy()
    for t in range(steps):
        X, stat, _ = orc.run(p.A, p.b, X, 1, seed=seed, step0=t, U=U, log_sigma=ls)
        assert not stat.any()
        U, ls, v, lam = orc.dikin_train_step(p.A, p.b, X, U, v, k_pow=4, eta=eta, kappa=kappa)
    assert gu.rel_err(X_gpu, X) <= 1e-9
    assert np.abs(ls_gpu - ls).max() <= 1e-9 * max(1.0, np.abs(ls).max())
    assert np.abs(U_gpu - U).max() <= 1e-8 * np.abs(U).max()


def test_mean_state_outside_is_reported():
    # states whose mean violates a row (set without validation): the fit
    # reports MHAR_FIT_FAILED at mhar_sync, and every later fit step leaves
    # the covariance unchanged until it is set again
    p = inst.hypercube(3, 8)
    gu.announce("dikin bad mean")
    _, ch = gu.make(p, "fp64", path="general")
    ch.precond_create(2, "dikin")
    U0, ls0 = (a.cpu().numpy() for a in ch.precond_get())
    assert ch.sync() == 0
    dev = gu.device()
    ch.set_state(torch.tensor(np.tile([1.5, 0.0, 0.0], (8, 1)), device=dev), 0)
    ch.precond_loss()
    assert ch.sync() & mhar.FIT_FAILED
    ch.set_state(torch.tensor(p.X0, device=dev), 0)
    ch.precond_train(2, 0.5)
    U1, ls1 = (a.cpu().numpy() for a in ch.precond_get())
    assert ch.sync() & mhar.FIT_FAILED
    assert np.array_equal(U1, U0) and np.array_equal(ls1, ls0)
    ch.precond_set(torch.tensor(U0, device=dev), torch.tensor(ls0, device=dev))
    assert ch.sync() & mhar.FIT_FAILED == 0


def _share_on_top_axes(U, ls, Q, sides, r):
    Sig = U @ U.T + np.diag(np.exp(2 * ls))
    top = Q[:, np.argsort(sides)[::-1][:r]]
    return float(np.trace(top.T @ Sig @ top) / np.trace(Sig))


def test_fit_gains_on_rotated_box():
    """Scaled-down rotated box (n = 200, sides log-uniform in [1e-3, 1],
    1600 extra halfspaces, 1024 walks from the centre): 200 burn-in steps of
    the Dikin fit at rank 16, frozen, then 4000 steps recorded every 4th,
    against the same 4200 steps with isotropic directions."""
    n, r, z = 200, 16, 1024
    p, Q, sides = inst.rotbox(n=n, m_extra=8 * n, z=z, seed=33)
    rng = np.random.default_rng(5)
    exact = ((rng.random((20000, n)) - 0.5) * sides) @ Q.T
    out = {}
    for mode in ("plain", "dikin"):
        gu.announce("dikin gain", mode)
        _, ch = gu.make(p, "bf16x3", seed=1)
        if mode == "dikin":
            ch.precond_create(r, "dikin")
            ch.precond_train(200, 0.5)
            ch.precond_freeze()
            U, ls = (a.cpu().numpy() for a in ch.precond_get())
            out["share"] = _share_on_top_axes(U, ls, Q, sides, r)
        else:
            ch.step(200)
        rec = ch.record(4000, 4, 64).cpu().numpy()
        X, st = gu.state(ch)
        assert not st.any() and gu.feasible(p, X)
        cols = np.arange(0, n, 10)
        ess, _ = min_marginal_ess(rec[:, :, cols])
        ks = max(ks_two_sample(X[:, j], exact[:, j]) for j in cols)
        out[mode] = (ess, ks)
        gu.announce("dikin gain", mode, "ess", round(ess, 1), "ks", round(ks, 3))
    # the trace of the fitted covariance sits on the r longest of n axes
    assert out["share"] >= 0.5, out
    assert out["dikin"][1] < 0.8 * out["plain"][1], out
    assert out["dikin"][0] > 1.5 * out["plain"][0], out
