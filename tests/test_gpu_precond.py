"""The learned direction covariance on the GPU against the FP64 oracle.

  * NLL and gradient (Woodbury form on the GPU) vs the oracle's dense
    n x n evaluation on the same states (itself pinned by scipy and finite
    differences);
  * one preconditioned step from a shared state vs the oracle (<= 1e-11);
  * the burn-in training loop (step, gradient, Adam) vs the same loop driven
    through the oracle, over 8 steps;
  * target preservation: a frozen random covariance keeps exact-uniform
    starts uniform;
  * gain: on an ill-conditioned rotated box the trained covariance raises the
    min-marginal ESS of the same number of steps."""
import numpy as np
import pytest
import torch
from scipy import stats

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd.stats import min_marginal_ess

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _random_cov(n, r, seed):
    rng = np.random.default_rng(seed)
    return 0.3 * rng.standard_normal((n, r)), 0.2 * rng.standard_normal(n)


@pytest.mark.parametrize("n,r,z", [(12, 3, 40), (70, 16, 300)])
def test_loss_and_gradient_parity(orc, n, r, z):
    p = inst.rotbox(n=n, m_extra=4 * n, z=z, seed=21)[0]
    gu.announce("precond loss", n, r, z)
    _, ch = gu.make(p, "fp32")
    ch.step(40)
    X, _ = gu.state(ch)
    ch.precond_create(r)
    U, ls = _random_cov(n, r, 3)
    dev = gu.device()
    ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    nll, gU, gl = ch.precond_loss()
    torch.cuda.synchronize()
    want_nll, want_gU, want_gl = orc.precond_nll(U, ls, X)
    assert abs(nll.item() - want_nll) <= 1e-10 * max(1.0, abs(want_nll))
    assert np.abs(gU.cpu().numpy() - want_gU).max() <= 1e-10 * max(1.0, np.abs(want_gU).max())
    assert np.abs(gl.cpu().numpy() - want_gl).max() <= 1e-10 * max(1.0, np.abs(want_gl).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_preconditioned_step_parity(orc, prec):
    p = inst.rotbox(n=30, m_extra=120, z=40, seed=22)[0]
    n, r = 30, 5
    gu.announce("precond step", prec)
    _, ch = gu.make(p, prec)
    ch.precond_create(r)
    U, ls = _random_cov(n, r, 4)
    dev = gu.device()
    ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    Xt, _, _ = orc.run(p.A, p.b, p.X0, 11, seed=0, U=U, log_sigma=ls)
    want, st, _ = orc.run(p.A, p.b, Xt, 1, seed=0, step0=11, U=U, log_sigma=ls)
    ch.set_state(torch.tensor(Xt, device=dev), 11)
    ch.step(1)
    got, gst = gu.state(ch)
    assert not gst.any() and not st.any()
    assert gu.rel_err(got, want) <= 1e-11
    # short horizon with the same frozen covariance
    _, ch2 = gu.make(p, prec)
    ch2.precond_create(r)
    ch2.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    ch2.precond_freeze()
    ch2.step(20)
    got2, _ = gu.state(ch2)
    want2, _, _ = orc.run(p.A, p.b, p.X0, 20, seed=0, U=U, log_sigma=ls)
    assert gu.rel_err(got2, want2) <= 1e-8


def test_training_loop_parity(orc):
    p = inst.rotbox(n=16, m_extra=60, z=64, seed=23)[0]
    n, r, lr = 16, 4, 0.05
    gu.announce("precond training")
    _, ch = gu.make(p, "fp32")
    ch.precond_create(r)
    U0, ls0 = (t.cpu().numpy() for t in ch.precond_get())
    assert np.all(ls0 == 0.0) and 0 < np.abs(U0).max() < 0.1
    ch.precond_train(8, lr)
    U_gpu, ls_gpu = (t.cpu().numpy() for t in ch.precond_get())
    X_gpu, st = gu.state(ch)
    # the same loop through the oracle (log scales start at 0, so V = U)
    U, V, ls = U0.copy(), U0.copy(), ls0.copy()
    mom = (np.zeros_like(U), np.zeros_like(U), np.zeros_like(ls), np.zeros_like(ls))
    X = p.X0.copy()
    for t in range(8):
        X, _, _ = orc.run(p.A, p.b, X, 1, seed=0, step0=t, U=U, log_sigma=ls)
        V, ls, mom, U = orc.precond_train_step(V, ls, mom, X, t + 1, lr)
    assert not st.any()
    assert gu.rel_err(X_gpu, X) <= 1e-8
    assert np.abs(U_gpu - U).max() <= 1e-8 and np.abs(ls_gpu - ls).max() <= 1e-8


def test_frozen_covariance_keeps_uniform_target():
    rng = np.random.default_rng(30)
    n, z, r = 5, 3000, 2
    p = inst.hypercube(n, z, inst.exact_cube(rng, z, n))
    gu.announce("precond invariance")
    _, ch = gu.make(p, "fp32")
    ch.precond_create(r)
    U, ls = _random_cov(n, r, 5)
    dev = gu.device()
    ch.precond_set(torch.tensor(3 * U, device=dev), torch.tensor(2 * ls, device=dev))
    ch.precond_freeze()
    ch.step(25)
    X, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.uniform(-1, 2).cdf).pvalue > 1e-3


def test_learned_covariance_raises_ess():
    """Rotated box n=20, sides log-uniform in [1e-2, 1]: 300 burn-in steps
    (training or plain), then 2000 recorded steps of 64 walks each."""
    n = 20
    p = inst.rotbox(n=n, m_extra=40, z=64, seed=24, side_lo=1e-2)[0]
    gu.announce("precond gain")
    _, plain = gu.make(p, "fp32")
    plain.step(300)
    rp = plain.record(2000, 1, 64).cpu().numpy()
    ess_plain, _ = min_marginal_ess(rp)
    _, learned = gu.make(p, "fp32")
    learned.precond_create(8)
    learned.precond_train(300, 0.05)
    learned.precond_freeze()
    rl = learned.record(2000, 1, 64).cpu().numpy()
    ess_learned, _ = min_marginal_ess(rl)
    print(f"  min-marginal ESS plain {ess_plain:.1f}, learned {ess_learned:.1f}", flush=True)
    assert gu.feasible(p, rl.reshape(-1, n))
    assert ess_learned > 2.0 * ess_plain
