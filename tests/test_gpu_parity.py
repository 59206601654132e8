"""Parity of the HIP path against the FP64 CPU oracle (through the C ABI).

The HAR map is chaotic: a 1e-15 perturbation of a state grows to ~1e-12
after 100 steps and to O(1) after ~1000 (measured on the oracle itself).
Parity is therefore checked
  * per step: from the same state (taken from the oracle), one GPU step and
    one oracle step agree to 1e-11 (relative, max over walks/coordinates);
  * over 100 steps from the start: agree to within twice the oracle's own
    sensitivity to one-ulp perturbations of every state (computed per case on
    the CPU: 8e-15 to 1.1e-10 on these cases), since the GPU's states differ
    from the oracle's only by ulps of log, sin and cos in the directions;
in every product precision, since the chord is always evaluated exactly in
FP64.  Long runs are judged statistically (test_gpu_stats.py)."""
import numpy as np
import pytest

from oracle import Oracle

from . import gpu_util as gu

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "bf16x3"]


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["cube10", "randpoly", "simplex_cut", "rotbox", "split3", "split3_xcd"])
def test_one_step_parity(orc, case, prec):
    p = gu.small_cases()[case]
    P = gu.oracle_projection(orc, p)
    gu.announce("one-step", case, prec)
    prob, ch = gu.make(p, prec, recompute_every=5)
    X = p.X0
    for t in (0, 7, 23):
        Xt, st, _ = orc.run(p.A, p.b, p.X0, t, seed=0, P=P)
        want, st1, _ = orc.run(p.A, p.b, Xt, 1, seed=0, P=P, step0=t)
        ch.set_state(__import__("torch").tensor(Xt, device=gu.device()), t)
        ch.step(1)
        got, gst = gu.state(ch)
        assert not gst.any() and not st1.any()
        err = gu.rel_err(got, want)
        print(f"  t={t} rel err {err:.2e}", flush=True)
        assert err <= 1e-11, (case, prec, t, err)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["cube10", "randpoly", "simplex_cut", "rotbox", "split3", "split3_xcd"])
def test_short_horizon_parity(orc, case, prec):
    p = gu.small_cases()[case]
    P = gu.oracle_projection(orc, p)
    gu.announce("100-step", case, prec)
    prob, ch = gu.make(p, prec, recompute_every=7)
    ch.step(100)
    got, gst = gu.state(ch)
    want, st, _ = orc.run(p.A, p.b, p.X0, 100, seed=0, P=P)
    err = gu.rel_err(got, want)
    tol = max(1e-13, 2.0 * gu.ulp_sensitivity(orc, p, 100, P=P))
    print(f"  rel err after 100 steps {err:.2e} (bound {tol:.2e})", flush=True)
    assert not gst.any()
    assert err <= tol, (case, prec, err, tol)
    assert gu.feasible(p, got)


def test_projection_matches_oracle(orc):
    p = gu.small_cases()["simplex_cut"]
    gu.announce("projection")
    prob, ch = gu.make(p, "fp32")
    got = prob.projection().cpu().numpy()
    rc, want = orc.projection(p.n, p.A_eq)
    assert rc == 0
    assert np.abs(got - want).max() <= 1e-13


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_bench_size_sampled_parity(orc, prec):
    """The benchmark workload at full size (n=100, m=2000, z=1024): one step from
    a mid-run state, checked on a sample of 96 walks computed by the oracle one
    by one, plus feasibility of every walk."""
    import torch
    from paper_2104_07097_amd import instances as inst
    p = inst.randpoly()
    gu.announce("bench-size", prec)
    prob, ch = gu.make(p, prec, recompute_every=50)
    ch.step(60)
    Xt, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, Xt)
    ch.set_state(torch.tensor(Xt, device=gu.device()), 60)
    ch.step(1)
    got, st = gu.state(ch)
    sample = np.random.default_rng(0).choice(p.z, size=96, replace=False)
    for k in sample:
        want, _, _ = orc.run(p.A, p.b, Xt[k:k + 1], 1, seed=0, chain_offset=int(k), step0=60)
        err = gu.rel_err(got[k:k + 1], want)
        assert err <= 1e-11, (k, err)
    assert gu.feasible(p, got)
