"""The tiled path (screening GEMM over 256-row x 128-walk tiles, chords kernel,
FP64 recompute GEMM) against the FP64 oracle, and against the single-kernel
path.

Both paths evaluate the chord exactly in FP64 with the same code and draw the
same directions and theta, so their trajectories must be bitwise equal even
though their screening products round differently.  The shapes span several
row and walk tiles with ragged tails (m_pad not a multiple of 256, z_pad not a
multiple of 128)."""
import numpy as np
import pytest
import torch

from oracle import Oracle
from paper_2104_07097_amd import instances as inst

from . import gpu_util as gu

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16x3"]


def cases():
    return {
        "blocks": inst.randpoly(n=33, m=600, z=150, seed=41),
        "simplex_cut": inst.simplex_cut(n=30, m_extra=200, m_eq_extra=3, z=40, seed=12),
        "rotbox": inst.rotbox(n=40, m_extra=200, z=33, seed=13)[0],
        "wide": inst.randpoly(n=200, m=700, z=20, seed=42),
    }


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["blocks", "simplex_cut", "rotbox", "wide"])
def test_tiled_one_step_parity(orc, case, prec):
    p = cases()[case]
    P = gu.oracle_projection(orc, p)
    gu.announce("tiled one-step", case, prec)
    prob, ch = gu.make(p, prec, recompute_every=5, path="tiled")
    assert ch.stats()["kernel"] == 3
    for t in (0, 7, 23):
        Xt, _, _ = orc.run(p.A, p.b, p.X0, t, seed=0, P=P)
        want, st1, _ = orc.run(p.A, p.b, Xt, 1, seed=0, P=P, step0=t)
        ch.set_state(torch.tensor(Xt, device=gu.device()), t)
        ch.step(1)
        got, gst = gu.state(ch)
        assert not gst.any() and not st1.any()
        err = gu.rel_err(got, want)
        print(f"  t={t} rel err {err:.2e}", flush=True)
        assert err <= 1e-11, (case, prec, t, err)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["blocks", "simplex_cut", "rotbox", "wide"])
def test_tiled_short_horizon_parity(orc, case, prec):
    p = cases()[case]
    P = gu.oracle_projection(orc, p)
    gu.announce("tiled 100-step", case, prec)
    prob, ch = gu.make(p, prec, recompute_every=7, path="tiled")
    ch.step(100)
    got, gst = gu.state(ch)
    want, _, _ = orc.run(p.A, p.b, p.X0, 100, seed=0, P=P)
    err = gu.rel_err(got, want)
    tol = max(1e-13, 2.0 * gu.ulp_sensitivity(orc, p, 100, P=P))
    print(f"  rel err after 100 steps {err:.2e} (bound {tol:.2e})", flush=True)
    assert not gst.any()
    assert err <= tol, (case, prec, err, tol)
    assert gu.feasible(p, got)


@pytest.mark.parametrize("prec", PRECS)
def test_tiled_equals_general_bitwise(prec):
    p = cases()["blocks"]
    gu.announce("tiled vs general", prec)
    _, a = gu.make(p, prec, recompute_every=9, path="tiled")
    _, b = gu.make(p, prec, recompute_every=9, path="general")
    for k in (1, 13, 50):
        a.step(k)
        b.step(k)
    Xa, sa = gu.state(a)
    Xb, sb = gu.state(b)
    assert not sa.any() and not sb.any()
    assert np.array_equal(Xa, Xb)
    # recorded trajectories (every step) agree too
    ra = a.record(20, 1, 16).cpu().numpy()
    rb = b.record(20, 1, 16).cpu().numpy()
    assert np.array_equal(ra, rb)


def test_tiled_precisions_agree_bitwise():
    p = cases()["wide"]
    gu.announce("tiled fp32 vs bf16x3")
    _, a = gu.make(p, "fp32", recompute_every=11, path="tiled")
    _, b = gu.make(p, "bf16x3", recompute_every=11, path="tiled")
    a.step(77)
    b.step(77)
    Xa, _ = gu.state(a)
    Xb, _ = gu.state(b)
    assert np.array_equal(Xa, Xb)


def test_tiled_learned_covariance_step(orc):
    p = inst.rotbox(n=30, m_extra=300, z=40, seed=22)[0]
    n, r = 30, 5
    gu.announce("tiled precond step")
    _, ch = gu.make(p, "bf16x3", path="tiled")
    ch.precond_create(r)
    rng = np.random.default_rng(4)
    U, ls = 0.3 * rng.standard_normal((n, r)), 0.2 * rng.standard_normal(n)
    dev = gu.device()
    ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    Xt, _, _ = orc.run(p.A, p.b, p.X0, 11, seed=0, U=U, log_sigma=ls)
    want, st, _ = orc.run(p.A, p.b, Xt, 1, seed=0, step0=11, U=U, log_sigma=ls)
    ch.set_state(torch.tensor(Xt, device=dev), 11)
    ch.step(1)
    got, gst = gu.state(ch)
    assert not gst.any() and not st.any()
    assert gu.rel_err(got, want) <= 1e-11


def test_tiled_full_size_sampled_parity(orc):
    """The simplex-with-equalities workload at full size (n=500, m=5500 with 5
    equalities, z=4096) on the tiled path: one step from a mid-run state,
    checked on 48 walks computed by the oracle one by one, plus feasibility
    of every walk."""
    p = inst.simplex_cut()
    P = gu.oracle_projection(orc, p)
    gu.announce("tiled full-size simplex_cut")
    _, ch = gu.make(p, "bf16x3", recompute_every=50)
    assert ch.stats()["kernel"] == 3
    ch.step(40)
    Xt, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, Xt)
    ch.set_state(torch.tensor(Xt, device=gu.device()), 40)
    ch.step(1)
    got, st = gu.state(ch)
    assert not st.any()
    sample = np.random.default_rng(1).choice(p.z, size=48, replace=False)
    for k in sample:
        want, _, _ = orc.run(p.A, p.b, Xt[k:k + 1], 1, seed=0, P=P, chain_offset=int(k), step0=40)
        err = gu.rel_err(got[k:k + 1], want)
        assert err <= 1e-11, (k, err)
    assert gu.feasible(p, got)


@pytest.mark.parametrize("fig", ["simplex", "hypercube"])
def test_tiled_large_n_parity(orc, fig):
    """n = 1500 (beyond the single-kernel paths' 1152): the tiled path is chosen
    automatically; one step from a mid-run state against the oracle on every
    walk, and 12 steps from the start."""
    n, z = 1500, 24
    p = inst.simplex(n, z) if fig == "simplex" else inst.hypercube(n, z)
    P = gu.oracle_projection(orc, p)
    gu.announce("tiled large n", fig)
    _, ch = gu.make(p, "bf16x3", recompute_every=5)
    assert ch.stats()["kernel"] == 3
    ch.step(12)
    got12, st = gu.state(ch)
    want12, _, _ = orc.run(p.A, p.b, p.X0, 12, seed=0, P=P)
    assert not st.any()
    assert gu.rel_err(got12, want12) <= 1e-9
    ch.set_state(torch.tensor(want12, device=gu.device()), 12)
    ch.step(1)
    got, st = gu.state(ch)
    want, _, _ = orc.run(p.A, p.b, want12, 1, seed=0, P=P, step0=12)
    assert not st.any()
    assert gu.rel_err(got, want) <= 1e-11
    assert gu.feasible(p, got)
