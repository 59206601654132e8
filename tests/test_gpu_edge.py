"""Edge cases and invariants of the HIP path (through the C ABI)."""
import numpy as np
import pytest
import torch

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_chain_split_and_determinism(prec):
    p = inst.randpoly(n=20, m=150, z=40, seed=3)
    gu.announce("chain split", prec)
    _, ch = gu.make(p, prec)
    ch.step(25)
    full, _ = gu.state(ch)
    _, ch2 = gu.make(p, prec)
    ch2.step(25)
    again, _ = gu.state(ch2)
    assert np.array_equal(full, again)  # bitwise run to run
    pa = inst.randpoly(n=20, m=150, z=17, seed=3)
    _, ca = gu.make(pa, prec)
    ca.step(25)
    a, _ = gu.state(ca)
    pb = inst.randpoly(n=20, m=150, z=23, seed=3)
    _, cb = gu.make(pb, prec, chain_offset=17)
    cb.step(25)
    b, _ = gu.state(cb)
    assert np.array_equal(full, np.vstack([a, b]))  # global chain ids in the counter


def test_resume_is_bitwise():
    p = inst.randpoly(n=12, m=90, z=20, seed=4)
    gu.announce("resume")
    _, ch = gu.make(p, "fp32", recompute_every=10)
    ch.step(40)
    full, _ = gu.state(ch)
    _, c2 = gu.make(p, "fp32", recompute_every=10)
    c2.step(20)
    mid, _ = gu.state(c2)
    _, c3 = gu.make(p, "fp32", recompute_every=10)
    c3.set_state(torch.tensor(mid, device=gu.device()), 20)
    c3.step(20)
    resumed, _ = gu.state(c3)
    assert np.array_equal(full, resumed)


def test_single_walk_and_interval():
    orc = Oracle()
    A = np.array([[1.0], [-1.0]])
    b = np.array([7.5, -2.0])
    p = inst.Polytope("interval", A, b, np.array([[6.9]]))
    gu.announce("interval z=1")
    for prec in ("fp64", "fp32", "bf16x3"):
        _, ch = gu.make(p, prec)
        ch.step(200)
        got, st = gu.state(ch)
        want, _, _ = orc.run(A, b, p.X0, 200, seed=0)
        assert not st.any()
        assert abs(got[0, 0] - want[0, 0]) <= 1e-12


def test_unbounded_flag():
    A = np.array([[1.0]])
    b = np.array([1.0])
    p = inst.Polytope("halfline", A, b, np.zeros((3, 1)))
    gu.announce("unbounded")
    _, ch = gu.make(p, "fp32")
    ch.step(5)
    X, st = gu.state(ch)
    assert np.all(st & mhar.CHAIN_UNBOUNDED)
    assert np.all(X == 0.0)
    assert ch.sync() & mhar.CHAIN_UNBOUNDED


def test_not_interior_and_rank_deficient():
    dev = gu.device()
    p = inst.hypercube(3, 2)
    X0 = p.X0.copy()
    X0[1, 2] = 1.0
    gu.announce("not interior")
    with pytest.raises(mhar.MharError) as ei:
        gu.make(p, "fp32", X0=X0)
    assert ei.value.code == mhar.E_NOT_INTERIOR
    q = inst.simplex(6, 2)
    A_eq = np.vstack([q.A_eq, 2 * q.A_eq])
    with pytest.raises(mhar.MharError) as ei:
        mhar.Problem(torch.tensor(q.A, device=dev), torch.tensor(q.b, device=dev),
                     torch.tensor(A_eq, device=dev), torch.tensor([1.0, 2.0], device=dev))
    assert ei.value.code == mhar.E_RANK_DEFICIENT
    bad = q.X0.copy()
    bad[0, 0] += 1e-6  # off the equality plane
    with pytest.raises(mhar.MharError) as ei:
        gu.make(q, "fp32", X0=bad)
    assert ei.value.code == mhar.E_NOT_INTERIOR


def test_record_matches_steps():
    orc = Oracle()
    p = inst.randpoly(n=9, m=60, z=20, seed=5)
    gu.announce("record")
    _, ch = gu.make(p, "fp64")
    rec = ch.record(40, 4, 7).cpu().numpy()
    assert rec.shape == (10, 7, 9)
    _, _, want = orc.run(p.A, p.b, p.X0, 40, seed=0, rec_stride=4, rec_chains=7)
    assert gu.rel_err(rec, want) <= 1e-9
    assert ch.step_count() == 40
    ch.step(0)
    assert ch.step_count() == 40
    s = ch.stats()
    assert s["steps"] == 40 and s["chain_steps"] == 800 and s["exact_rows"] > 0


def test_largest_n():
    orc = Oracle()
    p = inst.randpoly(n=1152, m=1300, z=18, seed=6)
    gu.announce("n=1152")
    for prec in ("fp32", "bf16x3", "fp64"):
        _, ch = gu.make(p, prec, recompute_every=3)
        ch.step(4)
        got, st = gu.state(ch)
        want, _, _ = orc.run(p.A, p.b, p.X0, 4, seed=0)
        assert not st.any()
        assert gu.rel_err(got, want) <= 1e-9, prec


@pytest.mark.parametrize("path", ["auto", "general", "tiled", "lane"])
def test_nan_inputs_rejected(path):
    """A NaN in A, b or a start point makes that walk's start slack NaN, which
    the interior check rejects on every kernel path."""
    dev = gu.device()
    base = inst.randpoly(n=12, m=50, z=5, seed=9)
    cases = []
    A = base.A.copy()
    A[3, 4] = np.nan
    cases.append((A, base.b, base.X0))
    b = base.b.copy()
    b[7] = np.nan
    cases.append((base.A, b, base.X0))
    X0 = base.X0.copy()
    X0[2, 1] = np.nan
    cases.append((base.A, base.b, X0))
    gu.announce("nan inputs", path)
    for A_, b_, X_ in cases:
        prob = mhar.Problem(torch.tensor(A_, device=dev), torch.tensor(b_, device=dev),
                            precision="fp32", path=path)
        with pytest.raises(mhar.MharError) as ei:
            mhar.Chains(prob, torch.tensor(X_, device=dev))
        assert ei.value.code == mhar.E_NOT_INTERIOR


def test_unbounded_flag_tiled():
    # the half-line x <= 1: every line through a start point is unbounded below
    A = np.array([[1.0]])
    b = np.array([1.0])
    p = inst.Polytope("halfline", A, b, np.zeros((20, 1)))
    gu.announce("unbounded tiled")
    _, ch = gu.make(p, "bf16x3", path="tiled")
    ch.step(3)
    X, st = gu.state(ch)
    assert np.all(st & mhar.CHAIN_UNBOUNDED)
    assert np.all(X == 0.0)


@pytest.mark.parametrize("path,prec", [("tiled", "bf16x3"), ("general", "fp64")])
def test_repeated_facets_overflow_the_candidate_lists(path, prec):
    """Every facet of the cube [-1,1]^n written k times: the copies of a facet
    tie, so each walk has at least 2k exact candidate rows and a 16-walk tile
    more than 32k, past the staged batch of 96 candidates and the tile's list
    of 512 (the rest is evaluated where it is found); the copies of a facet
    lie in every 64-row group, so the tile also flags more (walk, group)
    pairs than its list of 512 holds.  One step and five steps must still
    be the oracle's, and every walk must evaluate its 2k tied rows."""
    n, k, z = 40, 48, 32
    eye = np.eye(n)
    A = np.vstack([np.tile(eye, (k, 1)), np.tile(-eye, (k, 1))])
    X0 = np.random.default_rng(9).uniform(-0.5, 0.5, size=(z, n))
    p = inst.Polytope("repeated_cube", A, np.ones(2 * n * k), X0)
    orc = Oracle()
    gu.announce("repeated facets", path, prec, "m", p.m)
    _, ch = gu.make(p, prec, recompute_every=4, path=path)
    ch.step(1)
    got, st = gu.state(ch)
    want, wst, _ = orc.run(p.A, p.b, X0, 1, seed=0)
    assert not st.any() and not wst.any()
    assert gu.rel_err(got, want) <= 1e-11
    assert ch.stats()["exact_rows"] >= 2 * k * z
    ch.step(4)
    got5, st = gu.state(ch)
    want5, _, _ = orc.run(p.A, p.b, X0, 5, seed=0)
    assert not st.any()
    assert gu.rel_err(got5, want5) <= 1e-10
    assert gu.feasible(p, got5)
