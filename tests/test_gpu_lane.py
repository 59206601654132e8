"""The lane path (a group of lanes per walk, every row evaluated exactly
each step) against the general kernel and the oracle.

It draws the same directions (the projection's A_eq h summed in the order of
the other paths' wave reduction) and evaluates every row with the same
sequential FP64 formula the other paths use for their candidate rows; the
chord ends of a walk's lanes are combined by an exact minimum.  So its
trajectories must be bitwise those of the general kernel.  Shapes cover each
register template (n <= 8, 16, 32), both group sizes (4 lanes per walk
for n <= 8 and with equalities above 16, 8 otherwise), the variant for
33..64 coordinates that keeps x and d in LDS, equality constraints, and walk
counts that leave a partial last wave."""
import numpy as np
import pytest
import torch

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def cases():
    rng = np.random.default_rng(77)
    cube_start = rng.uniform(-0.5, 0.5, size=(70, 15))
    return {
        "cube3": inst.hypercube(3, 70),
        "cube15": inst.hypercube(15, 70, cube_start),
        "simplex5": inst.simplex(5, 70),
        "simplex15": inst.simplex(15, 130),
        "randpoly20": inst.randpoly(n=20, m=45, z=70, seed=71),
        "cube32": inst.hypercube(32, 70),
        "simplex_cut30": inst.simplex_cut(n=30, m_extra=12, m_eq_extra=2, z=70, seed=72),
        # rows of 33..64 coordinates: the variant with x, d and the draws in LDS
        "cube40": inst.hypercube(40, 70, rng.uniform(-0.5, 0.5, size=(70, 40))),
        "simplex50": inst.simplex(50, 45),
        "simplex_cut64": inst.simplex_cut(n=64, m_extra=30, m_eq_extra=3, z=70, seed=75),
    }


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("case", list(cases()))
def test_lane_equals_general_bitwise(case):
    p = cases()[case]
    gu.announce("lane vs general", case)
    _, a = gu.make(p, "fp64", recompute_every=9, path="lane")
    _, b = gu.make(p, "fp64", recompute_every=9, path="general")
    for k in (1, 12, 40):
        a.step(k)
        b.step(k)
    Xa, sa = gu.state(a)
    Xb, sb = gu.state(b)
    assert a.stats()["kernel"] == 4 and b.stats()["kernel"] == 1
    assert not sa.any() and not sb.any()
    assert np.array_equal(Xa, Xb)
    ra = a.record(20, 3, 16).cpu().numpy()
    rb = b.record(20, 3, 16).cpu().numpy()
    assert np.array_equal(ra, rb)
    assert gu.feasible(p, Xa)


@pytest.mark.parametrize("case", ["cube15", "simplex15", "simplex_cut30"])
def test_lane_short_horizon_parity(orc, case):
    p = cases()[case]
    P = gu.oracle_projection(orc, p)
    gu.announce("lane 30-step", case)
    _, ch = gu.make(p, "fp32", path="lane")
    ch.step(30)
    got, gst = gu.state(ch)
    want, st, _ = orc.run(p.A, p.b, p.X0, 30, seed=0, P=P)
    err = gu.rel_err(got, want)
    print(f"  rel err after 30 steps {err:.2e}", flush=True)
    assert not gst.any() and not st.any()
    assert err <= 1e-8, (case, err)


def test_lane_stats_and_auto_choice():
    p = cases()["cube3"]
    gu.announce("lane stats")
    _, ch = gu.make(p, "fp32")            # AUTO: n = 3, m = 6 takes the lane path
    ch.step(25)
    s = ch.stats()
    assert s["kernel"] == 4
    assert s["exact_rows"] == 6 * 70 * 25
    big = inst.randpoly(n=40, m=300, z=20, seed=73)
    _, ch2 = gu.make(big, "fp32")         # n > 32: not the lane path
    ch2.step(2)
    assert ch2.stats()["kernel"] != 4


@pytest.mark.parametrize("n,m", [(65, 80), (64, 400)])
def test_lane_rejects_large_shapes(n, m):
    """n above 64, or n above 32 with A too large for the LDS of the wide variant."""
    p = inst.randpoly(n=n, m=m, z=4, seed=74)
    gu.announce("lane", f"n={n}", f"m={m}")
    with pytest.raises(mhar.MharError) as ei:
        gu.make(p, "fp32", path="lane")
    assert ei.value.code == mhar.E_UNSUPPORTED


def test_lane_handle_in_batch_and_after():
    """A lane handle stepped inside a batch (general kernel, whose slack it
    must first recompute) and then alone again follows the trajectory of a
    handle that only ever ran the general kernel."""
    p = cases()["simplex15"]
    gu.announce("lane handle in a batch")
    _, a = gu.make(p, "fp32", path="lane")
    _, b = gu.make(p, "fp32", path="general")
    a.step(7)
    b.step(7)
    bat = mhar.Batch([a])
    bat.step(11)
    bat.close()
    b.step(11)
    a.step(5)
    b.step(5)
    Xa, sa = gu.state(a)
    Xb, sb = gu.state(b)
    assert not sa.any() and not sb.any()
    assert np.array_equal(Xa, Xb)
    assert a.stats()["kernel"] == 4


def test_lane_handle_with_covariance_and_state_reset():
    """A learned covariance on a lane handle moves it to the general kernel
    (which first recomputes the slack the lane path does not keep); detached,
    it returns to the lane path; a new state set on it is stepped like any
    other.  At every stage the trajectory is bitwise that of a handle that
    only ever ran the general kernel."""
    p = cases()["randpoly20"]
    dev = gu.device()
    gu.announce("lane handle, covariance and state reset")
    _, a = gu.make(p, "fp32", path="lane")
    _, b = gu.make(p, "fp32", path="general")
    for ch in (a, b):
        ch.step(5)
    rng = np.random.default_rng(3)
    U = torch.tensor(0.05 * rng.standard_normal((p.A.shape[1], 2)), device=dev)
    ls = torch.tensor(np.full(p.A.shape[1], np.log(0.9)), device=dev)
    for ch in (a, b):
        ch.precond_create(2)
        ch.precond_set(U, ls)
        ch.precond_freeze()
        ch.step(9)
    Xa, sa = gu.state(a)
    Xb, sb = gu.state(b)
    assert a.stats()["kernel"] == 1
    assert not sa.any() and not sb.any()
    assert np.array_equal(Xa, Xb)
    for ch in (a, b):
        ch.precond_destroy()
        ch.step(6)
    Xa, _ = gu.state(a)
    Xb, _ = gu.state(b)
    assert a.stats()["kernel"] == 4
    assert np.array_equal(Xa, Xb)
    X = torch.tensor(p.X0, device=dev)
    for ch in (a, b):
        ch.set_state(X, 100)
        ch.step(4)
    Xa, sa = gu.state(a)
    Xb, sb = gu.state(b)
    assert not sa.any() and not sb.any()
    assert np.array_equal(Xa, Xb)
