"""Walks started at the Chebyshev centre (S4.2, Model CCHC) on the device path.

The centre is the one-time host-side linear programme of
paper_2104_07097_amd.start (pinned by closed forms in test_start.py); the
walks then run on the GPU.  On the random polytope (n = 100, m = 2000,
1024 walks) and on the cut simplex (n = 500, 5 equalities, 5500 rows,
4096 walks): the library's interior check accepts the centre, one step
matches the oracle on sampled walks, and every walk stays feasible over
a short run."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar
from paper_2104_07097_amd.start import chebyshev_center, start_points

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return Oracle()


@pytest.mark.parametrize("name,prec", [("randpoly", "fp32"), ("randpoly", "bf16x3"),
                                       ("simplex_cut", "bf16x3")])
def test_walks_from_chebyshev_centre(orc, name, prec):
    p = inst.randpoly() if name == "randpoly" else inst.simplex_cut()
    gu.announce("chebyshev start", name, prec, "n", p.n, "m", p.m, "z", p.z)
    x, r = chebyshev_center(p.A, p.b, p.A_eq, p.b_eq)
    assert r > 0.0
    X0 = start_points(p.A, p.b, p.z, p.A_eq, p.b_eq) if name == "randpoly" else np.tile(x, (p.z, 1))
    # the interior check runs inside chain creation and raises if it fails
    _, ch = gu.make(p, prec, X0=X0)
    assert ch.sync() == 0
    ch.step(1)
    got, st = gu.state(ch)
    assert not st.any()
    P = gu.oracle_projection(orc, p)
    for k in np.random.default_rng(4).choice(p.z, size=24, replace=False):
        want, wst, _ = orc.run(p.A, p.b, X0[k:k + 1], 1, seed=0, chain_offset=int(k), P=P)
        assert not wst.any()
        err = gu.rel_err(got[k:k + 1], want)
        assert err <= 1e-11, (k, err)
    ch.step(30)
    got, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, got)


def test_centre_is_interior_on_device_but_point_past_a_facet_is_not():
    """The same check rejects a start just past a facet: the centre moved
    along the normal of its nearest row to (1 + 1e-9) times that row's slack."""
    p = inst.randpoly(n=20, m=80, z=4, seed=3)
    x, r = chebyshev_center(p.A, p.b)
    s = p.b - p.A @ x
    i = int(np.argmin(s / np.linalg.norm(p.A, axis=1)))
    edge = x + (1.0 + 1e-9) * (s[i] / np.dot(p.A[i], p.A[i])) * p.A[i]
    assert p.b[i] - p.A[i] @ edge < 0.0
    X0 = np.tile(x, (p.z, 1))
    gu.announce("chebyshev interior check")
    _, ch = gu.make(p, "fp64", X0=X0)
    assert ch.sync() == 0
    X0[2] = edge
    with pytest.raises(mhar.MharError) as ei:
        gu.make(p, "fp64", X0=X0)
    assert ei.value.code == mhar.E_NOT_INTERIOR
