"""The register-resident kernel at every padded row length it is built for
(lda = 32 .. 256, one template per 32 columns), against the general kernel.

Both kernels draw the same directions and theta and evaluate the chord
exactly in FP64 in the same order, so their trajectories must be bitwise
equal however their screening products round.  The resident kernel reads A
from the packed operand copy made at problem setup (one layout per row
length) and screens with its own product-form test, so this covers both for
every template.  Row lengths are ragged (n not a multiple of 32); the walk
counts leave a partial last tile of 16 walks; odd templates run with one
workgroup per walk tile, even ones with rows split over several workgroups
that exchange chord ends."""
import numpy as np
import pytest

from paper_2104_07097_amd import instances as inst

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def _case(nk):
    n = 32 * nk - 3
    m = 300 if nk % 2 else 1100 + 40 * nk   # m_pad <= 512: one workgroup; above: split
    return inst.randpoly(n=n, m=m, z=37, seed=100 + nk)


def _run(p, prec, path, steps):
    _, ch = gu.make(p, prec, recompute_every=6, path=path)
    ch.step(steps)
    X, st = gu.state(ch)
    return X, st, ch.stats()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("nk", range(1, 9))
def test_resident_equals_general_every_row_length(nk, prec):
    p = _case(nk)
    gu.announce("resident vs general", f"n={p.A.shape[1]}", f"m={p.A.shape[0]}", prec)
    Xr, sr, stats = _run(p, prec, "resident", 25)
    assert stats["kernel"] == 2
    assert (stats["split"] > 1) == (nk % 2 == 0)
    Xg, sg, _ = _run(p, prec, "general", 25)
    assert not sr.any() and not sg.any()
    assert np.array_equal(Xr, Xg)
    assert gu.feasible(p, Xr)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_resident_equals_general_with_equalities(prec):
    p = inst.simplex_cut(n=60, m_extra=700, m_eq_extra=2, z=37, seed=120)
    gu.announce("resident vs general, equalities", prec)
    Xr, sr, stats = _run(p, prec, "resident", 25)
    assert stats["kernel"] == 2
    Xg, sg, _ = _run(p, prec, "general", 25)
    assert not sr.any() and not sg.any()
    assert np.array_equal(Xr, Xg)
    assert gu.feasible(p, Xr)


def test_resident_at_its_largest_shape():
    """n = 256 and m = 8192: the longest rows and the widest split (16
    co-resident workgroups per walk tile) the resident kernel takes."""
    p = inst.randpoly(n=256, m=8192, z=20, seed=130)
    gu.announce("resident largest shape")
    Xr, sr, stats = _run(p, "bf16x3", "resident", 12)
    assert stats["kernel"] == 2 and stats["split"] == 16
    Xg, sg, _ = _run(p, "bf16x3", "general", 12)
    assert not sr.any() and not sg.any()
    assert np.array_equal(Xr, Xg)


def test_resident_rejects_more_rows():
    from paper_2104_07097_amd import mhar
    p = inst.randpoly(n=40, m=8193, z=4, seed=131)
    gu.announce("resident m=8193")
    with pytest.raises(mhar.MharError) as ei:
        gu.make(p, "fp32", path="resident")
    assert ei.value.code == mhar.E_UNSUPPORTED
