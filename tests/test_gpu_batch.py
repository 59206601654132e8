"""Batched persistent launches over problems of uneven n and m."""
import numpy as np
import pytest

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def _problems():
    return [inst.randpoly(n=20, m=120, z=32, seed=41),
            inst.randpoly(n=50, m=700, z=48, seed=42),
            inst.simplex_cut(n=25, m_extra=150, m_eq_extra=2, z=20, seed=43),
            inst.cube10(16),
            inst.rotbox(n=40, m_extra=160, z=20, seed=44)[0],
            inst.randpoly(n=140, m=2500, z=64, seed=45)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp64"])
def test_batch_equals_individual_runs(prec):
    probs = _problems()
    gu.announce("batch", prec)
    singles = []
    for p in probs:
        _, ch = gu.make(p, prec)
        ch.step(30)
        singles.append(gu.state(ch)[0])
    made = [gu.make(p, prec) for p in probs]
    batch = mhar.Batch([ch for _, ch in made])
    batch.step(12)
    batch.step(18)
    for (prob, ch), want, p in zip(made, singles, probs):
        got, st = gu.state(ch)
        assert not st.any()
        assert np.array_equal(got, want), p.name
        assert ch.step_count() == 30
    # after the batch is gone, the handles keep stepping on their own kernels
    batch.close()
    _, ch = made[1]
    ch.step(5)
    orc = Oracle()
    p = probs[1]
    want, _, _ = orc.run(p.A, p.b, p.X0, 35, seed=0)
    got, _ = gu.state(ch)
    assert gu.rel_err(got, want) <= 1e-8


def test_batch_rejects_mixed_precision():
    p = inst.cube10(16)
    _, a = gu.make(p, "fp32")
    _, b = gu.make(p, "bf16x3")
    gu.announce("batch mixed")
    with pytest.raises(mhar.MharError) as ei:
        mhar.Batch([a, b])
    assert ei.value.code == mhar.E_INVALID_ARG


def _mixed_problems():
    # the first runs the tiled path on its own, the next two the resident kernel
    # (tiled inside a batch), the fourth the resident kernel and the last the
    # lane path (both the general kernel inside a batch)
    return [inst.randpoly(n=300, m=1200, z=200, seed=51),
            inst.simplex_cut(n=150, m_extra=2000, m_eq_extra=3, z=150, seed=52),
            inst.rotbox(n=200, m_extra=1500, z=100, seed=53)[0],
            inst.randpoly(n=30, m=200, z=40, seed=54),
            inst.cube10(16)]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_grouped_tiled_batch_equals_individual_runs(prec):
    """Large problems of a batch run grouped tiled launches (one table of tiles
    over all of them), small ones the persistent general kernel.  Handles are
    stepped apart first by different amounts, so their recompute schedules
    (R = 7) are out of phase inside the batch; the result must be bitwise that
    of stepping each handle alone."""
    probs = _mixed_problems()
    offsets = [0, 3, 5, 1, 2]
    gu.announce("grouped batch", prec)
    singles = []
    for p, off in zip(probs, offsets):
        _, ch = gu.make(p, prec, recompute_every=7)
        ch.step(off + 30)
        singles.append(gu.state(ch)[0])
    made = [gu.make(p, prec, recompute_every=7) for p in probs]
    for (_, ch), off in zip(made, offsets):
        if off:
            ch.step(off)
    batch = mhar.Batch([ch for _, ch in made])
    # inside the batch the three large problems run the grouped tiled path
    assert [ch.stats()["kernel"] for _, ch in made] == [3, 3, 3, 1, 1]
    batch.step(13)
    batch.step(17)
    for (_, ch), want, p in zip(made, singles, probs):
        got, st = gu.state(ch)
        assert not st.any(), p.name
        assert np.array_equal(got, want), p.name
    batch.close()
