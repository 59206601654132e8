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


def _packed(probs, prec, seed=0, X0s=None):
    import torch
    dev = gu.device()
    t = lambda a: torch.tensor(a, device=dev, dtype=torch.float64)
    X0s = X0s or [p.X0 for p in probs]
    return mhar.PackedBatch.from_lists([t(p.A) for p in probs], [t(p.b) for p in probs],
                                       [t(x) for x in X0s], seed=seed, precision=prec)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32"])
def test_packed_batch_matches_handles_and_oracle(prec):
    """Packed creation (one device array per field, host offsets): 14
    inequality-only problems, n from 20 to 400 with ragged walk counts, some
    on the grouped tiled launches and some on the general kernel.  After 20
    steps every walk equals the handle-built batch whose walk ids continue
    across problems, and sampled walks match the oracle."""
    probs = inst.batched(count=12, z_each=64, seed=46)
    probs.append(inst.randpoly(n=300, m=5000, z=130, seed=47))
    probs.append(inst.randpoly(n=23, m=90, z=17, seed=48))
    gu.announce("packed batch", prec, len(probs), "problems")
    pb = _packed(probs, prec, seed=5)
    pb.step(20)
    base = np.cumsum([0] + [p.z for p in probs])
    made = [gu.make(p, prec, seed=5, chain_offset=int(base[i])) for i, p in enumerate(probs)]
    batch = mhar.Batch([ch for _, ch in made])
    batch.step(20)
    orc = Oracle()
    rng = np.random.default_rng(6)
    for i, p in enumerate(probs):
        got, st = pb.state(i)
        got, st = got.cpu().numpy(), st.cpu().numpy()
        want, wst = gu.state(made[i][1])
        assert not st.any() and np.array_equal(got, want), p.name
        if i % 4 == 0 or i == len(probs) - 1:
            for k in rng.choice(p.z, size=2, replace=False):
                ref, _, _ = orc.run(p.A, p.b, p.X0[k:k + 1], 20, seed=5, chain_offset=int(base[i] + k))
                assert gu.rel_err(got[k:k + 1], ref) <= 1e-9, (p.name, k)
    batch.close()
    pb.close()


def test_packed_batch_rejects_a_start_outside():
    probs = [inst.randpoly(n=20, m=100, z=8, seed=49), inst.randpoly(n=30, m=200, z=8, seed=50)]
    X0s = [probs[0].X0, probs[1].X0.copy()]
    X0s[1][3, 0] = 10.0
    gu.announce("packed batch outside")
    with pytest.raises(mhar.MharError) as ei:
        _packed(probs, "fp32", X0s=X0s)
    assert ei.value.code == mhar.E_NOT_INTERIOR and "problem 1" in str(ei.value)
    # nothing is left behind: the same shapes build cleanly afterwards
    pb = _packed(probs, "fp32")
    pb.step(3)
    assert not pb.state(1)[1].any()
    pb.close()
