"""Checkpoint and restore of the chain and training state (mhar_checkpoint /
mhar_restore): continuing from a restored handle must give bitwise the
states and covariance of an uninterrupted run, for plain walks, for a
covariance trained by Adam on the states, and for the Dikin fit on the tiled
path; mismatched handles and truncated buffers are refused."""
import numpy as np
import pytest
import torch

from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_plain_walks_resume_bitwise():
    p = inst.randpoly(n=24, m=200, z=40, seed=71)
    gu.announce("checkpoint plain")
    _, a = gu.make(p, "fp32", recompute_every=9, seed=5)
    a.step(23)
    blob = a.checkpoint()
    a.step(31)
    want, wst = gu.state(a)
    _, b = gu.make(p, "fp32", recompute_every=9, seed=5)
    b.restore(blob)
    assert b.step_count() == 23
    b.step(31)
    got, gst = gu.state(b)
    assert np.array_equal(got, want) and np.array_equal(gst, wst)


def test_status_bits_survive():
    A = np.array([[1.0]])
    b = np.array([1.0])
    p = inst.Polytope("halfline", A, b, np.zeros((4, 1)))
    gu.announce("checkpoint status bits")
    _, a = gu.make(p, "fp64", path="general")
    a.step(2)
    blob = a.checkpoint()
    _, c = gu.make(p, "fp64", path="general")
    c.restore(blob)
    _, st = gu.state(c)
    assert np.all(st == mhar.CHAIN_UNBOUNDED)


@pytest.mark.parametrize("objective,prec,path,lr", [("states", "fp32", "general", 0.05),
                                                    ("dikin", "bf16x3", "tiled", 0.5)])
def test_training_resumes_bitwise(objective, prec, path, lr):
    p = inst.rotbox(n=40, m_extra=240, z=70, seed=72)[0]
    r = 6
    gu.announce("checkpoint training", objective)
    _, a = gu.make(p, prec, path=path, recompute_every=7, seed=2)
    a.precond_create(r, objective)
    a.precond_train(9, lr)
    blob = a.checkpoint()
    a.precond_train(8, lr)
    a.precond_freeze()
    a.step(12)
    want, _ = gu.state(a)
    wU, wl = (t.cpu().numpy() for t in a.precond_get())
    _, b = gu.make(p, prec, path=path, recompute_every=7, seed=2)
    b.precond_create(r, objective)
    b.restore(blob)
    b.precond_train(8, lr)
    b.precond_freeze()
    b.step(12)
    got, _ = gu.state(b)
    gU, gl = (t.cpu().numpy() for t in b.precond_get())
    assert np.array_equal(gU, wU) and np.array_equal(gl, wl)
    assert np.array_equal(got, want)
    # the frozen flag travels with the checkpoint
    frozen = b.checkpoint()
    _, c = gu.make(p, prec, path=path, recompute_every=7, seed=2)
    c.precond_create(r, objective)
    c.restore(frozen)
    with pytest.raises(mhar.MharError) as ei:
        c.precond_train(1, lr)
    assert ei.value.code == mhar.E_STATE


def test_mismatches_are_refused():
    p = inst.randpoly(n=10, m=40, z=16, seed=73)
    gu.announce("checkpoint refusals")
    _, a = gu.make(p, "fp32", seed=1)
    a.step(3)
    blob = a.checkpoint()
    _, other_seed = gu.make(p, "fp32", seed=2)
    with pytest.raises(mhar.MharError) as ei:
        other_seed.restore(blob)
    assert ei.value.code == mhar.E_STATE
    _, with_cov = gu.make(p, "fp32", seed=1)
    with_cov.precond_create(3)
    with pytest.raises(mhar.MharError) as ei:
        with_cov.restore(blob)
    assert ei.value.code == mhar.E_STATE
    q = inst.randpoly(n=10, m=40, z=17, seed=73)
    _, other_z = gu.make(q, "fp32", seed=1)
    with pytest.raises(mhar.MharError) as ei:
        other_z.restore(blob)
    assert ei.value.code == mhar.E_SHAPE
    _, fresh = gu.make(p, "fp32", seed=1)
    with pytest.raises(mhar.MharError) as ei:
        fresh.restore(blob[:-8])
    assert ei.value.code == mhar.E_INVALID_ARG
