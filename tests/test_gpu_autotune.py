"""The native path autotuner (mhar_chains_autotune): it tries every kernel
path a handle can take on the handle's own walks, keeps the fastest, and
the walks stay bitwise those of an untuned twin; a batch of tuned handles
runs each on the path its choice maps to."""
import math

import numpy as np
import pytest
import torch

from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def _tuned_and_twin(p, prec, trial, rank=0, path="auto"):
    _, tuned = gu.make(p, prec, path=path)
    _, twin = gu.make(p, prec, path=path)
    if rank:
        rng = np.random.default_rng(9)
        U = 0.02 * rng.standard_normal((p.n, rank))
        ls = 0.2 * rng.standard_normal(p.n) + math.log(0.05)
        dev = gu.device()
        for ch in (tuned, twin):
            ch.precond_create(rank)
            ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    res = tuned.autotune(trial)
    return tuned, twin, res


@pytest.mark.parametrize("name,prec,rank,path,expect", [
    ("randpoly", "bf16x3", 0, "auto", {"general", "resident", "tiled"}),
    ("cube10", "fp64", 0, "auto", {"general", "lane"}),
    # a covariance attached on the tiled path: both paths; attached on the
    # general kernel: the split screening has no buffers, the tiled path is not tried
    ("rotbox", "bf16x3", 8, "tiled", {"general", "tiled"}),
    ("rotbox", "bf16x3", 8, "auto", {"general"}),
])
def test_autotune_keeps_fastest_and_walks(name, prec, rank, path, expect):
    p = {"randpoly": inst.randpoly(n=100, m=2000, z=1024, seed=81),
         "cube10": inst.cube10(64),
         "rotbox": inst.rotbox(n=100, m_extra=800, z=256, seed=82)[0]}[name]
    gu.announce("autotune", name, prec, rank, path)
    trial = 12
    tuned, twin, res = _tuned_and_twin(p, prec, trial, rank, path)
    ms = res["ms_per_step"]
    assert set(ms) == expect, ms
    assert res["path"] == min(ms, key=ms.get)
    assert all(v > 0 for v in ms.values())
    twin.step(trial * len(ms))
    tuned.step(17)
    twin.step(17)
    a, sa = gu.state(tuned)
    b, sb = gu.state(twin)
    assert np.array_equal(a, b) and np.array_equal(sa, sb)
    assert tuned.step_count() == twin.step_count()
    assert tuned.stats()["kernel"] == mhar.PATHS[res["path"]]


def test_batch_runs_tuned_choices():
    probs = [inst.randpoly(n=100, m=2000, z=256, seed=83), inst.randpoly(n=48, m=600, z=128, seed=84)]
    gu.announce("autotune batch")
    made = [gu.make(p, "bf16x3") for p in probs]
    chosen = [ch.autotune(8)["path"] for _, ch in made]
    batch = mhar.Batch([ch for _, ch in made])
    batch.step(9)
    for (prob, ch), path in zip(made, chosen):
        kern = ch.stats()["kernel"]
        if path == "tiled":
            assert kern == mhar.PATHS["tiled"]
        elif path == "general":
            assert kern == mhar.PATHS["general"]
        else:
            assert kern in (mhar.PATHS["tiled"], mhar.PATHS["general"])
        assert not gu.state(ch)[1].any()
    batch.close()


def test_autotune_rejects_bad_trial_length():
    _, ch = gu.make(inst.cube10(16), "fp64")
    gu.announce("autotune bad args")
    with pytest.raises(mhar.MharError) as ei:
        ch.autotune(0)
    assert ei.value.code == mhar.E_INVALID_ARG
