"""Graph replays of the tiled path (mhar_chains_set_graph): the walks after
every call equal those of ordinary launches bit for bit, on unaligned call
lengths, with the program's own eager work and synchronisations between
the calls, with equalities and with a learned covariance (split screening)
whose values change between calls; sampled walks match the oracle."""
import math

import numpy as np
import pytest
import torch

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu

CASES = [
    ("randpoly", "bf16x3", 5, 10, 0),
    ("simplex_cut", "fp32", 4, 8, 0),
    ("rotbox", "bf16x3", 5, 5, 16),
]


def _problem(name):
    if name == "randpoly":
        return inst.randpoly(n=64, m=1500, z=128, seed=71)
    if name == "simplex_cut":
        return inst.simplex_cut(n=60, m_extra=900, m_eq_extra=3, z=96, seed=72)
    return inst.rotbox(n=100, m_extra=800, z=80, seed=73)[0]


def _cov(n, r, seed):
    rng = np.random.default_rng(seed)
    return 0.02 * rng.standard_normal((n, r)), 0.2 * rng.standard_normal(n) + math.log(0.05)


@pytest.mark.parametrize("name,prec,R,K,rank", CASES)
def test_graph_replays_equal_ordinary_launches(name, prec, R, K, rank):
    p = _problem(name)
    dev = gu.device()
    gu.announce("graph", name, prec, "R", R, "K", K, "rank", rank)
    _, eager = gu.make(p, prec, recompute_every=R, path="tiled")
    _, graph = gu.make(p, prec, recompute_every=R, path="tiled")
    graph.set_graph(K)
    if rank:
        U, ls = _cov(p.n, rank, 5)
        for ch in (eager, graph):
            ch.precond_create(rank)
            ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    total = 0
    for i, n in enumerate((7, 23, 3, 2 * K + 1, 40)):
        if rank and i == 3:
            # new covariance values between calls: the graph reads them from the device
            U, ls = _cov(p.n, rank, 6)
            for ch in (eager, graph):
                ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
        eager.step(n)
        graph.step(n)
        total += n
        # eager work of the program between replays
        torch.cuda.synchronize()
        assert float((torch.arange(1000, device=dev, dtype=torch.float64) * 2.0).sum()) == 999000.0
        a, sa = gu.state(eager)
        b, sb = gu.state(graph)
        assert np.array_equal(a, b) and np.array_equal(sa, sb), (i, n)
        assert graph.step_count() == eager.step_count() == total
    assert graph.stats()["kernel"] == mhar.PATHS["tiled"]
    assert gu.feasible(p, b)
    if rank == 0:
        orc = Oracle()
        P = gu.oracle_projection(orc, p)
        for k in (0, p.z - 1):
            want, _, _ = orc.run(p.A, p.b, p.X0[k:k + 1], total, seed=0, chain_offset=k, P=P)
            assert gu.rel_err(b[k:k + 1], want) <= 1e-9


def test_graph_steps_must_be_a_multiple_of_R():
    p = inst.randpoly(n=40, m=600, z=64, seed=74)
    _, ch = gu.make(p, "fp32", recompute_every=6, path="tiled")
    gu.announce("graph bad K")
    with pytest.raises(mhar.MharError) as ei:
        ch.set_graph(9)
    assert ei.value.code == mhar.E_INVALID_ARG
    with pytest.raises(mhar.MharError):
        ch.set_graph(-6)
    ch.set_graph(12)
    ch.set_graph(0)
    ch.step(13)
    assert not gu.state(ch)[1].any()
