"""Parity with the FP64 oracle on the full-size paths the benchmarks use, and
on the boundary branches.

  * learned covariances of rank 8, 13 and 64 (the blocked U eps loop and the
    split screening of the tiled path), on the general and tiled paths, with
    and without equalities: one step from shared states and 20 steps from
    the start;
  * the rotated box at full size (n = 1000, m = 10000, z = 8192) on the
    tiled path, plain and with a seeded rank-64 covariance: one step from a
    mid-run state on 48 sampled walks, computed by the oracle one by one,
    and feasibility of every walk;
  * a 32-problem batch (n from 20 to 400, m = ceil(4 n^1.5), 64 walks each)
    whose problems take both the grouped tiled and the general kernels:
    sampled walks of sampled problems after 20 batched steps;
  * walks on a facet, just below one, past one, at a vertex and with a NaN
    coordinate: positions and status bits after one step on every path
    (the oracle's branches are pinned in test_oracle_flags.py)."""
import math

import numpy as np
import pytest
import torch

from oracle import Oracle
from paper_2104_07097_amd import instances as inst
from paper_2104_07097_amd import mhar

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def orc():
    return Oracle()


def _cov(n, r, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((n, r)), 0.2 * rng.standard_normal(n)


CASES = [
    ("rotbox70", 8, "general", "fp32"),
    ("rotbox70", 13, "tiled", "bf16x3"),
    ("rotbox100", 64, "general", "fp64"),
    ("rotbox100", 64, "tiled", "fp32"),
    ("rotbox100", 64, "tiled", "bf16x3"),
    ("simplex80", 13, "tiled", "bf16x3"),
    ("simplex80", 64, "general", "fp32"),
]


def _problem(name):
    if name == "rotbox70":
        return inst.rotbox(n=70, m_extra=400, z=40, seed=51)[0]
    if name == "rotbox100":
        return inst.rotbox(n=100, m_extra=600, z=40, seed=52)[0]
    return inst.simplex_cut(n=80, m_extra=500, m_eq_extra=3, z=40, seed=53)


@pytest.mark.parametrize("name,r,path,prec", CASES)
def test_high_rank_covariance_parity(orc, name, r, path, prec):
    p = _problem(name)
    P = gu.oracle_projection(orc, p)
    U, ls = _cov(p.n, r, 7 + r)
    dev = gu.device()
    gu.announce("rank", name, r, path, prec)
    _, ch = gu.make(p, prec, recompute_every=6, path=path)
    ch.precond_create(r)
    ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    for t in (0, 9):
        Xt, _, _ = orc.run(p.A, p.b, p.X0, t, seed=0, P=P, U=U, log_sigma=ls)
        want, st, _ = orc.run(p.A, p.b, Xt, 1, seed=0, P=P, step0=t, U=U, log_sigma=ls)
        ch.set_state(torch.tensor(Xt, device=dev), t)
        ch.step(1)
        got, gst = gu.state(ch)
        assert not gst.any() and not st.any()
        assert gu.rel_err(got, want) <= 1e-11, (t, gu.rel_err(got, want))
    _, ch2 = gu.make(p, prec, recompute_every=6, path=path)
    ch2.precond_create(r)
    ch2.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    ch2.step(20)
    got, gst = gu.state(ch2)
    want, _, _ = orc.run(p.A, p.b, p.X0, 20, seed=0, P=P, U=U, log_sigma=ls)
    err = gu.rel_err(got, want)
    print(f"  20 steps: rel err {err:.2e}", flush=True)
    assert not gst.any() and err <= 1e-10
    assert gu.feasible(p, got)


@pytest.mark.parametrize("learned", [False, True])
def test_rotated_box_full_size_sampled_parity(orc, learned):
    p, _, _ = inst.rotbox()
    dev = gu.device()
    gu.announce("rotbox full size", "learned" if learned else "plain")
    _, ch = gu.make(p, "bf16x3", recompute_every=50)
    U = ls = None
    if learned:
        U, ls = _cov(p.n, 64, 61, scale=0.02)
        ls = ls + math.log(0.005)
        ch.precond_create(64)
        ch.precond_set(torch.tensor(U, device=dev), torch.tensor(ls, device=dev))
    assert ch.stats()["kernel"] == 3
    ch.step(40)
    Xt, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, Xt)
    ch.set_state(torch.tensor(Xt, device=dev), 40)
    ch.step(1)
    got, st = gu.state(ch)
    assert not st.any()
    sample = np.random.default_rng(2).choice(p.z, size=48, replace=False)
    for k in sample:
        want, _, _ = orc.run(p.A, p.b, Xt[k:k + 1], 1, seed=0, chain_offset=int(k), step0=40,
                             U=U, log_sigma=ls)
        err = gu.rel_err(got[k:k + 1], want)
        assert err <= 1e-11, (k, err)
    assert gu.feasible(p, got)


def _tiled_in_batch(p, z):
    m_pad = -(-p.m // 64) * 64
    lda = -(-p.n // 32) * 32
    z_pad = -(-z // 16) * 16
    return m_pad * lda >= (1 << 18) and z_pad >= 64


def test_batch_against_oracle(orc):
    probs = inst.batched(count=32, z_each=64)
    kinds = [_tiled_in_batch(p, p.z) for p in probs]
    assert any(kinds) and not all(kinds)
    gu.announce("batch vs oracle", len(probs), "problems,", sum(kinds), "tiled")
    made = [gu.make(p, "bf16x3") for p in probs]
    batch = mhar.Batch([ch for _, ch in made])
    batch.step(20)
    # sampled problems spanning n, both kinds; two walks each
    order = np.argsort([p.n for p in probs])
    pick = sorted(set(order[np.linspace(0, len(probs) - 1, 8).astype(int)]) |
                  {kinds.index(True), kinds.index(False)})
    rng = np.random.default_rng(3)
    for i in pick:
        p = probs[i]
        got, st = gu.state(made[i][1])
        assert not st.any() and gu.feasible(p, got), p.name
        for k in rng.choice(p.z, size=2, replace=False):
            want, _, _ = orc.run(p.A, p.b, p.X0[k:k + 1], 20, seed=0, chain_offset=int(k))
            err = gu.rel_err(got[k:k + 1], want)
            assert err <= 1e-9, (p.name, kinds[i], k, err)
    batch.close()


@pytest.mark.parametrize("prec,path", [("fp64", "general"), ("fp64", "lane"), ("fp32", "resident"),
                                       ("bf16x3", "tiled")])
def test_boundary_branches_match_oracle(orc, prec, path):
    """Facet, rounding below a facet, past a facet, vertex, NaN and an interior
    point, one walk each (several walks per kind so that different directions
    are drawn), set without validation and stepped once."""
    A = np.vstack([np.eye(3), -np.eye(3)])
    b = np.ones(6)
    kinds = [[1.0, 0.2, -0.3], [1.0 + 1e-13, 0.0, 0.0], [1.0 + 1e-9, 0.0, 0.0], [1.0, 1.0, 1.0],
             [np.nan, 0.0, 0.0], [0.1, -0.2, 0.3]]
    X = np.array([kinds[k % len(kinds)] for k in range(24)])
    p = inst.Polytope("cube3", A, b, np.zeros((24, 3)))
    gu.announce("boundary branches", prec, path)
    _, ch = gu.make(p, prec, path=path)
    ch.set_state(torch.tensor(X, device=gu.device()), 5)
    ch.step(1)
    got, gst = gu.state(ch)
    want, wst, _ = orc.run(A, b, X, 1, seed=0, step0=5)
    assert np.array_equal(gst, wst), (gst, wst)
    fin = np.isfinite(want)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.max(np.abs(got[fin] - want[fin]) / np.maximum(1.0, np.abs(want[fin]))) <= 1e-11
    assert (wst & 2).any() and (wst & 8).any() and (wst & 4).any()
