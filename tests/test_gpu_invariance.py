"""The samples do not depend on how the work is cut: into launches, or into
handles of fewer walks.

The chord of every step is the exact FP64 chord of a certified candidate set
(S4.4), and the random numbers of a step are keyed by (walk, step) alone, so
running the same steps as many short launches or as one long launch must give
bitwise the same states on every kernel path, although the screening state
differs (a resident launch starts from an exact slack recompute, because its
slack lives in registers only while it runs).
"""
import numpy as np
import pytest

from paper_2104_07097_amd import instances as inst

from . import gpu_util as gu

pytestmark = pytest.mark.gpu

KERNEL = {"general": 1, "resident": 2, "tiled": 3, "lane": 4}

CASES = {
    "resident": (lambda: inst.randpoly(n=37, m=300, z=50, seed=11), "resident", "bf16x3"),
    "resident_split3": (lambda: inst.randpoly(n=40, m=1300, z=40, seed=14), "resident", "fp32"),
    "resident_split3_bf16x3": (lambda: inst.randpoly(n=40, m=1300, z=40, seed=14), "resident", "bf16x3"),
    "general": (lambda: inst.randpoly(n=37, m=300, z=50, seed=11), "general", "fp32"),
    "tiled": (lambda: inst.simplex_cut(n=30, m_extra=200, m_eq_extra=3, z=40, seed=12), "tiled", "bf16x3"),
    "lane": (lambda: inst.cube10(16), "lane", "fp64"),
}


def _run(p, prec, path, steps, steps_per_launch=0, X0=None, offset=0):
    """States, status bits and kernel path after `steps` steps of walks X0
    (default: all of p's) whose global indices start at `offset`."""
    import torch
    from paper_2104_07097_amd import mhar
    dev = gu.device()
    t = lambda a: None if a is None else torch.tensor(a, device=dev, dtype=torch.float64)
    prob = mhar.Problem(t(p.A), t(p.b), t(p.A_eq), t(p.b_eq), precision=prec, recompute_every=6,
                        steps_per_launch=steps_per_launch, path=path)
    ch = mhar.Chains(prob, t(p.X0 if X0 is None else X0), seed=3, chain_offset=offset)
    ch.step(steps)
    X, st = gu.state(ch)
    kernel = ch.stats()["kernel"]
    ch.close()
    prob.close()
    return X, st, kernel


@pytest.mark.parametrize("case", sorted(CASES))
def test_short_launches_give_the_same_states(case):
    make, path, prec = CASES[case]
    p = make()
    gu.announce("launch length", case, f"n={p.A.shape[1]}", f"m={p.A.shape[0]}", prec)
    Xs, ss, ks = _run(p, prec, path, 37, steps_per_launch=5)    # 7 launches of 5 steps and one of 2
    Xl, sl, kl = _run(p, prec, path, 37, steps_per_launch=37)   # one launch
    assert ks == kl == KERNEL[path]
    assert not ss.any() and not sl.any()
    assert np.array_equal(Xs, Xl)
    assert not np.array_equal(Xs, p.X0)          # the walks moved
    assert gu.feasible(p, Xs)


@pytest.mark.parametrize("case", sorted(CASES))
def test_walks_do_not_depend_on_their_neighbours(case):
    """A walk's draws are keyed by its global index (the handle's chain offset
    plus its position), so a contiguous subset of the walks, run alone in a
    handle of its own, follows bitwise the same trajectories as inside the
    whole set, although tiles, workgroups and padding differ."""
    make, path, prec = CASES[case]
    p = make()
    z = p.X0.shape[0]
    k0, zs = z // 4 + 1, z // 2 - 1
    gu.announce("walk subset", case, f"z={z}", f"walks {k0}..{k0 + zs - 1}", prec)
    Xf, sf, kf = _run(p, prec, path, 23)
    Xs, ss, ks = _run(p, prec, path, 23, X0=p.X0[k0:k0 + zs], offset=k0)
    assert kf == ks == KERNEL[path]
    assert not sf.any() and not ss.any()
    assert np.array_equal(Xs, Xf[k0:k0 + zs])
