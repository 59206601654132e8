"""Helpers for the GPU tests: run the HIP path and the oracle on the same inputs."""
import numpy as np

import oracle as oracle_pkg
from paper_2104_07097_amd import instances as inst


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def announce(*parts):
    print("[gpu-case]", *parts, flush=True)


def make(p, precision, recompute_every=50, seed=0, chain_offset=0, X0=None, path="auto"):
    import torch
    from paper_2104_07097_amd import mhar
    dev = device()
    t = lambda a: None if a is None else torch.tensor(a, device=dev, dtype=torch.float64)
    prob = mhar.Problem(t(p.A), t(p.b), t(p.A_eq), t(p.b_eq), precision=precision,
                        recompute_every=recompute_every, path=path)
    ch = mhar.Chains(prob, t(p.X0 if X0 is None else X0), seed=seed, chain_offset=chain_offset)
    return prob, ch


def state(ch):
    import torch
    X, st = ch.state()
    torch.cuda.synchronize()
    return X.cpu().numpy(), st.cpu().numpy()


def oracle_projection(orc, p):
    if p.A_eq is None:
        return None
    rc, P = orc.projection(p.n, p.A_eq)
    assert rc == 0
    return P


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


def feasible(p, X, tol=1e-12):
    ok = np.all(X @ p.A.T <= p.b + tol * np.maximum(1.0, np.abs(p.b)))
    if p.A_eq is not None:
        ok = ok and np.abs(X @ p.A_eq.T - p.b_eq).max() <= 1e-9
    return bool(ok)


def small_cases():
    """Small polytopes spanning several tiles with ragged tails in n, m and z."""
    cases = {
        "cube10": inst.cube10(16),
        "randpoly": inst.randpoly(n=37, m=300, z=50, seed=11),
        "simplex_cut": inst.simplex_cut(n=30, m_extra=200, m_eq_extra=3, z=40, seed=12),
        "rotbox": inst.rotbox(n=40, m_extra=200, z=33, seed=13)[0],
        # rows split over 3 workgroups per walk tile (plain and XCD-aware mapping)
        "split3": inst.randpoly(n=40, m=1300, z=40, seed=14),
        "split3_xcd": inst.randpoly(n=64, m=1500, z=128, seed=15),
    }
    return cases


def ulp_sensitivity(orc, p, steps, P=None, reps=3):
    """How far the oracle's own trajectory moves after `steps` steps when each
    state is perturbed by one ulp (relative 2.2e-16, random signs) before every
    step: the scale of the difference that ulp-level disagreements of log, sin
    and cos in the directions (all that differs between the HIP path and the
    oracle) can grow to under the chaotic map.  Max relative error over reps."""
    Xa, _, _ = orc.run(p.A, p.b, p.X0, steps, seed=0, P=P)
    worst = 0.0
    for rep in range(reps):
        rng = np.random.default_rng(rep)
        Xb = p.X0.copy()
        for s in range(steps):
            Xb = Xb * (1 + 2.2e-16 * rng.choice([-1.0, 1.0], Xb.shape))
            Xb, _, _ = orc.run(p.A, p.b, Xb, 1, seed=0, P=P, step0=s)
        worst = max(worst, rel_err(Xb, Xa))
    return worst
