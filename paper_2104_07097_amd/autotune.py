"""Autotuner for the MHAR options of a problem shape.

For a shape bucket (n, m, m_eq, z rounded up to powers of two) it times short
runs of candidate option sets -- screening precision, exact-recompute period
R, steps per launch and kernel path -- on a synthetic problem of that shape, and caches
the fastest in a JSON file (``MHAR_AUTOTUNE_CACHE``, default
``~/.cache/mhar_autotune.json``).  Every candidate produces the same
trajectories (the chord is evaluated exactly in FP64 whatever the options),
so tuning only trades speed.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

from . import instances as inst
from . import mhar

DEFAULT_CANDIDATES = (
    [{"precision": p, "recompute_every": r, "steps_per_launch": 0, "path": "auto"}
     for p in ("fp32", "bf16x3") for r in (25, 50, 100)]
    + [{"precision": p, "recompute_every": 50, "steps_per_launch": 0, "path": path}
       for p in ("fp32", "bf16x3") for path in ("tiled", "general")]
    + [{"precision": "fp64", "recompute_every": 50, "steps_per_launch": 0, "path": "lane"}]
)


def _bucket(v: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1, v)))))


def shape_key(n: int, m: int, m_eq: int, z: int) -> str:
    return f"n{_bucket(n)}_m{_bucket(m)}_e{int(m_eq > 0)}_z{_bucket(z)}"


def cache_path() -> str:
    return os.environ.get("MHAR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mhar_autotune.json"))


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_options(p: inst.Polytope, opts: dict, steps: int = 200, warmup: int = 20) -> float:
    """Seconds per step of `p` under `opts` (HIP events on the current stream)."""
    import torch
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.tensor(a, device=dev, dtype=torch.float64)
    prob = mhar.Problem(t(p.A), t(p.b), t(p.A_eq), t(p.b_eq), **opts)
    ch = mhar.Chains(prob, t(p.X0))
    ch.step(warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    stream = torch.cuda.current_stream(dev)
    e0.record(stream)
    ch.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / steps
    ch.close()
    prob.close()
    return sec


def tune(p: inst.Polytope, candidates=None, steps: int = 200, use_cache: bool = True) -> dict:
    """Best option set for the shape of `p` (timed on `p` itself)."""
    key = shape_key(p.n, p.m, p.m_eq, p.z)
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if key in cache:
        return cache[key]["options"]
    results = []
    for opts in candidates or DEFAULT_CANDIDATES:
        try:
            results.append((time_options(p, opts, steps=steps), opts))
        except mhar.MharError as e:
            if e.code not in (mhar.E_UNSUPPORTED, mhar.E_SHAPE):
                raise   # a path that does not fit this shape is skipped; anything else is an error
    results.sort(key=lambda x: x[0])
    best_sec, best = results[0]
    if use_cache:
        cache[key] = {"options": best, "sec_per_step": best_sec,
                      "timings": [{"options": o, "sec_per_step": s} for s, o in results]}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1)
    return best


def tune_shape(n: int, m: int, z: int, seed: int = 0, **kw) -> dict:
    """Tune on a synthetic unit-norm Gaussian polytope of the given shape."""
    return tune(inst.randpoly(n=n, m=m, z=z, seed=seed), **kw)
