"""Seeded synthetic polytopes and start points (host side, numpy).

This module only *builds inputs*: constraint matrices, right-hand sides and
start points of the benchmark workloads, plus exact reference samplers for
the two polytopes whose uniform law has a closed form.  It contains none of
the sampler's arithmetic and is shared by the tests, the benchmark and the
oracle-driven checks.

Workloads (all synthetic, as in the paper's own experiments, S6):
  * ``hypercube(n)``  -- [-1, 1]^n written as [I; -I] x <= 1 (S6 definition)
  * ``simplex(n)``    -- {x >= 0, 1^T x = 1} (S6 definition)
  * ``cube10``        -- hypercube n=10, 16 chains from the origin
  * ``randpoly``      -- n=100, m=2000 unit-norm Gaussian rows, b=1
  * ``simplex_cut``   -- simplex n=500 + 4 Gaussian equalities through the
                         centre + 5000 Gaussian halfspaces just outside it
  * ``batched``       -- 256 random Gaussian-halfspace polytopes
  * ``rotbox``        -- rotated axis box with log-uniform sides + 8000
                         unit-norm halfspaces at distance 1
Instance seeds: numpy ``default_rng(1000 + k)`` for workload k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Polytope:
    """{x : A x <= b, A_eq x = b_eq} with start points X0 (z x n)."""

    name: str
    A: np.ndarray
    b: np.ndarray
    X0: np.ndarray
    A_eq: np.ndarray | None = None
    b_eq: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.A.shape[1]

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def m_eq(self) -> int:
        return 0 if self.A_eq is None else self.A_eq.shape[0]

    @property
    def z(self) -> int:
        return self.X0.shape[0]


def _unit_rows(rng, m, n):
    A = rng.standard_normal((m, n))
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    return A


def hypercube(n: int, z: int, start: np.ndarray | None = None) -> Polytope:
    A = np.vstack([np.eye(n), -np.eye(n)])
    b = np.ones(2 * n)
    X0 = np.zeros((z, n)) if start is None else np.array(start, dtype=np.float64).reshape(z, n)
    return Polytope(f"hypercube{n}", A, b, X0)


def simplex(n: int, z: int, start: np.ndarray | None = None) -> Polytope:
    A = -np.eye(n)
    b = np.zeros(n)
    A_eq = np.ones((1, n))
    b_eq = np.ones(1)
    if start is None:
        X0 = np.full((z, n), 1.0 / n)
    else:
        X0 = np.array(start, dtype=np.float64).reshape(z, n)
    return Polytope(f"simplex{n}", A, b, X0, A_eq, b_eq)


def cube10(z: int = 16) -> Polytope:
    """Hypercube n=10 (m=20) with z chains at the origin."""
    p = hypercube(10, z)
    p.name = "cube10"
    return p


def randpoly(n: int = 100, m: int = 2000, z: int = 1024, seed: int = 1001) -> Polytope:
    """Rows i.i.d. N(0, I) scaled to unit norm, b = 1 (contains the unit ball)."""
    rng = np.random.default_rng(seed)
    A = _unit_rows(rng, m, n)
    return Polytope(f"randpoly_n{n}_m{m}", A, np.ones(m), np.zeros((z, n)))


def simplex_cut(n: int = 500, m_extra: int = 5000, m_eq_extra: int = 4, z: int = 4096,
                seed: int = 1002) -> Polytope:
    """Simplex plus Gaussian equalities through c = 1/n and Gaussian halfspaces
    a_i ~ N(0, I) with b_i = a_i.c + (0.1/n)|a_i| (c stays strictly inside)."""
    rng = np.random.default_rng(seed)
    c = np.full(n, 1.0 / n)
    G = rng.standard_normal((m_eq_extra, n))
    A_eq = np.vstack([np.ones((1, n)), G])
    b_eq = A_eq @ c
    N = rng.standard_normal((m_extra, n))
    A = np.vstack([-np.eye(n), N])
    b = np.concatenate([np.zeros(n), N @ c + (0.1 / n) * np.linalg.norm(N, axis=1)])
    X0 = np.tile(c, (z, 1))
    return Polytope(f"simplex_cut_n{n}", A, b, X0, A_eq, b_eq)


def rotbox(n: int = 1000, m_extra: int = 8000, z: int = 8192, seed: int = 1004,
           side_lo: float = 1e-3):
    """Axis box with sides l_i = exp(U(ln side_lo, 0)) rotated by a Haar Q
    (QR of a Gaussian matrix with the sign fix of Mezzadri), as rows
    [Q^T; -Q^T] x <= l/2, plus m_extra unit-norm Gaussian halfspaces with
    b = 1.  Returns (Polytope, Q, sides)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    Q = Q * np.sign(np.diag(R))[None, :]
    sides = np.exp(rng.uniform(math.log(side_lo), 0.0, size=n))
    H = _unit_rows(rng, m_extra, n)
    A = np.vstack([Q.T, -Q.T, H])
    b = np.concatenate([sides / 2, sides / 2, np.ones(m_extra)])
    return Polytope(f"rotbox_n{n}", A, b, np.zeros((z, n))), Q, sides


def batched(count: int = 256, z_each: int = 256, n_lo: int = 20, n_hi: int = 400,
            seed: int = 1003) -> list[Polytope]:
    """`count` polytopes with n log-uniform in [n_lo, n_hi], m = ceil(4 n^1.5),
    unit-norm Gaussian rows, b = 1, z_each chains from the origin each."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(math.ceil(4 * n ** 1.5))
        A = _unit_rows(rng, m, n)
        out.append(Polytope(f"batched{p}_n{n}_m{m}", A, np.ones(m), np.zeros((z_each, n))))
    return out


def triangle(z: int, seed: int = 7) -> Polytope:
    """2-D triangle y >= 0, x + 1.5 y <= 2, -2 x + 0.5 y <= 0 (vertices (0,0),
    (2,0), (2/7, 8/7)); z chains at the interior point (5/6, 1/3)."""
    A = np.array([[0.0, -1.0], [1.0, 1.5], [-2.0, 0.5]])
    b = np.array([0.0, 2.0, 0.0])
    start = np.array([2.5 / 3.0, 1.0 / 3.0])
    return Polytope("triangle", A, b, np.tile(start, (z, 1)))


# --------------------------------------------------------------------------
# Exact reference samplers (the uniform law has a closed form)
# --------------------------------------------------------------------------

def exact_cube(rng, count: int, n: int) -> np.ndarray:
    """Uniform on [-1, 1]^n."""
    return rng.uniform(-1.0, 1.0, size=(count, n))


def exact_simplex(rng, count: int, n: int) -> np.ndarray:
    """Uniform on the simplex: normalised i.i.d. exponentials (Dirichlet(1,...,1))."""
    E = rng.exponential(size=(count, n))
    return E / E.sum(axis=1, keepdims=True)


def exact_by_rejection(rng, A, b, lo, hi, count: int, batch: int = 1 << 16) -> np.ndarray:
    """Uniform on {A x <= b} by rejection from the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    out = []
    have = 0
    while have < count:
        X = rng.uniform(lo, hi, size=(batch, lo.size))
        keep = X[np.all(X @ A.T <= b, axis=1)]
        out.append(keep)
        have += keep.shape[0]
    return np.vstack(out)[:count]
