"""Starting point of the walks: the Chebyshev centre of the polytope.

The paper (S4.2, Model CCHC) starts every walk at the centre of the largest
inscribed ball: maximise r over (x, r) subject to A_eq x = b_eq and
a_i x + r ||a_i||_2 <= b_i for every inequality row.  This is a one-time
host-side setup step, outside the per-step path; the linear programme is
solved with HiGHS through scipy.optimize.linprog.
"""
from __future__ import annotations

import numpy as np


def chebyshev_center(A, b, A_eq=None, b_eq=None) -> tuple[np.ndarray, float]:
    """(x, r): centre and radius of the largest ball (measured with the rows'
    2-norms, as in the paper's model) inside {A x <= b, A_eq x = b_eq}.

    Raises ValueError if the programme is infeasible or unbounded (an
    unbounded polytope, or r <= 0: no strictly interior point)."""
    from scipy.optimize import linprog

    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    m, n = A.shape
    norms = np.linalg.norm(A, axis=1)
    # variables (x, r); maximise r == minimise -r
    cost = np.zeros(n + 1)
    cost[-1] = -1.0
    A_ub = np.hstack([A, norms[:, None]])
    eq = None
    if A_eq is not None and np.size(A_eq):
        A_eq = np.asarray(A_eq, dtype=np.float64).reshape(-1, n)
        eq = (np.hstack([A_eq, np.zeros((A_eq.shape[0], 1))]),
              np.asarray(b_eq, dtype=np.float64).reshape(-1))
    bounds = [(None, None)] * n + [(0.0, None)]
    res = linprog(cost, A_ub=A_ub, b_ub=b, A_eq=None if eq is None else eq[0],
                  b_eq=None if eq is None else eq[1], bounds=bounds, method="highs")
    if res.status == 3:
        raise ValueError("the polytope is unbounded (the inscribed radius is not bounded)")
    if res.status != 0:
        raise ValueError(f"no Chebyshev centre: {res.message}")
    x, r = res.x[:n], float(res.x[n])
    if not r > 0.0:
        raise ValueError("the polytope has no strictly interior point (inscribed radius 0)")
    return x, r


def start_points(A, b, z: int, A_eq=None, b_eq=None) -> np.ndarray:
    """z copies of the Chebyshev centre (z x n), the paper's start for all walks."""
    x, _ = chebyshev_center(A, b, A_eq, b_eq)
    return np.tile(x, (int(z), 1))
