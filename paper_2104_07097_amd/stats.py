"""Host-side statistics for judging samplers: effective sample size,
Kolmogorov-Smirnov distances and the Friedman-Rafsky two-sample test.

The ESS estimator follows the multi-chain recipe of Gelman et al.,
*Bayesian Data Analysis* (3rd ed., S11.5) as used by Stan: split each chain
in half, pool within- and between-chain variances, and sum the
autocorrelations with Geyer's initial monotone sequence (Geyer 1992,
"Practical Markov chain Monte Carlo").  Autocovariances come from FFTs.
"""
from __future__ import annotations

import numpy as np


def _autocov(x: np.ndarray) -> np.ndarray:
    """Biased autocovariance of each row of x (chains x draws), all lags."""
    c, t = x.shape
    x = x - x.mean(axis=1, keepdims=True)
    size = 1
    while size < 2 * t:
        size *= 2
    f = np.fft.rfft(x, n=size, axis=1)
    ac = np.fft.irfft(f * np.conj(f), n=size, axis=1)[:, :t]
    return ac / t


def ess(draws: np.ndarray) -> float:
    """Effective sample size of one scalar quantity.

    draws: array (chains, iterations).  Returns the multi-chain ESS
    (split chains, Geyer initial monotone sequence)."""
    draws = np.asarray(draws, dtype=np.float64)
    if draws.ndim == 1:
        draws = draws[None, :]
    c, t = draws.shape
    half = t // 2
    if half < 4:
        return float(c * t)
    x = np.concatenate([draws[:, :half], draws[:, t - half:]], axis=0)
    m, n = x.shape
    acov = _autocov(x)
    chain_mean = x.mean(axis=1)
    chain_var = acov[:, 0] * n / (n - 1.0)
    w = chain_var.mean()
    b_over_n = chain_mean.var(ddof=1) if m > 1 else 0.0
    var_plus = w * (n - 1.0) / n + b_over_n
    if not var_plus > 0:
        return float(m * n)
    rho = 1.0 - (w - acov.mean(axis=0)) / var_plus
    rho[0] = 1.0
    # Geyer: pair sums P_k = rho_{2k} + rho_{2k+1}, stop at the first
    # non-positive pair, then enforce monotone decrease.
    pairs = []
    k = 0
    while 2 * k + 1 < n:
        p = rho[2 * k] + rho[2 * k + 1]
        if p <= 0:
            break
        pairs.append(p)
        k += 1
    pairs = np.minimum.accumulate(np.array(pairs)) if pairs else np.array([1.0])
    tau = -1.0 + 2.0 * pairs.sum()
    tau = max(tau, 1.0 / np.log10(m * n))
    return float(m * n / tau)


def split_rhat(draws: np.ndarray) -> float:
    """Split potential scale reduction R-hat of one scalar quantity (Gelman et
    al., BDA3 S11.4): chains (rows) cut in halves, sqrt(var_plus / W) with W
    the mean within-half variance and var_plus = (n-1)/n W + B/n.  Near 1 when
    the halves agree; well above 1 when the chains have not mixed."""
    draws = np.asarray(draws, dtype=np.float64)
    if draws.ndim == 1:
        draws = draws[None, :]
    t = draws.shape[1]
    half = t // 2
    x = np.concatenate([draws[:, :half], draws[:, t - half:]], axis=0)
    n = x.shape[1]
    w = x.var(axis=1, ddof=1).mean()
    b_over_n = x.mean(axis=1).var(ddof=1)
    var_plus = w * (n - 1.0) / n + b_over_n
    if not w > 0:
        return float("inf") if var_plus > 0 else 1.0
    return float(np.sqrt(var_plus / w))


def max_marginal_rhat(samples: np.ndarray) -> float:
    """samples: (iterations, chains, n).  The largest split R-hat over coordinates."""
    samples = np.asarray(samples, dtype=np.float64)
    return max(split_rhat(samples[:, :, j].T) for j in range(samples.shape[2]))


def min_marginal_ess(samples: np.ndarray) -> tuple[float, np.ndarray]:
    """samples: (iterations, chains, n).  Returns (min over coordinates, per-coordinate ESS)."""
    samples = np.asarray(samples, dtype=np.float64)
    per = np.array([ess(samples[:, :, j].T) for j in range(samples.shape[2])])
    return float(per.min()), per


def ks_distance(sample: np.ndarray, cdf) -> float:
    """One-sample Kolmogorov-Smirnov distance sup |F_n - F|."""
    x = np.sort(np.asarray(sample, dtype=np.float64))
    k = x.size
    f = cdf(x)
    upper = np.arange(1, k + 1) / k - f
    lower = f - np.arange(0, k) / k
    return float(max(upper.max(), lower.max()))


def ks_two_sample(a: np.ndarray, b: np.ndarray) -> float:
    """Two-sample Kolmogorov-Smirnov distance."""
    a = np.sort(np.asarray(a, dtype=np.float64))
    b = np.sort(np.asarray(b, dtype=np.float64))
    grid = np.concatenate([a, b])
    fa = np.searchsorted(a, grid, side="right") / a.size
    fb = np.searchsorted(b, grid, side="right") / b.size
    return float(np.abs(fa - fb).max())


def friedman_rafsky(x: np.ndarray, y: np.ndarray) -> tuple[int, float]:
    """Friedman-Rafsky multivariate two-sample test (Friedman & Rafsky, Ann.
    Statist. 7(4), 1979), the convergence check the paper applies to MHAR.

    Pool the samples (rows of x and y), build the Euclidean minimum spanning
    tree, and count runs R = (edges joining a point of x to a point of y) + 1.
    Under the null hypothesis of equal laws
      E[R]   = 2 m n / N + 1,
      Var[R] = 2 m n / (N (N - 1)) * [ (2 m n - N) / N
               + (C - N + 2) / ((N - 2)(N - 3)) * (N (N - 1) - 4 m n + 2) ],
    with m, n the sample sizes, N = m + n and C the number of pairs of tree
    edges that share a node.  Returns (R, z = (R - E[R]) / sd[R]); few runs
    (z very negative) mean the samples come from different laws."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m, n = len(x), len(y)
    N = m + n
    pts = np.vstack([x, y])
    # Prim's algorithm on squared Euclidean distances (same tree), one row of
    # distances at a time: O(N^2 dim) work, O(N) memory
    sq = np.einsum("ij,ij->i", pts, pts)
    in_tree = np.zeros(N, dtype=bool)
    best = np.full(N, np.inf)
    parent = np.full(N, -1, dtype=np.int64)
    best[0] = 0.0
    for _ in range(N):
        u = int(np.argmin(np.where(in_tree, np.inf, best)))
        in_tree[u] = True
        d = sq - 2.0 * (pts @ pts[u]) + sq[u]
        upd = (~in_tree) & (d < best)
        best[upd] = d[upd]
        parent[upd] = u
    child = np.nonzero(parent >= 0)[0]
    rows, cols = parent[child], child
    label = np.concatenate([np.zeros(m, dtype=bool), np.ones(n, dtype=bool)])
    cross = int(np.sum(label[rows] != label[cols]))
    R = cross + 1
    deg = np.bincount(np.concatenate([rows, cols]), minlength=N)
    C = float(np.sum(deg * (deg - 1) / 2.0))
    mn = float(m) * float(n)
    mean = 2.0 * mn / N + 1.0
    var = (2.0 * mn / (N * (N - 1.0))) * ((2.0 * mn - N) / N + (C - N + 2.0) / ((N - 2.0) * (N - 3.0))
                                          * (N * (N - 1.0) - 4.0 * mn + 2.0))
    return R, float((R - mean) / np.sqrt(var))
