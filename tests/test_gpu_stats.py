"""Statistical checks of the HIP path against closed-form uniform laws."""
import numpy as np
import pytest
from scipy import stats

from paper_2104_07097_amd import instances as inst

from . import gpu_util as gu

pytestmark = pytest.mark.gpu


def test_cube10_full_run_marginals():
    """Hypercube n=10, 16 walks from the origin, 10,000 steps, FP64 products."""
    p = inst.cube10(16)
    gu.announce("cube10 10k steps")
    _, ch = gu.make(p, "fp64")
    rec = ch.record(10000, 50, 16).cpu().numpy()
    X, st = gu.state(ch)
    assert not st.any()
    samples = rec[20:].reshape(-1, 10)
    assert gu.feasible(p, samples)
    for j in range(10):
        d = stats.kstest(samples[:, j], stats.uniform(-1, 2).cdf).statistic
        assert d < 0.06, (j, d)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_simplex_from_centre(prec):
    n, z = 10, 2000
    p = inst.simplex(n, z)
    gu.announce("simplex n=10", prec)
    _, ch = gu.make(p, prec)
    ch.step(400)
    X, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.beta(1, n - 1).cdf).pvalue > 1e-3


def test_triangle_vs_rejection():
    z = 4000
    p = inst.triangle(z)
    gu.announce("triangle")
    _, ch = gu.make(p, "fp32")
    ch.step(200)
    X, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, X)
    ref = inst.exact_by_rejection(np.random.default_rng(9), p.A, p.b, [0, 0], [2, 1], z)
    for v in ([1.0, 0.0], [0.0, 1.0], [0.6, 0.8], [0.8, -0.6], [-0.28, 0.96]):
        v = np.array(v)
        assert stats.ks_2samp(X @ v, ref @ v).pvalue > 1e-3


def test_cube_stationary_from_exact_start():
    rng = np.random.default_rng(20)
    n, z = 5, 3000
    p = inst.hypercube(n, z, inst.exact_cube(rng, z, n))
    gu.announce("cube stationarity")
    _, ch = gu.make(p, "bf16x3")
    ch.step(25)
    X, st = gu.state(ch)
    assert not st.any() and gu.feasible(p, X)
    for j in range(n):
        assert stats.kstest(X[:, j], stats.uniform(-1, 2).cdf).pvalue > 1e-3


@pytest.mark.parametrize("fig,n", [("simplex", 5), ("hypercube", 5), ("simplex", 15), ("hypercube", 15)])
def test_friedman_rafsky_paper_protocol(fig, n):
    """The paper's independence check (S6) at its settings for n = 5 and 15:
    z = 1000 walks from the centre, burn-in phi = (n-1)^3 or n^3 steps, then 5
    samples per walk phi steps apart against 5000 exact uniform points.  The
    paper accepts at z >= -1.64 (5 % one-sided); the gate here is 0.1 % so
    that it fails only for a real difference of laws."""
    import bench
    gu.announce("friedman-rafsky", fig, n)
    zval, steps, sec, flags = bench.fr_run(fig, n, seed=1)
    print(f"  FR z = {zval:+.2f} after {steps} steps", flush=True)
    assert flags == 0
    assert zval > -3.09
