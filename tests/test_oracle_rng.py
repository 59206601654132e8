"""Pins for the oracle's random streams (Philox4x32-10, uniforms, Box-Muller).

What fixes them from outside the oracle:
  * published Philox4x32-10 known-answer vectors (Random123), golden file;
  * rocRAND's independent open-source Philox, compiled on the host, on
    random counters and keys;
  * the documented stream layout (counter words, 52-bit uniform, Box-Muller
    pairing) evaluated from the raw block words;
  * distribution facts: uniforms strictly inside (0,1) and uniform (KS),
    normals with mean 0, variance 1, kurtosis 3, N(0,1) KS, uncorrelated pairs.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

from oracle import TAG_DIR, TAG_LOWRANK, TAG_THETA

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_published_kat(oracle):
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox(ctr, key) == want


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_source(oracle, tmp_path):
    exe = tmp_path / "kat"
    src = os.path.join(HERE, "golden", "philox_rocrand_kat.cpp")
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O1", "-o", str(exe), src], check=True,
                   capture_output=True)
    rng = np.random.default_rng(5)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    text = "\n".join(" ".join(f"{int(v):08x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    got = [[int(t, 16) for t in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for row, ref in zip(cases, got):
        assert oracle.philox(row[:4], row[4:]) == ref


def _words(oracle, seed, tag, chain, step, block):
    ctr = [block, chain & 0xFFFFFFFF, step & 0xFFFFFFFF, tag | ((step >> 32) << 4)]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    return oracle.philox(ctr, key)


def _u52(hi, lo):
    bits = ((hi << 32) | lo) >> 12
    return (bits + 0.5) * 2.0**-52


@pytest.mark.parametrize("seed,tag,chain,step,block", [
    (0, TAG_THETA, 0, 0, 0), (12345678901234, TAG_DIR, 77, 3, 5),
    (2**64 - 1, TAG_LOWRANK, 2**32 - 1, 2**40 + 17, 9)])
def test_stream_layout(oracle, seed, tag, chain, step, block):
    w = _words(oracle, seed, tag, chain, step, block)
    assert oracle.uniform(seed, tag, chain, step, block, 0) == _u52(w[0], w[1])
    assert oracle.uniform(seed, tag, chain, step, block, 1) == _u52(w[2], w[3])
    ua, ub = _u52(w[0], w[1]), _u52(w[2], w[3])
    rad = math.sqrt(-2.0 * math.log(ua))
    ang = 6.283185307179586 * ub
    for j, want in ((2 * block, rad * math.cos(ang)), (2 * block + 1, rad * math.sin(ang))):
        got = oracle.gauss(seed, tag, chain, step, j)
        assert abs(got - want) <= 4e-16 * max(1.0, abs(want))


def test_uniform_extremes_exact():
    # all-zero and all-one words give the two ends of the grid, both inside (0,1)
    assert _u52(0, 0) == 2.0**-53
    assert _u52(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0**-53


def test_uniforms_open_and_uniform(oracle):
    u = np.array([oracle.uniform(3, TAG_THETA, k, t, 0, 0) for k in range(200) for t in range(100)])
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_gauss_distribution(oracle):
    g = np.array([oracle.gauss(11, TAG_DIR, k, t, j)
                  for k in range(40) for t in range(50) for j in range(50)])
    assert abs(g.mean()) < 5 * (1 / math.sqrt(g.size))
    assert abs(g.var() - 1.0) < 5 * math.sqrt(2 / g.size)
    assert abs(stats.kurtosis(g, fisher=False) - 3.0) < 0.05
    assert stats.kstest(g, "norm").pvalue > 1e-3
    pairs = g.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5 / math.sqrt(pairs.shape[0])


def test_streams_distinct(oracle):
    # different tags, chains or steps give different blocks
    a = _words(oracle, 0, TAG_DIR, 1, 2, 0)
    assert a != _words(oracle, 0, TAG_THETA, 1, 2, 0)
    assert a != _words(oracle, 0, TAG_DIR, 2, 2, 0)
    assert a != _words(oracle, 0, TAG_DIR, 1, 3, 0)
    assert a != _words(oracle, 1, TAG_DIR, 1, 2, 0)
