"""Pins of the oracle's Philox4x64-10 and complex Gaussian."""
import math
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert philox.philox4x64_10_scalar(ctr, key) == out
    o = philox.philox4x64_10(np.array([ctr[0]], np.uint64), ctr[1], ctr[2], ctr[3], key[0], key[1])
    assert [int(x[0]) for x in o] == out


def test_philox_vs_numpy_bitgenerator():
    """numpy.random.Philox is an independent Philox4x64-10; it increments its
    counter before producing a block, so counter c yields block c+1."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.int64)]
        ctr = [int(x) for x in rng.integers(1, 2**62, 4, dtype=np.int64)]
        bg = np.random.Philox(key=np.array(key, np.uint64),
                              counter=np.array([ctr[0] - 1] + ctr[1:], np.uint64))
        ref = [int(x) for x in bg.random_raw(4)]
        assert philox.philox4x64_10_scalar(ctr, key) == ref
        vec = philox.philox4x64_10(np.array([ctr[0]], np.uint64), ctr[1], ctr[2], ctr[3], key[0], key[1])
        assert [int(x[0]) for x in vec] == ref


def test_uniform_open_interval():
    o = np.array([0, 2**64 - 1, 2**12 - 1, 2**12], dtype=np.uint64)
    u = philox.uniform52(o)
    assert u[0] == 2.0 ** -53 and 0.0 < u[0]
    assert u[1] == 1.0 - 2.0 ** -53 and u[1] < 1.0
    assert u[2] == u[0] and u[3] == 1.5 * 2.0 ** -52


def test_gaussian_distribution():
    """Real and imaginary parts i.i.d. N(0, 1/2): KS tests, |g|^2 ~ Exp(1)."""
    g = philox.gaussian_block(11, philox.tag(philox.PHASE_R, 3, 5), 100, 4000, 5).ravel()
    s = math.sqrt(0.5)
    assert stats.kstest(g.real, "norm", args=(0, s)).pvalue > 1e-3
    assert stats.kstest(g.imag, "norm", args=(0, s)).pvalue > 1e-3
    assert stats.kstest(np.abs(g) ** 2, "expon").pvalue > 1e-3
    assert abs(np.corrcoef(g.real, g.imag)[0, 1]) < 0.03


def test_gaussian_is_function_of_coordinates():
    """Entries depend only on (seed, tag, row, col): sub-blocks agree, tags and
    seeds decorrelate."""
    full = philox.gaussian_block(5, philox.tag(philox.PHASE_W, 2, 1), 0, 50, 8)
    part = philox.gaussian_block(5, philox.tag(philox.PHASE_W, 2, 1), 20, 10, 3)
    assert np.array_equal(full[20:30, :3], part)
    other = philox.gaussian_block(5, philox.tag(philox.PHASE_W, 2, 2), 0, 50, 8)
    seed2 = philox.gaussian_block(6, philox.tag(philox.PHASE_W, 2, 1), 0, 50, 8)
    assert not np.any(full == other) and not np.any(full == seed2)


def test_tag_fields_disjoint():
    assert philox.tag(1, 0, 0) == 1 << 56
    assert philox.tag(0, 1, 0) == 1 << 40
    assert philox.tag(4, 13, (1 << 40) - 1) >> 56 == 4
