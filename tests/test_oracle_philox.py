"""Pins of the oracle's counter-based Gaussian generator (CPU only)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        rows.append([int(w, 16) for w in line.split()])
    return rows


@pytest.mark.parametrize("row", _kat())
def test_philox_known_answers(row):
    got = philox.philox4x32_10(*[np.uint64(x) for x in row[:6]])
    assert [int(g) for g in got] == row[6:]


def test_uniforms_open_interval_exact():
    u = philox.uniforms_from_words(np.array([0, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 0.5 / 2**32 and u[1] == (2**32 - 0.5) / 2**32
    assert 0.0 < u[0] < u[1] < 1.0


def test_gaussian_moments_and_ks():
    z = philox.gaussian_block(400_000, slice_id=3, call_id=1, stream_id=0, seed=12345)
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert abs(stats.skew(z)) < 0.02
    assert abs(stats.kurtosis(z)) < 0.04
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_keys_give_independent_streams():
    a = philox.gaussian_block(100_000, 0, 0, 0, 7)
    for other in [(1, 0, 0, 7), (0, 1, 0, 7), (0, 0, 1, 7), (0, 0, 0, 8)]:
        b = philox.gaussian_block(100_000, *other)
        assert abs(np.corrcoef(a, b)[0, 1]) < 0.02
    # lanes within a group are uncorrelated as well (cos/sin pairs)
    g = a.reshape(-1, 4)
    c = np.corrcoef(g.T)
    assert np.abs(c - np.eye(4)).max() < 0.02


def test_omega_column_major_layout():
    n2, l = 13, 7
    om = philox.omega(n2, l, slice_id=5, call_id=2, stream_id=1, seed=99)
    flat = philox.gaussian_block(n2 * l, 5, 2, 1, 99)
    for i in range(n2):
        for c in range(l):
            assert om[i, c] == flat[i + n2 * c]
    # a prefix of a longer draw is the same draw (counter keyed, not stateful)
    assert np.array_equal(philox.gaussian_block(10, 5, 2, 1, 99), flat[:10])
