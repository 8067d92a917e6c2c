"""Pins for the oracle's random numbers (Philox4x64-10, uniforms, Box-Muller).

The multiplier is a standard Gaussian matrix (Definition defrndm: i.i.d. mean 0,
variance 1).  The generator is pinned against the published Random123
known-answer values and against numpy's independent Philox implementation; the
normals are pinned by distribution tests, not by retyping Box-Muller.
"""
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("row", _kat_rows())
def test_philox_known_answers(orc, row):
    ctr, key, want = row
    got = orc.philox(ctr, key)
    assert [int(x) for x in got] == want


def _numpy_blocks(seed, stream, nblocks):
    # numpy's Philox increments the 256-bit counter before each block, so start
    # one below (m=0, stream) to get blocks m = 0, 1, 2, ... of the stream.
    c = (stream << 64) - 1
    ctr = np.array([(c >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64), counter=ctr)
    return bg.random_raw(4 * nblocks)


@pytest.mark.parametrize("seed,stream", [(0, 1), (1, 1), (12345, 2), (2**63 + 7, 3), (2**64 - 1, 1)])
def test_philox_stream_matches_numpy(orc, seed, stream):
    n = 257
    got = orc.words(seed, stream, n)
    want = _numpy_blocks(seed, stream, n)
    np.testing.assert_array_equal(got, want)


def test_uniforms_open_interval_and_exact(orc):
    w = orc.words(7, 1, 1000)
    u = orc.uniforms(7, 1, 4000)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    # 52-bit integer plus one half, times 2^-52: exact in binary64.
    k = (w >> np.uint64(12)).astype(np.float64)
    np.testing.assert_array_equal((u * 2.0**52 - 0.5), k)
    assert u.min() >= 2.0**-53 and u.max() <= 1 - 2.0**-53


def test_normals_distribution(orc):
    z = orc.normals(2024, 1, 400_000)
    assert abs(z.mean()) < 5 * 1 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    ks = stats.kstest(z, "norm")
    assert ks.pvalue > 1e-3
    # the four outputs of one block are independent of each other
    zz = z[: (z.size // 4) * 4].reshape(-1, 4)
    c = np.corrcoef(zz.T)
    assert np.max(np.abs(c - np.eye(4))) < 0.01
    # higher moments of N(0,1): skew 0, kurtosis 3
    assert abs(stats.skew(z)) < 0.02
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 0.05


def test_normals_pairs_share_radius(orc):
    # Box-Muller: both members of a pair lie on one circle whose squared radius
    # is -2 ln of the first uniform of the pair; a swapped uniform breaks this.
    z = orc.normals(5, 2, 4000).reshape(-1, 4)
    u = orc.uniforms(5, 2, 4000).reshape(-1, 4)
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u[:, 0]), rtol=1e-13)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2 * np.log(u[:, 2]), rtol=1e-13)
    # and the angle of the pair is 2 pi times the second uniform of the pair
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]), 2 * np.pi)
    np.testing.assert_allclose(ang, 2 * np.pi * u[:, 1], atol=1e-9)


def test_streams_and_seeds_differ(orc):
    a = orc.normals(1, 1, 64)
    b = orc.normals(1, 2, 64)
    c = orc.normals(2, 1, 64)
    assert not np.allclose(a, b) and not np.allclose(a, c)
    # prefix property: element e does not depend on how many are drawn
    np.testing.assert_array_equal(orc.normals(1, 1, 10), a[:10])
