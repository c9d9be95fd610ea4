"""Pins of the oracle's Philox4x64-10 against numpy's independent implementation."""
import numpy as np
import pytest
import scipy.stats

from oracle import philox


def numpy_philox_block(counter, key):
    # numpy's Philox increments its 256-bit counter before producing a block, so starting one
    # below the counter yields the block for `counter` itself (c0 >= 1 avoids the borrow).
    c = np.array(counter, dtype=np.uint64)
    c[0] -= np.uint64(1)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=c)
    return bg.random_raw(4)


def test_matches_numpy_philox():
    rng = np.random.default_rng(123)
    for _ in range(300):
        ctr = [int(v) for v in rng.integers(1, 2**63, size=4, dtype=np.uint64)]
        ctr[1] = int(rng.integers(0, 2**20))
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.uint64)]
        ref = numpy_philox_block(ctr, key)
        got = philox.philox4x64(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))
        assert [int(g) for g in got] == [int(r) for r in ref]


def test_vectorised_matches_scalar():
    idx = np.arange(1, 200, dtype=np.uint64)
    x = philox.philox4x64(idx, 7, 3, 1, 99, 0)
    for k in (0, 5, 198):
        ref = numpy_philox_block([int(idx[k]), 7, 3, 1], [99, 0])
        assert [int(v[k]) for v in x] == [int(r) for r in ref]


def test_uniform_range_and_chi2():
    x0, _, _, _ = philox.philox4x64(np.arange(400000, dtype=np.uint64), 1, 2, 0, 42, 0)
    u = philox.uniform(x0)
    assert u.min() >= 0.0 and u.max() < 1.0
    counts, _ = np.histogram(u, bins=100, range=(0, 1))
    chi2 = ((counts - 4000.0) ** 2 / 4000.0).sum()
    assert scipy.stats.chi2.sf(chi2, 99) > 1e-4


def test_gaussian_ks():
    x0, x1, _, _ = philox.philox4x64(np.arange(200000, dtype=np.uint64), 0, 0, 1, 5, 0)
    z = philox.gaussian(x0, x1)
    assert np.all(np.isfinite(z))
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4


def test_uniform_edges():
    assert philox.uniform(np.array([0], dtype=np.uint64))[0] == 0.0
    top = philox.uniform(np.array([np.iinfo(np.uint64).max], dtype=np.uint64))[0]
    assert top == 1.0 - 2.0 ** -53
    z = philox.gaussian(np.array([np.iinfo(np.uint64).max], dtype=np.uint64), np.array([0], dtype=np.uint64))
    assert z[0] == 0.0
