"""Pins of the oracle's generator and transforms (CPU)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

HERE = os.path.dirname(os.path.abspath(__file__))


def load_kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(t, 16) for t in line.split()])
    return rows


def test_philox_known_answers():
    rows = load_kat()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32_10(*[np.uint64(v) for v in r[:4]], r[4], r[5])
        assert [int(x) for x in out] == r[6:]


def test_philox_vectorised_equals_scalar():
    ks = np.arange(100, 164, dtype=np.uint64)
    vec = philox.words(12345, ks, 7, 3, 1)
    for i, k in enumerate(ks):
        sc = philox.words(12345, k, 7, 3, 1)
        assert [int(v[i]) for v in vec] == [int(v) for v in sc]


def test_key_from_seed_splits_64_bits():
    assert philox.key_from_seed(0) == (0, 0)
    assert philox.key_from_seed((5 << 32) | 9) == (9, 5)


def test_uniform_grid_exact_in_fp32():
    x = np.array([0, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint64)
    u = philox.uniform(x)
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24
    assert u[2] == 3.0 * 2.0 ** -24
    assert u[3] == 1.0 - 2.0 ** -24
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    assert np.all((u > 0) & (u < 1))


def test_uniforms_are_uniform():
    w = philox.raw_words(0, 1, 2, 3, 0, 1 << 16).astype(np.uint64)
    u = philox.uniform(w)
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # lag-1 pairs independent: correlation within 5 standard errors
    r = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(r) < 5.0 / np.sqrt(u.size)


def test_normals_moments_and_ks():
    z = philox.outer_normals(7, np.arange(4096), 3, 27).reshape(-1)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the pair (cos, sin) of one Box-Muller draw is uncorrelated
    zz = philox.outer_normals(7, np.arange(1 << 15), 0, 2)
    r = np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]
    assert abs(r) < 5.0 / np.sqrt(zz.shape[0])


def test_inner_prefix_property():
    """The first n_b' draws of a path are the same for every n_b >= n_b' (common numbers)."""
    a = philox.inner_uniforms(0, np.arange(10), 3, 2)
    b = philox.inner_uniforms(0, np.arange(10), 17, 2)
    assert np.array_equal(a, b[:, :3, :])


def test_streams_are_distinct():
    o = philox.words(0, 5, 0, 0, 0)
    i = philox.words(0, 5, 0, 0, 1)
    assert [int(v) for v in o] != [int(v) for v in i]
