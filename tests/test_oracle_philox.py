"""Pins of the oracle's noise: Philox4x64-10 and the Box-Muller law."""

import math
import os

import numpy as np
import pytest

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def _kat_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat_rows())
def test_published_known_answers(ctr, key, expect):
    out = philox.philox4x64_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
    assert [int(x) for x in out] == expect


def _numpy_block(ctr, key):
    """NumPy's Philox advances its 256-bit counter before producing a block, so the block
    for counter C is the first output of a generator started at C - 1 (mod 2^256)."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)]
    g = np.random.Philox(key=np.array([int(key[0]), int(key[1])], dtype=np.uint64),
                         counter=np.array(words, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def test_against_numpy_philox():
    rng = np.random.default_rng(123)
    ctrs = rng.integers(0, 2**63, size=(64, 4), dtype=np.int64).astype(np.uint64)
    ctrs[:8, 0] = np.arange(8, dtype=np.uint64)     # small block indices as used for noise
    ctrs[:8, 3] = 0
    keys = rng.integers(0, 2**63, size=(64, 2), dtype=np.int64).astype(np.uint64)
    out = philox.philox4x64_10(ctrs, keys)
    for i in range(64):
        assert [int(x) for x in out[i]] == _numpy_block(ctrs[i], keys[i])


def test_uniform_extremes_are_exact():
    u = philox.uniforms23(np.array([0, (1 << 64) - 1, 1 << 41], dtype=np.uint64))
    assert u[0] == 0.5 * 2.0 ** -23
    assert u[1] == 1.0 - 2.0 ** -24
    assert u[2] == 1.5 * 2.0 ** -23
    assert np.all(np.float32(u) == u)    # exactly representable in FP32 too


def test_noise_is_standard_normal():
    n = 200_000
    x = philox.noise_event(seed=7, event=3, n=n // 9 + 1, n_feat=9).ravel()
    m, v = x.mean(), x.var()
    assert abs(m) < 5.0 / math.sqrt(x.size)
    assert abs(v - 1.0) < 5.0 * math.sqrt(2.0 / x.size)
    # Kolmogorov-Smirnov distance to N(0,1), well below the 1e-3-level critical value
    xs = np.sort(x)
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(xs / math.sqrt(2.0)))
    ks = np.max(np.abs(cdf - (np.arange(1, xs.size + 1) / xs.size)))
    assert ks < 1.95 / math.sqrt(xs.size)
    # every feature column has the same law (block / lane assignment is not degenerate)
    cols = philox.noise_event(seed=7, event=3, n=20000, n_feat=9)
    assert np.all(np.abs(cols.mean(axis=0)) < 0.05)
    assert np.all(np.abs(cols.std(axis=0) - 1.0) < 0.05)
    assert abs(np.corrcoef(cols.T)[np.triu_indices(9, 1)]).max() < 0.05


def test_noise_keys():
    a = philox.noise_event(1, 0, 10)
    assert np.array_equal(a, philox.noise_event(1, 0, 10))
    assert not np.allclose(a, philox.noise_event(2, 0, 10))
    assert not np.allclose(a, philox.noise_event(1, 1, 10))
    # slot i's noise does not depend on the event length
    assert np.array_equal(philox.noise_event(1, 5, 4), philox.noise_event(1, 5, 30)[:4])
    # the batch form keys by position in the batch
    off = np.array([0, 3, 3, 8])
    b = philox.noise_batch(9, off)
    assert np.array_equal(b[3:8], philox.noise_event(9, 2, 5))


def test_box_muller_pairs_share_radius():
    """z_a^2 + z_b^2 = -2 ln u_a for the pair built from words (0, 1)."""
    ctr = np.zeros((1, 4), dtype=np.uint64)
    ctr[0, 1] = 4
    ctr[0, 2] = 2
    w = philox.philox4x64_10(ctr, np.array([11, 0], dtype=np.uint64))
    u = philox.uniforms23(w)[0]
    x = philox.noise_event(11, 2, 5)[4]
    assert math.isclose(x[0] ** 2 + x[1] ** 2, -2.0 * math.log(u[0]), rel_tol=1e-12)
    assert math.isclose(x[2] ** 2 + x[3] ** 2, -2.0 * math.log(u[2]), rel_tol=1e-12)
    assert math.isclose(math.atan2(x[1], x[0]) % (2 * math.pi), 2 * math.pi * u[1], rel_tol=1e-12)
