"""Pins of the oracle's building blocks: LayerNorm, GELU, softmax, Linear, attention."""

import itertools
import math

import numpy as np
import pytest

from oracle import net


def test_layer_norm_constant_row_gives_shift():
    g = np.linspace(0.5, 2.0, 16)
    s = np.linspace(-1.0, 1.0, 16)
    z = np.full((3, 16), 4.25)
    np.testing.assert_array_equal(net.layer_norm(z, g, s), np.broadcast_to(s, (3, 16)))


def test_layer_norm_moments_and_affine_invariance():
    rng = np.random.default_rng(0)
    z = rng.standard_normal((5, 64)) * 30.0 + 7.0      # var >> eps: eps effect < 1e-8
    y = net.layer_norm(z, np.ones(64), np.zeros(64))
    np.testing.assert_allclose(y.mean(axis=1), 0.0, atol=1e-12)
    np.testing.assert_allclose(y.var(axis=1), 1.0, rtol=1e-7)     # biased variance
    y2 = net.layer_norm(3.0 * z - 11.0, np.ones(64), np.zeros(64))
    np.testing.assert_allclose(y2, y, atol=1e-7)
    # gain and shift act per feature after normalisation
    g, s = rng.standard_normal(64), rng.standard_normal(64)
    np.testing.assert_allclose(net.layer_norm(z, g, s), y * g + s, atol=1e-12)


def test_layer_norm_epsilon_and_biased_variance():
    # a two-valued row [a, -a]: biased variance a^2, normalised value a / sqrt(a^2 + eps)
    a = 1e-3
    y = net.layer_norm(np.array([[a, -a]]), np.ones(2), np.zeros(2))
    assert math.isclose(y[0, 0], a / math.sqrt(a * a + 1e-5), rel_tol=1e-14)


def test_gelu_textbook_values():
    # GELU(1) = Phi(1) (standard normal CDF at one standard deviation)
    assert math.isclose(float(net.gelu(np.array(1.0))), 0.8413447460685429, rel_tol=1e-15)
    assert float(net.gelu(np.array(0.0))) == 0.0
    # odd part: GELU(x) - GELU(-x) = x (erf is odd)
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(net.gelu(x) - net.gelu(-x), x, atol=1e-14)
    # tails: GELU(x) -> x for large x, -> 0 for very negative x
    assert abs(float(net.gelu(np.array(10.0))) - 10.0) < 1e-20
    assert abs(float(net.gelu(np.array(-10.0)))) < 1e-20
    # agrees with the standard library's erf at points across the range
    for v in (-3.3, -0.7, 0.2, 1.9, 4.4):
        assert math.isclose(float(net.gelu(np.array(v))), 0.5 * v * (1 + math.erf(v / math.sqrt(2))),
                            rel_tol=1e-14)


def test_softmax_rows():
    rng = np.random.default_rng(1)
    S = rng.standard_normal((4, 7)) * 5
    P = net.softmax_rows(S)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(net.softmax_rows(S + 123.0), P, atol=1e-15)
    big = net.softmax_rows(np.array([[1000.0, 1000.0, -1000.0]]))
    np.testing.assert_allclose(big, [[0.5, 0.5, 0.0]], atol=1e-15)


def test_linear_is_rows_times_in_out_matrix():
    x = np.array([[1.0, 2.0]])
    W = np.array([[1.0, 10.0, 100.0], [1000.0, 10000.0, 100000.0]])   # [in=2, out=3]
    b = np.array([0.5, 0.25, 0.125])
    np.testing.assert_array_equal(net.linear(x, W, b), [[2001.5, 20010.25, 200100.125]])


def test_attention_single_key_returns_value():
    rng = np.random.default_rng(2)
    Q = rng.standard_normal((5, 32))
    K = rng.standard_normal((1, 32))
    V = rng.standard_normal((1, 32))
    np.testing.assert_allclose(net.attention(Q, K, V, 4), np.broadcast_to(V, (5, 32)), atol=1e-15)


def test_attention_zero_query_is_mean_of_values():
    rng = np.random.default_rng(3)
    K = rng.standard_normal((9, 16))
    V = rng.standard_normal((9, 16))
    out = net.attention(np.zeros((2, 16)), K, V, 2)
    np.testing.assert_allclose(out, np.broadcast_to(V.mean(axis=0), (2, 16)), atol=1e-15)


def test_attention_heads_are_separate_and_scaled():
    # two heads of width 2; head 0 sees a dominant key 0, head 1 a dominant key 1
    Q = np.array([[10.0, 0.0, 0.0, 10.0]])
    K = np.array([[10.0, 0.0, 0.0, 0.0], [0.0, 0.0, 0.0, 10.0]])
    V = np.array([[1.0, 2.0, 3.0, 4.0], [5.0, 6.0, 7.0, 8.0]])
    out = net.attention(Q, K, V, 2)
    s = 100.0 / math.sqrt(2.0)          # score gap with scale 1/sqrt(dh), dh = 2
    p = 1.0 / (1.0 + math.exp(-s))
    np.testing.assert_allclose(out[0, :2], p * V[0, :2] + (1 - p) * V[1, :2], rtol=1e-14)
    np.testing.assert_allclose(out[0, 2:], (1 - p) * V[0, 2:] + p * V[1, 2:], rtol=1e-14)


def test_attention_permutations():
    rng = np.random.default_rng(4)
    Q, K, V = (rng.standard_normal((6, 16)) for _ in range(3))
    out = net.attention(Q, K, V, 4)
    pk = rng.permutation(6)
    np.testing.assert_allclose(net.attention(Q, K[pk], V[pk], 4), out, atol=1e-14)
    pq = rng.permutation(6)
    np.testing.assert_allclose(net.attention(Q[pq], K, V, 4), out[pq], atol=1e-14)


@pytest.mark.parametrize("nq,nk", [(1, 1), (2, 3), (3, 2), (3, 3)])
def test_attention_brute_force_tiny(nq, nk):
    """Scalar loops over every (query, key, feature) triple for tiny sets."""
    rng = np.random.default_rng(10 * nq + nk)
    H, dh = 2, 3
    Q, K, V = rng.standard_normal((nq, H * dh)), rng.standard_normal((nk, H * dh)), \
        rng.standard_normal((nk, H * dh))
    ref = np.zeros((nq, H * dh))
    for h, i in itertools.product(range(H), range(nq)):
        sc = [sum(Q[i, h * dh + a] * K[j, h * dh + a] for a in range(dh)) / math.sqrt(dh)
              for j in range(nk)]
        w = [math.exp(s) for s in sc]
        tot = sum(w)
        for a in range(dh):
            ref[i, h * dh + a] = sum(w[j] * V[j, h * dh + a] for j in range(nk)) / tot
    np.testing.assert_allclose(net.attention(Q, K, V, H), ref, rtol=1e-13, atol=1e-14)


def test_time_features():
    E = 32
    phi0 = net.time_features(0.0, E)
    np.testing.assert_array_equal(phi0, np.r_[np.zeros(16), np.ones(16)])
    t = 0.37
    phi = net.time_features(t, E)
    # k = 0 has unit frequency; the last frequency is 10000^(-15/16)
    assert math.isclose(phi[0], math.sin(t), rel_tol=1e-15)
    assert math.isclose(phi[16], math.cos(t), rel_tol=1e-15)
    assert math.isclose(phi[15], math.sin(t * 10000.0 ** (-15 / 16)), rel_tol=1e-14)
    np.testing.assert_allclose(phi[:16] ** 2 + phi[16:] ** 2, 1.0, atol=1e-15)
