"""Pins of the oracle's reco-multiplicity law (CPU).

The law (a stand-in: the paper says the model can emit extra, pile-up-like particles but not
how their number is drawn) is N_reco = min(n_max, N - lost + fakes), lost ~ Binomial(N, q) and
fakes ~ Binomial(M, p) from disjoint Philox words, 0 for an event without truth particles.
What fixes it independently of the code:
- the exact thresholds floor(x 2^64) at dyadic x;
- the degenerate laws (q = p = 0: the truth count; q near 1: all particles lost);
- the binomial means and variances over many events, at 5 sigma;
- lost and fakes uncorrelated (they must use different words);
- the clamp at n_max;
- the stream is keyed by (seed, event index) alone, separate from the noise stream.
"""

import numpy as np
import pytest

from oracle import multiplicity as mult
from oracle.philox import philox4x64_10


def test_thresholds_are_exact_at_dyadic_probabilities():
    assert mult.threshold(0.0) == 0
    assert mult.threshold(0.5) == 1 << 63
    assert mult.threshold(0.25) == 1 << 62
    assert mult.threshold(1.0 - 2.0 ** -53) == (1 << 64) - (1 << 11)
    with pytest.raises(ValueError):
        mult.threshold(1.0)
    with pytest.raises(ValueError):
        mult.threshold(-0.1)


def test_degenerate_laws():
    off = np.array([0, 0, 5, 5, 205, 206], dtype=np.int64)
    assert np.array_equal(mult.reco_offsets(off, 3, 0.0, 0.0, 0, 1000), off)
    # fakes with p = 0 add nothing; M trials with every word accepted cannot be asked for
    # (p < 1), but p = 1 - 2^-53 accepts all but a vanishing share
    assert np.array_equal(mult.reco_offsets(off, 3, 0.0, 0.0, 500, 1000), off)
    r = mult.reco_offsets(off, 3, 0.0, 1.0 - 2.0 ** -53, 40, 1000)
    assert np.array_equal(np.diff(r), np.where(np.diff(off) > 0, np.diff(off) + 40, 0))
    r = mult.reco_offsets(off, 3, 1.0 - 2.0 ** -53, 0.0, 0, 1000)
    assert r[-1] == 0
    # events without truth particles never get slots, whatever the fake law
    r = mult.reco_offsets(np.array([0, 0, 0], dtype=np.int64), 9, 0.0, 0.5, 100, 1000)
    assert r[-1] == 0


def test_loss_count_follows_the_binomial_law():
    n, E, q = 200, 400, 0.3
    off = np.arange(E + 1, dtype=np.int64) * n
    kept = np.diff(mult.reco_offsets(off, 11, q, 0.0, 0, 1000))
    lost = n - kept
    mean, var = lost.mean(), lost.var(ddof=1)
    assert abs(mean - n * q) < 5 * np.sqrt(n * q * (1 - q) / E)
    # variance of a sample variance of a (near-normal) binomial: 2 sigma^4 / (E - 1)
    s2 = n * q * (1 - q)
    assert abs(var - s2) < 5 * s2 * np.sqrt(2.0 / (E - 1))


def test_fake_count_follows_the_binomial_law_and_is_independent_of_losses():
    E, n, M, p, q = 2000, 64, 64, 0.25, 0.5
    off = np.arange(E + 1, dtype=np.int64) * n
    lost = np.array([n - mult.reco_count(5, e, n, q, 0.0, 0, 1000) for e in range(E)])
    fakes = np.array([mult.reco_count(5, e, n, 0.0, p, M, 1000) - n for e in range(E)])
    both = np.diff(mult.reco_offsets(off, 5, q, p, M, 1000))
    # the combined law is the two separate draws (disjoint words of one stream)
    assert np.array_equal(both, n - lost + fakes)
    assert abs(fakes.mean() - M * p) < 5 * np.sqrt(M * p * (1 - p) / E)
    s2 = M * p * (1 - p)
    assert abs(fakes.var(ddof=1) - s2) < 5 * s2 * np.sqrt(2.0 / (E - 1))
    # if losses and fakes read the same words they would be strongly correlated (M = N)
    corr = np.corrcoef(lost, fakes)[0, 1]
    assert abs(corr) < 5 / np.sqrt(E)


def test_clamp_at_the_particle_limit():
    off = np.array([0, 390, 400], dtype=np.int64)
    r = np.diff(mult.reco_offsets(off, 2, 0.0, 1.0 - 2.0 ** -53, 50, 400))
    assert list(r) == [400, 60]


def test_stream_is_keyed_by_seed_and_event_only():
    # an event's count does not depend on the events around it
    off_a = np.array([0, 30, 80, 81], dtype=np.int64)
    off_b = np.array([0, 7, 57, 300], dtype=np.int64)      # event 1 has 50 particles in both
    ra = np.diff(mult.reco_offsets(off_a, 4, 0.2, 0.1, 30, 1000))
    rb = np.diff(mult.reco_offsets(off_b, 4, 0.2, 0.1, 30, 1000))
    assert ra[1] == rb[1]
    # the words are Philox4x64-10 with key (seed, 1) at counters (c, event, 0, 0), not the
    # noise stream's key (seed, 0)
    w = mult.event_words(77, 3, 10)
    ctr = np.array([[0, 3, 0, 0], [1, 3, 0, 0], [2, 3, 0, 0]], dtype=np.uint64)
    assert np.array_equal(w, philox4x64_10(ctr, np.array([77, 1], np.uint64)).reshape(-1)[:10])
    assert not np.array_equal(w, philox4x64_10(ctr, np.array([77, 0], np.uint64)).reshape(-1)[:10])
    # different seeds give different counts somewhere
    off = np.arange(101, dtype=np.int64) * 50
    assert not np.array_equal(mult.reco_offsets(off, 1, 0.2, 0.2, 20, 1000),
                              mult.reco_offsets(off, 2, 0.2, 0.2, 20, 1000))
