"""Reco multiplicity of each event before the flow is integrated — oracle side.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the HIP path.

The paper's neural model need not emit one reco particle per truth particle. It can add
particles that correspond to no truth particle: pile-up-like "fake" particles that it
generates implicitly (Sec. 2.2, the pile-up paragraph; the configuration appendix on the
CMS model's pile-up). How the count is drawn is not described, so a stand-in law is read
here. For event e (its index within the call) with N truth particles:

    N_reco = min(n_max, N - lost + fakes)   when N > 0, and 0 when N = 0
    lost   = number of i < N     with w_i     < thr(q)   (each truth particle is missed
                                                           with probability q)
    fakes  = number of j < M     with w_(N+j) < thr(p)   (M Bernoulli trials of success
                                                           probability p: Binomial(M, p),
                                                           close to Poisson(M p) for small p)

where w_0, w_1, ... are the 64-bit output words of Philox4x64-10 with key (seed, 1) at the
counters (c, e, 0, 0), c = 0, 1, 2, ..., the four words of each counter taken in order, and
thr(x) = floor(x 2^64), an exact integer for a double x in [0, 1). Events without truth
particles get no reco slot, since a reco slot needs truth particles to attend to.

Every decision is an integer comparison, so the GPU must reproduce the counts bit for bit.
The key differs from the noise key (seed, 0), so the counts and the slot noise are
independent streams.
"""

import numpy as np

from .philox import MASK64, philox4x64_10

MAX_FAKE_TRIALS = 4096


def threshold(x: float) -> int:
    """floor(x 2^64) for x in [0, 1): the integer below which a uniform 64-bit word falls
    with probability x."""
    if not (0.0 <= x < 1.0):
        raise ValueError("probability must lie in [0, 1)")
    return int(np.floor(np.ldexp(np.float64(x), 64)))


def event_words(seed: int, event: int, n_words: int) -> np.ndarray:
    """The first n_words Philox words of an event's multiplicity stream (uint64)."""
    n_ctr = (n_words + 3) // 4
    ctr = np.zeros((n_ctr, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n_ctr, dtype=np.uint64)
    ctr[:, 1] = np.uint64(event)
    w = philox4x64_10(ctr, np.array([seed & MASK64, 1], dtype=np.uint64))
    return w.reshape(-1)[:n_words]


def reco_count(seed: int, event: int, n_truth: int, loss_prob: float, fake_prob: float,
               fake_trials: int, n_max: int) -> int:
    """N_reco of one event under the law above."""
    if not (0 <= fake_trials <= MAX_FAKE_TRIALS):
        raise ValueError("fake_trials out of range")
    if n_truth <= 0:
        return 0
    tq, tp = threshold(loss_prob), threshold(fake_prob)
    w = event_words(seed, event, n_truth + fake_trials)
    lost = sum(1 for i in range(n_truth) if int(w[i]) < tq)
    fakes = sum(1 for j in range(fake_trials) if int(w[n_truth + j]) < tp)
    return min(n_max, n_truth - lost + fakes)


def reco_offsets(truth_offsets, seed: int, loss_prob: float, fake_prob: float, fake_trials: int,
                 n_max: int) -> np.ndarray:
    """CSR offsets [E + 1] of the reco slots of a call whose truth events have the given
    offsets: the exclusive prefix sum of the per-event counts."""
    off = np.asarray(truth_offsets, dtype=np.int64)
    counts = [reco_count(seed, e, int(off[e + 1] - off[e]), loss_prob, fake_prob, fake_trials, n_max)
              for e in range(len(off) - 1)]
    return np.r_[0, np.cumsum(counts, dtype=np.int64)].astype(np.int64)
