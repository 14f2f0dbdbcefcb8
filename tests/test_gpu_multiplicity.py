"""Reco multiplicities drawn on the device (GPU) under the stand-in law (truth particles
missed with probability q, Binomial(M, p) fake slots, the n_max clamp; Sec. 2.2: the model can
emit particles that match no truth particle). The counts are integer work, so they must equal
the oracle's bit for bit: on the base workload's truth with several laws, on empty events,
at the clamp and with the extreme probabilities. Then the drawn counts feed the sampler and the
result is compared with the oracle run on the oracle's own counts (BF16 tolerance 2e-2)."""

import numpy as np
import pytest

from oracle import multiplicity as mult
from oracle import sample
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu

LAWS = [(0.0, 0.0, 0), (0.05, 0.25, 64), (0.3, 0.01, 4096), (0.0, 1.0 - 2.0 ** -53, 17),
        (1.0 - 2.0 ** -53, 0.5, 3)]


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


@pytest.mark.parametrize("q,p,M", LAWS)
def test_counts_equal_the_oracle_bit_for_bit(env, q, p, M):
    _, fmd = env
    off, _ = events.truth_events(512, ("uniform", 20, 200), seed=31)
    sizes = np.diff(off)
    sizes[::7] = 0                                   # empty events
    sizes[5] = 999                                   # near and at the clamp
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    for seed, n_max in ((1, 1000), (2 ** 64 - 5, 150)):
        got = fmd.reco_multiplicity(off, seed, q, p, M, n_max)
        want = mult.reco_offsets(off, seed, q, p, M, n_max)
        assert np.array_equal(got, want), (seed, n_max)


def test_invalid_laws_are_rejected(env):
    _, fmd = env
    off = np.array([0, 3, 5], dtype=np.int64)
    for q, p, M in ((1.0, 0.0, 0), (0.0, -0.1, 0), (0.0, 0.1, 4097), (0.0, 0.1, -1)):
        with pytest.raises(fmd.FmdError):
            fmd.reco_multiplicity(off, 1, q, p, M, 100)
    with pytest.raises(fmd.FmdError):
        fmd.reco_multiplicity(np.array([0, 3, 2], dtype=np.int64), 1, 0.0, 0.0, 0, 100)


def test_drawn_counts_feed_the_sampler(env):
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(configs.BF16)
    flat = params.draw(cfg, seed=0)
    off, feat = events.truth_events(10, ("uniform", 20, 200), seed=32)
    q, p, M = 0.1, 0.2, 80
    roff = fmd.reco_multiplicity(off, 9, q, p, M, cfg.n_max)
    assert np.array_equal(roff, mult.reco_offsets(off, 9, q, p, M, cfg.n_max))
    assert not np.array_equal(roff, off)
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, torch.from_numpy(feat).cuda(), 9, sched, reco_offsets=roff).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, cfg, off, feat, sched, seed=9,
                          reco_offsets=mult.reco_offsets(off, 9, q, p, M, cfg.n_max))
    assert out.shape == ref.shape
    assert errors.normwise_rel_err(out, ref).max() < 2e-2
