"""Reco multiplicities that differ from the truth multiplicities (Sec. 2.2: the reco slots
self-attend and cross-attend to the event's truth particles), on the GPU against the FP64
oracle: more and fewer reco slots than truth particles, events with truth particles and no
reco slot, a truth side much larger than the reco side, key counts spanning several
attention chunks and query tiles, and the equal-count case bit for bit against the plain
sampler. Tolerances as for the sampler: FP32 1e-4 and BF16 2e-2 normwise per feature."""

import numpy as np
import pytest

from oracle import sample
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _reco_offsets(off, rng, lo, hi, n_max):
    """Reco counts = truth count scaled by a factor in [lo, hi], at least one slot where the
    event has truth particles, at most n_max; every third event gets none."""
    n = np.diff(off)
    r = np.minimum(np.maximum(np.rint(n * rng.uniform(lo, hi, len(n))), 1), n_max).astype(np.int64)
    r[n == 0] = 0
    r[::3] = 0
    return np.r_[0, np.cumsum(r)].astype(np.int64)


def _events_with_counts(n_truth, seed):
    off = np.r_[0, np.cumsum(n_truth)].astype(np.int64)
    return off, events.particles(np.random.default_rng(seed), int(off[-1]))


def test_small_model_matches_oracle(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, seed=3, perturbed=True)
    n_truth = [5, 12, 1, 30, 0, 7, 40, 3, 16, 9, 25, 2, 64]
    n_reco = [9, 4, 1, 64, 0, 0, 40, 8, 1, 20, 13, 2, 17]
    off, feat = _events_with_counts(n_truth, 41)
    roff = np.r_[0, np.cumsum(n_reco)].astype(np.int64)
    sched = configs.Schedule(configs.RK4, 3)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, dev(torch, feat), 5, sched, reco_offsets=roff).cpu().numpy()
    host = m.simulate(off, feat, 5, sched, reco_offsets=roff)
    m.close()
    assert out.shape == (roff[-1], 9) and np.array_equal(out, host)
    ref = sample.simulate(flat, cfg, off, feat, sched, seed=5, reco_offsets=roff)
    assert errors.normwise_rel_err(out, ref).max() < 1e-4


@pytest.mark.parametrize("lo,hi", [(0.5, 1.6), (0.01, 0.05)])
def test_base_bf16_fused_path_matches_oracle(env, lo, hi):
    """The BF16 fused kernels at the base shape; the second case has one to a few reco slots
    against hundreds of truth particles (the workspace is sized by the truth side)."""
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(configs.BF16)
    flat = params.draw(cfg, seed=0)
    off, feat = events.truth_events(6, ("uniform", 90, 300), seed=42)
    roff = _reco_offsets(off, np.random.default_rng(2), lo, hi, cfg.n_max)
    sched = configs.Schedule(configs.EULER, 4)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, dev(torch, feat), 9, sched, reco_offsets=roff).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, cfg, off, feat, sched, seed=9, reco_offsets=roff)
    assert np.all(np.isfinite(out))
    assert errors.normwise_rel_err(out, ref).max() < 2e-2


@pytest.mark.parametrize("precision", [configs.FP32, configs.BF16])
def test_equal_counts_reproduce_the_plain_sampler_bitwise(env, precision):
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(precision)
    flat = params.draw(cfg, seed=1)
    off, feat = events.truth_events(20, ("uniform", 1, 150), seed=43)
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(cfg, flat)
    a = m.simulate(off, dev(torch, feat), 2, sched).cpu().numpy()
    b = m.simulate(off, dev(torch, feat), 2, sched, reco_offsets=off).cpu().numpy()
    c = m.simulate(off, dev(torch, feat), 2, sched).cpu().numpy()
    m.close()
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_event_alone_equals_event_in_batch_and_layouts_alternate(env):
    """Per-event results do not depend on the other events (the event alone sits behind
    empty events so that it keeps its noise index), and two calls with the same token
    counts but different reco layouts (cross-attention work lists) each give their own
    result when they alternate on one model."""
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(configs.BF16)
    flat = params.draw(cfg, seed=2)
    off, feat = events.truth_events(10, ("uniform", 10, 200), seed=44)
    roff = _reco_offsets(off, np.random.default_rng(3), 0.3, 2.0, cfg.n_max)
    sched = configs.Schedule(configs.EULER, 3)
    m = fmd.Model(cfg, flat)
    full = m.simulate(off, dev(torch, feat), 4, sched, reco_offsets=roff).cpu().numpy()
    for e in (1, 5, 8):
        a, b = off[e], off[e + 1]
        ra, rb = roff[e], roff[e + 1]
        alone = np.r_[np.zeros(e + 1, np.int64), b - a]
        ralone = np.r_[np.zeros(e + 1, np.int64), rb - ra]
        one = m.simulate(alone, dev(torch, feat[a:b]), 4, sched, reco_offsets=ralone)
        assert np.array_equal(one.cpu().numpy(), full[ra:rb])
    r2 = np.r_[0, np.cumsum(np.diff(roff)[::-1])].astype(np.int64)
    other = m.simulate(off, dev(torch, feat), 4, sched, reco_offsets=r2).cpu().numpy()
    again = m.simulate(off, dev(torch, feat), 4, sched, reco_offsets=roff).cpu().numpy()
    assert np.array_equal(again, full)
    m.close()
    m2 = fmd.Model(cfg, flat)
    fresh = m2.simulate(off, dev(torch, feat), 4, sched, reco_offsets=r2).cpu().numpy()
    m2.close()
    assert np.array_equal(other, fresh)


def test_full_base_workload_with_scaled_reco_counts(env):
    """All 4096 events of the base workload in one call, with per-event reco counts scaled
    by a seeded factor in [0.8, 1.3] (the bench's reco leg), in the bench's precision and
    schedule; sampled events against the oracle."""
    torch, fmd = env
    w = configs.BASE_BF16
    off, feat = events.for_workload(w)
    n = np.diff(off)
    f = np.random.default_rng(11).uniform(0.8, 1.3, len(n))
    r = np.where(n > 0, np.clip(np.rint(n * f), 1, w.model.n_max), 0).astype(np.int64)
    roff = np.r_[0, np.cumsum(r)].astype(np.int64)
    flat = params.draw(w.model, w.weight_seed)
    m = fmd.Model(w.model, flat)
    out = m.simulate(off, dev(torch, feat), w.noise_seed, w.schedule, reco_offsets=roff).cpu().numpy()
    m.close()
    assert out.shape == (roff[-1], 9) and np.all(np.isfinite(out))
    ids = [0, 1777, 4095]
    ref = sample.simulate_events(flat, w.model, off, feat, w.schedule, seed=w.noise_seed,
                                 event_ids=ids, reco_offsets=roff)
    got = np.concatenate([out[roff[e]:roff[e + 1]] for e in ids])
    assert errors.normwise_rel_err(got, np.concatenate(ref)).max() < 2e-2


@pytest.mark.parametrize("precision", [configs.FP32, configs.BF16])
def test_plain_and_reco_calls_alternate_on_one_output_buffer(env, precision):
    """A reco call (50 truth particles, 30 reco slots) and a plain call (30 particles) have
    the same reco-side shapes, so only the cross-attention work list tells their stage
    graphs apart. Alternating them on one model and one output buffer must give each call
    the result a fresh model gives."""
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(precision)
    flat = params.draw(cfg, seed=4)
    off50, f50 = _events_with_counts([50], 45)
    off30 = np.array([0, 30], np.int64)
    f30 = f50[:30].copy()
    roff = np.array([0, 30], np.int64)
    sched = configs.Schedule(configs.EULER, 2)
    out = torch.empty((30, 9), dtype=torch.float32, device="cuda")

    def fresh(o, f, r):
        m2 = fmd.Model(cfg, flat)
        y = m2.simulate(o, dev(torch, f), 6, sched, reco_offsets=r).cpu().numpy()
        m2.close()
        return y

    want_reco, want_plain = fresh(off50, f50, roff), fresh(off30, f30, None)
    assert not np.array_equal(want_reco, want_plain)
    m = fmd.Model(cfg, flat)
    for _ in range(2):
        a = m.simulate(off50, dev(torch, f50), 6, sched, out=out, reco_offsets=roff).cpu().numpy()
        b = m.simulate(off30, dev(torch, f30), 6, sched, out=out).cpu().numpy()
        assert np.array_equal(a, want_reco) and np.array_equal(b, want_plain)
    m.close()
