"""Continuous-batching server (GPU): results alone = in the mix, admission by budget,
failure handling."""

import time

import numpy as np
import pytest

from oracle import sample
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu

CFG = configs.SMALL_MODEL


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def _requests(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        off, feat = events.truth_events(int(rng.integers(1, 9)), ("uniform", 1, 64), seed=100 + i)
        sched = (configs.Schedule(configs.RK4, 2), configs.Schedule(configs.EULER, 3),
                 configs.Schedule(configs.MIDPOINT, 3))[i % 3]
        out.append((off, feat, 1000 + i, sched))
    return out


def _alone(fmd, flat, reqs, precision=configs.FP32):
    m = fmd.Model(CFG.with_precision(precision), flat)
    res = [m.simulate(off, feat, seed, sched) for off, feat, seed, sched in reqs]
    m.close()
    return res


@pytest.mark.parametrize("precision", [configs.FP32, configs.BF16])
def test_mix_equals_alone_bitwise(env, precision):
    torch, fmd = env
    flat = params.draw(CFG, 7, perturbed=True)
    reqs = _requests(10)
    alone = _alone(fmd, flat, reqs, precision)
    m = fmd.Model(CFG.with_precision(precision), flat)
    srv = fmd.Server(m, hbm_budget_bytes=256 << 20)
    ids = [srv.submit(off, feat, seed, sched) for off, feat, seed, sched in reqs]
    for rid, ref in zip(ids, alone):
        out, st = srv.wait(rid)
        assert np.array_equal(out, ref)
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
    info = srv.info()
    assert info["iterations"] >= 8 and info["resident_requests"] == 0
    srv.close()
    m.close()


def _reco_offsets(off, seed):
    """Per-event reco counts from 0 to 2x the truth count (none where there is no truth)."""
    n = np.diff(off)
    r = np.random.default_rng(seed).integers(0, 2 * n + 1)
    r = np.minimum(r, 64)
    return np.r_[0, np.cumsum(np.where(n > 0, r, 0))].astype(np.int64)


@pytest.mark.parametrize("cfg", [CFG, configs.BASE_MODEL.with_precision(configs.BF16)],
                         ids=["small-fp32", "base-bf16"])
def test_reco_counts_in_the_mix_equal_alone_bitwise(env, cfg):
    """Requests with reco counts that differ from their truth counts (more, fewer, none),
    mixed with plain requests: each equals fmd_simulate_reco / fmd_simulate alone."""
    torch, fmd = env
    flat = params.draw(cfg, 11, perturbed=True)
    reqs = _requests(8, seed=5)
    roffs = [_reco_offsets(off, 50 + i) if i % 4 != 3 else None
             for i, (off, _, _, _) in enumerate(reqs)]
    m = fmd.Model(cfg, flat)
    alone = [m.simulate(off, feat, seed, sched, reco_offsets=ro)
             for (off, feat, seed, sched), ro in zip(reqs, roffs)]
    srv = fmd.Server(m, hbm_budget_bytes=512 << 20)
    ids = [srv.submit(off, feat, seed, sched, reco_offsets=ro)
           for (off, feat, seed, sched), ro in zip(reqs, roffs)]
    for rid, ref, ro in zip(ids, alone, roffs):
        out, _ = srv.wait(rid)
        assert out.shape == ref.shape and np.array_equal(out, ref)
    srv.close()
    m.close()
    assert any(ro is not None and ro[-1] > off[-1] for ro, (off, *_) in zip(roffs, reqs))
    assert any(ro is not None and ro[-1] < off[-1] for ro, (off, *_) in zip(roffs, reqs))


@pytest.mark.parametrize("cfg", [configs.ModelCfg(d_model=64, n_blocks=2, n_heads=2, n_max=64),
                                 configs.BASE_MODEL],
                         ids=["d64-heads32", "base-fused"])
def test_mix_equals_alone_bitwise_heads_of_32(env, cfg):
    # BF16 with heads of 32 keeps the cross K/V cache head-major: the server writes each
    # admitted request's rows into the planes at its pool offset
    torch, fmd = env
    cfg = cfg.with_precision(configs.BF16)
    flat = params.draw(cfg, 9, perturbed=True)
    reqs = _requests(6, seed=3)
    m = fmd.Model(cfg, flat)
    alone = [m.simulate(off, feat, seed, sched) for off, feat, seed, sched in reqs]
    srv = fmd.Server(m, hbm_budget_bytes=512 << 20)
    ids = [srv.submit(off, feat, seed, sched) for off, feat, seed, sched in reqs]
    for rid, ref in zip(ids, alone):
        out, _ = srv.wait(rid)
        assert np.array_equal(out, ref)
    srv.close()
    m.close()


def test_staggered_arrivals_overlap_and_match(env):
    torch, fmd = env
    flat = params.draw(CFG, 3)
    reqs = _requests(6, seed=5)
    alone = _alone(fmd, flat, reqs)
    m = fmd.Model(CFG, flat)
    srv = fmd.Server(m, hbm_budget_bytes=256 << 20)
    ids = []
    for r in reqs:
        ids.append(srv.submit(*r))
        time.sleep(0.002)
    results = [srv.wait(i) for i in ids]
    for (out, st), ref in zip(results, alone):
        assert np.array_equal(out, ref)
    # the first request was still running when later ones were admitted
    admits = [st["t_admit_ns"] for _, st in results]
    assert min(st["t_done_ns"] for _, st in results[:1]) > admits[1]
    srv.close()
    m.close()


def test_server_matches_oracle(env):
    torch, fmd = env
    flat = params.draw(CFG, 4, perturbed=True)
    off, feat = events.truth_events(5, ("uniform", 1, 50), seed=8)
    sched = configs.Schedule(configs.RK4, 3)
    m = fmd.Model(CFG, flat)
    srv = fmd.Server(m, hbm_budget_bytes=64 << 20)
    out, _ = srv.wait(srv.submit(off, feat, 9, sched))
    srv.close()
    m.close()
    ref = sample.simulate(flat, CFG, off, feat, sched, seed=9)
    assert errors.normwise_rel_err(out, ref).max() < 1e-4


def test_tight_budget_queues_requests_and_rejects_oversize(env):
    torch, fmd = env
    flat = params.draw(CFG, 1)
    m = fmd.Model(CFG, flat)
    probe = fmd.Server(m, hbm_budget_bytes=64 << 20)
    bpt = probe.info()["bytes_per_token"]
    probe.close()
    reqs = [(off, feat, s, sch) for off, feat, s, sch in _requests(8, seed=9)]
    biggest = max(int(r[0][-1]) for r in reqs)
    # one request at a time, at most (pool ranges are whole 64-row tiles)
    budget = (-(-biggest // 64) * 64 + 256 + 8) * bpt
    alone = _alone(fmd, flat, reqs)
    srv = fmd.Server(m, hbm_budget_bytes=budget)
    assert srv.info()["pool_tokens"] >= biggest
    ids = [srv.submit(*r) for r in reqs]
    outs = [srv.wait(i) for i in ids]
    for (out, _), ref in zip(outs, alone):
        assert np.array_equal(out, ref)
    big_off = np.array([0, 60, 120, 180, 240, 300], dtype=np.int64)
    big_feat = events.particles(np.random.default_rng(0), 300)
    if srv.info()["pool_tokens"] < 300:
        with pytest.raises(fmd.FmdError) as e:
            srv.submit(big_off, big_feat, 0, configs.Schedule(configs.EULER, 1))
        assert e.value.status == fmd.E_BUDGET
    srv.close()
    m.close()


def test_model_is_owned_while_a_server_exists(env):
    torch, fmd = env
    flat = params.draw(CFG, 1)
    m = fmd.Model(CFG, flat)
    srv = fmd.Server(m, hbm_budget_bytes=32 << 20)
    off, feat = events.truth_events(2, ("uniform", 3, 5), seed=1)
    with pytest.raises(fmd.FmdError) as e:
        m.simulate(off, feat, 0, configs.Schedule(configs.EULER, 1))
    assert e.value.status == fmd.E_STATE
    assert fmd.lib().fmd_model_destroy(m._h) == fmd.E_STATE
    with pytest.raises(fmd.FmdError):
        fmd.Server(m, hbm_budget_bytes=32 << 20)
    srv.close()
    out = m.simulate(off, feat, 0, configs.Schedule(configs.EULER, 1))
    assert out.shape == (off[-1], 9)
    m.close()


def test_empty_request_and_destroy_with_pending_work(env):
    torch, fmd = env
    flat = params.draw(CFG, 1)
    m = fmd.Model(CFG, flat)
    srv = fmd.Server(m, hbm_budget_bytes=64 << 20)
    rid = srv.submit(np.array([0, 0, 0]), np.zeros((0, 9), np.float32), 3, configs.Schedule())
    out, st = srv.wait(rid)
    assert out.shape == (0, 9)
    for r in _requests(12, seed=2):
        srv.submit(r[0], r[1], r[2], configs.Schedule(configs.RK4, 40))
    srv.close()                        # cancels whatever has not finished; must not hang
    m.close()


def test_invalid_submissions(env):
    torch, fmd = env
    flat = params.draw(CFG, 1)
    m = fmd.Model(CFG, flat)
    srv = fmd.Server(m, hbm_budget_bytes=64 << 20)
    with pytest.raises(fmd.FmdError) as e:
        srv.submit([0, 3, 2], np.zeros((3, 9), np.float32), 0, configs.Schedule())
    assert e.value.status == fmd.E_INVALID
    with pytest.raises(fmd.FmdError) as e:
        srv.submit([0, 70], np.zeros((70, 9), np.float32), 0, configs.Schedule())
    assert e.value.status == fmd.E_UNSUPPORTED
    with pytest.raises(fmd.FmdError) as e:
        srv.submit([0, 2], np.zeros((2, 9), np.float32), 0, configs.Schedule(configs.EULER, 0))
    assert e.value.status == fmd.E_INVALID
    srv.close()
    m.close()
