"""Fused BF16 block kernels (GPU): LN1 + QKV, the self-attention projection with the
residual update + LN2 + cross query, and the cross-attention projection + LN3 + whole MLP.

They are checked against the FP64 oracle (normwise 2e-2, the BF16 tolerance) and against
the unfused BF16 GEMM path, on ragged events that span several 128-row tiles, and for the
invariances that hold exactly: an event alone equals the event inside a batch, graph
replay equals eager launches.
"""

import dataclasses

import numpy as np
import pytest

from oracle import net, sample
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu

CFG = dataclasses.replace(configs.BASE_MODEL.with_precision(configs.BF16), n_max=1000)


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _inputs(sizes, seed):
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    feat = events.particles(np.random.default_rng(seed), int(off[-1]))
    x = np.random.default_rng(seed + 1).standard_normal((off[-1], 9)).astype(np.float32)
    t = np.linspace(0.02, 0.98, len(sizes)).astype(np.float32)
    return off, feat, x, t


@pytest.mark.parametrize("sizes", [[1, 127, 128, 129, 0, 3], [700, 5, 300], [1000]])
def test_fused_velocity_matches_oracle_and_unfused(env, sizes):
    torch, fmd = env
    flat = params.draw(CFG, seed=6, perturbed=True)
    off, feat, x, t = _inputs(sizes, 20 + len(sizes))
    m = fmd.Model(CFG, flat)
    args = (off, dev(torch, feat), dev(torch, x), dev(torch, t))
    v_fused = m.velocity(*args).cpu().numpy()
    m.fused_enable(False)
    v_gemm = m.velocity(*args).cpu().numpy()
    m.close()
    P = net.unpack(flat, CFG)
    ref = np.concatenate([net.velocity(P, feat[off[e]:off[e + 1]], x[off[e]:off[e + 1]], float(t[e]))
                          for e in range(len(sizes)) if sizes[e]])
    assert np.all(np.isfinite(v_fused))
    assert errors.normwise_rel_err(v_fused, ref).max() < 2e-2
    assert errors.normwise_rel_err(v_gemm, ref).max() < 2e-2
    assert errors.normwise_rel_err(v_fused, v_gemm).max() < 2e-2
    assert not np.array_equal(v_fused, v_gemm)        # the two paths really differ


def test_embedding_in_the_qkv_kernel_changes_nothing(env):
    """Block 0's QKV kernel forms the input embedding itself (FUSED_EMBED) in the order of
    the embedding kernel: velocity (per-event times) and a whole integration (stage times)
    are bitwise the same as with the embedding kernel."""
    torch, fmd = env
    flat = params.draw(CFG, seed=8, perturbed=True)
    off, feat, x, t = _inputs([1, 127, 128, 129, 0, 3, 260], 40)
    m = fmd.Model(CFG, flat)
    args = (off, dev(torch, feat), dev(torch, x), dev(torch, t))
    sched = configs.Schedule(configs.RK4, 2)
    res = {}
    for mask in (fmd.FUSED_ALL, fmd.FUSED_ALL & ~fmd.FUSED_EMBED):
        m.fused_enable(mask)
        res[mask] = (m.velocity(*args).cpu().numpy(),
                     m.simulate(off, dev(torch, feat), 3, sched).cpu().numpy())
    m.close()
    a, b = res.values()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_fused_integration_matches_oracle(env):
    torch, fmd = env
    flat = params.draw(CFG, seed=7, perturbed=True)
    off, feat = events.truth_events(5, ("uniform", 20, 200), seed=41)
    sched = configs.Schedule(configs.RK4, 4)
    m = fmd.Model(CFG, flat)
    out = m.simulate(off, dev(torch, feat), 11, sched).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, CFG, off, feat, sched, seed=11)
    assert errors.normwise_rel_err(out, ref).max() < 2e-2


def test_fused_event_alone_equals_event_in_batch_bitwise(env):
    torch, fmd = env
    flat = params.draw(CFG, 0, perturbed=True)
    off, feat = events.truth_events(30, ("uniform", 1, 200), seed=32)
    x0 = np.random.default_rng(5).standard_normal((off[-1], 9)).astype(np.float32)
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(CFG, flat)
    full = m.simulate_from_state(off, dev(torch, feat), dev(torch, x0), sched).cpu().numpy()
    for e in (0, 13, 29):
        a, b = off[e], off[e + 1]
        one = m.simulate_from_state(np.array([0, b - a]), dev(torch, feat[a:b]),
                                    dev(torch, x0[a:b]), sched).cpu().numpy()
        assert np.array_equal(one, full[a:b])
    m.close()


def test_fused_graph_replay_equals_eager(env):
    torch, fmd = env
    flat = params.draw(CFG, 3, perturbed=True)
    off, feat = events.truth_events(9, ("uniform", 1, 200), seed=15)
    feat_d = dev(torch, feat)
    sched = configs.Schedule(configs.RK4, 3)
    m = fmd.Model(CFG, flat)
    m.graphs_enable(False)
    eager = m.simulate(off, feat_d, 4, sched).cpu().numpy()
    m.graphs_enable(True)
    g1 = m.simulate(off, feat_d, 4, sched).cpu().numpy()
    g2 = m.simulate(off, feat_d, 4, sched).cpu().numpy()
    # switching the kernels drops the captured graph
    m.fused_enable(False)
    u = m.simulate(off, feat_d, 4, sched).cpu().numpy()
    m.fused_enable(True)
    g3 = m.simulate(off, feat_d, 4, sched).cpu().numpy()
    m.close()
    assert np.array_equal(eager, g1) and np.array_equal(g1, g2) and np.array_equal(g1, g3)
    assert not np.array_equal(u, g1)


def test_fused_kernels_only_where_they_exist(env):
    torch, fmd = env
    for cfg in (configs.BASE_MODEL, configs.SMALL_MODEL.with_precision(configs.BF16)):
        m = fmd.Model(cfg, params.draw(cfg, 0))
        with pytest.raises(fmd.FmdError) as e:
            m.fused_enable(True)
        assert e.value.status == fmd.E_UNSUPPORTED
        m.fused_enable(False)
        assert m.kernel_name(fmd.K_GEMM_QKV) == "k_gemm_qkv"
        m.close()
    m = fmd.Model(CFG, params.draw(CFG, 0))
    assert m.kernel_name(fmd.K_GEMM_QKV) == "k_fused_qkv"
    m.close()


def test_graph_recaptured_when_only_event_lengths_change(env):
    # same event and token counts, different lengths: the attention work bins differ, so a
    # cached graph must not be replayed
    torch, fmd = env
    flat = params.draw(CFG, 4, perturbed=True)
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(CFG, flat)
    outs = {}
    for sizes in ([400, 10, 10, 10], [10, 10, 10, 400], [108, 108, 108, 106]):
        off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
        feat = events.particles(np.random.default_rng(3), int(off[-1]))
        res = []
        for g in (False, True):
            m.graphs_enable(g)
            res.append(m.simulate(off, dev(torch, feat), 8, sched).cpu().numpy())
        outs[tuple(sizes)] = res
    m.close()
    for eager, graph in outs.values():
        assert np.array_equal(eager, graph)


@pytest.mark.parametrize("heads", [4, 16])
def test_bf16_width_256_with_other_head_counts_runs_unfused(env, heads):
    """The fused kernels write 8 head-major planes of width 32, so a BF16 d = 256 model with
    4 or 16 heads must take the GEMM path (and say so) and still match the oracle."""
    torch, fmd = env
    cfg = dataclasses.replace(CFG, n_heads=heads)
    flat = params.draw(cfg, seed=8, perturbed=True)
    off, feat, x, t = _inputs([40, 0, 130, 7], 70 + heads)
    m = fmd.Model(cfg, flat)
    with pytest.raises(fmd.FmdError):
        m.fused_enable(True)
    m.timing_enable(True)
    v = m.velocity(off, dev(torch, feat), dev(torch, x), dev(torch, t)).cpu().numpy()
    sched = configs.Schedule(configs.RK4, 2)
    out = m.simulate(off, dev(torch, feat), 3, sched).cpu().numpy()
    fused_launches = m.timing_read(fmd.K_FUSED_MLP)[1] + m.timing_read(fmd.K_FUSED_OQC)[1]
    gemm_launches = m.timing_read(fmd.K_GEMM_UP)[1]
    m.close()
    assert fused_launches == 0 and gemm_launches > 0
    P = net.unpack(flat, cfg)
    ref = np.concatenate([net.velocity(P, feat[off[e]:off[e + 1]], x[off[e]:off[e + 1]], float(t[e]))
                          for e in range(4) if off[e + 1] > off[e]])
    assert errors.normwise_rel_err(v, ref).max() < 2e-2
    ref_s = sample.simulate(flat, cfg, off, feat, sched, seed=3)
    assert errors.normwise_rel_err(out, ref_s).max() < 2e-2
