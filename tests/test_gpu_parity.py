"""End-to-end parity of the HIP sampling path with the FP64 oracle (GPU).

Tolerances (normwise per feature, the worst feature): FP32 path 1e-4 for whole
integrations and 1e-5 for one velocity evaluation; BF16 path 2e-2, with the pT and eta
response mean and width within 1% of the oracle's.
"""

import dataclasses
import os

import numpy as np
import pytest

from oracle import net, philox, sample
from tests._gpu import fmd_lib, normwise, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_base_rk4x16_first256.npz")


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------------------------------
# integrator and state update against the closed form of a linear field

@pytest.mark.parametrize("scheme,K", [(configs.EULER, 1), (configs.EULER, 20), (configs.RK4, 1),
                                      (configs.RK4, 16), (configs.MIDPOINT, 1),
                                      (configs.MIDPOINT, 32)])
def test_linear_field_closed_form(env, scheme, K):
    torch, fmd = env
    alpha, beta = -0.7, 1.9
    off = np.array([0, 3, 3, 40], dtype=np.int64)
    x0 = np.random.default_rng(3).standard_normal((40, 9)).astype(np.float32)
    m = fmd.linear_field(alpha, beta)
    out = m.simulate_from_state(off, dev(torch, np.zeros((40, 9), np.float32)), dev(torch, x0),
                                configs.Schedule(scheme, K)).cpu().numpy()
    h = 1.0 / K
    g = 1.0
    for k in range(K):
        t = k * h
        if scheme == configs.EULER:
            g *= 1 + h * (alpha + beta * t)
        elif scheme == configs.MIDPOINT:
            g *= 1 + h * (alpha + beta * (t + h / 2)) * (1 + h * (alpha + beta * t) / 2)
        else:
            a, mid, e = alpha + beta * t, alpha + beta * (t + h / 2), alpha + beta * (t + h)
            k2 = mid * (1 + h * a / 2)
            k3 = mid * (1 + h * k2 / 2)
            k4 = e * (1 + h * k3)
            g *= 1 + h / 6 * (a + 2 * k2 + 2 * k3 + k4)
    np.testing.assert_allclose(out, g * x0.astype(np.float64), rtol=3e-6, atol=1e-6)
    m.close()


# ---------------------------------------------------------------------------------------
# one velocity evaluation

@pytest.mark.parametrize("cfg", [configs.SMALL_MODEL, configs.BASE_MODEL,
                                 configs.SMALL_MODEL.with_precision(configs.BF16),
                                 configs.BASE_MODEL.with_precision(configs.BF16)])
def test_velocity_matches_oracle(env, cfg):
    torch, fmd = env
    cfg = dataclasses.replace(cfg, n_max=1000)
    flat = params.draw(cfg, seed=4, perturbed=True)
    sizes = [1, 2, 0, 17, 64, 65, 40] if cfg.d_model == 64 else [1, 33, 0, 130, 200]
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    feat = events.particles(np.random.default_rng(8), int(off[-1]))
    x = np.random.default_rng(9).standard_normal((off[-1], 9)).astype(np.float32)
    t = np.linspace(0.05, 0.95, len(sizes)).astype(np.float32)
    m = fmd.Model(cfg, flat)
    v = m.velocity(off, dev(torch, feat), dev(torch, x), dev(torch, t)).cpu().numpy()
    m.close()
    P = net.unpack(flat, cfg)
    ref = np.concatenate([net.velocity(P, feat[off[e]:off[e + 1]], x[off[e]:off[e + 1]], float(t[e]))
                          for e in range(len(sizes)) if sizes[e]])
    err = errors.normwise_rel_err(v, ref).max()
    assert err < (1e-5 if cfg.precision == configs.FP32 else 2e-2), err


# ---------------------------------------------------------------------------------------
# whole integrations

def test_small_workload_fp32_all_events(env):
    torch, fmd = env
    w = configs.SMALL
    off, feat = events.for_workload(w)
    flat = params.draw(w.model, w.weight_seed)
    m = fmd.Model(w.model, flat)
    out = m.simulate(off, dev(torch, feat), w.noise_seed, w.schedule).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, w.model, off, feat, w.schedule, seed=w.noise_seed)
    err = errors.normwise_rel_err(out, ref)
    assert err.max() < 1e-4, err


def test_small_workload_perturbed_params_rk4(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    off, feat = events.truth_events(16, ("uniform", 1, 48), seed=21)
    flat = params.draw(cfg, seed=5, perturbed=True)
    sched = configs.Schedule(configs.RK4, 5)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, dev(torch, feat), 3, sched).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, cfg, off, feat, sched, seed=3)
    assert errors.normwise_rel_err(out, ref).max() < 1e-4


@pytest.mark.parametrize("cfg,tol", [(configs.SMALL_MODEL, 1e-4),
                                     (configs.BASE_MODEL.with_precision(configs.BF16), 2e-2)])
def test_midpoint_integration_matches_oracle(env, cfg, tol):
    torch, fmd = env
    off, feat = events.truth_events(8, ("uniform", 1, 48), seed=22)
    flat = params.draw(cfg, seed=6, perturbed=True)
    sched = configs.Schedule(configs.MIDPOINT, 6)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, dev(torch, feat), 4, sched).cpu().numpy()
    m.close()
    ref = sample.simulate(flat, cfg, off, feat, sched, seed=4)
    assert errors.normwise_rel_err(out, ref).max() < tol


def test_integrators_at_equal_evaluation_budget(env, capsys):
    """Euler 64 steps, midpoint 32, RK4 16 (64 evaluations each) on the FP32 path against a
    fine oracle integration (RK4, 64 steps): the step count and scheme trade speed for
    quality; at equal cost the higher order wins by orders of magnitude."""
    torch, fmd = env
    cfg = configs.BASE_MODEL
    off, feat = events.truth_events(4, ("uniform", 20, 60), seed=23)
    flat = params.draw(cfg, seed=0)
    ref = sample.simulate(flat, cfg, off, feat, configs.Schedule(configs.RK4, 64), seed=7)
    m = fmd.Model(cfg, flat)
    errs = {}
    for name, sched in (("euler", configs.Schedule(configs.EULER, 64)),
                        ("midpoint", configs.Schedule(configs.MIDPOINT, 32)),
                        ("rk4", configs.Schedule(configs.RK4, 16))):
        assert sched.evals == 64
        out = m.simulate(off, dev(torch, feat), 7, sched).cpu().numpy()
        errs[name] = float(errors.normwise_rel_err(out, ref).max())
    m.close()
    with capsys.disabled():
        print(f"\nerror vs fine oracle at 64 evaluations: {errs}")
    assert errs["rk4"] < errs["midpoint"] < errs["euler"]
    assert errs["rk4"] < 1e-3


def _golden():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden oracle outputs missing (tests/golden/make_oracle_outputs.py)")
    z = np.load(GOLDEN)
    return z["offsets"], z["reco"]


@pytest.mark.parametrize("precision,n_check,tol", [(configs.FP32, 128, 1e-4), (configs.BF16, 256, 2e-2)])
def test_base_workload_full_size(env, precision, n_check, tol):
    """All 4096 events in one call, the bench launch configuration; the leading subset is
    compared with the stored oracle outputs."""
    torch, fmd = env
    w = configs.BASE_FP32
    g_off, g_reco = _golden()
    off, feat = events.for_workload(w)
    cfg = w.model.with_precision(precision)
    flat = params.draw(cfg, w.weight_seed)
    m = fmd.Model(cfg, flat)
    out = m.simulate(off, dev(torch, feat), w.noise_seed, w.schedule).cpu().numpy()
    m.close()
    assert np.all(np.isfinite(out))
    assert np.array_equal(off[:len(g_off)], g_off)
    rows = int(g_off[n_check])
    err = errors.normwise_rel_err(out[:rows], g_reco[:rows])
    assert err.max() < tol, err
    if precision == configs.BF16:
        r = errors.response(out[:rows], feat[:rows])
        r0 = errors.response(g_reco[:rows], feat[:rows])
        assert errors.response_agrees(r, r0, 0.01), (r, r0)


# ---------------------------------------------------------------------------------------
# invariances and edge cases

def test_event_alone_equals_event_in_batch_bitwise(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 0, perturbed=True)
    off, feat = events.truth_events(40, ("uniform", 1, 60), seed=31)
    x0 = np.random.default_rng(4).standard_normal((off[-1], 9)).astype(np.float32)
    sched = configs.Schedule(configs.RK4, 2)
    for prec in (configs.FP32, configs.BF16):
        m = fmd.Model(cfg.with_precision(prec), flat)
        full = m.simulate_from_state(off, dev(torch, feat), dev(torch, x0), sched).cpu().numpy()
        for e in (0, 7, 39):
            a, b = off[e], off[e + 1]
            one = m.simulate_from_state(np.array([0, b - a]), dev(torch, feat[a:b]), dev(torch, x0[a:b]),
                                        sched).cpu().numpy()
            assert np.array_equal(one, full[a:b])
        # reversed event order: per-event results unchanged
        order = np.arange(40)[::-1]
        off_r, feat_r = events.subset(off, feat, order)
        _, x_r = events.subset(off, x0, order)
        rev = m.simulate_from_state(off_r, dev(torch, feat_r), dev(torch, x_r), sched).cpu().numpy()
        for i, e in enumerate(order):
            assert np.array_equal(rev[off_r[i]:off_r[i + 1]], full[off[e]:off[e + 1]])
        m.close()


def test_seeded_noise_is_keyed_by_event_index(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 0)
    off, feat = events.truth_events(5, ("uniform", 3, 9), seed=2)
    sched = configs.Schedule(configs.EULER, 3)
    m = fmd.Model(cfg, flat)
    a = m.simulate(off, dev(torch, feat), 11, sched).cpu().numpy()
    x0 = philox.noise_batch(11, off).astype(np.float32)
    b = m.simulate_from_state(off, dev(torch, feat), dev(torch, x0), sched).cpu().numpy()
    m.close()
    assert normwise(a, b) < 1e-5


def test_reco_slot_permutation_equivariance(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 1, perturbed=True)
    off = np.array([0, 50], dtype=np.int64)
    feat = events.particles(np.random.default_rng(3), 50)
    x0 = np.random.default_rng(5).standard_normal((50, 9)).astype(np.float32)
    perm = np.random.default_rng(6).permutation(50)
    m = fmd.Model(cfg, flat)
    sched = configs.Schedule(configs.RK4, 3)
    a = m.simulate_from_state(off, dev(torch, feat), dev(torch, x0), sched).cpu().numpy()
    b = m.simulate_from_state(off, dev(torch, feat), dev(torch, x0[perm]), sched).cpu().numpy()
    m.close()
    assert normwise(b, a[perm]) < 1e-5


def test_host_and_device_buffers_agree(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 0)
    off, feat = events.truth_events(9, ("uniform", 1, 30), seed=7)
    sched = configs.Schedule(configs.EULER, 4)
    m = fmd.Model(cfg, flat)
    d = m.simulate(off, dev(torch, feat), 5, sched).cpu().numpy()
    h = m.simulate(off, feat, 5, sched)
    m.close()
    assert isinstance(h, np.ndarray) and np.array_equal(d, h)


def test_nan_truth_stays_in_its_event(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 0)
    off, feat = events.truth_events(6, ("uniform", 5, 20), seed=9)
    sched = configs.Schedule(configs.EULER, 2)
    m = fmd.Model(cfg, flat)
    clean = m.simulate(off, dev(torch, feat), 1, sched).cpu().numpy()
    bad = feat.copy()
    bad[off[2]:off[3]] = np.nan
    dirty = m.simulate(off, dev(torch, bad), 1, sched).cpu().numpy()
    m.close()
    keep = np.ones(off[-1], bool)
    keep[off[2]:off[3]] = False
    assert np.array_equal(dirty[keep], clean[keep])
    assert np.all(np.isnan(dirty[~keep]))


def test_event_above_n_max_is_rejected(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL          # n_max = 64
    m = fmd.Model(cfg, params.draw(cfg, 0))
    off = np.array([0, 10, 75], dtype=np.int64)
    with pytest.raises(fmd.FmdError) as e:
        m.simulate(off, dev(torch, np.zeros((75, 9), np.float32)), 0, configs.Schedule())
    assert e.value.status == fmd.E_UNSUPPORTED
    m.close()


def test_workspace_regrows_and_shrinks(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 0)
    m = fmd.Model(cfg, flat)
    sched = configs.Schedule(configs.EULER, 2)
    outs = {}
    for n in (3, 40, 2):
        off, feat = events.truth_events(n, ("uniform", 1, 64), seed=n)
        outs[n] = (off, feat, m.simulate(off, dev(torch, feat), 2, sched).cpu().numpy())
    m.close()
    for n, (off, feat, out) in outs.items():
        ref = sample.simulate(flat, cfg, off, feat, sched, seed=2)
        assert errors.normwise_rel_err(out, ref).max() < 1e-4


def test_graph_replay_equals_eager_launches(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 2, perturbed=True)
    off, feat = events.truth_events(12, ("uniform", 1, 60), seed=13)
    feat_d = dev(torch, feat)
    for sched in (configs.Schedule(configs.RK4, 3), configs.Schedule(configs.EULER, 5)):
        m = fmd.Model(cfg, flat)
        m.graphs_enable(False)
        eager = m.simulate(off, feat_d, 4, sched).cpu().numpy()
        m.graphs_enable(True)
        out1 = torch.empty((off[-1], 9), dtype=torch.float32, device="cuda")
        g1 = m.simulate(off, feat_d, 4, sched, out=out1).cpu().numpy()       # captures
        g2 = m.simulate(off, feat_d, 4, sched, out=out1).cpu().numpy()       # replays cached graph
        g3 = m.simulate(off, feat_d, 4, sched).cpu().numpy()                 # new output: recapture
        m.close()
        assert np.array_equal(eager, g1) and np.array_equal(g1, g2) and np.array_equal(g1, g3)


def test_graph_cache_follows_new_inputs_of_the_same_shape(env):
    torch, fmd = env
    cfg = configs.SMALL_MODEL
    flat = params.draw(cfg, 2)
    off, feat = events.truth_events(8, ("uniform", 5, 30), seed=14)
    feat2 = events.particles(np.random.default_rng(99), int(off[-1]))
    sched = configs.Schedule(configs.EULER, 3)
    m = fmd.Model(cfg, flat)
    out = torch.empty((off[-1], 9), dtype=torch.float32, device="cuda")
    a = m.simulate(off, dev(torch, feat), 1, sched, out=out).cpu().numpy()
    b = m.simulate(off, dev(torch, feat2), 1, sched, out=out).cpu().numpy()
    m.close()
    ref_b = sample.simulate(flat, cfg, off, feat2, sched, seed=1)
    assert errors.normwise_rel_err(b, ref_b).max() < 1e-4
    assert not np.array_equal(a, b)
