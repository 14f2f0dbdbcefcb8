"""Pins of the oracle's velocity network and sampler by invariances and reductions.

The paper prints no network values, so the composed network is pinned through the
properties its definition forces: set symmetry (reco slots equivariant, truth set
invariant), single-element attention collapsing to its value path, softmax shift
invariance making key biases irrelevant, and zeroed weights reducing sub-blocks to the
identity on the residual stream.
"""

import numpy as np
import pytest

from oracle import net, sample as simulate
from oracle.ode import EULER, RK4
from workload import configs, events, params

CFG = configs.SMALL_MODEL


def _setup(n_truth=6, perturbed=True, seed=0):
    flat = params.draw(CFG, seed=seed, perturbed=perturbed)
    _, feat = events.truth_events(1, ("fixed", n_truth), seed=11)
    x = np.random.default_rng(12).standard_normal((n_truth, 9))
    return flat, feat.astype(np.float64), x


def test_reco_slot_permutation_equivariance():
    flat, u, x = _setup()
    P = net.unpack(flat, CFG)
    perm = np.random.default_rng(0).permutation(len(x))
    v = net.velocity(P, u, x, 0.3)
    np.testing.assert_allclose(net.velocity(P, u, x[perm], 0.3), v[perm], rtol=1e-12, atol=1e-13)
    out = simulate.simulate_event(P, u, x, RK4, 3)
    np.testing.assert_allclose(simulate.simulate_event(P, u, x[perm], RK4, 3), out[perm],
                               rtol=1e-11, atol=1e-12)


def test_truth_permutation_invariance():
    flat, u, x = _setup()
    P = net.unpack(flat, CFG)
    perm = np.random.default_rng(1).permutation(len(u))
    np.testing.assert_allclose(net.velocity(P, u[perm], x, 0.8), net.velocity(P, u, x, 0.8),
                               rtol=1e-12, atol=1e-13)


def test_truth_matters_and_time_matters():
    flat, u, x = _setup()
    P = net.unpack(flat, CFG)
    v = net.velocity(P, u, x, 0.5)
    u2 = u.copy()
    u2[0, 0] += 1.0
    assert np.abs(net.velocity(P, u2, x, 0.5) - v).max() > 1e-3
    assert np.abs(net.velocity(P, u, x, 0.6) - v).max() > 1e-4


def test_single_slot_self_attention_ignores_query_and_key_weights():
    """N = 1: softmax over one key is 1, so self-attention returns the V row and the Q and K
    columns of W_qkv (and their biases) cannot change v; the V columns can."""
    flat, u, x = _setup(n_truth=1)
    d = CFG.d_model
    v0 = net.velocity(net.unpack(flat, CFG), u, x, 0.4)
    f2 = flat.copy()
    nm = params.named(CFG, f2)
    rng = np.random.default_rng(5)
    for l in range(CFG.n_blocks):
        nm[f"blk{l}.W_qkv"][:, :2 * d] = rng.standard_normal((d, 2 * d))
        nm[f"blk{l}.b_qkv"][:2 * d] = rng.standard_normal(2 * d)
        nm[f"blk{l}.W_qc"][:] = rng.standard_normal((d, d))      # cross: one truth key
        nm[f"blk{l}.W_kc"][:] = rng.standard_normal((d, d))
    np.testing.assert_allclose(net.velocity(net.unpack(f2, CFG), u, x, 0.4), v0,
                               rtol=1e-11, atol=1e-12)
    nm[f"blk0.W_qkv"][:, 2 * d:] *= 1.5
    assert np.abs(net.velocity(net.unpack(f2, CFG), u, x, 0.4) - v0).max() > 1e-4


def test_key_biases_are_irrelevant_query_biases_are_not():
    """Adding b_k to every key adds q.b_k to a whole score row: softmax is unchanged."""
    flat, u, x = _setup()
    d = CFG.d_model
    v0 = net.velocity(net.unpack(flat, CFG), u, x, 0.2)
    f2 = flat.copy()
    nm = params.named(CFG, f2)
    rng = np.random.default_rng(6)
    for l in range(CFG.n_blocks):
        nm[f"blk{l}.b_qkv"][d:2 * d] += rng.standard_normal(d)
        nm[f"blk{l}.b_kc"][:] += rng.standard_normal(d)
    np.testing.assert_allclose(net.velocity(net.unpack(f2, CFG), u, x, 0.2), v0,
                               rtol=1e-10, atol=1e-11)
    nm["blk0.b_qkv"][:d] += rng.standard_normal(d)
    assert np.abs(net.velocity(net.unpack(f2, CFG), u, x, 0.2) - v0).max() > 1e-5


def test_zero_block_outputs_cut_truth_and_slot_coupling():
    """W_o = W_oc = W_dn = 0 with zero biases: every block is the identity on the
    residual stream, so v no longer depends on the truth set and each slot evolves on its
    own (v of one slot equals v of that slot alone)."""
    flat, u, x = _setup(perturbed=False)
    nm = params.named(CFG, flat)
    for l in range(CFG.n_blocks):
        for w in ("W_o", "W_oc", "W_dn"):
            nm[f"blk{l}.{w}"][:] = 0.0
    P = net.unpack(flat, CFG)
    v = net.velocity(P, u, x, 0.7)
    np.testing.assert_allclose(net.velocity(P, u[:2] * 3.0, x, 0.7), v, rtol=1e-12, atol=1e-13)
    for i in range(len(x)):
        np.testing.assert_allclose(net.velocity(P, u, x[i:i + 1], 0.7)[0], v[i],
                                   rtol=1e-12, atol=1e-13)


def test_state_embedding_enters_once():
    """With every matrix but W_xin and W_out zeroed and unit LayerNorms, the velocity of
    one slot is LN(x W_xin + b_xin + b_time) W_out: only the embedding path remains."""
    flat = params.draw(CFG, seed=3)
    nm = params.named(CFG, flat)
    for name in nm:
        if name.startswith("blk") and ".W_" in name or name in ("W_time",):
            nm[name][:] = 0.0
    nm["b_time"][:] = np.linspace(-1, 1, CFG.d_model)
    P = net.unpack(flat, CFG)
    x = np.array([[0.3, -1.2, 2.0, 1, 0, 0, 0, 0, -1.0]])
    h = x @ P["W_xin"] + P["b_time"]
    hn = (h - h.mean()) / np.sqrt(h.var() + 1e-5)
    np.testing.assert_allclose(net.velocity(P, np.zeros((3, 9)), x, 0.9), hn @ P["W_out"],
                               rtol=1e-12, atol=1e-13)


def test_simulate_batch_matches_per_event_and_handles_empty_events():
    w = configs.SMALL
    off = np.array([0, 3, 3, 7], dtype=np.int64)      # middle event is empty
    feat = events.particles(np.random.default_rng(0), 7)
    flat = params.draw(w.model, 0)
    sch = configs.Schedule(EULER, 2)
    out = simulate.simulate(flat, w.model, off, feat, sch, seed=1)
    assert out.shape == (7, 9)
    P = net.unpack(flat, w.model)
    from oracle.philox import noise_event
    e2 = simulate.simulate_event(P, feat[3:7].astype(np.float64), noise_event(1, 2, 4), EULER, 2)
    np.testing.assert_allclose(out[3:7], e2, rtol=1e-14)


def test_float32_diagnostic_mode_is_close_but_not_the_reference():
    flat, u, x = _setup()
    v64 = net.velocity(net.unpack(flat, CFG), u, x, 0.5)
    v32 = net.velocity(net.unpack(flat, CFG, np.float32), u, x, 0.5)
    assert v32.dtype == np.float32
    err = np.abs(v32 - v64).max() / np.abs(v64).max()
    assert 0 < err < 1e-5


def test_unpack_rejects_wrong_length():
    flat = params.draw(CFG, 0)
    with pytest.raises(ValueError):
        net.unpack(flat[:-1], CFG)
    assert params.count(CFG) == flat.size


def test_decode():
    x = np.array([[0.0, 1.5, 3.5, 0.1, 0.9, 0.2, 0.0, 0.0, -1.7]])
    d = simulate.decode(x)
    assert d["pt"][0] == 10.0 and d["eta"][0] == 1.5
    assert np.isclose(d["phi"][0], 3.5 - 2 * np.pi)
    assert d["cls"][0] == 1 and d["q"][0] == -1
