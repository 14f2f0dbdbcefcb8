"""Pins of the oracle with reco multiplicities that differ from the truth multiplicities
(the model can emit more or fewer reco particles than truth particles; Sec. 2.2: the reco
slots attend to each other and, through cross-attention, to the event's truth set).

The properties the definition forces when N_reco != N_truth: cross-attention normalises
over the truth particles only (duplicated truth particles change nothing), a single truth
particle makes the cross-attention queries and keys irrelevant, the truth enters only
through cross-attention, set symmetry on both sides, and the noise of a reco slot depends
on (seed, event, slot) alone."""

import numpy as np
import pytest

from oracle import net, sample
from oracle.ode import EULER, RK4
from oracle.philox import noise_event
from workload import configs, events, params

CFG = configs.SMALL_MODEL


def _setup(n_truth, n_reco, seed=0):
    P = net.unpack(params.draw(CFG, seed=seed, perturbed=True), CFG)
    u = events.particles(np.random.default_rng(21), n_truth).astype(np.float64)
    x = np.random.default_rng(22).standard_normal((n_reco, 9))
    return P, u, x


@pytest.mark.parametrize("n_truth,n_reco", [(3, 7), (6, 2)])
def test_set_symmetry_with_unequal_counts(n_truth, n_reco):
    P, u, x = _setup(n_truth, n_reco)
    v = net.velocity(P, u, x, 0.4)
    assert v.shape == (n_reco, 9)
    pr = np.random.default_rng(1).permutation(n_reco)
    pt = np.random.default_rng(2).permutation(n_truth)
    np.testing.assert_allclose(net.velocity(P, u, x[pr], 0.4), v[pr], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(net.velocity(P, u[pt], x, 0.4), v, rtol=1e-12, atol=1e-13)


def test_duplicated_truth_particles_change_nothing():
    """Equal keys share the softmax weight equally and carry the same value row: three
    copies of each truth particle give the same velocity as one copy."""
    P, u, x = _setup(2, 5)
    v = net.velocity(P, u, x, 0.7)
    np.testing.assert_allclose(net.velocity(P, np.repeat(u, 3, axis=0), x, 0.7), v,
                               rtol=1e-11, atol=1e-12)
    assert np.abs(net.velocity(P, u[:1], x, 0.7) - v).max() > 1e-4


def test_single_truth_particle_makes_cross_queries_and_keys_irrelevant():
    P, u, x = _setup(1, 4)
    v = net.velocity(P, u, x, 0.2)
    rng = np.random.default_rng(5)
    for B in P["blocks"]:
        B["W_qc"] = B["W_qc"] + rng.standard_normal(B["W_qc"].shape)
        B["b_kc"] = B["b_kc"] + rng.standard_normal(B["b_kc"].shape)
        B["W_kc"] = B["W_kc"] * 3.0
    np.testing.assert_allclose(net.velocity(P, u, x, 0.2), v, rtol=1e-11, atol=1e-12)
    for B in P["blocks"]:
        B["W_vc"] = B["W_vc"] * 2.0
    assert np.abs(net.velocity(P, u, x, 0.2) - v).max() > 1e-4


def test_truth_enters_only_through_cross_attention():
    """With the cross-attention output projection zeroed, any truth set of any size gives
    the same velocity."""
    P, u, x = _setup(5, 3)
    for B in P["blocks"]:
        B["W_oc"] = np.zeros_like(B["W_oc"])
        B["b_oc"] = np.zeros_like(B["b_oc"])
    v = net.velocity(P, u, x, 0.5)
    u2 = events.particles(np.random.default_rng(9), 2).astype(np.float64)
    np.testing.assert_allclose(net.velocity(P, u2, x, 0.5), v, rtol=1e-12, atol=1e-13)


def test_reco_noise_depends_on_slot_not_on_truth_count():
    a = noise_event(7, 3, 10)
    np.testing.assert_array_equal(a[:4], noise_event(7, 3, 4))
    flat = params.draw(CFG, 0)
    off = np.array([0, 2, 5], dtype=np.int64)
    feat = events.particles(np.random.default_rng(0), 5)
    roff = np.array([0, 4, 5], dtype=np.int64)
    sch = configs.Schedule(EULER, 2)
    outs = sample.simulate_events(flat, CFG, off, feat, sch, seed=7, reco_offsets=roff)
    assert [len(o) for o in outs] == [4, 1]
    P = net.unpack(flat, CFG)
    ref = sample.simulate_event(P, feat[2:5].astype(np.float64), noise_event(7, 1, 1), EULER, 2)
    np.testing.assert_allclose(outs[1], ref, rtol=1e-14)


def test_default_reco_offsets_are_the_truth_offsets():
    flat = params.draw(CFG, 0)
    off = np.array([0, 3, 3, 6], dtype=np.int64)
    feat = events.particles(np.random.default_rng(1), 6)
    sch = configs.Schedule(RK4, 1)
    a = sample.simulate(flat, CFG, off, feat, sch, seed=2)
    b = sample.simulate(flat, CFG, off, feat, sch, seed=2, reco_offsets=off)
    np.testing.assert_array_equal(a, b)


def test_reco_without_truth_and_bad_offsets_are_rejected():
    flat = params.draw(CFG, 0)
    off = np.array([0, 2, 2], dtype=np.int64)
    feat = events.particles(np.random.default_rng(0), 2)
    sch = configs.Schedule(EULER, 1)
    with pytest.raises(ValueError, match="no truth"):
        sample.simulate(flat, CFG, off, feat, sch, seed=1, reco_offsets=[0, 2, 3])
    with pytest.raises(ValueError):
        sample.simulate(flat, CFG, off, feat, sch, seed=1, reco_offsets=[0, 3, 2])
    # an event may have truth particles and no reco slot
    out = sample.simulate(flat, CFG, off, feat, sch, seed=1, reco_offsets=[0, 0, 0])
    assert out.shape == (0, 9)
