"""Pins of the event-observables oracle (Sec. 2.4: H_T, MET, lepton isolation in a
Delta R < 0.4 cone): a worked example with hand-derived values, the phi wrap, invariances,
degenerate events, and a brute-force double loop in plain Python on random events."""

import math

import numpy as np
import pytest

from oracle import observables as ob

CH, EL, MU, NH, PH = range(5)


def particle(pt, eta, phi, cls, q=0.0):
    f = np.zeros(9, dtype=np.float32)
    f[0], f[1], f[2] = math.log(pt / 10.0), eta, phi
    f[3 + cls] = 1.0
    f[8] = q
    return f


def test_worked_example():
    # electron (20 GeV at eta 0, phi 0); hadron 5 GeV at Delta R 0.3; photon 3 GeV at
    # Delta R 0.5; muon 10 GeV at (0.1, 0.1): Delta R to the electron sqrt(0.02)
    ev = np.stack([particle(20, 0.0, 0.0, EL, -1), particle(5, 0.3, 0.0, CH, 1),
                   particle(3, 0.0, 0.5, PH), particle(10, 0.1, 0.1, MU, 1)])
    ht, met, iso = ob.event_observables(ev)
    assert ht == pytest.approx(38.0, rel=1e-6)
    px = 20 + 5 + 3 * math.cos(0.5) + 10 * math.cos(0.1)
    py = 3 * math.sin(0.5) + 10 * math.sin(0.1)
    assert met == pytest.approx(math.hypot(px, py), rel=1e-6)
    # electron: hadron (0.3) and muon (0.141) inside, photon (0.5) outside
    assert iso[0] == pytest.approx((5 + 10) / 20, rel=1e-6)
    # muon: electron (0.141) and hadron (sqrt(0.05) = 0.224) inside, photon
    # (sqrt(0.01 + 0.16) = 0.412) outside
    assert iso[3] == pytest.approx((20 + 5) / 10, rel=1e-6)
    assert np.isnan(iso[1]) and np.isnan(iso[2])


def test_phi_wraps_around():
    ev = np.stack([particle(10, 0.0, 3.1, MU), particle(4, 0.0, -3.1, CH),
                   particle(7, 0.0, 3.1 + 4 * math.pi, NH), particle(9, 0.0, 3.1 + 0.6, PH)])
    _, _, iso = ob.event_observables(ev)
    # -3.1 is 0.083 away across the boundary; 3.1 + 4 pi is the same direction; +0.6 is out
    assert iso[0] == pytest.approx((4 + 7) / 10, rel=1e-6)


def test_single_particles_and_empty_events():
    ht, met, iso = ob.event_observables(np.zeros((0, 9), np.float32))
    assert (ht, met, len(iso)) == (0.0, 0.0, 0)
    ht, met, iso = ob.event_observables(particle(25, 1.0, 2.0, EL)[None])
    assert ht == pytest.approx(25) and met == pytest.approx(25) and iso[0] == 0.0
    # back to back, equal pT: no missing momentum
    ev = np.stack([particle(30, 0.0, 0.7, CH), particle(30, 1.0, 0.7 - math.pi, NH)])
    assert ob.event_observables(ev)[1] == pytest.approx(0.0, abs=1e-5)


def test_rotation_in_phi_leaves_everything_unchanged():
    rng = np.random.default_rng(4)
    ev = np.stack([particle(float(rng.uniform(1, 50)), float(rng.uniform(-1, 1)),
                            float(rng.uniform(-3, 3)), int(rng.integers(5))) for _ in range(40)])
    rot = ev.copy()
    rot[:, 2] += np.float32(0.25)
    a, b = ob.event_observables(ev), ob.event_observables(rot)
    assert a[0] == pytest.approx(b[0]) and a[1] == pytest.approx(b[1], rel=1e-5)
    far = np.abs(np.nan_to_num(a[2]) - np.nan_to_num(b[2]))
    # a shift can move a pair across the float32 cone edge only by rounding; none does here
    assert far.max() < 1e-9


def _brute(ev):
    """Plain-Python double loop with the same float32 cone decision."""
    f32 = np.float32
    n = len(ev)
    pts = [10.0 * math.exp(float(ev[i, 0])) for i in range(n)]
    cls = [max(range(5), key=lambda c: (ev[i, 3 + c], -c)) for i in range(n)]
    ht = sum(pts)
    met = math.hypot(sum(p * math.cos(float(ev[i, 2])) for i, p in enumerate(pts)),
                     sum(p * math.sin(float(ev[i, 2])) for i, p in enumerate(pts)))
    iso = [float("nan")] * n
    for i in range(n):
        if cls[i] not in (EL, MU):
            continue
        s = 0.0
        for j in range(n):
            if j == i:
                continue
            deta = f32(ev[i, 1]) - f32(ev[j, 1])
            d = f32(ev[i, 2]) - f32(ev[j, 2])
            dphi = f32(d - f32(2 * np.pi) * f32(np.rint(f32(d * f32(1 / (2 * np.pi))))))
            if f32(f32(deta * deta) + f32(dphi * dphi)) < f32(0.16):
                s += pts[j]
        iso[i] = s / pts[i]
    return ht, met, np.array(iso)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = 60
    ev = np.zeros((n, 9), np.float32)
    ev[:, 0] = rng.normal(0, 1, n)
    ev[:, 1] = rng.uniform(-0.6, 0.6, n)            # dense enough for many cone members
    ev[:, 2] = rng.uniform(-4, 4, n)                 # beyond [-pi, pi] on purpose
    ev[:, 3:8] = rng.normal(0, 1, (n, 5))
    ht, met, iso = ob.event_observables(ev)
    bht, bmet, biso = _brute(ev)
    assert ht == pytest.approx(bht, rel=1e-12) and met == pytest.approx(bmet, rel=1e-12)
    assert np.array_equal(np.isnan(iso), np.isnan(biso))
    ok = ~np.isnan(iso)
    assert ok.sum() > 10 and np.allclose(iso[ok], biso[ok], rtol=1e-12, atol=0)
    assert (iso[ok] > 0).sum() > 5


def test_batch_is_per_event():
    rng = np.random.default_rng(5)
    sizes = [0, 3, 1, 17, 0, 8]
    off = np.r_[0, np.cumsum(sizes)]
    feat = rng.normal(0, 0.5, (off[-1], 9)).astype(np.float32)
    ht, met, iso = ob.observables(off, feat)
    for e in range(len(sizes)):
        h, m, i = ob.event_observables(feat[off[e]:off[e + 1]])
        assert ht[e] == h and met[e] == m
        assert np.array_equal(iso[off[e]:off[e + 1]], i, equal_nan=True)
