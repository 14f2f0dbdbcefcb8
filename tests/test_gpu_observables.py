"""Event observables on the GPU (Sec. 2.4: H_T, MET, lepton isolation in a Delta R < 0.4
cone) against the FP64 oracle: synthetic particle sets with the base workload's
multiplicities, degenerate events, the phi wrap, events longer than one LDS tile, host and
device memory, and the output of the BF16 sampler itself.

The cone test and the class maximum are integer decisions taken in FP32 on both sides, so
the isolation sums cover the same particles; the sums are FP64 on both sides and the
results FP32, so the bar is the FP32 rounding of the result (relative 1e-6)."""

import math

import numpy as np
import pytest

from oracle import observables as ob
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, events, params

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def _check(ht, met, iso, off, feat):
    rht, rmet, riso = ob.observables(off, feat)
    assert np.allclose(ht, rht, rtol=RTOL, atol=1e-6)
    assert np.allclose(met, rmet, rtol=RTOL, atol=1e-4)
    assert np.array_equal(np.isnan(iso), np.isnan(riso))
    ok = ~np.isnan(riso)
    assert np.allclose(iso[ok], riso[ok], rtol=RTOL, atol=1e-7)
    return ok


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_matches_oracle_on_base_multiplicities(env):
    torch, fmd = env
    off, feat = events.truth_events(512, ("uniform", 20, 200), seed=8)
    feat = feat.copy()
    feat[:, 1] *= np.float32(0.3)        # narrower in eta: more particles inside the cones
    ht, met, iso = fmd.event_observables(off, _dev(torch, feat))
    ok = _check(ht.cpu().numpy(), met.cpu().numpy(), iso.cpu().numpy(), off, feat)
    assert ok.sum() > 1000 and (iso.cpu().numpy()[ok] > 0).sum() > 500


def test_degenerate_events_and_phi_wrap(env):
    torch, fmd = env

    def p(pt, eta, phi, cls):
        f = np.zeros(9, np.float32)
        f[0], f[1], f[2], f[3 + cls] = math.log(pt / 10), eta, phi, 1
        return f
    evs = [[], [p(20, 0, 0, 1)], [p(5, 0, 1, 0), p(6, 0.2, 1.1, 3)],
           [p(20, 0, 0, 1), p(5, 0.3, 0, 0), p(3, 0, 0.5, 4), p(10, 0.1, 0.1, 2)],
           [p(10, 0, 3.1, 2), p(4, 0, -3.1, 0), p(7, 0, 3.1 + 4 * math.pi, 3)], []]
    off = np.r_[0, np.cumsum([len(e) for e in evs])].astype(np.int64)
    feat = np.stack([x for e in evs for x in e]).astype(np.float32)
    ht, met, iso = fmd.event_observables(off, _dev(torch, feat))
    ht, met, iso = ht.cpu().numpy(), met.cpu().numpy(), iso.cpu().numpy()
    _check(ht, met, iso, off, feat)
    assert ht[0] == 0 and met[0] == 0 and ht[5] == 0
    assert iso[0] == 0.0                                     # a lone lepton
    assert iso[3] == pytest.approx(0.75, rel=RTOL) and iso[6] == pytest.approx(2.5, rel=RTOL)
    assert iso[7] == pytest.approx(1.1, rel=RTOL)            # across the phi boundary


def test_events_longer_than_one_tile_and_host_memory(env):
    torch, fmd = env
    off, feat = events.truth_events(3, ("uniform", 2500, 3000), seed=9)
    feat = feat.copy()
    feat[:, 1] *= np.float32(0.2)
    d = fmd.event_observables(off, _dev(torch, feat))
    h = fmd.event_observables(off, feat)                    # host arrays in and out
    for a, b in zip(d, h):
        assert np.array_equal(a.cpu().numpy(), b, equal_nan=True)
    _check(*h, off, feat)


def test_on_the_bf16_sampler_output(env):
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(configs.BF16)
    off, feat = events.truth_events(64, ("uniform", 20, 200), seed=10)
    m = fmd.Model(cfg, params.draw(cfg, 0))
    reco = m.simulate(off, _dev(torch, feat), 3, configs.Schedule(configs.EULER, 4))
    m.close()
    ht, met, iso = fmd.event_observables(off, reco)
    _check(ht.cpu().numpy(), met.cpu().numpy(), iso.cpu().numpy(), off, reco.cpu().numpy())
