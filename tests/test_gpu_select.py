"""Truth preprocessing on the GPU (model pT cut and particle limit) against the oracle:
offsets and selected rows are integer/copy work, so they must match exactly; on the base
workload's truth with both released models' settings, on ties and degenerate events, in
host and device memory, and feeding the sampler."""

import numpy as np
import pytest

from oracle import select as sel
from tests._gpu import fmd_lib, torch_cuda
from workload import configs, events, params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return torch_cuda(), fmd_lib()


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("cut,limit", [(0.5, 128), (0.25, 400), (2.0, 50), (20.0, 3)])
def test_matches_oracle_on_base_truth(env, cut, limit):
    torch, fmd = env
    off, feat = events.truth_events(1024, ("uniform", 20, 200), seed=12)
    o2, f2 = fmd.truth_select(off, _dev(torch, feat), cut, limit)
    r_off, r_feat = sel.select(off, feat, cut, limit)
    assert np.array_equal(o2, r_off)
    assert np.array_equal(f2.cpu().numpy(), r_feat)
    if cut > 0.5 or limit < 200:                    # the truth law clips pT at 0.5 GeV, N <= 200
        assert r_off[-1] < off[-1]
    else:
        assert np.array_equal(r_off, off)


def test_ties_degenerate_events_and_host_memory(env):
    torch, fmd = env
    rng = np.random.default_rng(3)
    sizes = [0, 1, 5, 300, 0, 2000, 7]
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    feat = rng.normal(0, 0.3, (off[-1], 9)).astype(np.float32)
    feat[:, 0] = np.round(rng.normal(-1, 1.0, off[-1]) * 4) / 4    # many exact ties
    feat[off[2]:off[3], 0] = -9.0                                     # an event wholly cut
    for cut, limit in ((0.5, 64), (0.5, 0), (1.0, 1000), (3.0, 1)):
        r_off, r_feat = sel.select(off, feat, cut, limit)
        d_off, d_feat = fmd.truth_select(off, _dev(torch, feat), cut, limit)
        h_off, h_feat = fmd.truth_select(off, feat, cut, limit)
        assert np.array_equal(d_off, r_off) and np.array_equal(h_off, r_off)
        assert np.array_equal(d_feat.cpu().numpy(), r_feat) and np.array_equal(h_feat, r_feat)


def test_selected_truth_feeds_the_sampler(env):
    torch, fmd = env
    cfg = configs.BASE_MODEL.with_precision(configs.BF16)
    off, feat = events.truth_events(16, ("uniform", 20, 200), seed=13)
    o2, f2 = fmd.truth_select(off, _dev(torch, feat), 0.5, 128)
    m = fmd.Model(cfg, params.draw(cfg, 0))
    reco = m.simulate(o2, f2, 1, configs.Schedule(configs.EULER, 2))
    m.close()
    assert reco.shape[0] == o2[-1] and bool(torch.isfinite(reco).all())
