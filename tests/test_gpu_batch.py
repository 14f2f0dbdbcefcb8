"""Batching form at full size (GPU): 65,536 events with heavy-tailed multiplicities
(log-normal, median 60, sigma 0.8, clipped to [1, 1000]; 5.39 M particles), BF16 network of
the base workload, RK4 16, in one call: every output finite, selected events against the
stored FP64 oracle outputs (normwise 2e-2), and the largest event bitwise the same alone."""

import os

import numpy as np
import pytest

from tests._gpu import fmd_lib, torch_cuda
from workload import configs, errors, events, params

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_batch_rk4x16_selected.npz")


def test_batch_workload_full_size():
    torch = torch_cuda()
    fmd = fmd_lib()
    if not os.path.exists(GOLDEN):
        pytest.skip("golden oracle outputs missing (tests/golden/make_oracle_outputs.py)")
    z = np.load(GOLDEN)
    ids = z["event_ids"]
    w = configs.BATCH_BF16
    off, feat = events.for_workload(w)
    flat = params.draw(w.model, w.weight_seed)
    m = fmd.Model(w.model, flat)
    feat_d = torch.from_numpy(feat).cuda()
    out_d = m.simulate(off, feat_d, w.noise_seed, w.schedule)
    torch.cuda.synchronize()
    out = out_d.cpu().numpy()
    assert np.all(np.isfinite(out))
    got = np.concatenate([out[off[e]:off[e + 1]] for e in ids])
    err = errors.normwise_rel_err(got, z["reco"])
    assert err.max() < 2e-2, err

    # the largest event alone, from the same noise (keyed by its index in the big call)
    e = int(ids[np.argmax(z["sizes"])])
    n = int(off[e + 1] - off[e])
    x0_all = torch.empty((off[-1], 9), dtype=torch.float32, device="cuda")
    fmd.noise(w.noise_seed, off, 9, x0_all)
    x0 = x0_all[off[e]:off[e + 1]].contiguous()
    one = m.simulate_from_state(np.array([0, n]), feat_d[off[e]:off[e + 1]].contiguous(), x0,
                                w.schedule).cpu().numpy()
    m.close()
    assert np.array_equal(one, out[off[e]:off[e + 1]])
