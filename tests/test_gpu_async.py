"""Sampling calls enqueue work without waiting (GPU): each call's host-built arrays (offsets,
attention work lists, stage table) go through one of two pinned staging sets, so calls issued
back to back on one stream, with different event sets, must give exactly what the same calls
give one at a time with the stream synchronized after each."""

import numpy as np
import pytest

from tests._gpu import fmd_lib, torch_cuda
from workload import configs, events, params

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [configs.FP32, configs.BF16])
def test_back_to_back_calls_equal_synchronized_calls(precision):
    torch, fmd = torch_cuda(), fmd_lib()
    cfg = (configs.SMALL_MODEL if precision == configs.FP32 else
           configs.BASE_MODEL).with_precision(precision)
    flat = params.draw(cfg, seed=0)
    sets = [events.truth_events(n, ("uniform", 5, 60), seed=40 + n) for n in (9, 23, 4, 15, 30)]
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(cfg, flat)
    feats = [torch.from_numpy(f).cuda() for _, f in sets]
    ref = []
    for (off, _), f in zip(sets, feats):
        ref.append(m.simulate(off, f, 11, sched).cpu().numpy())
        torch.cuda.synchronize()
    outs = [torch.empty((int(off[-1]), 9), dtype=torch.float32, device="cuda") for off, _ in sets]
    for _ in range(2):
        for (off, _), f, o in zip(sets, feats, outs):
            m.simulate(off, f, 11, sched, out=o)
        torch.cuda.synchronize()
        for r, o in zip(ref, outs):
            assert np.array_equal(o.cpu().numpy(), r)
    m.close()
