"""The autotuner on the fused BF16 path (GPU): for the sizes a call runs it times the attention
query tile (work items of 64, 128 or 192 queries) and the row tile of block 0's QKV kernel and of
the OQC kernel (64 or 128 rows), keeps the fastest, and
reports them in the tuning table. Every candidate must give bitwise-identical results, so the
choice cannot change what is computed: each combination is forced in turn and the sampler's
output compared bit for bit, on ragged events that span several tiles and key chunks (an event
of 1, of 64 and 65 queries, one above 128, one of 300; last key chunks of every shortened
length)."""

import dataclasses
import itertools

import numpy as np
import pytest

from tests._gpu import fmd_lib, torch_cuda
from workload import configs, events, params

pytestmark = pytest.mark.gpu

CFG = dataclasses.replace(configs.BASE_MODEL.with_precision(configs.BF16), n_max=1000)


def test_candidates_are_tuned_reported_and_bitwise_equal():
    torch, fmd = torch_cuda(), fmd_lib()
    sizes = [1, 64, 65, 200, 0, 129, 37, 128, 300, 5, 96, 97, 161, 224]
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    feat = torch.from_numpy(events.particles(np.random.default_rng(6), int(off[-1]))).cuda()
    flat = params.draw(CFG, seed=0, perturbed=True)
    sched = configs.Schedule(configs.RK4, 2)
    m = fmd.Model(CFG, flat)
    tuned = m.simulate(off, feat, 4, sched).cpu().numpy()
    table = m.tuning_table()["entries"]
    sites = {e["site"]: e for e in table}
    for name, n in (("attn_query_tile", 3), ("fused_qkv", 2), ("fused_oqc", 2)):
        assert name in sites, table
        assert len(sites[name]["candidates_us"]) == n
    assert sites["attn_query_tile"]["BM"] in (64, 128, 192)
    bucket = sites["fused_oqc"]["tokens_log2"]
    assert all(e["tokens_log2"] == bucket for e in table)
    outs = []
    for a, q, o in itertools.product((0, 1, 2), (0, 1), (0, 1)):
        m.tuning_set(fmd.TUNE_ATTN_QUERY_TILE, bucket, a)
        m.tuning_set(fmd.TUNE_FUSED_QKV, bucket, q)
        m.tuning_set(fmd.TUNE_FUSED_OQC, bucket, o)
        outs.append(((a, q, o), m.simulate(off, feat, 4, sched).cpu().numpy()))
    with pytest.raises(fmd.FmdError):
        m.tuning_set(fmd.TUNE_FUSED_OQC, bucket, 2)
    with pytest.raises(fmd.FmdError):
        m.tuning_set(fmd.TUNE_ATTN_QUERY_TILE, bucket, 3)
    with pytest.raises(fmd.FmdError):
        m.tuning_set(0, bucket, 0)           # GEMM sites are not set this way
    m.close()
    assert np.isfinite(tuned).all()
    for combo, out in outs:
        assert np.array_equal(out, tuned), combo
