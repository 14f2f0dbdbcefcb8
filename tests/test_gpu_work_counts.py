"""Algorithmic work that the timing counters credit (GPU): the flops each kernel class adds
up over one sampling call must equal the per-event count of the method (28 d^2 N per block
for the matrix products, 8 d N^2 per block for the two attentions, 4 F d N for the input
embedding and the output head), split by kernel as the fused path runs it:

  block 0's QKV kernel       6 d^2 T + 2 F d T (embedding folded in)
  self / cross attention     4 d sum(N^2) and 4 d sum(N N_truth) per block
  OQC kernel                 4 d^2 T per block (W_o, W_qc)
  MLP kernel, blocks < L-1   24 d^2 T (W_oc, W_up, W_dn, next block's W_qkv)
  MLP kernel, last block     18 d^2 T + 2 F d T (output head folded in)

so the roofline figures derived from the counters rest on the method's flop count and
nothing else.
"""

import dataclasses

import numpy as np
import pytest

from tests._gpu import fmd_lib, torch_cuda
from workload import configs, events, params

pytestmark = pytest.mark.gpu

CFG = dataclasses.replace(configs.BASE_MODEL.with_precision(configs.BF16), n_max=1000)


def test_flop_counters_follow_the_per_event_formula():
    torch, fmd = torch_cuda(), fmd_lib()
    sizes = [23, 0, 140, 64, 65, 7, 200, 31]
    off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    feat = events.particles(np.random.default_rng(5), int(off[-1]))
    flat = params.draw(CFG, seed=0)
    sched = configs.Schedule(configs.RK4, 2)
    evals = sched.evals
    m = fmd.Model(CFG, flat)
    assert m.kernel_name(fmd.K_FUSED_MLP) == "k_fused_mlp"
    m.timing_enable(True)
    m.simulate(off, torch.from_numpy(feat).cuda(), 1, sched)
    torch.cuda.synchronize()
    got = {cls: m.timing_read(cls)[2] for cls in (fmd.K_GEMM_QKV, fmd.K_ATTN_SELF, fmd.K_ATTN_CROSS,
                                                   fmd.K_FUSED_OQC, fmd.K_FUSED_MLP)}
    m.close()
    d, L, F = CFG.d_model, CFG.n_blocks, 9
    n = np.array(sizes, dtype=np.float64)
    T, n2 = n.sum(), (n * n).sum()
    want = {
        fmd.K_GEMM_QKV: evals * (6 * d * d * T + 2 * F * d * T),
        fmd.K_ATTN_SELF: evals * L * 4 * d * n2,
        fmd.K_ATTN_CROSS: evals * L * 4 * d * n2,
        fmd.K_FUSED_OQC: evals * L * 4 * d * d * T,
        fmd.K_FUSED_MLP: evals * ((L - 1) * 24 * d * d * T + 18 * d * d * T + 2 * F * d * T),
    }
    for cls, w in want.items():
        assert got[cls] == pytest.approx(w, rel=1e-9), (cls, got[cls], w)
    total = evals * (L * (28 * d * d * T + 8 * d * n2) + 4 * F * d * T)
    assert sum(got.values()) == pytest.approx(total, rel=1e-9)
