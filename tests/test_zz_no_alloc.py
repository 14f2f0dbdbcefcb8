"""The allocation-free truth selection (GPU), called through the C ABI: its offsets and rows
must equal those of the allocating entry point bit for bit (integer and copy work), on two
calls in a row, the second smaller than the first, so that values the first call left in the
shared scratch array cannot leak into the second. Also: the limits of the fixed scratch and
the device-memory requirement are rejected on the host before anything is launched."""

import numpy as np
import pytest

from tests._gpu import fmd_lib, torch_cuda
from workload import events

pytestmark = pytest.mark.gpu


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_no_alloc_selection_equals_the_allocating_call_on_two_calls():
    torch, fmd = torch_cuda(), fmd_lib()
    big_off, big_feat = events.truth_events(3000, ("uniform", 20, 200), seed=21)
    rng = np.random.default_rng(4)
    sizes = [0, 3, 250, 1, 0, 90]
    small_off = np.r_[0, np.cumsum(sizes)].astype(np.int64)
    small_feat = rng.normal(0, 0.5, (small_off[-1], 9)).astype(np.float32)
    small_feat[:, 0] = np.round(rng.normal(-1, 1.0, small_off[-1]) * 4) / 4   # exact ties
    for off, feat, cut, limit in ((big_off, big_feat, 0.5, 128), (small_off, small_feat, 0.5, 40)):
        f_d = _dev(torch, feat)
        out = torch.full((max(int(off[-1]), 1), 9), float("nan"), dtype=torch.float32, device="cuda")
        o1, r1 = fmd.truth_select_noalloc(off, f_d, cut, limit, out)
        o2, r2 = fmd.truth_select(off, f_d, cut, limit)
        assert np.array_equal(o1, o2)
        assert np.array_equal(r1.cpu().numpy(), r2.cpu().numpy())
        assert o1[-1] < off[-1]          # the cut and the limit removed particles


def test_no_alloc_selection_rejects_what_the_scratch_cannot_hold():
    torch, fmd = torch_cuda(), fmd_lib()
    off = np.zeros(65537 + 1, dtype=np.int64)       # 65537 empty events: one too many
    feat = torch.zeros((1, 9), dtype=torch.float32, device="cuda")
    with pytest.raises(fmd.FmdError) as e:
        fmd.truth_select_noalloc(off, feat, 0.5, 10, feat)
    assert e.value.status == -4                     # FMD_E_UNSUPPORTED
    off = np.array([0, 3], dtype=np.int64)
    with pytest.raises(fmd.FmdError) as e:          # host data: the call takes device data only
        fmd.truth_select_noalloc(off, np.zeros((3, 9), np.float32), 0.5, 10, feat)
    assert e.value.status == -1                     # FMD_E_INVALID
