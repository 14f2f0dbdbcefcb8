"""Shared helpers of the GPU tests (not collected)."""

import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def fmd_lib():
    from paper_2606_26089_amd import fmd
    fmd.lib()          # raises if the HIP library is missing: GPU tests never fall back
    return fmd


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32.
    Emulates the kernels' operand rounding for unit-level comparisons."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def normwise(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(y - ref)) / max(np.max(np.abs(ref)), 1e-300))
