"""Truth preprocessing before the sampler: FP64 oracle — TEST INFRASTRUCTURE ONLY.

For the neural backend the truth particles pass the model's selection before sampling: a
transverse-momentum cut and the model's particle limit, both fixed by the released model
(the pT cut from the model metadata in the configuration reference appendix: 0.25 GeV for
the CMS model, 0.5 GeV for the ALEPH one; the particle limits of the detector-backend table
and Sec. 2.2, "Event Generation": 400 and 128 particles).

Readings (the paper leaves these open):
  * A particle survives the cut when pT > cut (strictly). pT = 10 GeV exp(x0) in the state
    layout (reading R3); the decision is x0 > c0 with c0 = ln(cut / 10 GeV) rounded to
    float32, taken in float32 on the state value as stored.
  * An event with more survivors than the limit keeps the `limit` survivors of largest x0
    (largest pT); equal x0 keep the earlier particle. Kept particles stay in input order.
  * Events may become empty; the event count never changes.

Plain NumPy, one event at a time.
"""

import math

import numpy as np


def cut_threshold(pt_cut_gev: float) -> np.float32:
    """c0 = ln(cut / 10 GeV) as float32 (the cut applied to x0 = ln(pT / 10 GeV))."""
    return np.float32(math.log(pt_cut_gev / 10.0))


def select_event(feat: np.ndarray, pt_cut_gev: float, limit: int) -> np.ndarray:
    """Indices (ascending) of the particles of one event [n, 9] that the selection keeps."""
    x0 = np.asarray(feat, dtype=np.float32)[:, 0]
    idx = np.nonzero(x0 > cut_threshold(pt_cut_gev))[0]
    if len(idx) > limit:
        # largest x0 first, earlier index first among equals; then back to input order
        order = sorted(idx.tolist(), key=lambda i: (-float(x0[i]), i))
        idx = np.array(sorted(order[:limit]), dtype=np.int64)
    return idx


def select(offsets: np.ndarray, feat: np.ndarray, pt_cut_gev: float, limit: int):
    """(offsets_out [E+1], feat_out [T', 9]) of a CSR batch after the selection."""
    E = len(offsets) - 1
    out_off = np.zeros(E + 1, dtype=np.int64)
    rows = []
    for e in range(E):
        a = int(offsets[e])
        keep = select_event(feat[a:int(offsets[e + 1])], pt_cut_gev, limit)
        rows.append(a + keep)
        out_off[e + 1] = out_off[e] + len(keep)
    rows = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    return out_off, np.asarray(feat, dtype=np.float32)[rows]
