"""Pins of the truth-selection oracle (model pT cut and particle limit before sampling):
hand-made events with the expected survivors written out, the strict cut at the threshold,
ties under the limit, empty results, and a sort-based restatement on random events."""

import math

import numpy as np
import pytest

from oracle import select as sel


def ev(pts):
    f = np.zeros((len(pts), 9), np.float32)
    f[:, 0] = [math.log(p / 10.0) for p in pts]
    f[:, 1] = np.arange(len(pts))            # tags the particles
    return f


def test_cut_only():
    f = ev([0.3, 5.0, 0.2, 1.0, 0.6])
    assert sel.select_event(f, 0.5, 128).tolist() == [1, 3, 4]
    assert sel.select_event(f, 0.25, 128).tolist() == [0, 1, 3, 4]


def test_cut_is_strict_at_the_float32_threshold():
    f = np.zeros((3, 9), np.float32)
    c0 = sel.cut_threshold(0.5)
    f[:, 0] = [c0, np.nextafter(c0, np.float32(np.inf)), np.nextafter(c0, np.float32(-np.inf))]
    assert sel.select_event(f, 0.5, 10).tolist() == [1]


def test_limit_keeps_the_hardest_in_input_order():
    f = ev([3.0, 50.0, 7.0, 1.0, 50.0, 20.0])
    # limit 3: 50 (1), 50 (4), 20 (5); output in input order
    assert sel.select_event(f, 0.5, 3).tolist() == [1, 4, 5]
    # limit 1 among the equal 50s: the earlier one
    assert sel.select_event(f, 0.5, 1).tolist() == [1]
    assert sel.select_event(f, 0.5, 0).tolist() == []


def test_batch_offsets_and_rows():
    evs = [ev([1.0, 2.0]), ev([0.1]), ev([]), ev([9.0, 0.4, 8.0, 7.0])]
    off = np.r_[0, np.cumsum([len(e) for e in evs])].astype(np.int64)
    feat = np.concatenate(evs)
    o2, f2 = sel.select(off, feat, 0.5, 2)
    assert o2.tolist() == [0, 2, 2, 2, 4]
    assert f2[:, 1].tolist() == [0, 1, 0, 2]          # tags: event 3 keeps 9.0 and 8.0
    assert np.array_equal(f2[2:, 0], feat[[3, 5], 0])


@pytest.mark.parametrize("seed", [0, 1])
def test_restated_with_a_stable_sort(seed):
    rng = np.random.default_rng(seed)
    x0 = rng.normal(-1, 1.5, 300).astype(np.float32)
    x0[rng.integers(0, 300, 40)] = x0[0]               # many exact ties
    f = np.zeros((300, 9), np.float32)
    f[:, 0] = x0
    for cut, lim in ((0.25, 400), (0.5, 128), (2.0, 50), (0.5, 10)):
        got = sel.select_event(f, cut, lim)
        surv = np.nonzero(x0 > np.float32(math.log(cut / 10)))[0]
        # stable argsort of -x0 keeps the input order among equal values
        best = surv[np.argsort(-x0[surv], kind="stable")][:lim]
        assert got.tolist() == sorted(best.tolist())
        assert len(got) == min(lim, len(surv))
