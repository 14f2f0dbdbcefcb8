"""Write the FP64 oracle's outputs for selected events of the benchmark workloads.

The oracle takes seconds to minutes per event on these workloads, which is too slow to
recompute inside a GPU test. This script runs only ``oracle`` on the seeded inputs of
``workload`` and stores the raw ODE state at t = 1:
  base   first 256 events of the 4096-event workload (d=256, 6 blocks, RK4 16). The first
         128 are the FP32 parity subset; all 256 are the BF16 one.
  batch  events of the 65,536-event heavy-tailed workload (log-normal multiplicity, median
         60, clipped to [1, 1000]): the first 8, the largest event and one event near 400
         particles. Noise is keyed by each event's index in the full call.
The small workload (64 events) is fast and is recomputed in the tests.

Usage: python tests/golden/make_oracle_outputs.py [--which base|batch|all] [--processes 8]
"""

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sample  # noqa: E402
from workload import configs, events, params  # noqa: E402

OUT_BASE = os.path.join(HERE, "oracle_base_rk4x16_first256.npz")
OUT_BATCH = os.path.join(HERE, "oracle_batch_rk4x16_selected.npz")


def batch_event_ids(offsets):
    n = np.diff(offsets)
    ids = list(range(8))
    ids.append(int(np.argmax(n)))
    ids.append(int(np.argmin(np.abs(n - 400))))
    return sorted(set(ids))


def make_base(processes, n_events=256):
    w = configs.BASE_FP32
    off, feat = events.for_workload(w, n_events)
    flat = params.draw(w.model, w.weight_seed)
    t = time.time()
    out = sample.simulate(flat, w.model, off, feat, w.schedule, seed=w.noise_seed,
                          processes=processes)
    np.savez(OUT_BASE, offsets=off, reco=out, seconds=time.time() - t, processes=processes)
    print(f"wrote {OUT_BASE}: {n_events} events, {len(out)} rows")


def make_batch(processes):
    w = configs.BATCH_BF16
    off, feat = events.for_workload(w)
    flat = params.draw(w.model, w.weight_seed)
    ids = batch_event_ids(off)
    t = time.time()
    outs = sample.simulate_events(flat, w.model, off, feat, w.schedule, seed=w.noise_seed,
                                  event_ids=ids, processes=processes)
    np.savez(OUT_BATCH, event_ids=np.array(ids), sizes=np.diff(off)[ids],
             reco=np.concatenate(outs), seconds=time.time() - t, processes=processes)
    print(f"wrote {OUT_BATCH}: events {ids} sizes {np.diff(off)[ids].tolist()}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--which", default="all", choices=("base", "batch", "all"))
    ap.add_argument("--processes", type=int, default=os.cpu_count())
    a = ap.parse_args()
    if a.which in ("base", "all"):
        make_base(a.processes)
    if a.which in ("batch", "all"):
        make_batch(a.processes)


if __name__ == "__main__":
    main()
