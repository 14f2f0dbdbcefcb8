"""Write the FP64 oracle's outputs for the leading events of the benchmark workloads.

The base workload (4096 events, N ~ U{20..200}, d=256, 6 blocks, 8 heads, RK4 16) takes
seconds per event in the oracle, too slow to recompute inside a GPU test. This script
runs only ``oracle`` on the seeded inputs of ``workload`` and stores the raw ODE state
at t = 1 of the first 256 events (the first 128 are the FP32 parity subset, all 256 the
BF16 one). The small workload (64 events) is fast and is recomputed in the tests.

Usage: python tests/golden/make_oracle_outputs.py [--processes 8]
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

OUT = os.path.join(HERE, "oracle_base_rk4x16_first256.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--processes", type=int, default=os.cpu_count())
    ap.add_argument("--events", type=int, default=256)
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    w = configs.BASE_FP32
    off, feat = events.for_workload(w, a.events)
    flat = params.draw(w.model, w.weight_seed)
    t = time.time()
    out = sample.simulate(flat, w.model, off, feat, w.schedule, seed=w.noise_seed,
                          processes=a.processes)
    dt = time.time() - t
    np.savez(OUT, offsets=off, reco=out, seconds=dt, processes=a.processes)
    print(f"wrote {OUT}: {a.events} events, {len(out)} rows, {dt:.1f} s on {a.processes} processes")


if __name__ == "__main__":
    main()
