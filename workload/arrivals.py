"""Open-loop Poisson request streams for the serving form.

A request carries 1..512 events (integer-uniform) whose multiplicities follow the
heavy-tailed law of the batching workload, and asks for either Euler 20 or RK4 16 with
probability one half each. Inter-arrival gaps are exponential with mean
E[events per request] / rate, so that the offered load is ``rate`` events per second.
"""

from dataclasses import dataclass

import numpy as np

from .configs import EULER, RK4, Schedule
from .events import multiplicities, particles


@dataclass
class Request:
    t_arrive: float          # seconds from stream start
    offsets: np.ndarray      # int64 [n+1]
    feat: np.ndarray         # float32 [T, 9]
    seed: int
    schedule: Schedule


def stream(rate: float, n_requests: int, seed: int = 3, events_per_request=(1, 512),
           mult=("lognormal", 60.0, 0.8, 1, 1000), schedules=None):
    rng = np.random.default_rng(seed)
    if schedules is None:
        schedules = (Schedule(EULER, 20), Schedule(RK4, 16))
    lo, hi = events_per_request
    mean_events = 0.5 * (lo + hi)
    gaps = rng.exponential(mean_events / rate, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(n_requests):
        n_ev = int(rng.integers(lo, hi + 1))
        n = multiplicities(rng, n_ev, mult)
        offsets = np.zeros(n_ev + 1, dtype=np.int64)
        np.cumsum(n, out=offsets[1:])
        feat = particles(rng, int(offsets[-1]))
        sched = schedules[int(rng.integers(0, len(schedules)))]
        out.append(Request(float(t[r]), offsets, feat, int(rng.integers(0, 2**62)), sched))
    return out
