"""Per-event sampling driver — oracle side.

simulate(truth sets, seed, schedule) -> reco sets, the problem the paper states for its
detector backends (Sec. 1, program summary: truth-level particles in, detector-level
reconstructed particles out) with the neural backend's sampler (Sec. 2.2). Each event is
handled alone: its noise is drawn from (seed, event index), its own truth encoding is
formed, and the ODE is integrated over its N reco slots, one per truth particle (the
reco multiplicity equals the truth multiplicity in every workload here; the paper's
model can add particles, a mechanism it does not describe).

``decode`` maps a 9-feature state back to particle quantities for physics checks:
pT = 10 GeV exp(x0), eta = x1, phi wrapped to [-pi, pi), class = argmax x[3:8],
charge = clamp(round(x8), -1, 1).
"""

from concurrent.futures import ProcessPoolExecutor

import numpy as np

from .net import unpack, velocity
from .ode import integrate
from .philox import noise_event


def simulate_event(P, u, x0, scheme, n_steps, t0=0.0, t1=1.0):
    if len(x0) == 0:
        return np.zeros((0, P["cfg"].f_reco))
    return integrate(lambda x, t: velocity(P, u, x, t), x0, scheme, n_steps, t0, t1)


def _worker(args):
    flat, cfg, u, x0, scheme, n_steps, t0, t1, dtype = args
    P = unpack(flat, cfg, dtype)
    return simulate_event(P, u, x0, scheme, n_steps, t0, t1)


def _pool_init():
    # one BLAS thread per worker process: the pool already spans the cores
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def simulate_events(flat, cfg, offsets, feat, schedule, seed=None, x0=None, event_ids=None,
                    dtype=np.float64, processes=1, progress=None):
    """Run events of a CSR batch; returns the list of per-event [N_e, 9] outputs.

    ``event_ids`` selects events (default all); noise uses the event's index in the batch.
    ``x0`` ([T, 9], same CSR) replaces the seeded noise when given.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    E = len(offsets) - 1
    ids = range(E) if event_ids is None else event_ids
    jobs = []
    for e in ids:
        a, b = int(offsets[e]), int(offsets[e + 1])
        u = np.asarray(feat[a:b], dtype=np.float64)
        if x0 is not None:
            xe = np.asarray(x0[a:b], dtype=np.float64)
        else:
            xe = noise_event(seed, e, b - a, cfg.f_reco)
        jobs.append((flat, cfg, u, xe, schedule.scheme, schedule.n_steps,
                     schedule.t0, schedule.t1, dtype))
    out = []
    if processes > 1 and len(jobs) > 1:
        with ProcessPoolExecutor(processes, initializer=_pool_init) as ex:
            for r in ex.map(_worker, jobs, chunksize=1):
                out.append(r)
                if progress:
                    progress(len(out), len(jobs))
        return out
    for j in jobs:
        out.append(_worker(j))
        if progress:
            progress(len(out), len(jobs))
    return out


def simulate(flat, cfg, offsets, feat, schedule, seed=None, x0=None, dtype=np.float64,
             processes=1):
    """Whole CSR batch -> [T, 9] FP64 reco state (the raw ODE state at t1)."""
    outs = simulate_events(flat, cfg, offsets, feat, schedule, seed, x0, None, dtype, processes)
    return np.concatenate(outs) if outs else np.zeros((0, cfg.f_reco))


def decode(x):
    x = np.asarray(x, dtype=np.float64)
    pt = 10.0 * np.exp(x[:, 0])
    eta = x[:, 1]
    phi = (x[:, 2] + np.pi) % (2.0 * np.pi) - np.pi
    cls = np.argmax(x[:, 3:8], axis=1)
    q = np.clip(np.rint(x[:, 8]), -1, 1)
    return {"pt": pt, "eta": eta, "phi": phi, "cls": cls, "q": q}
