"""Per-event sampling driver — oracle side.

simulate(truth sets, seed, schedule) -> reco sets, the problem the paper states for its
detector backends (Sec. 1, program summary: truth-level particles in, detector-level
reconstructed particles out) with the neural backend's sampler (Sec. 2.2). Each event is
handled alone: its noise is drawn from (seed, event index), its own truth encoding is
formed, and the ODE is integrated over its reco slots: one per truth particle by default,
or the per-event reco multiplicities the caller gives (``reco_offsets``). The paper's model
can emit more or fewer reco particles than truth particles but does not describe how the
count is chosen; the network itself needs no change for it, since self-attention runs over
the reco slots and cross-attention from them to the event's truth particles (Sec. 2.2).
A reco slot needs at least one truth particle to attend to.

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
                    dtype=np.float64, processes=1, progress=None, reco_offsets=None):
    """Run events of a CSR batch; returns the list of per-event [N_reco_e, 9] outputs.

    ``event_ids`` selects events (default all); noise uses the event's index in the batch.
    ``reco_offsets`` ([E + 1], default ``offsets``) gives the reco multiplicities; the noise
    of an event's reco slot s is the generator's draw for (event, s) whatever the truth count.
    ``x0`` ([T_reco, 9], CSR by ``reco_offsets``) replaces the seeded noise when given.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    E = len(offsets) - 1
    roff = offsets if reco_offsets is None else np.asarray(reco_offsets, dtype=np.int64)
    if len(roff) != E + 1 or roff[0] != 0 or np.any(np.diff(roff) < 0):
        raise ValueError("reco_offsets must be non-decreasing from 0, one entry per event + 1")
    ids = range(E) if event_ids is None else event_ids
    jobs = []
    for e in ids:
        a, b = int(offsets[e]), int(offsets[e + 1])
        ra, rb = int(roff[e]), int(roff[e + 1])
        if rb > ra and b == a:
            raise ValueError(f"event {e} has reco slots but no truth particle")
        u = np.asarray(feat[a:b], dtype=np.float64)
        if x0 is not None:
            xe = np.asarray(x0[ra:rb], dtype=np.float64)
        else:
            xe = noise_event(seed, e, rb - ra, cfg.f_reco)
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
             processes=1, reco_offsets=None):
    """Whole CSR batch -> [T_reco, 9] FP64 reco state (the raw ODE state at t1)."""
    outs = simulate_events(flat, cfg, offsets, feat, schedule, seed, x0, None, dtype, processes,
                           reco_offsets=reco_offsets)
    return np.concatenate(outs) if outs else np.zeros((0, cfg.f_reco))


def decode(x):
    x = np.asarray(x, dtype=np.float64)
    pt = 10.0 * np.exp(x[:, 0])
    eta = x[:, 1]
    phi = (x[:, 2] + np.pi) % (2.0 * np.pi) - np.pi
    cls = np.argmax(x[:, 3:8], axis=1)
    q = np.clip(np.rint(x[:, 8]), -1, 1)
    return {"pt": pt, "eta": eta, "phi": phi, "cls": cls, "q": q}
