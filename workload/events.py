"""Synthetic truth events.

Every event is a variable-length set of generator-level particles (the paper's input to
the detector model, Sec. 1 and Sec. 2.1). No event file of the paper's benchmark is
available, so particles are drawn from the laws of the benchmark configurations:

* log pT ~ N(log 10 GeV, 1) clipped (not resampled) to [0.5, 500] GeV;
* eta ~ U[-2.5, 2.5]; phi ~ U[-pi, pi);
* class uniform over the five particle-flow classes, in the order the paper lists them
  for its demonstration (charged hadron, electron, muon, neutral hadron, photon);
* charge +-1 with equal probability for the three charged classes, 0 for the neutral two.

A particle is stored as 9 FP32 features ``[ln(pT/10 GeV), eta, phi, onehot5(class), q]``.
Events are stored in CSR form: ``offsets[E+1]`` (int64, offsets[0] = 0) and
``feat[offsets[E], 9]``. Multiplicities are drawn for all events first, then particle
fields for all particles, so the first k events of a draw do not depend on E.
"""

import numpy as np

from .configs import F_FEAT

N_CLASSES = 5
CHARGED_CLASSES = (0, 1, 2)


def multiplicities(rng: np.random.Generator, n_events: int, law: tuple) -> np.ndarray:
    kind = law[0]
    if kind == "uniform":
        lo, hi = law[1], law[2]
        return rng.integers(lo, hi + 1, size=n_events).astype(np.int64)
    if kind == "lognormal":
        median, sigma, lo, hi = law[1:]
        z = rng.standard_normal(n_events)
        return np.clip(np.rint(median * np.exp(sigma * z)), lo, hi).astype(np.int64)
    if kind == "fixed":
        return np.full(n_events, law[1], dtype=np.int64)
    raise ValueError(f"unknown multiplicity law {law!r}")


def particles(rng: np.random.Generator, n: int) -> np.ndarray:
    """Draw n particles and return their 9-feature rows (float32)."""
    z = rng.standard_normal(n)
    pt = np.clip(10.0 * np.exp(z), 0.5, 500.0)
    eta = rng.uniform(-2.5, 2.5, n)
    phi = rng.uniform(-np.pi, np.pi, n)
    cls = rng.integers(0, N_CLASSES, n)
    sign = np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0)
    q = np.where(np.isin(cls, CHARGED_CLASSES), sign, 0.0)
    feat = np.zeros((n, F_FEAT), dtype=np.float64)
    feat[:, 0] = np.log(pt / 10.0)
    feat[:, 1] = eta
    feat[:, 2] = phi
    feat[np.arange(n), 3 + cls] = 1.0
    feat[:, 8] = q
    return feat.astype(np.float32)


def truth_events(n_events: int, law: tuple, seed: int = 2):
    """Return (offsets int64 [E+1], feat float32 [T, 9])."""
    rng = np.random.default_rng(seed)
    n = multiplicities(rng, n_events, law)
    offsets = np.zeros(n_events + 1, dtype=np.int64)
    np.cumsum(n, out=offsets[1:])
    feat = particles(rng, int(offsets[-1]))
    return offsets, feat


def for_workload(w, n_events: int | None = None):
    """Truth events of a workload; ``n_events`` < E gives the leading subset."""
    offsets, feat = truth_events(w.n_events, w.mult, w.truth_seed)
    if n_events is not None and n_events < w.n_events:
        offsets = offsets[: n_events + 1].copy()
        feat = feat[: offsets[-1]].copy()
    return offsets, feat


def subset(offsets: np.ndarray, feat: np.ndarray, idx) -> tuple:
    """Events ``idx`` (any order) of a CSR batch as a new CSR batch."""
    idx = np.asarray(idx, dtype=np.int64)
    n = offsets[idx + 1] - offsets[idx]
    out_off = np.zeros(len(idx) + 1, dtype=np.int64)
    np.cumsum(n, out=out_off[1:])
    rows = np.concatenate([np.arange(offsets[i], offsets[i + 1]) for i in idx]) if len(idx) else \
        np.zeros(0, dtype=np.int64)
    return out_off, feat[rows].copy()


def split(offsets: np.ndarray, feat: np.ndarray):
    """List of per-event [N_e, F] arrays."""
    return [feat[offsets[e]:offsets[e + 1]] for e in range(len(offsets) - 1)]


def join(event_list, n_feat: int = F_FEAT):
    offsets = np.zeros(len(event_list) + 1, dtype=np.int64)
    np.cumsum([len(a) for a in event_list], out=offsets[1:])
    feat = np.concatenate(event_list).astype(np.float32) if len(event_list) and offsets[-1] \
        else np.zeros((0, n_feat), dtype=np.float32)
    return offsets, feat
