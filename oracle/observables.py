"""Event-level observables of reconstructed events: FP64 oracle — TEST INFRASTRUCTURE ONLY.

Follows the event post-processing of Sec. 2.4: the scalar transverse-momentum sum H_T and
the missing transverse momentum of each event (recomputed from the particles), and the
isolation of each electron or muon, R_iso = (sum of the pT of the other particles of the
event inside the cone Delta R = sqrt(Delta eta^2 + Delta phi^2) < 0.4 around it) / pT of the
lepton (the isolation equation of Sec. 2.4, sums excluding the lepton itself).

Readings (the paper leaves these open):
  * Kinematics come from the 9-slot particle state of the model (reading R3): pT = 10 GeV x
    exp(x0), eta = x1, phi = x2, class = first maximum of x3..x7 in the order charged
    hadron, electron, muon, neutral hadron, photon. Leptons are the electron and muon
    classes.
  * The cone sums run over every other particle of the event, charged, neutral and photon
    alike. The exclusion of final-state-radiation photon candidates has no definition in
    the paper and is not applied.
  * Delta phi = d - 2 pi rint(d / (2 pi)) with d = phi_i - phi_j (the state's phi is not
    confined to [-pi, pi]). A particle is inside the cone when Delta eta^2 + Delta phi^2 <
    0.16. That test, and the class maximum, decide integers from floating point, so they
    are taken in float32 with separate multiplies and adds, the device's precision; every
    sum is FP64 here.
  * MET is the magnitude of the vector sum of (pT cos phi, pT sin phi) over the event.
  * Particles that are not leptons get NaN isolation; an empty event has H_T = MET = 0.

Plain NumPy, one event at a time; the brute-force double loop in the tests pins it.
"""

import numpy as np

CLASS_ELECTRON = 1
CLASS_MUON = 2
CONE_R2 = np.float32(0.16)
TWO_PI_F32 = np.float32(2.0 * np.pi)
INV_TWO_PI_F32 = np.float32(1.0 / (2.0 * np.pi))


def decode(feat: np.ndarray):
    """(pT FP64, eta float32, phi float32, class int) of particles [n, 9] (reading R3)."""
    f = np.asarray(feat, dtype=np.float32)
    pt = 10.0 * np.exp(f[:, 0].astype(np.float64))
    cls = np.argmax(f[:, 3:8], axis=1)          # first maximum, float32 comparisons
    return pt, f[:, 1], f[:, 2], cls


def in_cone(eta_i, phi_i, eta, phi) -> np.ndarray:
    """Delta R < 0.4 of particle i against the arrays eta, phi, decided in float32."""
    deta = np.float32(eta_i) - eta.astype(np.float32)
    d = np.float32(phi_i) - phi.astype(np.float32)
    dphi = d - TWO_PI_F32 * np.rint(d * INV_TWO_PI_F32).astype(np.float32)
    r2 = deta * deta + dphi * dphi               # float32 products and sum, no fused form
    return r2 < CONE_R2


def event_observables(feat: np.ndarray):
    """H_T, MET and per-particle isolation of one event's particles [n, 9]."""
    n = len(feat)
    iso = np.full(n, np.nan)
    if n == 0:
        return 0.0, 0.0, iso
    pt, eta, phi, cls = decode(feat)
    phi64 = phi.astype(np.float64)
    ht = float(pt.sum())
    met = float(np.hypot((pt * np.cos(phi64)).sum(), (pt * np.sin(phi64)).sum()))
    for i in range(n):
        if cls[i] != CLASS_ELECTRON and cls[i] != CLASS_MUON:
            continue
        inside = in_cone(eta[i], phi[i], eta, phi)
        inside[i] = False                          # the lepton itself is excluded
        iso[i] = float(pt[inside].sum()) / pt[i]
    return ht, met, iso


def observables(offsets: np.ndarray, feat: np.ndarray):
    """(ht [E], met [E], iso [T]) of a CSR batch of reconstructed events."""
    E = len(offsets) - 1
    ht, met = np.zeros(E), np.zeros(E)
    iso = np.full(int(offsets[-1]), np.nan)
    for e in range(E):
        a, b = int(offsets[e]), int(offsets[e + 1])
        ht[e], met[e], iso[a:b] = event_observables(feat[a:b])
    return ht, met, iso
