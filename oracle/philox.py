"""Philox4x64-10 and the Gaussian noise that starts the flow — oracle side.

The flow is integrated from a standard-normal sample (conditional flow matching starts
from noise; paper Sec. 2.2 and its flow-matching references). The paper names no
generator; this project fixes a counter-based one so that every particle slot's noise is
a pure function of (seed, event index, slot), independent of batching:

* Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 256-bit counter (c0..c3) and 128-bit key (k0, k1). A round
  multiplies c0 and c2 by the constants M0, M1 into 128-bit products and forms
  (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key is bumped
  by the Weyl constants between rounds.
* key = (seed, 0); counter = (b, slot, event, 0); block b = 0, 1, 2 feeds features
  0-3, 4-7 and 8.
* uniform u = ((w >> 41) + 1/2) * 2^-23 for each 64-bit word w (exact in FP32 and FP64,
  never 0 or 1).
* Box-Muller on word pairs (0, 1) and (2, 3): r = sqrt(-2 ln u_a),
  z_a = r cos(2 pi u_b), z_b = r sin(2 pi u_b).

Everything here is exact integer arithmetic on uint64 arrays plus the FP64 transform.
"""

import numpy as np

MASK64 = (1 << 64) - 1
M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """128-bit product of uint64 arrays: (hi, lo), by 32-bit limbs."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(counter, key):
    """Philox4x64-10 bijection.

    counter: uint64 array [..., 4]; key: uint64 array [..., 2] (broadcast).
    Returns uint64 array [..., 4].
    """
    with np.errstate(over="ignore"):
        c = np.array(counter, dtype=np.uint64, copy=True)
        k = np.array(np.broadcast_to(np.asarray(key, dtype=np.uint64), c.shape[:-1] + (2,)),
                     dtype=np.uint64, copy=True)
        c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
        k0, k1 = k[..., 0], k[..., 1]
        for r in range(10):
            if r:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        return np.stack([c0, c1, c2, c3], axis=-1)


def uniforms23(words: np.ndarray) -> np.ndarray:
    """Top 23 bits of each word, centred: ((w >> 41) + 0.5) * 2^-23, in FP64."""
    return ((np.asarray(words, dtype=np.uint64) >> np.uint64(41)).astype(np.float64) + 0.5) \
        * 2.0 ** -23


def _box_muller(ua: np.ndarray, ub: np.ndarray):
    r = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return r * np.cos(ang), r * np.sin(ang)


def noise_event(seed: int, event: int, n: int, n_feat: int = 9) -> np.ndarray:
    """x0 for one event of n slots: [n, n_feat] FP64 standard normals."""
    assert n_feat <= 12
    n_blocks = (n_feat + 3) // 4
    slots = np.arange(n, dtype=np.uint64)
    out = np.zeros((n, 4 * n_blocks))
    for b in range(n_blocks):
        ctr = np.zeros((n, 4), dtype=np.uint64)
        ctr[:, 0] = b
        ctr[:, 1] = slots
        ctr[:, 2] = np.uint64(event)
        w = philox4x64_10(ctr, np.array([seed & MASK64, 0], dtype=np.uint64))
        u = uniforms23(w)
        z0, z1 = _box_muller(u[:, 0], u[:, 1])
        z2, z3 = _box_muller(u[:, 2], u[:, 3])
        out[:, 4 * b + 0], out[:, 4 * b + 1] = z0, z1
        out[:, 4 * b + 2], out[:, 4 * b + 3] = z2, z3
    return out[:, :n_feat]


def noise_batch(seed: int, offsets, n_feat: int = 9) -> np.ndarray:
    """x0 for a CSR batch; event index = position within the batch."""
    offsets = np.asarray(offsets, dtype=np.int64)
    parts = [noise_event(seed, e, int(offsets[e + 1] - offsets[e]), n_feat)
             for e in range(len(offsets) - 1)]
    return np.concatenate(parts) if parts else np.zeros((0, n_feat))
