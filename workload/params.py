"""Seeded parameters of the stand-in velocity network.

The paper's trained checkpoints are not available, so the network is a stand-in with
seeded random weights: every matrix is drawn N(0, 1/fan_in) with fan_in its input width,
biases are zero, LayerNorm gains one and shifts zero. A second flavour (``perturbed``)
also draws biases, gains and shifts, so that those paths are exercised.

Flat layout (FP32, this exact order; every matrix is [in, out] row-major and is applied
as y = x W + b). With d = d_model, F = 9, E = t_embed_dim, R = mlp_ratio:

    W_tin[F,d]  b_tin[d]  g_t[d]  s_t[d]          truth encoder Linear + LayerNorm
    W_xin[F,d]  b_xin[d]                          state input embedding
    W_time[E,d] b_time[d]                         time embedding Linear
    per block:
      g1[d] s1[d]  W_qkv[d,3d] b_qkv[3d]  W_o[d,d] b_o[d]          self-attention
      g2[d] s2[d]  W_qc[d,d] b_qc[d]  W_kc[d,d] b_kc[d]  W_vc[d,d] b_vc[d]  W_oc[d,d] b_oc[d]
      g3[d] s3[d]  W_up[d,Rd] b_up[Rd]  W_dn[Rd,d] b_dn[d]          MLP
    g_f[d] s_f[d]  W_out[d,F] b_out[F]                              output head

The columns of W_qkv are [Q | K | V]; head h owns columns [h*dh, (h+1)*dh) of each.
This module only lays out and draws numbers; the two consumers unpack it on their own.
"""

import numpy as np

from .configs import ModelCfg


def layout(cfg: ModelCfg):
    """List of (name, shape, kind) in flat order; kind in {'w', 'b', 'g', 's'}."""
    d, F, E, R = cfg.d_model, cfg.f_truth, cfg.t_embed_dim, cfg.mlp_ratio
    Fo = cfg.f_reco
    out = [("W_tin", (F, d), "w"), ("b_tin", (d,), "b"), ("g_t", (d,), "g"), ("s_t", (d,), "s"),
           ("W_xin", (Fo, d), "w"), ("b_xin", (d,), "b"),
           ("W_time", (E, d), "w"), ("b_time", (d,), "b")]
    for l in range(cfg.n_blocks):
        p = f"blk{l}."
        out += [(p + "g1", (d,), "g"), (p + "s1", (d,), "s"),
                (p + "W_qkv", (d, 3 * d), "w"), (p + "b_qkv", (3 * d,), "b"),
                (p + "W_o", (d, d), "w"), (p + "b_o", (d,), "b"),
                (p + "g2", (d,), "g"), (p + "s2", (d,), "s"),
                (p + "W_qc", (d, d), "w"), (p + "b_qc", (d,), "b"),
                (p + "W_kc", (d, d), "w"), (p + "b_kc", (d,), "b"),
                (p + "W_vc", (d, d), "w"), (p + "b_vc", (d,), "b"),
                (p + "W_oc", (d, d), "w"), (p + "b_oc", (d,), "b"),
                (p + "g3", (d,), "g"), (p + "s3", (d,), "s"),
                (p + "W_up", (d, R * d), "w"), (p + "b_up", (R * d,), "b"),
                (p + "W_dn", (R * d, d), "w"), (p + "b_dn", (d,), "b")]
    out += [("g_f", (d,), "g"), ("s_f", (d,), "s"), ("W_out", (d, Fo), "w"), ("b_out", (Fo,), "b")]
    return out


def count(cfg: ModelCfg) -> int:
    return int(sum(np.prod(s) for _, s, _ in layout(cfg)))


def draw(cfg: ModelCfg, seed: int = 0, perturbed: bool = False) -> np.ndarray:
    """Flat float32 parameter vector.

    Matrices consume one ``default_rng(seed)`` stream in layout order. With ``perturbed``
    a second stream (seed + 1000) then draws biases ~ N(0, 0.1^2), gains 1 + N(0, 0.1^2)
    and shifts ~ N(0, 0.1^2), again in layout order.
    """
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, kind in layout(cfg):
        if kind == "w":
            parts.append((rng.standard_normal(shape) / np.sqrt(shape[0])).ravel())
        elif kind == "g":
            parts.append(np.ones(shape))
        else:
            parts.append(np.zeros(shape))
    if perturbed:
        rng2 = np.random.default_rng(seed + 1000)
        for i, (name, shape, kind) in enumerate(layout(cfg)):
            if kind == "b" or kind == "s":
                parts[i] = 0.1 * rng2.standard_normal(shape).ravel()
            elif kind == "g":
                parts[i] = 1.0 + 0.1 * rng2.standard_normal(shape).ravel()
    return np.concatenate(parts).astype(np.float32)


def named(cfg: ModelCfg, flat: np.ndarray) -> dict:
    """Views of a flat vector by name (used by tests to edit single tensors)."""
    out, o = {}, 0
    for name, shape, _ in layout(cfg):
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    assert o == flat.size, (o, flat.size)
    return out
