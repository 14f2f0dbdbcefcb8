"""The stand-in velocity network, FP64, one event at a time — oracle side.

The paper (Sec. 2.2) gives the model as a learned vector field over the reconstructed
particle set, conditioned on the event's truth particles, and defers its architecture to
earlier work. The stand-in used here (a reading, not the paper's trained model):

* truth encoder: c = LN_t(u W_tin + b_tin), u the 9 truth features per particle;
* time features: phi(t) = [sin(w_k t) | cos(w_k t)], w_k = 10000^(-k/(E/2)),
  k < E/2, on the unscaled time t in [0, 1];
* input: H = x W_xin + b_xin + (phi(t) W_time + b_time), x the 9-feature state;
* per block, pre-LayerNorm residual sub-blocks
    H += SelfAttn(LN1(H)) W_o + b_o          (over the event's own reco slots)
    H += CrossAttn(LN2(H), c) W_oc + b_oc    (keys/values from the truth encoding)
    H += GELU(LN3(H) W_up + b_up) W_dn + b_dn
* head: v = LN_f(H) W_out + b_out.

LayerNorm: (z - mean) / sqrt(var + 1e-5) * g + s with the biased variance over the
feature axis. GELU: z/2 (1 + erf(z / sqrt 2)). Attention per head: softmax over the
event's keys of Q K^T / sqrt(dh), rows max-subtracted; no padding ever exists here.
"""

import math

import numpy as np
from scipy.special import erf as _erf

LN_EPS = 1e-5


def _shapes(cfg):
    """Flat-parameter order (independent restatement of the documented layout)."""
    d, F, Fo, E, R = cfg.d_model, cfg.f_truth, cfg.f_reco, cfg.t_embed_dim, cfg.mlp_ratio
    head = [("W_tin", (F, d)), ("b_tin", (d,)), ("g_t", (d,)), ("s_t", (d,)),
            ("W_xin", (Fo, d)), ("b_xin", (d,)), ("W_time", (E, d)), ("b_time", (d,))]
    block = [("g1", (d,)), ("s1", (d,)), ("W_qkv", (d, 3 * d)), ("b_qkv", (3 * d,)),
             ("W_o", (d, d)), ("b_o", (d,)), ("g2", (d,)), ("s2", (d,)),
             ("W_qc", (d, d)), ("b_qc", (d,)), ("W_kc", (d, d)), ("b_kc", (d,)),
             ("W_vc", (d, d)), ("b_vc", (d,)), ("W_oc", (d, d)), ("b_oc", (d,)),
             ("g3", (d,)), ("s3", (d,)), ("W_up", (d, R * d)), ("b_up", (R * d,)),
             ("W_dn", (R * d, d)), ("b_dn", (d,))]
    tail = [("g_f", (d,)), ("s_f", (d,)), ("W_out", (d, Fo)), ("b_out", (Fo,))]
    return head, block, tail


def unpack(flat, cfg, dtype=np.float64) -> dict:
    """Flat FP32 vector -> dict of arrays (upcast to ``dtype``); blocks in P['blocks']."""
    flat = np.asarray(flat)
    head, block, tail = _shapes(cfg)
    pos = 0

    def take(shape):
        nonlocal pos
        n = int(np.prod(shape))
        a = flat[pos:pos + n].astype(dtype).reshape(shape)
        pos += n
        return a

    P = {name: take(s) for name, s in head}
    P["blocks"] = [{name: take(s) for name, s in block} for _ in range(cfg.n_blocks)]
    P.update({name: take(s) for name, s in tail})
    if pos != flat.size:
        raise ValueError(f"parameter vector has {flat.size} values, layout needs {pos}")
    P["cfg"] = cfg
    return P


def linear(x, W, b):
    """y = x W + b with W stored [in, out]."""
    return x @ W + b


def layer_norm(z, g, s, eps=LN_EPS):
    mu = z.mean(axis=-1, keepdims=True)
    var = ((z - mu) ** 2).mean(axis=-1, keepdims=True)
    return (z - mu) / np.sqrt(var + eps) * g + s


def gelu(z):
    """Exact GELU through the error function (SciPy's vectorised erf)."""
    z = np.asarray(z)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)).astype(z.dtype))


def softmax_rows(S):
    S = S - S.max(axis=-1, keepdims=True)
    E = np.exp(S)
    return E / E.sum(axis=-1, keepdims=True)


def attention(Q, K, V, n_heads):
    """Multi-head scaled dot-product attention of one event.

    Q [Nq, d], K and V [Nk, d]; head h uses columns [h dh, (h+1) dh). Returns [Nq, d].
    """
    Nq, d = Q.shape
    dh = d // n_heads
    out = np.empty((Nq, d), dtype=Q.dtype)
    scale = 1.0 / math.sqrt(dh)
    for h in range(n_heads):
        sl = slice(h * dh, (h + 1) * dh)
        P = softmax_rows((Q[:, sl] @ K[:, sl].T) * scale)
        out[:, sl] = P @ V[:, sl]
    return out


def time_features(t, E):
    """phi(t) in R^E: sines then cosines of w_k t, w_k = 10000^(-k/(E/2))."""
    half = E // 2
    w = 10000.0 ** (-np.arange(half, dtype=np.float64) / half)
    a = float(t) * w
    return np.concatenate([np.sin(a), np.cos(a)])


def encode_truth(P, u):
    return layer_norm(linear(u, P["W_tin"], P["b_tin"]), P["g_t"], P["s_t"])


def velocity(P, u, x, t):
    """v(x, t | truth u) for one event: u [N_truth, 9], x [N_reco, 9] -> [N_reco, 9]."""
    cfg = P["cfg"]
    dt = P["W_xin"].dtype
    u = np.asarray(u, dtype=dt)
    x = np.asarray(x, dtype=dt)
    c = encode_truth(P, u)
    temb = linear(time_features(t, cfg.t_embed_dim).astype(dt), P["W_time"], P["b_time"])
    H = linear(x, P["W_xin"], P["b_xin"]) + temb
    d = cfg.d_model
    for B in P["blocks"]:
        A = layer_norm(H, B["g1"], B["s1"])
        qkv = linear(A, B["W_qkv"], B["b_qkv"])
        O = attention(qkv[:, :d], qkv[:, d:2 * d], qkv[:, 2 * d:], cfg.n_heads)
        H = H + linear(O, B["W_o"], B["b_o"])
        A = layer_norm(H, B["g2"], B["s2"])
        Q = linear(A, B["W_qc"], B["b_qc"])
        Kc = linear(c, B["W_kc"], B["b_kc"])
        Vc = linear(c, B["W_vc"], B["b_vc"])
        O = attention(Q, Kc, Vc, cfg.n_heads)
        H = H + linear(O, B["W_oc"], B["b_oc"])
        A = layer_norm(H, B["g3"], B["s3"])
        H = H + linear(gelu(linear(A, B["W_up"], B["b_up"])), B["W_dn"], B["b_dn"])
    return linear(layer_norm(H, P["g_f"], P["s_f"]), P["W_out"], P["b_out"])
