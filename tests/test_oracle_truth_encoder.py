"""Pins of the oracle's truth encoder c = LN_t(u W_tin + b_tin) and of the time features.

The paper conditions the sampled vector field on the event's truth particles (Sec. 2.2) and
prints no values of the network, so the encoder is pinned by rows whose LayerNorm has a
closed form:

* a constant pre-activation row (every column of W_tin equal, b_tin constant) has zero
  deviation from its mean, so its LayerNorm is the shift s_t, whatever the gain;
* a row of +a and -a in equal numbers has mean 0 and biased variance a^2, so its LayerNorm
  is sign_j a / sqrt(a^2 + eps) g_t[j] + s_t[j]: with |a| of order sqrt(eps) the eps term
  changes the result by tens of percent.

The same rows are then pushed through the whole velocity field with every other path cut
(self-attention, MLP and all but one cross-attention value path zeroed, one truth particle so
the softmax is exactly 1, W_oc = I), where v = LN_f(h + c W_vc + b_vc) W_out + b_out with h
the input embedding. The expected value is computed with scalar Python sums (math.fsum),
not the oracle's vectorised LayerNorm. The time features are pinned at t = 0, where the
sines vanish and the cosines are 1.

Each pin is checked to fail when a plausible mistake is planted in the oracle (LN_t dropped,
gain and shift swapped, a wrong eps, the state embedding's weights used for the truth).
"""

import math

import numpy as np
import pytest

from oracle import net
from workload import configs, params

CFG = configs.SMALL_MODEL       # d = 64, 2 blocks, 4 heads
D = CFG.d_model
EPS = 1e-5


def _ln_scalar(z, g, s, eps=EPS):
    """LayerNorm of one row by scalar sums (biased variance over the row)."""
    n = len(z)
    mu = math.fsum(z) / n
    var = math.fsum((zi - mu) ** 2 for zi in z) / n
    r = 1.0 / math.sqrt(var + eps)
    return np.array([(zi - mu) * r * gi + si for zi, gi, si in zip(z, g, s)])


def _row_matvec(x, W, b):
    """x W + b for one row by scalar sums."""
    return np.array([math.fsum(x[i] * W[i, j] for i in range(len(x))) + b[j]
                     for j in range(W.shape[1])])


def _encoder_params(kind, seed=0):
    """Perturbed parameters (gains and shifts differ from 1 and 0 and from one another) with
    W_tin and b_tin set so that u W_tin + b_tin has a closed-form LayerNorm."""
    flat = params.draw(CFG, seed=seed, perturbed=True)
    nm = params.named(CFG, flat)
    w = np.random.default_rng(seed + 7).standard_normal(9) * 0.3
    if kind == "constant":
        nm["W_tin"][:] = w[:, None]                  # every column the same
        nm["b_tin"][:] = 0.25
    else:                                             # +a in even columns, -a in odd ones
        sign = np.where(np.arange(D) % 2 == 0, 1.0, -1.0)
        nm["W_tin"][:] = w[:, None] * sign[None, :]
        nm["b_tin"][:] = 0.0
    return flat, nm, w


def _expected_c(kind, nm, w, u_row):
    g = nm["g_t"].astype(np.float64)
    s = nm["s_t"].astype(np.float64)
    if kind == "constant":
        return s.copy()
    a = math.fsum(float(u_row[i]) * float(np.float32(w[i])) for i in range(9))
    sign = np.where(np.arange(D) % 2 == 0, 1.0, -1.0)
    return sign * a / math.sqrt(a * a + EPS) * g + s


def _u_row(scale):
    u = np.array([0.7, -1.1, 2.3, 0, 0, 1, 0, 0, -1.0])
    return u * scale


# ---- the encoder alone ----------------------------------------------------------------

@pytest.mark.parametrize("kind,scale", [("constant", 1.0), ("pm", 1.0), ("pm", 3e-3)])
def test_encoder_closed_form(kind, scale):
    flat, nm, w = _encoder_params(kind)
    P = net.unpack(flat, CFG)
    u = _u_row(scale)[None, :]
    c = net.encode_truth(P, u)[0]
    ref = _expected_c(kind, nm, w, u[0])
    np.testing.assert_allclose(c, ref, rtol=1e-9, atol=1e-12)


def test_pm_row_is_sensitive_to_eps():
    """At |a| ~ sqrt(eps) the closed form differs by > 10% between eps = 1e-5 and eps = 0,
    so the comparison above fixes eps."""
    _, nm, w = _encoder_params("pm")
    a = math.fsum(float(_u_row(3e-3)[i]) * float(np.float32(w[i])) for i in range(9))
    assert abs(a) < 10 * math.sqrt(EPS)
    assert abs(a / math.sqrt(a * a + EPS) - math.copysign(1.0, a)) > 0.1


# ---- the encoder inside the velocity field ------------------------------------------------

def _truth_path_params(kind):
    """Cut every path but the truth value path of block 0's cross-attention:
    W_qkv = 0 and b_qkv = 0 (self-attention values 0), W_o = 0, b_o = 0; W_up = 0, b_up = 0
    (GELU(0) = 0), b_dn = 0; block 0: W_oc = I, b_oc = 0; later blocks: W_oc = 0, b_oc = 0."""
    flat, nm, w = _encoder_params(kind)
    for l in range(CFG.n_blocks):
        p = f"blk{l}."
        for name in ("W_qkv", "b_qkv", "W_o", "b_o", "W_up", "b_up", "b_dn", "b_oc"):
            nm[p + name][:] = 0.0
        nm[p + "W_oc"][:] = np.eye(D) if l == 0 else 0.0
    return flat, nm, w


def _expected_velocity(nm, kind, w, u_row, x_row, t):
    f64 = {k: v.astype(np.float64) for k, v in nm.items()}
    c = _expected_c(kind, nm, w, u_row)
    # input embedding h = x W_xin + b_xin + phi(t) W_time + b_time; at t = 0 phi is
    # 16 zeros (sines) then 16 ones (cosines)
    assert t == 0.0
    half = CFG.t_embed_dim // 2
    phi0 = np.r_[np.zeros(half), np.ones(half)]
    h = _row_matvec(x_row, f64["W_xin"], f64["b_xin"]) + \
        _row_matvec(phi0, f64["W_time"], f64["b_time"])
    vc = _row_matvec(c, f64["blk0.W_vc"], f64["blk0.b_vc"])
    hf = _ln_scalar(h + vc, f64["g_f"], f64["s_f"])
    return _row_matvec(hf, f64["W_out"], f64["b_out"])


def _truth_path_error(kind, scale=1.0):
    flat, nm, w = _truth_path_params(kind)
    P = net.unpack(flat, CFG)
    u = _u_row(scale)[None, :]
    x = np.random.default_rng(3).standard_normal((3, 9))     # three reco slots, one truth
    v = net.velocity(P, u, x, 0.0)
    ref = np.stack([_expected_velocity(nm, kind, w, u[0], x[i], 0.0) for i in range(3)])
    return np.abs(v - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("kind,scale", [("constant", 1.0), ("pm", 1.0), ("pm", 3e-3)])
def test_truth_value_path_closed_form(kind, scale):
    assert _truth_path_error(kind, scale) < 1e-10


def test_time_features_at_zero_enter_the_embedding():
    """With W_time != 0, t = 0 and every block and the truth cut, the velocity of a slot is
    LN_f(x W_xin + b_xin + sum of W_time's cosine rows + b_time) W_out + b_out."""
    flat = params.draw(CFG, seed=4, perturbed=True)
    nm = params.named(CFG, flat)
    for l in range(CFG.n_blocks):
        for name in ("W_o", "b_o", "W_oc", "b_oc", "W_dn", "b_dn"):
            nm[f"blk{l}.{name}"][:] = 0.0
    P = net.unpack(flat, CFG)
    x = np.array([[0.3, -1.2, 2.0, 0, 1, 0, 0, 0, 1.0]])
    f64 = {k: v.astype(np.float64) for k, v in nm.items()}
    half = CFG.t_embed_dim // 2
    cos_rows = np.array([math.fsum(f64["W_time"][k, j] for k in range(half, 2 * half))
                         for j in range(D)])
    h = _row_matvec(x[0], f64["W_xin"], f64["b_xin"]) + cos_rows + f64["b_time"]
    ref = _row_matvec(_ln_scalar(h, f64["g_f"], f64["s_f"]), f64["W_out"], f64["b_out"])
    v = net.velocity(P, np.zeros((2, 9)), x, 0.0)[0]
    np.testing.assert_allclose(v, ref, rtol=1e-10, atol=1e-12)


# ---- planted mistakes must fail the pins --------------------------------------------------

def _planted(monkeypatch, variant):
    ln = net.layer_norm

    def enc(P, u):
        z = net.linear(u, P["W_tin"], P["b_tin"])
        if variant == "no_ln":
            return z
        if variant == "swap":
            return ln(z, P["s_t"], P["g_t"])
        if variant == "eps0":
            return ln(z, P["g_t"], P["s_t"], eps=0.0)
        if variant == "w_xin":
            return ln(net.linear(u, P["W_xin"], P["b_tin"]), P["g_t"], P["s_t"])
        raise ValueError(variant)

    monkeypatch.setattr(net, "encode_truth", enc)


@pytest.mark.parametrize("variant", ["no_ln", "swap", "eps0", "w_xin"])
def test_planted_encoder_mistakes_are_caught(monkeypatch, variant):
    _planted(monkeypatch, variant)
    with np.errstate(invalid="ignore", divide="ignore"):
        errs = [_truth_path_error(k, s) for k, s in (("constant", 1.0), ("pm", 1.0), ("pm", 3e-3))]
    # caught: some pin is off by more than 1e-3 (or not finite, as 0/0 with eps = 0)
    assert not all(np.isfinite(e) and e < 1e-3 for e in errs), (variant, errs)


def test_planted_time_feature_order_is_caught(monkeypatch):
    """Cosines first instead of sines first changes phi(0) and fails the t = 0 pin."""
    orig = net.time_features

    def swapped(t, E):
        f = orig(t, E)
        return np.r_[f[E // 2:], f[:E // 2]]

    monkeypatch.setattr(net, "time_features", swapped)
    with pytest.raises(AssertionError):
        test_time_features_at_zero_enter_the_embedding()
