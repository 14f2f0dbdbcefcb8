"""Error measures between two sets of outputs (any two sources).

``normwise_rel_err``: for each feature f over all real rows,
    err_f = max_i |y[i,f] - ref[i,f]| / max_i |ref[i,f]|,
the per-feature reading of "max relative error per output feature" that stays defined
when single reference values are near zero. The worst feature is the headline number.

``response``: per particle paired with the truth particle of the same CSR index,
r_pT = pT_reco / pT_truth and r_eta = eta_reco - eta_truth, summarised by sample mean
and width (population standard deviation) plus the 16-84% half width.
"""

import numpy as np


def normwise_rel_err(y, ref) -> np.ndarray:
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    if y.size == 0:
        return np.zeros(y.shape[-1] if y.ndim else 0)
    num = np.max(np.abs(y - ref), axis=0)
    den = np.max(np.abs(ref), axis=0)
    return num / np.where(den > 0, den, 1.0)


def elementwise_rel_err(y, ref) -> np.ndarray:
    """Diagnostic: max_i |dy| / (|ref| + rms_f) per feature."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = np.sqrt(np.mean(ref * ref, axis=0))
    return np.max(np.abs(y - ref) / (np.abs(ref) + rms), axis=0)


def response(reco, truth) -> dict:
    reco = np.asarray(reco, dtype=np.float64)
    truth = np.asarray(truth, dtype=np.float64)
    r_pt = np.exp(reco[:, 0] - truth[:, 0])          # ratio of 10 GeV * exp(x0)
    r_eta = reco[:, 1] - truth[:, 1]
    out = {}
    for name, r in (("pt", r_pt), ("eta", r_eta)):
        q16, q84 = np.quantile(r, [0.16, 0.84])
        out[name] = {"mean": float(np.mean(r)), "width": float(np.std(r)),
                     "half_width_68": float(0.5 * (q84 - q16))}
    return out


def response_agrees(resp, resp_ref, frac: float = 0.01) -> bool:
    ok = True
    for name in ("pt", "eta"):
        m, w = resp[name]["mean"], resp[name]["width"]
        m0, w0 = resp_ref[name]["mean"], resp_ref[name]["width"]
        ok &= abs(m - m0) <= frac * max(abs(m0), w0)
        ok &= abs(w - w0) <= frac * w0
    return bool(ok)
