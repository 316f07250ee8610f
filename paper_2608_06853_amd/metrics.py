"""Evaluation metrics of the Model Evaluation subsection, on host arrays.

These are reporting steps outside the differentiable hot path: the images and
slowness maps they take come from the library.

* sound-speed MAE (Eq. 13) and RMSE of an estimated map against the true one;
* contrast (dB) and CNR of an anechoic region against its surroundings, with
  contrast = 20 log10(mu_in / mu_out) and CNR = |mu_in - mu_out| /
  sqrt(var_in + var_out) on the envelope (Rodriguez-Molares et al.); the regions
  are the disc r < 0.7 R inside the cyst and the annulus 1.3 R < r < 2 R around
  it (the paper drew its regions by hand).
"""
from __future__ import annotations

import numpy as np


def speed_errors(s_est: np.ndarray, c_true: np.ndarray) -> dict:
    """MAE and RMSE in m/s between 1/s_est and c_true (both on the same nodes, mm/us)."""
    d = (1.0 / np.asarray(s_est, dtype=np.float64) - np.asarray(c_true, dtype=np.float64)) * 1000.0
    return {"mae_mps": float(np.mean(np.abs(d))), "rmse_mps": float(np.sqrt(np.mean(d * d)))}


def contrast_cnr(env: np.ndarray, xz: np.ndarray, centre, radius: float) -> dict:
    """Contrast (dB) and CNR of the envelope ``env`` at points ``xz`` for a cyst."""
    env = np.asarray(env, dtype=np.float64)
    r = np.hypot(xz[:, 0] - centre[0], xz[:, 1] - centre[1])
    inside = r < 0.7 * radius
    outside = (r > 1.3 * radius) & (r < 2.0 * radius)
    if inside.sum() < 3 or outside.sum() < 3:
        return {"contrast_db": float("nan"), "cnr": float("nan")}
    mi, mo = env[inside].mean(), env[outside].mean()
    vi, vo = env[inside].var(), env[outside].var()
    return {"contrast_db": float(20.0 * np.log10(max(mi, 1e-30) / max(mo, 1e-30))),
            "cnr": float(abs(mi - mo) / np.sqrt(vi + vo + 1e-30))}
