"""Evaluation metrics of the Model Evaluation subsection, on host arrays.

These are reporting steps outside the differentiable hot path: the images and
slowness maps they take come from the library.

* sound-speed MAE (Eq. 13) and RMSE of an estimated map against the true one;
* contrast (dB) and CNR of an anechoic region against its surroundings, with
  contrast = 20 log10(mu_in / mu_out) and CNR = |mu_in - mu_out| /
  sqrt(var_in + var_out) on the envelope (Rodriguez-Molares et al.); the regions
  are the disc r < 0.7 R inside the cyst and the annulus 1.3 R < r < 2 R around
  it (the paper drew its regions by hand);
* the generalised CNR of the same regions (Rodriguez-Molares et al.): one minus
  the overlap of the two envelope histograms, over 100 common bins;
* the lateral -6 dB width of a point target: along the image row of the
  envelope peak near the target, the distance between the two half-amplitude
  crossings (linear interpolation between columns);
* the Tenengrad sharpness change eta between an aberrated and a corrected image:
  both envelopes are log-compressed to a 60 dB display range, the corrected
  image is scaled so that its 80th-percentile amplitude equals the aberrated
  one's, a lateral Sobel filter is applied, the filtered amplitudes are summed
  from 10 mm depth down, and eta = 100 (S_corrected / S_aberrated - 1).
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
            "cnr": float(abs(mi - mo) / np.sqrt(vi + vo + 1e-30)),
            "gcnr": gcnr(env[inside], env[outside])}


def gcnr(a: np.ndarray, b: np.ndarray, bins: int = 100) -> float:
    """1 - sum_k min(p_a(k), p_b(k)) over ``bins`` common bins of the two samples."""
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    lo, hi = min(a.min(), b.min()), max(a.max(), b.max())
    if not hi > lo:
        return 0.0
    edges = np.linspace(lo, hi, bins + 1)
    pa = np.histogram(a, edges)[0] / a.size
    pb = np.histogram(b, edges)[0] / b.size
    return float(1.0 - np.minimum(pa, pb).sum())


def log_compress(env: np.ndarray, dyn_range_db: float = 60.0) -> np.ndarray:
    """Envelope [depth][angle] -> display amplitude in [0, 1] over dyn_range_db."""
    env = np.asarray(env, dtype=np.float64)
    db = 20.0 * np.log10(np.maximum(env, 1e-30) / max(float(env.max()), 1e-30))
    return np.clip(db + dyn_range_db, 0.0, dyn_range_db) / dyn_range_db


def lateral_sobel(img: np.ndarray) -> np.ndarray:
    """3x3 Sobel derivative along the lateral (last) axis, edge rows/columns replicated."""
    p = np.pad(img, 1, mode="edge")
    d = p[:, 2:] - p[:, :-2]                       # central difference across columns
    return d[:-2] + 2.0 * d[1:-1] + d[2:]          # [1, 2, 1] smoothing along depth


def tenengrad_change(env_aberrated: np.ndarray, env_corrected: np.ndarray, depth_mm: np.ndarray,
                     min_depth_mm: float = 10.0) -> float:
    """eta (%) for envelopes [depth][angle] with row depths ``depth_mm``."""
    a = log_compress(env_aberrated)
    c = log_compress(env_corrected)
    pa, pc = np.percentile(a, 80.0), np.percentile(c, 80.0)
    if pc > 0:
        c = c * (pa / pc)
    rows = np.asarray(depth_mm) >= min_depth_mm
    sa = float(np.abs(lateral_sobel(a))[rows].sum())
    sc = float(np.abs(lateral_sobel(c))[rows].sum())
    return 100.0 * (sc / sa - 1.0) if sa > 0 else float("nan")


def point_width(env: np.ndarray, col_mm: np.ndarray, row: int, col: int, search: int = 3) -> float:
    """Lateral -6 dB width (mm) of the peak of envelope ``env`` [rows][cols] nearest
    (row, col); ``col_mm`` gives the lateral position of every column, for all
    rows ([cols]) or per row ([rows][cols]).  NaN if the half-amplitude level is
    not crossed on both sides."""
    env = np.asarray(env, dtype=np.float64)
    r0, r1 = max(row - search, 0), min(row + search + 1, env.shape[0])
    c0, c1 = max(col - search, 0), min(col + search + 1, env.shape[1])
    win = env[r0:r1, c0:c1]
    pr, pc = np.unravel_index(np.argmax(win), win.shape)
    pr, pc = pr + r0, pc + c0
    line = env[pr]
    col_mm = np.asarray(col_mm, dtype=np.float64)
    if col_mm.ndim == 2:
        col_mm = col_mm[pr]
    while pc > 0 and line[pc - 1] > line[pc]:          # climb to the row's local maximum
        pc -= 1
    while pc < line.size - 1 and line[pc + 1] > line[pc]:
        pc += 1
    half = 0.5 * line[pc]
    pos = []
    for step in (-1, 1):
        k = pc
        while 0 <= k + step < line.size and line[k + step] > half:
            k += step
        if not 0 <= k + step < line.size:
            return float("nan")
        a, b = line[k], line[k + step]          # a > half >= b
        t = (a - half) / (a - b)
        pos.append(col_mm[k] + t * (col_mm[k + step] - col_mm[k]))
    return float(abs(pos[1] - pos[0]))
