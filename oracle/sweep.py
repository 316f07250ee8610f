"""Global sound-speed sweep with the adaptive (dynamic) CMPE grid.

Paper: Sound Speed Estimation subsection (CMPE evaluated over a discrete range
of global speeds, the lowest CMPE initialises the grid; the dynamic grid moves
the CMPE pixels and kernel spacing with the active speed so the same speckle
is observed) and Model Implementation (sweep from 1340 to 1740 m/s, 3x3 kernel
at lambda/2).

Readings: the sweep step is 10 m/s; the reference grid is laid out for
c_ref = 1.540 mm/us, and at speed c_g every pixel's depth below the lens
surface is scaled by c_g/c_ref along its polar angle while the kernel spacing
becomes c_g/(2 f_c).  For radial rays through the concentric lens this keeps
the round-trip time exactly fixed.  For a linear array with a flat lens the
depth below the lens plane is scaled straight down, which keeps it fixed for
rays normal to the lens.

The static grid of the earlier method (the comparison of the model-initialisation
results) is laid out once for 1500 m/s: every speed of the sweep is evaluated on
the pixels and kernel spacing of c_g = 1.500 mm/us.
"""
from __future__ import annotations

import numpy as np

from .fermat import is_linear
from . import cmpe
from .model import Problem, LossParams, forward


def sweep_speeds(lo: float = 1.340, hi: float = 1.740, step: float = 0.010) -> np.ndarray:
    n = int(round((hi - lo) / step)) + 1
    return lo + step * np.arange(n)


def scaled_centres(centres: np.ndarray, elem_xz: np.ndarray, d_lens: float, c_g: float,
                   c_ref: float) -> np.ndarray:
    if is_linear(elem_xz):
        # flat lens: depth below the lens plane scaled straight down
        zl = float(elem_xz[0, 1]) + d_lens
        return np.stack([centres[:, 0], zl + (centres[:, 1] - zl) * (c_g / c_ref)], axis=1)
    rl = float(np.hypot(elem_xz[0, 0], elem_xz[0, 1])) + d_lens
    rho = np.hypot(centres[:, 0], centres[:, 1])
    th = np.arctan2(centres[:, 0], centres[:, 1])
    rho_g = rl + (rho - rl) * (c_g / c_ref)
    return np.stack([rho_g * np.sin(th), rho_g * np.cos(th)], axis=1)


def sweep(prob: Problem, lp: LossParams, fc: float, c_ref: float = 1.540,
          speeds: np.ndarray | None = None, dynamic: bool = True, static_c: float = 1.500,
          rho_band: float | None = None):
    """CMPE for each homogeneous speed.  Returns (speeds, cmpe values, best speed);
    with ``rho_band`` also, per speed, (n_valid, number of pairs with energy whose
    rho lies within rho_band of rho_thresh)."""
    speeds = sweep_speeds() if speeds is None else speeds
    x0, z0, dx, dz, nx, nz = prob.grid
    vals, info = [], []
    for c_g in speeds:
        if dynamic:
            cen = scaled_centres(prob.centres, prob.elem_xz, prob.d_lens, c_g, c_ref)
            sp = c_g / (2.0 * fc)
        else:
            cen = scaled_centres(prob.centres, prob.elem_xz, prob.d_lens, static_c, c_ref)
            sp = static_c / (2.0 * fc)
        p = Problem(**{**prob.__dict__, "centres": cen, "spacing": sp, "_cache": {}})
        s = np.full((nz, nx), 1.0 / c_g)
        f = forward(p, s, lp, keep=rho_band is not None)
        vals.append(f["cmpe"])
        if rho_band is not None:
            d = cmpe.cmpe(f["bsub"], p.n_patch, lp.rho_thresh)
            pos = (d["ex"] > cmpe.MIN_ENERGY) & (d["ey"] > cmpe.MIN_ENERGY)
            info.append((f["n_valid"], int(np.sum(pos & (np.abs(d["rho"] - lp.rho_thresh)
                                                           < rho_band)))))
    vals = np.array(vals)
    best = float(speeds[int(np.argmin(vals))])
    if rho_band is not None:
        return speeds, vals, best, info
    return speeds, vals, best
