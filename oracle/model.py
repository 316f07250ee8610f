"""The whole differentiable beamformer: travel times -> DAS -> loss -> gradient.

Paper: Fig. 1 steps (b)-(g); Eqs. 1-8 (model), Eq. 12 (objective), the Sound
Speed Estimation and Model Implementation subsections (slowness grid, bent rays
refracted with the global mean speed, reverse-mode gradient back to the grid).

Readings (beyond those of the step modules):
* c_med is the arithmetic mean of c = 1/s over the grid nodes;
* the refraction points, c_med, the apodisation masks and the CMPE validity
  masks are held constant when differentiating (stop-gradient);
* the objective may add a speckle-brightness term -w_sb * SB / SB_ref
  (SB_ref > 0 given by the caller; w_sb = 0 gives the paper's Eq. 12).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry, fermat, path, das, cmpe, reg


@dataclass
class LossParams:
    w1: float = 10.0
    kx1: float = 0.01
    kz1: float = 0.01
    w2: float = 100.0
    kx2: float = 0.001
    kz2: float = 0.001
    rho_thresh: float = 0.9
    w_sb: float = 0.0
    sb_ref: float = 1.0


@dataclass
class Problem:
    elem_xz: np.ndarray          # [N][2] mm
    d_lens: float                # mm
    c_lens: float                # mm/us
    t_ttp: float                 # us
    centres: np.ndarray          # [n_pix][2] patch centres, mm
    patch: int                   # points per side of a patch
    spacing: float               # mm, patch point spacing
    t0: float                    # us
    fs: float                    # MHz
    fd: float                    # MHz
    block: int                   # S
    fnum: float                  # F
    n_seg: int                   # ray segments
    grid: tuple                  # (x0, z0, dx, dz, nx, nz)
    iq: np.ndarray | None = None  # [N][N][Ns] complex
    n_search: int = 0            # discrete refraction candidates (0: continuous root)
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n_elem(self):
        return self.elem_xz.shape[0]

    @property
    def n_patch(self):
        return self.patch * self.patch

    def points(self) -> np.ndarray:
        if "pts" not in self._cache:
            self._cache["pts"] = geometry.patch_points(self.centres, self.patch,
                                                       self.spacing).reshape(-1, 2)
        return self._cache["pts"]

    def apod(self) -> np.ndarray:
        if "h" not in self._cache:
            th = geometry.element_orientation(self.elem_xz)
            xp, zp = geometry.element_frame(self.elem_xz, th, self.points())
            self._cache["h"] = geometry.apodization(xp, zp, self.fnum)
        return self._cache["h"]


def c_mean(s: np.ndarray) -> float:
    return float(np.mean(1.0 / s.astype(np.float64)))


def rays(prob: Problem, s: np.ndarray, mask: np.ndarray | None = None,
         c_med: float | None = None):
    """Refraction of every masked (element, point) ray at c_med = mean(1/s)
    (or at the given ``c_med``, which tests use to hold it fixed).

    Returns (a_idx, p_idx, dict) for the selected rays."""
    pts = prob.points()
    if mask is None:
        mask = prob.apod()
    ai, pi = np.nonzero(mask)
    cm = c_mean(s) if c_med is None else c_med
    if prob.n_search >= 2 and prob.d_lens > 0:
        r = fermat.discrete_refract(prob.elem_xz, prob.d_lens, prob.c_lens, cm, pts,
                                    prob.n_search, pairs=(ai, pi))
    else:
        r = fermat.refract(prob.elem_xz, prob.d_lens, prob.c_lens, cm, pts, pairs=(ai, pi))
    return ai, pi, r


def travel_times(prob: Problem, s: np.ndarray, mask: np.ndarray | None = None,
                 c_med: float | None = None):
    """T[a][p] = L1/c_lens + L2 * trapezoid sum of bicubic slowness (Eqs. 1, 8).

    Entries outside ``mask`` (default: the apodisation) are NaN."""
    pts = prob.points()
    if mask is None:
        mask = prob.apod()
    ai, pi, r = rays(prob, s, mask, c_med)
    tm = path.medium_time(s.astype(np.float64), prob.grid, r["ref_x"], r["ref_z"],
                          pts[pi, 0], pts[pi, 1], r["l2"], prob.n_seg)
    T = np.full(mask.shape, np.nan)
    T[ai, pi] = r["l1"] / prob.c_lens + tm
    return T


def forward(prob: Problem, s: np.ndarray, lp: LossParams, keep: bool = False,
            c_med: float | None = None):
    """Loss terms (dict) at slowness ``s`` [nz][nx]."""
    h = prob.apod()
    T = travel_times(prob, s, h, c_med)
    Tz = np.where(h, T, 0.0)
    bblk = das.das_blocks(prob.iq, Tz, h, t0=prob.t0, fs=prob.fs, fd=prob.fd,
                          t_ttp=prob.t_ttp, block=prob.block)
    bsub = cmpe.subaperture_images(bblk)
    l_cmpe, nv, cmap, _ = cmpe.cmpe_loss(bsub, prob.n_patch, lp.rho_thresh)
    sb = cmpe.speckle_brightness(bblk, prob.n_patch) / lp.sb_ref
    x0, z0, dx, dz, nx, nz = prob.grid
    tv, sv = reg.reg_terms(s.astype(np.float64), dx, dz, lp.kx1, lp.kz1, lp.kx2, lp.kz2)
    total = l_cmpe + lp.w1 * tv + lp.w2 * sv - lp.w_sb * sb
    out = dict(cmpe=l_cmpe, tv=tv, sv=sv, sb=sb, total=total, n_valid=nv, cmpe_map=cmap,
               cf=cmpe.coherence_factor(bblk, prob.n_patch),
               cmcc=cmpe.cmcc_map(bsub, prob.n_patch))
    if keep:
        out.update(T=T, bblk=bblk, bsub=bsub)
    return out


def loss_and_grad(prob: Problem, s: np.ndarray, lp: LossParams, c_med: float | None = None):
    """(terms, dL/ds) by the analytic adjoint (reverse order of ``forward``)."""
    f = forward(prob, s, lp, keep=True, c_med=c_med)
    h = prob.apod()
    gsub = cmpe.cmpe_loss_grad(f["bsub"], prob.n_patch, lp.rho_thresh)
    gblk = cmpe.subaperture_images_adjoint(gsub)
    if lp.w_sb != 0.0:
        gblk = gblk - (lp.w_sb / lp.sb_ref) * cmpe.speckle_brightness_grad(f["bblk"], prob.n_patch)
    Tz = np.where(h, f["T"], 0.0)
    g = das.das_blocks_adjoint_T(prob.iq, Tz, h, gblk, t0=prob.t0, fs=prob.fs, fd=prob.fd,
                                 t_ttp=prob.t_ttp, block=prob.block)
    pts = prob.points()
    ai, pi, r = rays(prob, s, h, c_med)
    gs = path.medium_time_adjoint(g[ai, pi], prob.grid, r["ref_x"], r["ref_z"],
                                  pts[pi, 0], pts[pi, 1], r["l2"], prob.n_seg)
    x0, z0, dx, dz, nx, nz = prob.grid
    gs = gs + reg.reg_grad(s.astype(np.float64), dx, dz, lp.kx1, lp.kz1, lp.kx2, lp.kz2,
                           lp.w1, lp.w2)
    f["g_T"] = g
    f["g_blk"] = gblk
    return f, gs
