"""The whole differentiable beamformer: travel times -> DAS -> loss -> gradient.

Paper: Fig. 1 steps (b)-(g); Eqs. 1-8 (model), Eq. 12 (objective), the Sound
Speed Estimation and Model Implementation subsections (slowness grid, bent rays
refracted with the global mean speed, reverse-mode gradient back to the grid).

Lens models (``lens``): ``Problem.lens_model`` selects the bent-ray model
(Eqs. 7-8, the default), the conventional model (Eq. 6: straight rays from the
elements plus a scalar lens offset) or no lens correction (straight rays only).

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

from . import geometry, fermat, path, das, cmpe, reg, lens


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
    lens_model: str = "bent"     # "bent" (Eqs. 7-8), "conventional" (Eq. 6) or "none"
    c_ref: float = lens.C_REF    # mm/us, reference speed of the conventional lens offset
    _cache: dict = field(default_factory=dict, repr=False)

    @property
    def n_elem(self):
        return self.elem_xz.shape[0]

    @property
    def ray_d_lens(self) -> float:
        """Lens thickness the rays refract through (0: straight rays from the elements)."""
        return lens.ray_lens_thickness(self.lens_model, self.d_lens)

    @property
    def tau_offset(self) -> float:
        """Scalar added to every round trip (time-to-peak, plus the conventional
        model's lens offset)."""
        return lens.round_trip_offset(self.lens_model, self.d_lens, self.c_lens, self.t_ttp,
                                      self.c_ref)

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
    d = prob.ray_d_lens
    if prob.n_search >= 2 and d > 0:
        r = fermat.discrete_refract(prob.elem_xz, d, prob.c_lens, cm, pts, prob.n_search,
                                    pairs=(ai, pi))
    else:
        r = fermat.refract(prob.elem_xz, d, prob.c_lens, cm, pts, pairs=(ai, pi))
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
                          t_ttp=prob.tau_offset, block=prob.block)
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
                                 t_ttp=prob.tau_offset, block=prob.block)
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


def loss_and_grad_parts(prob: Problem, s: np.ndarray, lp: LossParams,
                        c_med: float | None = None, rho_band: float = 0.0) -> dict:
    """The additive pieces of ``loss_and_grad`` over the pixels of ``prob``, so that
    disjoint pixel sets can be evaluated separately and combined (``combine_parts``).

    Every term of the objective except the regularisers is a sum over pixels of
    per-pixel quantities (the CMPE pairs and the speckle brightness belong to one
    patch each), and the gradient is linear in the image gradient; the travel
    times depend on the whole grid only through c_med, which is held constant.
    Returns the sums sum_err (|arg C| over valid pairs), n_valid and sum_sb
    (|B|^2 at the patch centres), the pixel count, and the gradients of sum_err
    and of sum_sb with respect to the slowness grid (the second only when
    lp.w_sb != 0).  With rho_band > 0 it also counts the pairs with energy whose
    rho lies within rho_band of rho_thresh (n_near: where a lower precision may
    judge validity differently)."""
    f = forward(prob, s, lp, keep=True, c_med=c_med)
    h = prob.apod()
    n_pix = prob.centres.shape[0]
    nv = f["n_valid"]
    Tz = np.where(h, f["T"], 0.0)
    pts = prob.points()
    ai, pi, r = rays(prob, s, h, c_med)

    def to_grid(gblk):
        g = das.das_blocks_adjoint_T(prob.iq, Tz, h, gblk, t0=prob.t0, fs=prob.fs, fd=prob.fd,
                                     t_ttp=prob.tau_offset, block=prob.block)
        return path.medium_time_adjoint(g[ai, pi], prob.grid, r["ref_x"], r["ref_z"],
                                        pts[pi, 0], pts[pi, 1], r["l2"], prob.n_seg)

    # d(sum of |arg C| over valid pairs)/dB: the mean's gradient times n_valid
    g_err = to_grid(cmpe.subaperture_images_adjoint(
        nv * cmpe.cmpe_loss_grad(f["bsub"], prob.n_patch, lp.rho_thresh)))
    g_sb = None
    if lp.w_sb != 0.0:
        # d(sum over centres of |B|^2)/dB: the mean's gradient times the pixel count
        g_sb = to_grid(n_pix * cmpe.speckle_brightness_grad(f["bblk"], prob.n_patch))
    n_near = 0
    if rho_band > 0.0:
        d = cmpe.cmpe(f["bsub"], prob.n_patch, lp.rho_thresh)
        pos = (d["ex"] > cmpe.MIN_ENERGY) & (d["ey"] > cmpe.MIN_ENERGY)
        n_near = int(np.sum(pos & (np.abs(d["rho"] - lp.rho_thresh) < rho_band)))
    return dict(sum_err=f["cmpe"] * nv, n_valid=nv, sum_sb=f["sb"] * lp.sb_ref * n_pix,
                n_pix=n_pix, grad_err=g_err, grad_sb=g_sb, n_near=n_near)


def combine_parts(parts: list, s: np.ndarray, lp: LossParams, grid) -> tuple:
    """(terms, dL/ds) of the objective over the union of the pixel sets of ``parts``
    (from ``loss_and_grad_parts`` at the same slowness): L_CMPE is the mean over
    all valid pairs, SB the mean over all pixels, plus the regularisers of Eqs.
    10-11 on the grid."""
    nv = sum(p["n_valid"] for p in parts)
    n_pix = sum(p["n_pix"] for p in parts)
    sum_err = sum(p["sum_err"] for p in parts)
    l_cmpe = sum_err / nv if nv > 0 else 0.0
    sb = sum(p["sum_sb"] for p in parts) / n_pix / lp.sb_ref
    x0, z0, dx, dz, nx, nz = grid
    s64 = s.astype(np.float64)
    tv, sv = reg.reg_terms(s64, dx, dz, lp.kx1, lp.kz1, lp.kx2, lp.kz2)
    total = l_cmpe + lp.w1 * tv + lp.w2 * sv - lp.w_sb * sb
    g = reg.reg_grad(s64, dx, dz, lp.kx1, lp.kz1, lp.kx2, lp.kz2, lp.w1, lp.w2)
    if nv > 0:
        g = g + sum(p["grad_err"] for p in parts) / nv
    if lp.w_sb != 0.0:
        g = g - (lp.w_sb / (lp.sb_ref * n_pix)) * sum(p["grad_sb"] for p in parts)
    terms = dict(cmpe=l_cmpe, tv=tv, sv=sv, sb=sb, total=total, n_valid=nv)
    return terms, g
