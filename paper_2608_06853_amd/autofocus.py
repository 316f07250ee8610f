"""Autofocus driver over the library.

* ``Beamformer`` owns one library context for an acquisition (array, lens,
  channel-data format), an evaluation grid and a slowness grid;
* ``CmpeLoss`` is a ``torch.autograd.Function``: its forward runs the library's
  forward pass (travel times, DAS, CMPE, regularisers) and keeps only the
  gradient with respect to the block images; its backward recomputes the
  travel-time table and runs the hand-written adjoints (under a memory budget
  the library's chunked loss-and-gradient call runs in the forward instead);
* ``sweep`` is the global-speed initialisation with the dynamic CMPE grid and
  ``plain_autofocus`` the plain iterative method (Sections II-C and III-A of the
  paper; the optimiser is Adam instead of the plain descent of Eq. 9).

Every step of the method runs in libaf.so; this module sequences the calls and
holds the tensors they read and write.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, replace

import numpy as np
import torch

from . import _lib


@dataclass
class Acquisition:
    elem_xz: np.ndarray      # [N][2] mm, centre of curvature at the origin
    d_lens: float            # mm
    c_lens: float            # mm/us
    t_ttp: float             # us
    fs: float                # MHz
    t0: float                # us
    fd: float                # MHz (demodulation = centre frequency)
    n_samples: int
    lens_mode: int = _lib.LENS_BENT   # beamformer's lens model (_lib.LENS_*)
    c_ref: float = 1.540     # mm/us, reference speed of the conventional lens offset


@dataclass
class Imaging:
    centres: np.ndarray      # [n_pix][2] patch centres, mm
    patch: int               # 1 or 3
    spacing: float           # mm (lambda/2)
    block: int               # S
    fnum: float              # F of |x'| <= (F/2) z'
    n_seg: int


@dataclass
class Grid:
    nx: int
    nz: int
    x0: float
    z0: float
    dx: float
    dz: float

    @property
    def shape(self):
        return (self.nz, self.nx)


def is_linear(acq: Acquisition) -> bool:
    """Every element on one line z = const: a linear array with a flat lens (the
    library's own test of the array shape)."""
    z = acq.elem_xz[:, 1]
    return bool(np.max(np.abs(z - z[0])) <= 1e-9 * (1.0 + np.max(np.abs(acq.elem_xz[:, 0]))))


SWEEP_MIN, SWEEP_MAX = 1.340, 1.740   # mm/us, the global sweep's range (Section III-A)


class Beamformer:
    """Library context bound to one acquisition, evaluation grid and slowness grid."""

    def __init__(self, acq: Acquisition, img: Imaging, grid: Grid, device: int = 0,
                 n_search: int = 0, deterministic: bool = False, memory_budget: int = 0):
        """``n_search`` = 0 refracts at the exact Fermat root, >= 2 by the discrete
        search over that many lens points; ``deterministic`` fixes the reduction
        order of the gradient (bit-for-bit repeatable, a few percent slower);
        ``memory_budget`` > 0 bounds the device memory of the per-point buffers
        (bytes) by recomputing the travel times in the gradient pass."""
        self.acq, self.grid = acq, grid
        self.device = torch.device("cuda", device)
        self.ctx = _lib.Context(device)
        self.ctx.set_lens(acq.d_lens, acq.c_lens, acq.t_ttp, acq.lens_mode, acq.c_ref)
        self.ctx.set_refraction_search(n_search)
        self.ctx.set_deterministic(deterministic)
        self.ctx.set_memory_budget(memory_budget)
        self.img = None
        self.set_imaging(img)
        self.s = None

    def set_imaging(self, img: Imaging, keep_slowness: bool = True):
        """New evaluation grid.  The slowness is set again unless the caller sets a
        new one next (keep_slowness=False)."""
        a = self.acq
        self.ctx.set_geometry(a.elem_xz, img.centres, img.patch, img.spacing, a.n_samples, a.fs,
                              a.t0, a.fd, img.block, img.fnum, img.n_seg)
        self.img = img
        self.dynamic = None
        if keep_slowness and getattr(self, "s", None) is not None:
            self.set_slowness(self.s)

    def set_dynamic_grid(self, c_ref: float, fc: float, c_min: float = SWEEP_MIN,
                         c_max: float = SWEEP_MAX):
        """The library's dynamic CMPE grid over the current pixels (laid out for c_ref);
        af_set_sweep_speed then moves them.  The slowness is set again."""
        self.ctx.set_dynamic_grid(c_ref, fc, c_min, c_max)
        self.dynamic = (c_ref, fc, c_min, c_max)
        s = getattr(self, "s", None)
        self.set_slowness(s if s is not None else
                          torch.full(self.grid.shape, 1.0 / c_ref, device=self.device))

    def set_speed(self, c_g: float, c_ref: float, fc: float):
        """Points of the dynamic grid of speed c_g (set up for (c_ref, fc) on first use)."""
        d = self.dynamic
        if d is None or d[:2] != (c_ref, fc) or not d[2] <= c_g <= d[3]:
            self.set_dynamic_grid(c_ref, fc, min(SWEEP_MIN, c_g), max(SWEEP_MAX, c_g))
        self.ctx.set_sweep_speed(c_g)

    def set_slowness(self, s: torch.Tensor):
        g = self.grid
        s = s.detach().to(self.device, torch.float32).contiguous()
        self.ctx.set_slowness(g.nx, g.nz, g.x0, g.z0, g.dx, g.dz, s)
        self.s = s

    @property
    def n_points(self) -> int:
        return self.ctx.query(_lib.Q_P)

    @property
    def n_blk(self) -> int:
        return self.ctx.query(_lib.Q_NBLK)

    def empty_terms(self):
        return torch.zeros(_lib.N_TERMS, device=self.device, dtype=torch.float32)

    def loss_and_grad(self, iq, lp, s=None, want_grad=True):
        if s is not None:
            self.set_slowness(s)
        terms = self.empty_terms()
        grad = torch.empty(self.grid.shape, device=self.device) if want_grad else None
        self.ctx.loss_and_grad(iq, lp, terms, grad)
        return terms, grad

    def beamform(self, iq, s=None, blocks=False, maps=True):
        if s is not None:
            self.set_slowness(s)
        P = self.n_points
        nb = self.n_blk
        img = torch.empty(P, device=self.device, dtype=torch.complex64)
        mp = torch.empty(3 * self.img.centres.shape[0], device=self.device) if maps else None
        blk = torch.empty(nb * nb * P, device=self.device, dtype=torch.complex64) if blocks else None
        self.ctx.beamform(iq, blk, img, mp)
        return img, mp, blk

    def channel_images(self, iq, s=None):
        """Receive-channel images [n_elem][points] (complex64) at the slowness."""
        if s is not None:
            self.set_slowness(s)
        n = self.acq.elem_xz.shape[0]
        out = torch.empty(n * self.n_points, device=self.device, dtype=torch.complex64)
        self.ctx.channel_images(iq, out)
        return out.view(n, self.n_points)

    def lag_one_coherence(self, iq, s=None):
        """Per-pixel lag-one coherence [n_pix] at the slowness."""
        if s is not None:
            self.set_slowness(s)
        out = torch.empty(self.img.centres.shape[0], device=self.device)
        self.ctx.lag_one_coherence(iq, out)
        return out

    def travel_times(self, s=None):
        if s is not None:
            self.set_slowness(s)
        out = torch.empty(self.acq.elem_xz.shape[0] * self.n_points, device=self.device)
        self.ctx.travel_times(out)
        return out.view(self.acq.elem_xz.shape[0], self.n_points)


class CmpeLoss(torch.autograd.Function):
    """total = L_CMPE + w1 R_TV + w2 R_SV - w_sb SB/SB_ref as a function of the slowness.

    forward keeps only dL/dB^blk (no travel-time table); backward recomputes the
    table at the same slowness and runs the DAS and path adjoints.  Under a memory
    budget the library's chunked call forms the gradient in the forward (it
    recomputes each chunk's table there) and only the gradient grid is kept."""

    @staticmethod
    def forward(ctx, s, bf: Beamformer, iq, lp):
        bf.set_slowness(s)
        terms = bf.empty_terms()
        ctx.bf, ctx.iq, ctx.lp = bf, iq, lp
        if bf.ctx.query(_lib.Q_CHUNKS) > 1:
            grad = torch.empty(bf.grid.shape, device=bf.device)
            bf.ctx.loss_and_grad(iq, lp, terms, grad)
            ctx.grad, ctx.gblk = grad, None
        else:
            gblk = torch.empty(bf.ctx.query(_lib.Q_GBLK_ELEMS), device=bf.device,
                               dtype=torch.complex64)
            bf.ctx.forward(iq, lp, terms, gblk)
            ctx.grad, ctx.gblk = None, gblk
        ctx.save_for_backward(s)
        ctx.mark_non_differentiable(terms)
        return terms[_lib.TERM_TOTAL].clone(), terms

    @staticmethod
    def backward(ctx, g_total, g_terms):
        (s,) = ctx.saved_tensors
        bf = ctx.bf
        grad = ctx.grad
        if grad is None:
            bf.set_slowness(s)
            grad = torch.empty(bf.grid.shape, device=bf.device)
            bf.ctx.backward(ctx.iq, ctx.lp, ctx.gblk, grad)
        return (g_total * grad).view_as(s), None, None, None


def cmpe_loss(s: torch.Tensor, bf: Beamformer, iq: torch.Tensor, lp) -> tuple:
    """(total, terms) with total differentiable in ``s`` through the library's adjoint."""
    return CmpeLoss.apply(s, bf, iq, lp)


def sweep_speeds(lo=1.340, hi=1.740, step=0.010) -> np.ndarray:
    n = int(round((hi - lo) / step)) + 1
    return lo + step * np.arange(n)


def sweep(bf: Beamformer, iq, lp, fc: float, c_ref: float = 1.540, speeds=None, dynamic=True,
          static_c: float = 1.500):
    """CMPE of homogeneous speeds (Section II-C, model initialisation).  With
    ``dynamic`` every speed c_g is evaluated on the grid laid out for c_g; without,
    every speed is evaluated on the one grid laid out for ``static_c`` (the static
    grid the dynamic one replaces).  Leaves ``bf`` on the grid of the best speed
    (dynamic) or the static grid, with a uniform slowness.  Returns
    (speeds, values, best).  The library moves the points (af_set_dynamic_grid,
    af_sweep); the pixels of ``bf.img`` are the layout of c_ref."""
    speeds = sweep_speeds() if speeds is None else np.asarray(speeds, dtype=np.float64)
    lo = min(float(speeds.min()), static_c if not dynamic else np.inf)
    hi = max(float(speeds.max()), static_c if not dynamic else -np.inf)
    d = bf.dynamic
    if d is None or d[:2] != (c_ref, fc) or not (d[2] <= lo and hi <= d[3]):
        bf.set_dynamic_grid(c_ref, fc, lo, hi)
    vals = torch.empty(len(speeds), device=bf.device)
    best = bf.ctx.sweep(iq, lp, speeds, dynamic, static_c, vals)
    bf.s = torch.full(bf.grid.shape, 1.0 / best, device=bf.device)
    return speeds, vals.cpu().numpy().astype(np.float64), best


@dataclass
class History:
    terms: list = field(default_factory=list)
    times: list = field(default_factory=list)


def calibrated(bf: Beamformer, iq, lp, s: torch.Tensor):
    """Copy of ``lp`` whose speckle-brightness reference is SB at slowness ``s``."""
    probe = _lib.LossParams(*[getattr(lp, n) for n, _ in _lib.LossParams._fields_])
    probe.sb_ref = 1.0
    bf.set_slowness(s)
    terms = bf.empty_terms()
    bf.ctx.loss_and_grad(iq, probe, terms, None)
    sb = float(terms[_lib.TERM_SB].item())
    out = _lib.LossParams(*[getattr(lp, n) for n, _ in _lib.LossParams._fields_])
    out.sb_ref = sb if sb > 0 else 1.0
    return out


def plain_autofocus(bf: Beamformer, iq, lp, ap, n_iter: int, s0: torch.Tensor | None = None,
                    record_every: int = 1, stop_below: float | None = None,
                    calibrate_sb: bool = True):
    """Adam iterations of the plain method from ``s0`` (default: the context's slowness).

    Returns (s, History).  With ``stop_below`` the loop stops at the first
    iteration whose CMPE is at or below it (the terms of every iteration are read
    back only when a stop criterion or recording needs them).  With a speckle
    term, its reference SB_ref is the speckle brightness at the starting slowness."""
    s = (bf.s if s0 is None else s0).detach().clone().to(bf.device, torch.float32).contiguous()
    if lp.w_sb != 0.0 and calibrate_sb:
        lp = calibrated(bf, iq, lp, s)
    m = torch.zeros_like(s)
    v = torch.zeros_like(s)
    terms = bf.empty_terms()
    hist = History()
    t_start = time.perf_counter()
    for it in range(1, n_iter + 1):
        bf.ctx.autofocus_step(iq, lp, ap, it, s, m, v, terms)
        if stop_below is not None or (record_every and it % record_every == 0):
            t = terms.cpu().numpy().copy()
            hist.terms.append(t)
            hist.times.append(time.perf_counter() - t_start)
            if stop_below is not None and t[_lib.TERM_CMPE] <= stop_below:
                break
    bf.s = s
    return s, hist
