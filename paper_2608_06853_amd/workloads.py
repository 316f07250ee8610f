"""Seeded synthetic workloads on the GPU: a configured ``Beamformer`` plus
channel data simulated by the library from a random medium of ``afsynth``.

The slowness grid covers the imaged sector at every speed of the dynamic-grid
sweep (depths stretched up to 1740/1540).
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

import afsynth
from . import _lib, autofocus as af

SWEEP_MAX = 1.740


LENS_MODELS = ("bent", "conventional", "none")


def geometry(cfg, lens_model: str = "bent"):
    """(acquisition, imaging, slowness grid, cover points) of ``cfg`` for one lens
    model of the beamformer:

    * ``bent``: the two-layer Fermat ray through the lens (Eqs. 7-8);
    * ``conventional``: straight rays from the elements plus the scalar round-trip
      lens offset of Eq. 6, which the library forms from the lens constants;
    * ``none``: straight rays from the elements, no lens term.

    Pixels are the same physical points in every model; the slowness grid of the
    straight-ray models also covers the element arc, where their rays start."""
    if lens_model not in LENS_MODELS:
        raise ValueError(f"lens model must be one of {LENS_MODELS}")
    arr, acq, img, met = cfg.array, cfg.acq, cfg.img, cfg.method
    elem = afsynth.element_positions(arr)
    centres = afsynth.pixel_centres(arr, img)
    sp = afsynth.patch_spacing(img, acq)
    smax = SWEEP_MAX / img.c_ref
    cover = np.concatenate([centres, afsynth.pixel_centres(arr, img, depth_scale=smax)])
    arr_box = arr if lens_model == "bent" else replace(arr, d_lens=0.0)
    x0, z0, dx, dz = afsynth.slowness_box(arr_box, cover, sp * smax, met.nx, met.nz)
    acqd = af.Acquisition(elem_xz=elem, d_lens=arr.d_lens, c_lens=arr.c_lens, t_ttp=arr.t_ttp,
                          fs=acq.fs, t0=acq.t0, fd=acq.fc, n_samples=acq.n_samples,
                          lens_mode=_lib.LENS_MODES[lens_model], c_ref=img.c_ref)
    imgd = af.Imaging(centres=centres, patch=img.patch, spacing=sp, block=met.block,
                      fnum=met.fnum, n_seg=met.n_seg)
    grid = af.Grid(nx=met.nx, nz=met.nz, x0=x0, z0=z0, dx=dx, dz=dz)
    return acqd, imgd, grid, cover


def simulate(bf: af.Beamformer, cfg, med, cover) -> torch.Tensor:
    """Channel data [N*N*Ns] complex64 on the GPU for medium ``med``."""
    arr, acq = cfg.array, cfg.acq
    sp = afsynth.patch_spacing(cfg.img, acq)
    sx0, sz0, sdx, sdz, snx, snz = afsynth.sim_box(arr, np.concatenate([cover, med.scat_xz]), sp,
                                                   cfg.sim_spacing)
    s_true = torch.from_numpy(
        (1.0 / afsynth.speed_on_grid(med, sx0, sz0, sdx, sdz, snx, snz)).astype(np.float32)
    ).to(bf.device)
    n = arr.n_elem
    iq = torch.empty(n * n * acq.n_samples, device=bf.device, dtype=torch.complex64)
    bf.ctx.simulate(med.scat_xz, med.scat_amp.astype(np.float32), snx, snz, sx0, sz0, sdx, sdz,
                    s_true, cfg.sim_nseg, acq.fc, acq.frac_bw, iq)
    return iq


def build(cfg, seed=None, device: int = 0, lens_model: str = "bent",
          deterministic: bool = False):
    """(Beamformer of ``lens_model`` at a uniform 1/c_ref slowness, channel data,
    medium).  The channel data always come from the bent-ray physics of the lens
    (the library's simulator uses the physical lens whatever the lens model);
    ``deterministic`` fixes the gradient's reduction order."""
    acqd, imgd, grid, cover = geometry(cfg, lens_model)
    bf = af.Beamformer(acqd, imgd, grid, device, deterministic=deterministic)
    med = afsynth.medium_for(cfg, seed)
    iq = simulate(bf, cfg, med, cover)
    bf.set_slowness(torch.full(grid.shape, 1.0 / cfg.img.c_ref, device=bf.device))
    return bf, iq, med


def true_speed_nodes(cfg, med, grid, sub: int = 8) -> np.ndarray:
    """True speed averaged over each node's cell (sub x sub samples), [nz][nx]."""
    off = (np.arange(sub) + 0.5) / sub - 0.5
    xs = grid.x0 + grid.dx * (np.arange(grid.nx)[:, None] + off[None, :])
    zs = grid.z0 + grid.dz * (np.arange(grid.nz)[:, None] + off[None, :])
    X = xs[None, :, None, :]
    Z = zs[:, None, :, None]
    c = afsynth.sample_speed(med, np.broadcast_to(X, (grid.nz, grid.nx, sub, sub)),
                             np.broadcast_to(Z, (grid.nz, grid.nx, sub, sub)))
    return c.mean(axis=(2, 3))


def loss_params(cfg, sb_ref: float = 1.0):
    from . import _lib
    m = cfg.method
    return _lib.loss_params(m.w1, m.kx1, m.kz1, m.w2, m.kx2, m.kz2, m.rho_thresh, m.w_sb, sb_ref)
