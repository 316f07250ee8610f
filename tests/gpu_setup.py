"""Shared set-up of GPU parity tests: one seeded workload fed to both the oracle
and the library (inputs come from afsynth / the oracle simulator only)."""
from __future__ import annotations

import functools
import os
from dataclasses import replace

import numpy as np

import afsynth
import problems
from oracle import model

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    """Builds the library when it is missing or older than its sources."""
    from paper_2608_06853_amd import build
    return build.ensure_built()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


# A case on the tiny 32-element array small enough for the oracle: 8 blocks,
# 24 x 20 pixels (480 patches -> 18 tiles, ragged tail), 8 x 8 slowness grid.
C1_SMALL = afsynth.configs.C1.with_(
    name="c1_small",
    img=afsynth.ImgCfg(n_depth=24, n_angle=20, depth_min=3.0, depth_max=55.0),
    n_scat_random=1200,
)

MICRO = afsynth.configs.MICRO

# A linear array whose deeper pixels see more of its 24 blocks (48 elements in
# blocks of 2) than the CMPE stage can stage in LDS: their tiles run that stage
# from device memory, the shallow ones from LDS.  12 x 8 pixels from 4 to 24 mm.
_ML = afsynth.configs.MICRO_LINEAR
WIDE_LINEAR = _ML.with_(
    name="wide_linear",
    array=replace(_ML.array, n_elem=48),
    acq=replace(_ML.acq, n_samples=1024),
    img=afsynth.ImgCfg(n_depth=12, n_angle=8, depth_min=4.0, depth_max=24.0),
    method=replace(_ML.method, block=2),
)


@functools.lru_cache(maxsize=8)
def case(name: str, t0: float = 0.0, t_ttp: float = 0.0, patch: int = 3, block: int | None = None,
         perturb: float = 0.01, d_lens: float | None = None, n_search: int = 0,
         grid_nx: int | None = None, lens_model: str = "bent", rho: float = 0.5,
         grid_nz: int | None = None):
    """(cfg, oracle problem, iq complex64, s [nz][nx] float32, loss params).
    d_lens = 0 gives a lens-free array; lens_model "conventional" or "none" the
    straight-ray models of the beamformer (the channel data still come from the
    physical lens); n_search >= 2 the discrete refraction search; grid_nx and
    grid_nz replace the slowness grid's size; rho is the CMPE threshold."""
    base = {"micro": MICRO, "c1_small": C1_SMALL, "micro_linear": afsynth.configs.MICRO_LINEAR,
            "wide_linear": WIDE_LINEAR}[name]
    arr = replace(base.array, t_ttp=t_ttp)
    if d_lens is not None:
        arr = replace(arr, d_lens=d_lens)
    cfg = base.with_(array=arr, acq=replace(base.acq, t0=t0), img=replace(base.img, patch=patch))
    if block is not None:
        cfg = cfg.with_(method=replace(cfg.method, block=block))
    if grid_nx is not None:
        cfg = cfg.with_(method=replace(cfg.method, nx=grid_nx))
    if grid_nz is not None:
        cfg = cfg.with_(method=replace(cfg.method, nz=grid_nz))
    med = afsynth.medium_for(cfg)
    iq = problems.simulate_iq(cfg, med, n_seg=64).astype(np.complex64)
    prob = problems.problem(cfg, iq.astype(np.complex128))
    prob.n_search = n_search
    prob.lens_model = lens_model
    if lens_model != "bent":  # straight rays start at the elements: the grid covers them
        x0, z0, dx, dz, nx, nz = prob.grid
        zl = float(np.min(prob.elem_xz[:, 1])) - 0.25
        z1 = z0 + (nz - 1) * dz
        prob.grid = (x0, zl, dx, (z1 - zl) / (nz - 1), nx, nz)
    s_true = problems.true_slowness(cfg, med, prob)
    rng = np.random.default_rng(cfg.seed + 11)
    s = (s_true * (1.0 + perturb * rng.standard_normal(s_true.shape))).astype(np.float32)
    lp = problems.loss_params(cfg, sb_ref=float(np.mean(np.abs(iq)) ** 2 * 50.0))
    lp = model.LossParams(**{**lp.__dict__, "w_sb": 0.05, "rho_thresh": rho})
    return cfg, prob, iq, s, lp


def lib_params(lp):
    from paper_2608_06853_amd import _lib
    return _lib.loss_params(lp.w1, lp.kx1, lp.kz1, lp.w2, lp.kx2, lp.kz2, lp.rho_thresh, lp.w_sb,
                            lp.sb_ref)


def beamformer(cfg, prob, device=0):
    from paper_2608_06853_amd import autofocus as af
    from paper_2608_06853_amd import _lib
    acq = af.Acquisition(elem_xz=prob.elem_xz, d_lens=prob.d_lens, c_lens=prob.c_lens,
                         t_ttp=prob.t_ttp, fs=prob.fs, t0=prob.t0, fd=prob.fd,
                         n_samples=prob.iq.shape[2], lens_mode=_lib.LENS_MODES[prob.lens_model],
                         c_ref=prob.c_ref)
    img = af.Imaging(centres=prob.centres, patch=prob.patch, spacing=prob.spacing,
                     block=prob.block, fnum=prob.fnum, n_seg=prob.n_seg)
    x0, z0, dx, dz, nx, nz = prob.grid
    grid = af.Grid(nx=nx, nz=nz, x0=x0, z0=z0, dx=dx, dz=dz)
    return af.Beamformer(acq, img, grid, device, n_search=prob.n_search)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-30))
