"""Builds oracle problems from the seeded workload configurations (test glue)."""
from __future__ import annotations

import numpy as np

import afsynth
from oracle import model, simulate


def geometry(cfg, depth_scale_max: float = 1.0):
    arr, img, acq, met = cfg.array, cfg.img, cfg.acq, cfg.method
    elem = afsynth.element_positions(arr)
    centres = afsynth.pixel_centres(arr, img)
    sp = afsynth.patch_spacing(img, acq)
    cover = afsynth.pixel_centres(arr, img, depth_scale=depth_scale_max)
    x0, z0, dx, dz = afsynth.slowness_box(arr, np.concatenate([centres, cover]),
                                          sp * depth_scale_max, met.nx, met.nz)
    grid = (x0, z0, dx, dz, met.nx, met.nz)
    return elem, centres, sp, grid


def problem(cfg, iq=None, depth_scale_max: float = 1.0):
    arr, img, acq, met = cfg.array, cfg.img, cfg.acq, cfg.method
    elem, centres, sp, grid = geometry(cfg, depth_scale_max)
    return model.Problem(elem_xz=elem, d_lens=arr.d_lens, c_lens=arr.c_lens, t_ttp=arr.t_ttp,
                         centres=centres, patch=img.patch, spacing=sp, t0=acq.t0, fs=acq.fs,
                         fd=acq.fc, block=met.block, fnum=met.fnum, n_seg=met.n_seg,
                         grid=grid, iq=iq)


def loss_params(cfg, sb_ref=1.0):
    m = cfg.method
    return model.LossParams(w1=m.w1, kx1=m.kx1, kz1=m.kz1, w2=m.w2, kx2=m.kx2, kz2=m.kz2,
                            rho_thresh=m.rho_thresh, w_sb=m.w_sb, sb_ref=sb_ref)


def true_slowness(cfg, medium, prob):
    x0, z0, dx, dz, nx, nz = prob.grid
    return 1.0 / afsynth.speed_on_grid(medium, x0, z0, dx, dz, nx, nz)


def simulate_iq(cfg, medium, n_seg=None):
    """Oracle-simulated channel data for ``medium`` (complex128)."""
    arr, acq = cfg.array, cfg.acq
    elem = afsynth.element_positions(arr)
    centres = afsynth.pixel_centres(arr, cfg.img)
    sp = afsynth.patch_spacing(cfg.img, acq)
    x0, z0, dx, dz, nx, nz = afsynth.sim_box(arr, np.concatenate([centres, medium.scat_xz]), sp,
                                             cfg.sim_spacing)
    s_true = 1.0 / afsynth.speed_on_grid(medium, x0, z0, dx, dz, nx, nz)
    return simulate.simulate(elem, arr.d_lens, arr.c_lens, arr.t_ttp, s_true,
                             (x0, z0, dx, dz, nx, nz), n_seg or cfg.sim_nseg,
                             medium.scat_xz, medium.scat_amp, t0=acq.t0, fs=acq.fs,
                             fd=acq.fc, ns=acq.n_samples, fc=acq.fc, frac_bw=acq.frac_bw)


def smooth_slowness(grid, seed):
    """Smooth seeded slowness around 1/1540 us/mm on the node grid (three plane
    waves of 1 % amplitude)."""
    x0, z0, dx, dz, nx, nz = grid
    rng = np.random.default_rng(seed)
    X, Z = np.meshgrid(np.linspace(0, 1, nx), np.linspace(0, 1, nz))
    s = np.full((nz, nx), 1.0 / 1.54)
    for _ in range(3):
        kx, kz, ph = rng.uniform(0.5, 2.0), rng.uniform(0.5, 2.0), rng.uniform(0, 2 * np.pi)
        s += 0.01 / 1.54 * np.cos(2 * np.pi * (kx * X + kz * Z) + ph)
    return s.astype(np.float32)


_sim = {}


def _sim_rows(rows):
    a = _sim
    return simulate.synthesize(a["T"], a["amp"], t_ttp=a["t_ttp"], t0=a["t0"], fs=a["fs"],
                               fd=a["fd"], ns=a["ns"], fc=a["fc"], frac_bw=a["frac_bw"],
                               rows=rows).astype(np.complex64)


def simulate_iq_parallel(cfg, medium, n_seg, workers=None):
    """Oracle-simulated channel data [N][N][Ns] (complex64) for ``medium``: the
    scatterer times in chunks of scatterers, the transmit records in parallel
    processes (fork, all host cores by default)."""
    import multiprocessing as mp
    import os
    arr, acq = cfg.array, cfg.acq
    elem = afsynth.element_positions(arr)
    centres = afsynth.pixel_centres(arr, cfg.img)
    sp = afsynth.patch_spacing(cfg.img, acq)
    grid = afsynth.sim_box(arr, np.concatenate([centres, medium.scat_xz]), sp, cfg.sim_spacing)
    x0, z0, dx, dz, nx, nz = grid
    s_true = 1.0 / afsynth.speed_on_grid(medium, x0, z0, dx, dz, nx, nz)
    # all elements together (the array's shape decides arc or line), scatterers in chunks
    T = np.concatenate([simulate.scatterer_times(elem, arr.d_lens, arr.c_lens, s_true, grid,
                                                 n_seg, medium.scat_xz[k:k + 128])
                        for k in range(0, medium.n_scat, 128)], axis=1)
    _sim.update(T=T, amp=medium.scat_amp, t_ttp=arr.t_ttp, t0=acq.t0, fs=acq.fs, fd=acq.fc,
                ns=acq.n_samples, fc=acq.fc, frac_bw=acq.frac_bw)
    workers = workers or min(16, os.cpu_count() or 1)
    n = arr.n_elem
    chunks = [list(range(t, min(t + 4, n))) for t in range(0, n, 4)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_sim_rows, chunks)
    return np.concatenate(parts)
