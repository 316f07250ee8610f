"""Array, pixel and grid layout (inputs only).

Element ``a`` of an ``N``-element curvilinear array of radius ``R`` sits at
polar angle ``(a - (N-1)/2) * pitch / R`` about the centre of curvature, so the
pitch is the arc length at the element radius.  The paper's simulated C5-2v
array (Simulations subsection: 49.6 mm radius, 0.5872 degree angular pitch,
508 um linear pitch) is consistent with that reading.  The lens outer surface
is the concentric arc of radius ``R + d_lens``.

A linear array (``radius = inf``) has its elements on the line z = 0 at
x = (a - (N-1)/2) * pitch, and a flat lens: the layer 0 <= z <= d_lens, whose
outer surface is the plane z = d_lens.
"""
from __future__ import annotations

import math

import numpy as np

from .configs import ArrayCfg, ImgCfg, AcqCfg


def is_linear(arr: ArrayCfg) -> bool:
    return math.isinf(arr.radius)


def lens_radius(arr: ArrayCfg) -> float:
    if is_linear(arr):
        raise ValueError("a linear array has a flat lens")
    return arr.radius + arr.d_lens


def element_polar_angles(arr: ArrayCfg) -> np.ndarray:
    a = np.arange(arr.n_elem, dtype=np.float64)
    return (a - (arr.n_elem - 1) / 2.0) * (arr.pitch / arr.radius)


def element_x(arr: ArrayCfg) -> np.ndarray:
    """Lateral positions of a linear array's elements."""
    a = np.arange(arr.n_elem, dtype=np.float64)
    return (a - (arr.n_elem - 1) / 2.0) * arr.pitch


def element_positions(arr: ArrayCfg) -> np.ndarray:
    """[N][2] float64 element centres (x, z) in mm."""
    if is_linear(arr):
        return np.stack([element_x(arr), np.zeros(arr.n_elem)], axis=1)
    th = element_polar_angles(arr)
    return np.stack([arr.radius * np.sin(th), arr.radius * np.cos(th)], axis=1)


def element_span(arr: ArrayCfg) -> tuple[float, float]:
    th = element_polar_angles(arr)
    return float(th[0]), float(th[-1])


def pixel_centres(arr: ArrayCfg, img: ImgCfg, depth_scale: float = 1.0) -> np.ndarray:
    """[n_depth * n_angle][2] float64 pixel (patch) centres, row-major [depth][angle].

    Depth is measured below the lens surface; ``depth_scale`` stretches every
    depth by the same factor (the caller decides what the factor means).
    """
    depth = np.linspace(img.depth_min, img.depth_max, img.n_depth) * depth_scale
    if is_linear(arr):
        xe = element_x(arr)
        x = np.linspace(xe[0], xe[-1], img.n_angle)
        X, Z = np.meshgrid(x, arr.d_lens + depth)
        return np.stack([X.ravel(), Z.ravel()], axis=1)
    th0, th1 = element_span(arr)
    ang = np.linspace(th0, th1, img.n_angle)
    rho = lens_radius(arr) + depth[:, None]
    x = rho * np.sin(ang)[None, :]
    z = rho * np.cos(ang)[None, :]
    return np.stack([x.ravel(), z.ravel()], axis=1)


def patch_spacing(img: ImgCfg, acq: AcqCfg, c: float | None = None) -> float:
    """Half a wavelength at speed ``c`` (default the reference speed)."""
    c = img.c_ref if c is None else c
    return c / (2.0 * acq.fc)


def _cover(arr: ArrayCfg, centres: np.ndarray, spacing: float, margin: float):
    """Axis-aligned box holding the lens arc over the imaged angles and every point
    (for a linear array: the lens plane over the element span and every point)."""
    pts_x = centres[:, 0]
    pts_z = centres[:, 1]
    if is_linear(arr):
        xe = element_x(arr)
        x_lo = min(float(pts_x.min()) - spacing, float(xe[0]))
        x_hi = max(float(pts_x.max()) + spacing, float(xe[-1]))
        z_lo = min(arr.d_lens, float(pts_z.min()) - spacing)
        z_hi = float(pts_z.max()) + spacing
        return x_lo - margin, x_hi + margin, z_lo - margin, z_hi + margin
    th0, th1 = element_span(arr)
    ang_pts = np.arctan2(pts_x, pts_z)
    th_abs = max(abs(th0), abs(th1), float(np.max(np.abs(ang_pts))))
    th_abs = min(th_abs + 1e-3, math.pi / 2 - 1e-6)
    rl = lens_radius(arr)
    x_lo = min(float(pts_x.min()) - spacing, -rl * math.sin(th_abs))
    x_hi = max(float(pts_x.max()) + spacing, rl * math.sin(th_abs))
    z_lo = min(rl * math.cos(th_abs), float(pts_z.min()) - spacing)
    z_hi = float(pts_z.max()) + spacing
    return x_lo - margin, x_hi + margin, z_lo - margin, z_hi + margin


def slowness_box(arr: ArrayCfg, centres: np.ndarray, spacing: float, nx: int, nz: int,
                 margin: float = 0.25) -> tuple[float, float, float, float]:
    """(x0, z0, dx, dz) of an nx-by-nz node grid covering the lens arc and all points."""
    x_lo, x_hi, z_lo, z_hi = _cover(arr, centres, spacing, margin)
    return x_lo, z_lo, (x_hi - x_lo) / (nx - 1), (z_hi - z_lo) / (nz - 1)


def sim_box(arr: ArrayCfg, centres: np.ndarray, spacing: float, node_spacing: float,
            margin: float = 1.0) -> tuple[float, float, float, float, int, int]:
    """Node grid at roughly ``node_spacing`` covering the same region (for the simulator)."""
    x_lo, x_hi, z_lo, z_hi = _cover(arr, centres, spacing, margin)
    nx = int(math.ceil((x_hi - x_lo) / node_spacing)) + 1
    nz = int(math.ceil((z_hi - z_lo) / node_spacing)) + 1
    return x_lo, z_lo, (x_hi - x_lo) / (nx - 1), (z_hi - z_lo) / (nz - 1), nx, nz
