"""Straight-ray path integral of slowness through the gridded map.

Paper: Eq. 1 (t_d as the line integral of 1/c), Eq. 8 (medium legs of the bent
ray) and the Model Implementation subsection: after leaving the lens each ray
is cut into N segments with N+1 end points, slowness is interpolated bicubically
at the end points and the travel time is a discrete sum.

Readings (the paper does not fix them):
* the cubic kernel is Keys' cubic convolution with a = -0.5, node indices
  clamped to the grid;
* the discrete sum is the trapezoid rule: L2 * [s_0/2 + s_1 + ... + s_{N-1} + s_N/2] / N.

Grid: node (i, j) of the [nz][nx] array sits at (x0 + j dx, z0 + i dz).
"""
from __future__ import annotations

import numpy as np

KEYS_A = -0.5


def keys_kernel(x: np.ndarray, a: float = KEYS_A) -> np.ndarray:
    """Keys (1981) cubic convolution kernel W(x)."""
    x = np.abs(np.asarray(x, dtype=np.float64))
    out = np.zeros_like(x)
    m1 = x <= 1.0
    m2 = (x > 1.0) & (x < 2.0)
    out[m1] = (a + 2.0) * x[m1] ** 3 - (a + 3.0) * x[m1] ** 2 + 1.0
    out[m2] = a * x[m2] ** 3 - 5.0 * a * x[m2] ** 2 + 8.0 * a * x[m2] - 4.0 * a
    return out


def bicubic_taps(grid, x: np.ndarray, z: np.ndarray):
    """Node indices and weights of the 4x4 taps around every point.

    ``grid`` = (x0, z0, dx, dz, nx, nz).  Returns (iz, ix, w) with iz, ix of
    shape (..., 4, 4) (clamped node indices) and w the tap weights
    W(u - j) W(v - i) evaluated at the unclamped tap positions.
    """
    x0, z0, dx, dz, nx, nz = grid
    u = (np.asarray(x, dtype=np.float64) - x0) / dx
    v = (np.asarray(z, dtype=np.float64) - z0) / dz
    j0 = np.floor(u)
    i0 = np.floor(v)
    offs = np.arange(-1, 3)
    jt = j0[..., None] + offs                      # (..., 4)
    it = i0[..., None] + offs
    wx = keys_kernel(u[..., None] - jt)
    wz = keys_kernel(v[..., None] - it)
    jc = np.clip(jt, 0, nx - 1).astype(np.int64)
    ic = np.clip(it, 0, nz - 1).astype(np.int64)
    iz = np.broadcast_to(ic[..., :, None], ic.shape + (4,))
    ix = np.broadcast_to(jc[..., None, :], jc.shape[:-1] + (4, 4))
    w = wz[..., :, None] * wx[..., None, :]
    return iz, ix, w


def bicubic(s: np.ndarray, grid, x, z) -> np.ndarray:
    """Bicubic interpolation of the node values ``s`` [nz][nx] at points (x, z)."""
    iz, ix, w = bicubic_taps(grid, x, z)
    return np.sum(w * s[iz, ix], axis=(-2, -1))


def trapezoid_weights(n_seg: int) -> np.ndarray:
    w = np.full(n_seg + 1, 1.0 / n_seg)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


def ray_points(ref_x, ref_z, px, pz, n_seg: int):
    """End points r_k = r_ref + (k/N)(p - r_ref), k = 0..N, for every ray (last axis k)."""
    k = np.arange(n_seg + 1) / n_seg
    rx = ref_x[..., None] + k * (px - ref_x)[..., None]
    rz = ref_z[..., None] + k * (pz - ref_z)[..., None]
    return rx, rz


def medium_time(s: np.ndarray, grid, ref_x, ref_z, px, pz, l2, n_seg: int) -> np.ndarray:
    """L2 * trapezoid sum of interpolated slowness along the medium leg."""
    rx, rz = ray_points(ref_x, ref_z, px, pz, n_seg)
    sk = bicubic(s, grid, rx, rz)
    return l2 * np.sum(sk * trapezoid_weights(n_seg), axis=-1)


def medium_time_adjoint(gbar: np.ndarray, grid, ref_x, ref_z, px, pz, l2, n_seg: int,
                        chunk: int = 20000) -> np.ndarray:
    """Gradient of sum(gbar * medium_time) with respect to the node values.

    The refraction point, L2 and the ray geometry are held fixed (they depend
    on the slowness only through the global mean speed, whose gradient is
    stopped).  Returns a [nz][nx] array.
    """
    x0, z0, dx, dz, nx, nz = grid
    out = np.zeros(nz * nx)
    tw = trapezoid_weights(n_seg)
    gbar, ref_x, ref_z, px, pz, l2 = (np.ravel(v) for v in (gbar, ref_x, ref_z, px, pz, l2))
    for s0 in range(0, gbar.shape[0], chunk):
        sl = slice(s0, s0 + chunk)
        rx, rz = ray_points(ref_x[sl], ref_z[sl], px[sl], pz[sl], n_seg)
        iz, ix, w = bicubic_taps(grid, rx, rz)
        coef = (gbar[sl] * l2[sl])[:, None, None, None] * tw[None, :, None, None] * w
        out += np.bincount((iz * nx + ix).ravel(), weights=coef.ravel(), minlength=nz * nx)
    return out.reshape(nz, nx)
