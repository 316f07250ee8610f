"""Deadzone first- and second-order regularisers on the sound-speed grid.

Paper: Objective Function subsection, Eqs. 10-12: D_k(x) = max(0, |x| - k),
R_TV = (1/N) sum [D_kx1(d_x c) + D_kz1(d_z c)],
R_SV = (1/N) sum [D_kx2(d_xx c) + D_kz2(d_zz c)],
finite differences in physical units, c = 1/s on the slowness grid.

Readings: first differences are forward differences over every valid stencil,
second differences are central over interior nodes, N = nx * nz, and the
derivative of D at |x| = k is taken as 0.
"""
from __future__ import annotations

import numpy as np


def deadzone(x: np.ndarray, k: float) -> np.ndarray:
    return np.maximum(0.0, np.abs(x) - k)


def deadzone_grad(x: np.ndarray, k: float) -> np.ndarray:
    return np.where(np.abs(x) > k, np.sign(x), 0.0)


def differences(c: np.ndarray, dx: float, dz: float):
    cx = (c[:, 1:] - c[:, :-1]) / dx
    cz = (c[1:, :] - c[:-1, :]) / dz
    cxx = (c[:, 2:] - 2.0 * c[:, 1:-1] + c[:, :-2]) / (dx * dx)
    czz = (c[2:, :] - 2.0 * c[1:-1, :] + c[:-2, :]) / (dz * dz)
    return cx, cz, cxx, czz


def reg_terms(s: np.ndarray, dx: float, dz: float, kx1, kz1, kx2, kz2):
    """(R_TV, R_SV) for slowness grid ``s`` [nz][nx]."""
    c = 1.0 / s
    n = c.size
    cx, cz, cxx, czz = differences(c, dx, dz)
    tv = (np.sum(deadzone(cx, kx1)) + np.sum(deadzone(cz, kz1))) / n
    sv = (np.sum(deadzone(cxx, kx2)) + np.sum(deadzone(czz, kz2))) / n
    return float(tv), float(sv)


def reg_grad(s: np.ndarray, dx: float, dz: float, kx1, kz1, kx2, kz2, w1: float, w2: float):
    """d(w1 R_TV + w2 R_SV)/ds, chained through dc/ds = -1/s^2."""
    c = 1.0 / s
    n = c.size
    cx, cz, cxx, czz = differences(c, dx, dz)
    gc = np.zeros_like(c)
    a = w1 * deadzone_grad(cx, kx1) / (n * dx)
    gc[:, 1:] += a
    gc[:, :-1] -= a
    a = w1 * deadzone_grad(cz, kz1) / (n * dz)
    gc[1:, :] += a
    gc[:-1, :] -= a
    a = w2 * deadzone_grad(cxx, kx2) / (n * dx * dx)
    gc[:, 2:] += a
    gc[:, 1:-1] -= 2.0 * a
    gc[:, :-2] += a
    a = w2 * deadzone_grad(czz, kz2) / (n * dz * dz)
    gc[2:, :] += a
    gc[1:-1, :] -= 2.0 * a
    gc[:-2, :] += a
    return gc * (-1.0 / (s * s))
