"""Element orientation, element frame and constant-f-number apodisation.

Paper: Section II-A (Straight-Ray Model), Eqs. 2-4.
"""
from __future__ import annotations

import numpy as np


def element_orientation(elem_xz: np.ndarray) -> np.ndarray:
    """Eq. 3: theta_a = -atan((z_{a+1} - z_{a-1}) / (x_{a+1} - x_{a-1})).

    Reading: the paper does not say what the two end elements use; they take
    the one-sided difference with their only neighbour.
    """
    x = np.asarray(elem_xz[:, 0], dtype=np.float64)
    z = np.asarray(elem_xz[:, 1], dtype=np.float64)
    n = x.shape[0]
    theta = np.empty(n)
    for a in range(n):
        lo = max(a - 1, 0)
        hi = min(a + 1, n - 1)
        theta[a] = -np.arctan((z[hi] - z[lo]) / (x[hi] - x[lo]))
    return theta


def element_frame(elem_xz: np.ndarray, theta: np.ndarray, pts: np.ndarray):
    """Eq. 2: coordinates (x', z') of every point in every element's frame.

    Returns two [N][P] arrays: x' = cos(th)(x - x_a) - sin(th)(z - z_a),
    z' = sin(th)(x - x_a) + cos(th)(z - z_a).
    """
    dx = pts[None, :, 0] - elem_xz[:, None, 0]
    dz = pts[None, :, 1] - elem_xz[:, None, 1]
    c = np.cos(theta)[:, None]
    s = np.sin(theta)[:, None]
    return c * dx - s * dz, s * dx + c * dz


def apodization(xp: np.ndarray, zp: np.ndarray, fnum: float) -> np.ndarray:
    """Eq. 4, binary: h_a(p) = [ |x'| <= (F/2) z' ].

    Reading: the printed form is used literally (F/2 multiplies z'), not the
    textbook z'/(2F).
    """
    return np.abs(xp) <= (fnum / 2.0) * zp


def patch_points(centres: np.ndarray, patch: int, spacing: float) -> np.ndarray:
    """[n_pix][patch*patch][2] evaluation points: a patch x patch kernel of points
    at ``spacing`` (lambda/2) around each centre (Model Implementation subsection).

    Point m of a patch has lateral offset (m % patch - patch//2) and axial offset
    (m // patch - patch//2), both in units of ``spacing`` along x and z.
    """
    h = patch // 2
    offs = np.array([[(m % patch - h) * spacing, (m // patch - h) * spacing]
                     for m in range(patch * patch)])
    return centres[:, None, :] + offs[None, :, :]
