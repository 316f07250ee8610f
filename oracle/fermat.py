"""Two-layer refraction through the lens by Fermat's principle.

Paper: Section II-B (Bent-Ray Model for Lens Compensation), Eqs. 7-8, and the
Model Implementation subsection (refraction points from the global mean speed).

Geometry: the centre of curvature is the origin; element a sits at radius R_a
and polar angle theta_a; the lens outer surface is the concentric arc of radius
R_L = R_a + d_lens.  For a point p at radius rho and polar angle theta_p the
travel time through the lens and a homogeneous medium of speed c_med via the
lens point L(phi) = R_L (sin phi, cos phi) is

    T(phi) = |L(phi) - e_a| / c_lens + |p - L(phi)| / c_med .

Reading: the paper searches a finite set of N_search candidate points; the
oracle's ``refract`` returns the continuous minimiser (the discrete search
converges to it).  It scans phi over [min(theta_a, theta_p), max(theta_a,
theta_p)] -- outside that interval both legs get longer -- and then bisects the
sign of dT/dphi inside the bracket around the best scanned point.

``discrete_refract`` is the paper's search itself.  The paper gives neither
N_search nor where the candidates lie; the reading here: N_search lens points
evenly spaced in polar angle over the interval that holds the minimiser -- from
the element's own polar angle theta_a to the polar angle theta_x where the
straight element-to-point segment crosses the lens arc when c_lens <= c_med
(Snell bends the lens leg towards the normal), else from theta_x to theta_p --
and the candidate of least T, the first one on ties.

A linear array (every element on one line z = z_e) has a flat lens: the layer
z_e <= z <= z_e + d_lens, refracting at the plane z_L = z_e + d_lens.  The lens
point is L(x) = (x, z_L) and

    T(x) = |L(x) - e_a| / c_lens + |p - L(x)| / c_med ;

``refract`` scans x over [min(x_a, x_p), max(x_a, x_p)] and bisects dT/dx;
``discrete_refract`` spaces its candidates in x over the same kind of interval
as on the arc (element to straight crossing for a slower lens, crossing to the
point otherwise).  d_lens = 0 means no lens: the straight ray from the element.
"""
from __future__ import annotations

import numpy as np


def _legs(phi, ex, ez, px, pz, rl):
    lx = rl * np.sin(phi)
    lz = rl * np.cos(phi)
    l1 = np.hypot(lx - ex, lz - ez)
    l2 = np.hypot(px - lx, pz - lz)
    return lx, lz, l1, l2


def travel_time_via(phi, ex, ez, px, pz, rl, c_lens, c_med):
    """T(phi) for every ray (arrays broadcast)."""
    _, _, l1, l2 = _legs(phi, ex, ez, px, pz, rl)
    return l1 / c_lens + l2 / c_med


def _dT(phi, ex, ez, px, pz, rl, c_lens, c_med):
    """dT/dphi: the tangential components of both legs at L(phi)."""
    lx, lz, l1, l2 = _legs(phi, ex, ez, px, pz, rl)
    tx = rl * np.cos(phi)
    tz = -rl * np.sin(phi)
    d1 = ((lx - ex) * tx + (lz - ez) * tz) / np.where(l1 > 0, l1, 1.0)
    d2 = ((lx - px) * tx + (lz - pz) * tz) / np.where(l2 > 0, l2, 1.0)
    return d1 / c_lens + d2 / c_med


def refract(elem_xz: np.ndarray, d_lens: float, c_lens: float, c_med: float,
            pts: np.ndarray, n_scan: int = 129, n_bisect: int = 64,
            pairs: tuple[np.ndarray, np.ndarray] | None = None):
    """Refraction point and legs for every (element, point) ray.

    ``pts`` is [P][2].  Without ``pairs`` every element-point combination is
    solved and the outputs are [N][P]; with ``pairs = (a_idx, p_idx)`` only
    those rays are solved and the outputs are 1-D.

    Returns dict(phi, l1, l2, t_hom, ref_x, ref_z): refraction angle on the
    lens arc, lens leg, medium leg, homogeneous travel time l1/c_lens + l2/c_med
    and the refraction point.
    """
    if is_linear(elem_xz):
        return _refract_flat(elem_xz, d_lens, c_lens, c_med, pts, pairs, n_scan, n_bisect)
    ex_all = np.asarray(elem_xz[:, 0], dtype=np.float64)
    ez_all = np.asarray(elem_xz[:, 1], dtype=np.float64)
    if pairs is None:
        ex = ex_all[:, None] * np.ones((1, pts.shape[0]))
        ez = ez_all[:, None] * np.ones((1, pts.shape[0]))
        px = np.ones((elem_xz.shape[0], 1)) * pts[None, :, 0]
        pz = np.ones((elem_xz.shape[0], 1)) * pts[None, :, 1]
    else:
        ai, pi = pairs
        ex, ez = ex_all[ai], ez_all[ai]
        px, pz = pts[pi, 0], pts[pi, 1]
    shape = ex.shape
    ex, ez, px, pz = (v.ravel().astype(np.float64) for v in (ex, ez, px, pz))
    ra = np.hypot(ex, ez)
    rl = ra + d_lens
    th_a = np.arctan2(ex, ez)
    th_p = np.arctan2(px, pz)
    lo = np.minimum(th_a, th_p)
    hi = np.maximum(th_a, th_p)

    # scan
    k = np.arange(n_scan) / (n_scan - 1)
    phis = lo[:, None] + (hi - lo)[:, None] * k[None, :]
    tt = travel_time_via(phis, ex[:, None], ez[:, None], px[:, None], pz[:, None],
                         rl[:, None], c_lens, c_med)
    best = np.argmin(tt, axis=1)
    b_lo = phis[np.arange(phis.shape[0]), np.maximum(best - 1, 0)]
    b_hi = phis[np.arange(phis.shape[0]), np.minimum(best + 1, n_scan - 1)]

    # bisect the sign of dT/dphi (a minimum has dT < 0 to its left, > 0 to its right)
    a_ = b_lo.copy()
    b_ = b_hi.copy()
    d_a = _dT(a_, ex, ez, px, pz, rl, c_lens, c_med)
    d_b = _dT(b_, ex, ez, px, pz, rl, c_lens, c_med)
    interior = (d_a < 0) & (d_b > 0)
    for _ in range(n_bisect):
        m = 0.5 * (a_ + b_)
        dm = _dT(m, ex, ez, px, pz, rl, c_lens, c_med)
        go_right = dm < 0
        a_ = np.where(interior & go_right, m, a_)
        b_ = np.where(interior & ~go_right, m, b_)
    phi = np.where(interior, 0.5 * (a_ + b_), phis[np.arange(phis.shape[0]), best])
    # end-point minima (degenerate or monotone brackets) keep the best scanned end
    lx, lz, l1, l2 = _legs(phi, ex, ez, px, pz, rl)
    out = dict(phi=phi, l1=l1, l2=l2, t_hom=l1 / c_lens + l2 / c_med, ref_x=lx, ref_z=lz)
    return {k_: v.reshape(shape) for k_, v in out.items()}


def brute_refract(elem_xz, d_lens, c_lens, c_med, pts, n_points=200001):
    """Minimum of T over ``n_points`` evenly spaced lens points spanning the whole
    element-to-point angular interval (pin for small cases only)."""
    res = np.empty((elem_xz.shape[0], pts.shape[0]))
    arg = np.empty_like(res)
    for a in range(elem_xz.shape[0]):
        ex, ez = elem_xz[a]
        ra = np.hypot(ex, ez)
        rl = ra + d_lens
        th_a = np.arctan2(ex, ez)
        for p in range(pts.shape[0]):
            px, pz = pts[p]
            th_p = np.arctan2(px, pz)
            phis = np.linspace(min(th_a, th_p), max(th_a, th_p), n_points)
            tt = travel_time_via(phis, ex, ez, px, pz, rl, c_lens, c_med)
            i = int(np.argmin(tt))
            res[a, p] = tt[i]
            arg[a, p] = phis[i]
    return res, arg


def _ray_arrays(elem_xz, pts, pairs):
    """Flattened element and point coordinates of every ray, and the output shape."""
    ex_all = np.asarray(elem_xz[:, 0], dtype=np.float64)
    ez_all = np.asarray(elem_xz[:, 1], dtype=np.float64)
    if pairs is None:
        n, p = elem_xz.shape[0], pts.shape[0]
        ex, ez = np.repeat(ex_all, p), np.repeat(ez_all, p)
        px, pz = np.tile(pts[:, 0], n), np.tile(pts[:, 1], n)
        shape = (n, p)
    else:
        ai, pi = pairs
        ex, ez, px, pz = ex_all[ai], ez_all[ai], pts[pi, 0], pts[pi, 1]
        shape = np.shape(ai)
    return [np.asarray(v, dtype=np.float64).ravel() for v in (ex, ez, px, pz)], shape


def discrete_refract(elem_xz: np.ndarray, d_lens: float, c_lens: float, c_med: float,
                     pts: np.ndarray, n_search: int,
                     pairs: tuple[np.ndarray, np.ndarray] | None = None):
    """The N_search refraction search (Model Implementation subsection): the best
    of ``n_search`` >= 2 candidate lens points per ray, candidates as read in the
    module docstring.  Same arguments (plus ``n_search``) and outputs as
    ``refract``."""
    assert n_search >= 2
    if is_linear(elem_xz):
        return _discrete_refract_flat(elem_xz, d_lens, c_lens, c_med, pts, n_search, pairs)
    (ex, ez, px, pz), shape = _ray_arrays(elem_xz, pts, pairs)
    rl = np.hypot(ex, ez) + d_lens
    th_a = np.arctan2(ex, ez)
    th_p = np.arctan2(px, pz)
    # where the straight segment e + t (p - e), t in [0, 1], meets |x| = rl
    dx, dz = px - ex, pz - ez
    qa = dx * dx + dz * dz
    qb = 2.0 * (ex * dx + ez * dz)
    qc = ex * ex + ez * ez - rl * rl
    t = np.where(qa > 0, (-qb + np.sqrt(np.maximum(qb * qb - 4.0 * qa * qc, 0.0)))
                 / (2.0 * np.where(qa > 0, qa, 1.0)), 0.0)
    t = np.clip(t, 0.0, 1.0)
    th_x = np.arctan2(ex + t * dx, ez + t * dz)
    if c_lens <= c_med:
        lo, hi = th_a, th_x
    else:
        lo, hi = th_x, th_p
    k = np.arange(n_search) / (n_search - 1)
    phis = lo[:, None] + (hi - lo)[:, None] * k[None, :]
    tt = travel_time_via(phis, ex[:, None], ez[:, None], px[:, None], pz[:, None], rl[:, None],
                         c_lens, c_med)
    best = np.argmin(tt, axis=1)          # first minimum on ties
    phi = phis[np.arange(phis.shape[0]), best]
    lx, lz, l1, l2 = _legs(phi, ex, ez, px, pz, rl)
    out = dict(phi=phi, l1=l1, l2=l2, t_hom=l1 / c_lens + l2 / c_med, ref_x=lx, ref_z=lz)
    return {k_: v.reshape(shape) for k_, v in out.items()}


def is_linear(elem_xz: np.ndarray) -> bool:
    """Every element on one line z = const (within 1e-9 of the array's size)."""
    z = np.asarray(elem_xz[:, 1], dtype=np.float64)
    return bool(np.max(np.abs(z - z[0])) <= 1e-9 * (1.0 + np.max(np.abs(elem_xz[:, 0]))))


def _flat_out(x, ex, ez, px, pz, d_lens, c_lens, c_med, shape):
    zl = ez + d_lens
    l1 = np.hypot(x - ex, zl - ez)
    l2 = np.hypot(px - x, pz - zl)
    out = dict(phi=x, l1=l1, l2=l2, t_hom=l1 / c_lens + l2 / c_med, ref_x=x, ref_z=zl)
    return {k_: v.reshape(shape) for k_, v in out.items()}


def _straight(ex, ez, px, pz, c_med, shape):
    l2 = np.hypot(px - ex, pz - ez)
    out = dict(phi=ex.copy(), l1=np.zeros_like(l2), l2=l2, t_hom=l2 / c_med, ref_x=ex.copy(),
               ref_z=ez.copy())
    return {k_: v.reshape(shape) for k_, v in out.items()}


def _refract_flat(elem_xz, d_lens, c_lens, c_med, pts, pairs, n_scan, n_bisect):
    (ex, ez, px, pz), shape = _ray_arrays(elem_xz, pts, pairs)
    if d_lens == 0.0:
        return _straight(ex, ez, px, pz, c_med, shape)
    zl = ez + d_lens

    def T(x):
        return np.hypot(x - ex_, d_lens) / c_lens + np.hypot(px_ - x, pz_ - zl_) / c_med

    def dT(x):
        l1 = np.hypot(x - ex, d_lens)
        l2 = np.hypot(px - x, pz - zl)
        return (x - ex) / l1 / c_lens - (px - x) / np.where(l2 > 0, l2, 1.0) / c_med

    lo = np.minimum(ex, px)
    hi = np.maximum(ex, px)
    k = np.arange(n_scan) / (n_scan - 1)
    xs = lo[:, None] + (hi - lo)[:, None] * k[None, :]
    ex_, px_, pz_, zl_ = ex[:, None], px[:, None], pz[:, None], zl[:, None]
    best = np.argmin(T(xs), axis=1)
    rows = np.arange(xs.shape[0])
    a_ = xs[rows, np.maximum(best - 1, 0)]
    b_ = xs[rows, np.minimum(best + 1, n_scan - 1)]
    interior = (dT(a_) < 0) & (dT(b_) > 0)
    for _ in range(n_bisect):
        m = 0.5 * (a_ + b_)
        right = dT(m) < 0
        a_ = np.where(interior & right, m, a_)
        b_ = np.where(interior & ~right, m, b_)
    x = np.where(interior, 0.5 * (a_ + b_), xs[rows, best])
    return _flat_out(x, ex, ez, px, pz, d_lens, c_lens, c_med, shape)


def _discrete_refract_flat(elem_xz, d_lens, c_lens, c_med, pts, n_search, pairs):
    (ex, ez, px, pz), shape = _ray_arrays(elem_xz, pts, pairs)
    if d_lens == 0.0:
        return _straight(ex, ez, px, pz, c_med, shape)
    zl = ez + d_lens
    # straight crossing of the segment e -> p with the plane z = zl
    frac = np.where(pz - ez > 0, d_lens / np.where(pz - ez > 0, pz - ez, 1.0), 0.0)
    xc = ex + (px - ex) * frac
    lo, hi = (ex, xc) if c_lens <= c_med else (xc, px)
    k = np.arange(n_search) / (n_search - 1)
    xs = lo[:, None] + (hi - lo)[:, None] * k[None, :]
    tt = (np.hypot(xs - ex[:, None], d_lens) / c_lens
          + np.hypot(px[:, None] - xs, pz[:, None] - zl[:, None]) / c_med)
    best = np.argmin(tt, axis=1)
    x = xs[np.arange(xs.shape[0]), best]
    return _flat_out(x, ex, ez, px, pz, d_lens, c_lens, c_med, shape)
