"""Pins of the oracle's lens refraction (Eq. 8) against closed forms, Snell's law
written with angles, and brute force over lens points."""
import json
import math
import os

import numpy as np

import afsynth
from oracle import fermat

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _setup(n=4, R=49.6, pitch=0.5083, d=0.90, n_pts=16, seed=0):
    elem = afsynth.element_positions(afsynth.ArrayCfg(n, R, pitch, d, 1.0))
    rng = np.random.default_rng(seed)
    rl = R + d
    rho = rl + rng.uniform(0.5, 60.0, n_pts)
    th = rng.uniform(-0.4, 0.4, n_pts)
    pts = np.stack([rho * np.sin(th), rho * np.cos(th)], axis=1)
    return elem, pts


def test_zero_thickness_is_straight_ray():
    elem, pts = _setup()
    r = fermat.refract(elem, 0.0, 0.9994, 1.54, pts)
    d = np.hypot(pts[None, :, 0] - elem[:, None, 0], pts[None, :, 1] - elem[:, None, 1])
    assert np.allclose(r["t_hom"], d / 1.54, rtol=1e-13, atol=0)


def test_equal_speeds_is_straight_ray():
    elem, pts = _setup()
    r = fermat.refract(elem, 0.9, 1.54, 1.54, pts)
    d = np.hypot(pts[None, :, 0] - elem[:, None, 0], pts[None, :, 1] - elem[:, None, 1])
    assert np.allclose(r["t_hom"], d / 1.54, rtol=1e-12, atol=0)


def test_radial_closed_form_table1_lens():
    # Table I, C5-2v (Phantoms): c_lens 999.4 m/s, d_lens 0.90 mm
    c_lens, d_lens = [GOLD["table1_lens_calibration"]["C5-2v (Phantoms)"][i] for i in (0, 1)]
    c_lens /= 1000.0
    elem, _ = _setup(n=5, d=d_lens)
    R = float(np.hypot(*elem[0]))
    th = np.arctan2(elem[:, 0], elem[:, 1])
    depth = np.array([3.0, 40.0])
    pts = np.concatenate([np.stack([(R + d_lens + dd) * np.sin(th), (R + d_lens + dd) * np.cos(th)], 1)
                          for dd in depth])
    r = fermat.refract(elem, d_lens, c_lens, 1.54, pts)
    for k, dd in enumerate(depth):
        for a in range(5):
            p = k * 5 + a
            assert abs(r["t_hom"][a, p] - (d_lens / c_lens + dd / 1.54)) < 1e-12
            assert abs(r["phi"][a, p] - th[a]) < 1e-12


def test_snell_law_at_refraction_point():
    elem, pts = _setup(n=6, n_pts=40, seed=3)
    c_lens, c_med = 0.9994, 1.52
    r = fermat.refract(elem, 0.9, c_lens, c_med, pts)
    for a in range(elem.shape[0]):
        for p in range(pts.shape[0]):
            lx, lz = r["ref_x"][a, p], r["ref_z"][a, p]
            normal = math.atan2(lx, lz)
            inc = math.atan2(lx - elem[a, 0], lz - elem[a, 1]) - normal
            out = math.atan2(pts[p, 0] - lx, pts[p, 1] - lz) - normal
            assert abs(math.sin(inc) / c_lens - math.sin(out) / c_med) < 1e-9


def test_brute_force_tiny():
    elem, pts = _setup(n=4, n_pts=16, seed=1)
    r = fermat.refract(elem, 0.9, 0.9994, 1.48, pts)
    tb, _ = fermat.brute_refract(elem, 0.9, 0.9994, 1.48, pts, n_points=400001)
    # the continuous minimiser can only be lower than a discrete search, and only by
    # the discretisation error (quadratic in the lens-point spacing)
    assert np.all(r["t_hom"] <= tb + 1e-13)
    assert np.max(tb - r["t_hom"]) < 1e-9


def test_discrete_search_equal_speeds_is_straight_ray():
    # the straight crossing is the last candidate, and the straight line is the fastest path
    elem, pts = _setup(n=5, n_pts=20, seed=4)
    for n in (2, 7, 64):
        r = fermat.discrete_refract(elem, 0.9, 1.54, 1.54, pts, n)
        d = np.hypot(pts[None, :, 0] - elem[:, None, 0], pts[None, :, 1] - elem[:, None, 1])
        assert np.allclose(r["t_hom"], d / 1.54, rtol=1e-13, atol=0)


def test_discrete_search_radial_closed_form():
    elem, _ = _setup(n=5, d=0.9)
    R = float(np.hypot(*elem[0]))
    th = np.arctan2(elem[:, 0], elem[:, 1])
    dd = 25.0
    pts = np.stack([(R + 0.9 + dd) * np.sin(th), (R + 0.9 + dd) * np.cos(th)], 1)
    r = fermat.discrete_refract(elem, 0.9, 0.9994, 1.54, pts, 16)
    for a in range(5):
        assert abs(r["t_hom"][a, a] - (0.9 / 0.9994 + dd / 1.54)) < 1e-12


def _discrete_errors(c_lens, c_med, ns):
    elem, pts = _setup(n=8, n_pts=60, seed=5)
    rc = fermat.refract(elem, 0.9, c_lens, c_med, pts)
    out = []
    for n in ns:
        rd = fermat.discrete_refract(elem, 0.9, c_lens, c_med, pts, n)
        gap = rd["t_hom"] - rc["t_hom"]
        # no lens point beats the exact stationary point (a minimum over the arc)
        assert gap.min() > -1e-13
        out.append(gap)
    return out


def test_discrete_search_converges_quadratically_to_the_root():
    # slow lens (c_lens < c_med): candidates from the element's apex to the straight
    # crossing; the error of a ray shrinks with the square of the candidate spacing
    g16, g64 = _discrete_errors(0.9994, 1.54, (16, 64))
    assert np.median(g64) < 1.3 * (15.0 / 63.0) ** 2 * np.median(g16)
    assert np.median(g64) < 1e-5 and g64.max() < 5e-3


def test_discrete_search_fast_lens_interval():
    # fast lens (c_lens > c_med): candidates from the straight crossing to the point's angle
    g16, g64 = _discrete_errors(2.2, 1.54, (16, 64))
    assert np.median(g64) < 1.3 * (15.0 / 63.0) ** 2 * np.median(g16)


def _crossing(e, p, rl):
    """Where the segment e -> p leaves the circle of radius rl (bisection on t)."""
    lo, hi = 0.0, 1.0
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if np.hypot(*(e + m * (p - e))) < rl:
            lo = m
        else:
            hi = m
    return e + 0.5 * (lo + hi) * (p - e)


def test_discrete_search_two_candidates_are_the_interval_ends():
    # slow lens: the candidates run from the lens apex above the element (lens leg
    # = d_lens, radial) to the straight crossing; with two candidates the better end wins
    elem, pts = _setup(n=6, n_pts=30, seed=6)
    d, cl, cm = 0.9, 0.9994, 1.54
    r2 = fermat.discrete_refract(elem, d, cl, cm, pts, 2)
    r64 = fermat.discrete_refract(elem, d, cl, cm, pts, 64)
    for a in range(elem.shape[0]):
        e = elem[a]
        rl = np.hypot(*e) + d
        apex = e * rl / np.hypot(*e)
        for p in range(pts.shape[0]):
            q = pts[p]
            t_apex = d / cl + np.hypot(*(q - apex)) / cm
            x = _crossing(e, q, rl)
            t_x = np.hypot(*(x - e)) / cl + np.hypot(*(q - x)) / cm
            assert abs(r2["t_hom"][a, p] - min(t_apex, t_x)) < 1e-11
            assert r64["t_hom"][a, p] <= min(t_apex, t_x) + 1e-11


# ---- linear array, flat lens (the L12-3v lens of Table I) ----

def _linear(n=6, pitch=0.3, n_pts=24, seed=7):
    elem = np.stack([(np.arange(n) - (n - 1) / 2) * pitch, np.zeros(n)], axis=1)
    rng = np.random.default_rng(seed)
    pts = np.stack([rng.uniform(-8.0, 8.0, n_pts), rng.uniform(1.5, 40.0, n_pts)], axis=1)
    return elem, pts


def _table1_l12():
    c_lens, d_lens = [GOLD["table1_lens_calibration"]["L12-3v"][i] for i in (0, 1)]
    return c_lens / 1000.0, d_lens


def test_flat_lens_equal_speeds_and_no_lens_are_straight():
    elem, pts = _linear()
    d = np.hypot(pts[None, :, 0] - elem[:, None, 0], pts[None, :, 1] - elem[:, None, 1])
    r = fermat.refract(elem, 0.67, 1.54, 1.54, pts)
    assert np.allclose(r["t_hom"], d / 1.54, rtol=1e-12, atol=0)
    r0 = fermat.refract(elem, 0.0, 1.0494, 1.54, pts)
    assert np.allclose(r0["t_hom"], d / 1.54, rtol=1e-14, atol=0)
    for n in (2, 9):
        rd = fermat.discrete_refract(elem, 0.67, 1.54, 1.54, pts, n)
        assert np.allclose(rd["t_hom"], d / 1.54, rtol=1e-13, atol=0)


def test_flat_lens_normal_incidence_closed_form():
    c_lens, d_lens = _table1_l12()
    elem, _ = _linear(n=5)
    depth = 20.0
    pts = np.stack([elem[:, 0], np.full(5, d_lens + depth)], axis=1)
    r = fermat.refract(elem, d_lens, c_lens, 1.54, pts)
    for a in range(5):
        assert abs(r["t_hom"][a, a] - (d_lens / c_lens + depth / 1.54)) < 1e-12
        assert abs(r["ref_x"][a, a] - elem[a, 0]) < 1e-12


def test_flat_lens_snell_law_with_angles():
    c_lens, d_lens = _table1_l12()
    elem, pts = _linear(n=6, n_pts=40, seed=8)
    c_med = 1.50
    r = fermat.refract(elem, d_lens, c_lens, c_med, pts)
    for a in range(elem.shape[0]):
        for p in range(pts.shape[0]):
            lx, lz = r["ref_x"][a, p], r["ref_z"][a, p]
            assert abs(lz - d_lens) < 1e-15
            inc = math.atan2(lx - elem[a, 0], lz - elem[a, 1])   # angle to the plane's normal
            out = math.atan2(pts[p, 0] - lx, pts[p, 1] - lz)
            assert abs(math.sin(inc) / c_lens - math.sin(out) / c_med) < 1e-9


def test_flat_lens_brute_force():
    c_lens, d_lens = _table1_l12()
    elem, pts = _linear(n=4, n_pts=12, seed=9)
    r = fermat.refract(elem, d_lens, c_lens, 1.48, pts)
    for a in range(4):
        for p in range(12):
            xs = np.linspace(min(elem[a, 0], pts[p, 0]), max(elem[a, 0], pts[p, 0]), 400001)
            tt = (np.hypot(xs - elem[a, 0], d_lens) / c_lens
                  + np.hypot(pts[p, 0] - xs, pts[p, 1] - d_lens) / 1.48)
            assert r["t_hom"][a, p] <= tt.min() + 1e-13
            assert tt.min() - r["t_hom"][a, p] < 1e-9


def test_flat_lens_discrete_search():
    c_lens, d_lens = _table1_l12()
    elem, pts = _linear(n=6, n_pts=30, seed=10)
    cm = 1.54
    rc = fermat.refract(elem, d_lens, c_lens, cm, pts)
    r2 = fermat.discrete_refract(elem, d_lens, c_lens, cm, pts, 2)
    g16 = fermat.discrete_refract(elem, d_lens, c_lens, cm, pts, 16)["t_hom"] - rc["t_hom"]
    g64 = fermat.discrete_refract(elem, d_lens, c_lens, cm, pts, 64)["t_hom"] - rc["t_hom"]
    assert g16.min() > -1e-13 and g64.min() > -1e-13
    assert np.median(g64) < 1.3 * (15.0 / 63.0) ** 2 * np.median(g16)
    for a in range(elem.shape[0]):
        xe = elem[a, 0]
        for p in range(pts.shape[0]):
            xp, zp = pts[p]
            # two candidates: above the element, and where the straight ray meets the plane
            t_up = d_lens / c_lens + math.hypot(xp - xe, zp - d_lens) / cm
            xc = xe + (xp - xe) * d_lens / zp
            t_x = math.hypot(xc - xe, d_lens) / c_lens + math.hypot(xp - xc, zp - d_lens) / cm
            assert abs(r2["t_hom"][a, p] - min(t_up, t_x)) < 1e-11
