"""Pins of the oracle's geometry (Eqs. 2-4) against closed forms and paper constants."""
import json
import math
import os

import numpy as np
import pytest

import afsynth
from oracle import geometry

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _arc(n=16, R=40.0, pitch=0.4):
    return afsynth.element_positions(afsynth.ArrayCfg(n, R, pitch, 1.0, 1.0))


def test_pitch_is_arc_length_paper_arithmetic():
    # Section III-B: 49.6 mm radius x 0.5872 deg angular pitch is stated as 508 um linear pitch.
    g = GOLD["simulated_c5_2v"]
    arc = g["radius_mm"] * math.radians(g["angular_pitch_deg"])
    assert abs(arc * 1000.0 - g["linear_pitch_um"]) < 1.0
    # and the input generator spaces elements by pitch/R in angle
    elem = _arc(8, g["radius_mm"], arc)
    ang = np.arctan2(elem[:, 0], elem[:, 1])
    assert np.allclose(np.diff(ang), math.radians(g["angular_pitch_deg"]), rtol=0, atol=1e-12)


def test_orientation_interior_equals_arc_normal():
    elem = _arc()
    th = geometry.element_orientation(elem)
    polar = np.arctan2(elem[:, 0], elem[:, 1])
    assert np.max(np.abs(th[1:-1] - polar[1:-1])) < 1e-13


def test_orientation_end_elements_one_sided():
    # reading: end elements use the chord to their only neighbour -> mid-angle of the two
    elem = _arc()
    th = geometry.element_orientation(elem)
    polar = np.arctan2(elem[:, 0], elem[:, 1])
    assert abs(th[0] - 0.5 * (polar[0] + polar[1])) < 1e-13
    assert abs(th[-1] - 0.5 * (polar[-1] + polar[-2])) < 1e-13


def test_frame_normal_tangent_and_isometry():
    elem = _arc()
    th = geometry.element_orientation(elem)
    a = 5
    n = np.array([math.sin(th[a]), math.cos(th[a])])
    t = np.array([math.cos(th[a]), -math.sin(th[a])])
    pts = np.stack([elem[a] + 7.0 * n, elem[a] + 3.0 * t, elem[a] - 2.0 * t + 4.0 * n])
    xp, zp = geometry.element_frame(elem, th, pts)
    assert np.allclose([xp[a, 0], zp[a, 0]], [0.0, 7.0], atol=1e-12)
    assert np.allclose([xp[a, 1], zp[a, 1]], [3.0, 0.0], atol=1e-12)
    assert np.allclose([xp[a, 2], zp[a, 2]], [-2.0, 4.0], atol=1e-12)
    rng = np.random.default_rng(0)
    q = rng.uniform(-20, 20, (50, 2)) + np.array([0, 60.0])
    xp, zp = geometry.element_frame(elem, th, q)
    d = np.hypot(q[None, :, 0] - elem[:, None, 0], q[None, :, 1] - elem[:, None, 1])
    assert np.allclose(np.hypot(xp, zp), d, rtol=1e-13)


def test_apodization_literal_and_contiguous():
    elem = _arc(32)
    th = geometry.element_orientation(elem)
    a = 10
    n = np.array([math.sin(th[a]), math.cos(th[a])])
    t = np.array([math.cos(th[a]), -math.sin(th[a])])
    F = 0.5
    z = 20.0
    inside = elem[a] + z * n + (F / 2 * z * 0.999) * t
    outside = elem[a] + z * n + (F / 2 * z * 1.001) * t
    xp, zp = geometry.element_frame(elem, th, np.stack([inside, outside]))
    h = geometry.apodization(xp, zp, F)
    assert h[a, 0] and not h[a, 1]
    # behind the element: never active
    xp, zp = geometry.element_frame(elem, th, (elem[a] - 1.0 * n)[None])
    assert not geometry.apodization(xp, zp, F)[a, 0]
    # on a convex arc the active elements of any point form one contiguous run
    cfg = afsynth.configs.C1
    pts = afsynth.pixel_centres(cfg.array, cfg.img)
    elem = afsynth.element_positions(cfg.array)
    th = geometry.element_orientation(elem)
    xp, zp = geometry.element_frame(elem, th, pts)
    h = geometry.apodization(xp, zp, cfg.method.fnum)
    for p in range(0, pts.shape[0], 37):
        idx = np.nonzero(h[:, p])[0]
        if idx.size:
            assert idx[-1] - idx[0] + 1 == idx.size


def test_patch_points():
    c = np.array([[1.0, 50.0], [-2.0, 60.0]])
    pts = geometry.patch_points(c, 3, 0.25)
    assert pts.shape == (2, 9, 2)
    assert np.allclose(pts[:, 4], c)
    assert np.allclose(pts[0, 0], [0.75, 49.75])
    assert np.allclose(pts[0, 8], [1.25, 50.25])
