"""Pins of the lens models (Eq. 6 and the straight-ray baseline) and of the glue
around the warm-start network (feature rounding, output resampling).

Eq. 6's conventional lens offset is a reading (the paper gives no formula): the
round trip through the lens along the element normal at c_lens instead of c_ref.
It is pinned by the one case where its physics is exact: a ray along the element
normal in a medium of speed c_ref, where the conventional round trip equals the
bent-ray round trip of Eqs. 7-8."""
import math

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import fermat, lens, model


def _arc(n=6, R=40.0, pitch=0.4):
    th = (np.arange(n) - (n - 1) / 2.0) * pitch / R
    return np.stack([R * np.sin(th), R * np.cos(th)], axis=1), th, R


def _prob(elem, d, c_lens, model_name, centres, grid, t_ttp=0.2):
    return model.Problem(elem_xz=elem, d_lens=d, c_lens=c_lens, t_ttp=t_ttp, centres=centres,
                         patch=1, spacing=0.25, t0=0.0, fs=20.0, fd=5.0, block=1, fnum=10.0,
                         n_seg=32, grid=grid, lens_model=model_name)


def test_conventional_round_trip_equals_bent_ray_on_the_normal():
    # Table I, C5-2v (Phantoms): c_lens 999.4 m/s, d_lens 0.90 mm
    d, c_lens, c_ref = 0.90, 0.9994, lens.C_REF
    elem, th, R = _arc()
    depths = np.array([3.0, 17.0, 55.0])
    a = 2
    centres = np.stack([(R + d + depths) * np.sin(th[a]), (R + d + depths) * np.cos(th[a])], 1)
    grid = (-20.0, 30.0, 1.0, 1.0, 41, 80)
    s = np.full((80, 41), 1.0 / c_ref)
    tb = model.travel_times(_prob(elem, d, c_lens, "bent", centres, grid), s,
                            mask=np.ones((6, 3), bool))
    pc = _prob(elem, d, c_lens, "conventional", centres, grid)
    tc = model.travel_times(pc, s, mask=np.ones((6, 3), bool))
    for p in range(3):
        rt_bent = 2.0 * tb[a, p] + 0.2
        rt_conv = 2.0 * tc[a, p] + pc.tau_offset
        # closed form of both: lens crossed at c_lens, the rest at c_ref
        closed = 2.0 * (d / c_lens + depths[p] / c_ref) + 0.2
        assert abs(rt_bent - closed) < 1e-11
        assert abs(rt_conv - closed) < 1e-11


def test_conventional_offset_special_cases():
    assert lens.conventional_offset(0.0, 0.9994) == 0.0           # no lens
    assert lens.conventional_offset(1.2, lens.C_REF) == 0.0        # lens at the reference speed
    assert lens.conventional_offset(1.0, 1.0) > 0.0                # slower lens: later echoes
    assert lens.conventional_offset(1.0, 2.0) < 0.0


def test_straight_ray_models_start_at_the_elements():
    """Without lens correction (and in the conventional model) the one-way time in a
    homogeneous medium is the straight element-to-point distance times s."""
    elem, th, R = _arc()
    rng = np.random.default_rng(1)
    centres = np.stack([rng.uniform(-6, 6, 5), rng.uniform(50, 70, 5)], 1)
    grid = (-20.0, 30.0, 1.0, 1.0, 41, 80)
    s = np.full((80, 41), 0.7)
    for name in ("none", "conventional"):
        T = model.travel_times(_prob(elem, 1.0, 1.0, name, centres, grid), s,
                               mask=np.ones((6, 5), bool))
        dist = np.hypot(centres[None, :, 0] - elem[:, None, 0], centres[None, :, 1] - elem[:, None, 1])
        assert np.max(np.abs(T - 0.7 * dist)) < 1e-12
    assert _prob(elem, 1.0, 1.0, "none", centres, grid).tau_offset == 0.2
    with pytest.raises(ValueError):
        _ = _prob(elem, 1.0, 1.0, "thin", centres, grid).tau_offset


def test_bf16_round_matches_torch_and_known_values():
    import torch
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, math.pi, -2.5, 0.0, 65504.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 3.140625, -2.5, 0.0, 65536.0])
    assert np.array_equal(ocnn.bf16_round(vals), want)
    x = np.random.default_rng(0).standard_normal(10000) * 10.0
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ocnn.bf16_round(x), ref.astype(np.float64))


def test_features_closed_forms():
    maps = np.array([[0.6, 1.1, 0.1], [0.3, 0.0, 1.3]])
    out = ocnn.features(maps, np.array([0.6, 0.3]), np.array([2.0, 3.0]))
    assert out.shape == (3, 2)
    assert np.allclose(out, [[0.0, 0.0], [1.0, -0.9], [-1.0, 3.0]], atol=1e-15)


def test_polar_to_grid_reproduces_linear_maps_and_clamps():
    r0, dr, t0, dt = 50.0, 2.0, -0.4, 0.05
    a = np.arange(12)[:, None]
    b = np.arange(17)[None, :]
    pmap = 0.3 + 0.01 * a - 0.02 * b                 # linear in the map indices
    nx, nz, x0, z0, dx, dz = 9, 11, -8.0, 52.0, 2.0, 2.0
    s = ocnn.polar_to_grid(pmap, r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, 0.65, 0.1, 0.0, 10.0)
    for i in range(nz):
        for j in range(nx):
            x, z = x0 + j * dx, z0 + i * dz
            u = (math.hypot(x, z) - r0) / dr
            v = (math.atan2(x, z) - t0) / dt
            if 0 <= u <= 11 and 0 <= v <= 16:        # inside: bilinear is exact on linear maps
                assert abs(s[i, j] - (0.65 + 0.1 * (0.3 + 0.01 * u - 0.02 * v))) < 1e-13
    # beyond the last radius the map's edge row is used
    far = ocnn.polar_to_grid(pmap, r0, dr, t0, dt, 1, 1, 0.0, 500.0, 1.0, 1.0, 0.0, 1.0, -9, 9)
    v = (0.0 - t0) / dt
    assert abs(far[0, 0] - (0.3 + 0.11 - 0.02 * v)) < 1e-13
    # the result is clamped to [s_lo, s_hi]
    c = ocnn.polar_to_grid(pmap - pmap.mean(), r0, dr, t0, dt, nx, nz, x0, z0, dx, dz, 0.65,
                           100.0, 0.6, 0.7)
    assert c.min() >= 0.6 and c.max() <= 0.7 and np.any(c == 0.6) and np.any(c == 0.7)
