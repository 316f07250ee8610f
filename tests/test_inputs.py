"""The seeded input generators (afsynth) for the linear array: element line,
pixel rows below the flat lens, a slowness box that holds the lens plane, and
media layered by depth."""
import numpy as np

import afsynth


def test_linear_array_layout():
    cfg = afsynth.configs.L1
    arr = cfg.array
    assert afsynth.is_linear(arr) and not afsynth.is_linear(afsynth.configs.C2.array)
    e = afsynth.element_positions(arr)
    assert np.allclose(e[:, 1], 0.0)
    assert np.allclose(np.diff(e[:, 0]), arr.pitch) and abs(e[:, 0].mean()) < 1e-12
    c = afsynth.pixel_centres(arr, cfg.img).reshape(cfg.img.n_depth, cfg.img.n_angle, 2)
    assert np.allclose(c[:, 0, 1], arr.d_lens + np.linspace(cfg.img.depth_min, cfg.img.depth_max,
                                                           cfg.img.n_depth))
    assert np.isclose(c[0, 0, 0], e[0, 0]) and np.isclose(c[0, -1, 0], e[-1, 0])
    cs = afsynth.pixel_centres(arr, cfg.img, depth_scale=1.2).reshape(c.shape)
    assert np.allclose(cs[..., 1] - arr.d_lens, 1.2 * (c[..., 1] - arr.d_lens))


def test_linear_box_covers_lens_plane_and_points():
    cfg = afsynth.configs.L1
    arr = cfg.array
    c = afsynth.pixel_centres(arr, cfg.img)
    sp = afsynth.patch_spacing(cfg.img, cfg.acq)
    x0, z0, dx, dz = afsynth.slowness_box(arr, c, sp, 16, 16)
    x1, z1 = x0 + 15 * dx, z0 + 15 * dz
    e = afsynth.element_positions(arr)
    assert z0 <= arr.d_lens and x0 <= e[0, 0] and x1 >= e[-1, 0]
    assert c[:, 0].min() - sp >= x0 and c[:, 0].max() + sp <= x1 and c[:, 1].max() + sp <= z1


def test_linear_medium_is_layered_by_depth():
    cfg = afsynth.configs.L1
    for seed, c_ph in ((30, 1.490), (31, 1.516), (32, 1.540)):
        med = afsynth.medium_for(cfg, seed)
        top = float(med.layer_r[0])
        assert med.layer_axis == "depth" and med.layer_c[-1] == c_ph
        x = np.linspace(-10, 10, 5)
        assert np.allclose(afsynth.sample_speed(med, x, np.full(5, top - 0.1)), 1.575)
        assert np.allclose(afsynth.sample_speed(med, x, np.full(5, top + 0.1)), c_ph)
        # no scatterer inside the cyst
        r = np.hypot(med.scat_xz[:, 0] - med.cyst_xz[0, 0], med.scat_xz[:, 1] - med.cyst_xz[0, 1])
        assert r.min() > med.cyst_r[0]
