"""Host-side evaluation metrics (reporting, outside the differentiable path)."""
import numpy as np

from paper_2608_06853_amd import metrics


def test_speed_errors():
    c_true = np.full((4, 5), 1.5)
    e = metrics.speed_errors(1.0 / np.full((4, 5), 1.51), c_true)
    assert abs(e["mae_mps"] - 10.0) < 1e-9 and abs(e["rmse_mps"] - 10.0) < 1e-9


def test_lateral_sobel_of_a_ramp():
    img = np.tile(np.arange(6.0), (5, 1))          # value = column index
    g = metrics.lateral_sobel(img)
    assert np.allclose(g[:, 1:-1], 8.0)            # (1 + 2 + 1) * (x+1 - (x-1))
    assert np.allclose(metrics.lateral_sobel(np.ones((4, 4))), 0.0)


def test_tenengrad_change():
    rng = np.random.default_rng(0)
    env = rng.rayleigh(1.0, (40, 30))
    depth = np.linspace(1.0, 60.0, 40)
    assert abs(metrics.tenengrad_change(env, env, depth)) < 1e-12
    # the same speckle with a brighter, sharper lateral edge scores higher
    sharp = env.copy()
    sharp[:, ::2] *= 3.0
    assert metrics.tenengrad_change(env, sharp, depth) > 0.0
    # rows above 10 mm are ignored
    top = env.copy()
    top[depth < 10.0] = rng.rayleigh(5.0, top[depth < 10.0].shape)
    assert abs(metrics.tenengrad_change(env, top, depth)) < 50.0


def test_contrast_cnr_of_an_empty_disc():
    rng = np.random.default_rng(1)
    xz = rng.uniform(-10, 10, (20000, 2))
    env = rng.rayleigh(1.0, 20000)
    r = np.hypot(xz[:, 0], xz[:, 1])
    env[r < 3.0] *= 0.01
    q = metrics.contrast_cnr(env, xz, (0.0, 0.0), 3.0)
    assert q["contrast_db"] < -30.0 and q["cnr"] > 0.5


def test_gcnr_limits():
    rng = np.random.default_rng(2)
    a = rng.rayleigh(1.0, 50000)
    assert metrics.gcnr(a, a) == 0.0
    assert metrics.gcnr(a, a + 100.0) == 1.0                  # disjoint supports
    b = rng.rayleigh(1.0, 50000)
    assert metrics.gcnr(a, b) < 0.05                           # same distribution
    # two unit-variance Gaussians d apart overlap by 2 Phi(-d/2): gCNR = 1 - that
    from math import erf, sqrt
    x = rng.standard_normal(400000)
    y = rng.standard_normal(400000) + 2.0
    ov = 1.0 + erf(-1.0 / sqrt(2.0))
    assert abs(metrics.gcnr(x, y) - (1.0 - ov)) < 0.02


def test_point_width_of_a_gaussian():
    # exp(-x^2 / (2 sig^2)) halves at x = sig sqrt(2 ln 2): width 2.3548 sig
    x = np.linspace(-5.0, 5.0, 401)
    sig = 0.6
    env = np.outer(np.exp(-np.linspace(-1, 1, 9) ** 2), np.exp(-x ** 2 / (2 * sig * sig)))
    w = metrics.point_width(env, x, 4, 205)
    assert abs(w - 2.0 * sig * np.sqrt(2.0 * np.log(2.0))) < 1e-3
    assert np.isnan(metrics.point_width(np.ones((3, 10)), np.arange(10.0), 1, 5))
