"""Pins of the oracle's path integral (Eq. 1 discretised) and bicubic interpolation."""
import numpy as np

from oracle import path

GRID = (-20.0, 30.0, 2.5, 3.0, 17, 15)  # x0, z0, dx, dz, nx, nz


def _nodes(grid=GRID):
    x0, z0, dx, dz, nx, nz = grid
    X, Z = np.meshgrid(x0 + dx * np.arange(nx), z0 + dz * np.arange(nz))
    return X, Z


def test_keys_kernel_partition_and_interpolation():
    f = np.linspace(0, 1, 101)
    w = np.stack([path.keys_kernel(1 + f), path.keys_kernel(f), path.keys_kernel(1 - f),
                  path.keys_kernel(2 - f)])
    assert np.allclose(w.sum(0), 1.0, atol=1e-15)
    assert path.keys_kernel(np.array([0.0]))[0] == 1.0
    assert np.all(path.keys_kernel(np.array([1.0, 2.0, 2.5])) == 0.0)
    # a = -0.5 reproduces quadratics: sum_j w_j (j - u)^2 = 0 for taps j at distances
    d = np.stack([-(1 + f), -f, 1 - f, 2 - f])
    assert np.allclose((w * d).sum(0), 0.0, atol=1e-14)
    assert np.allclose((w * d * d).sum(0), 0.0, atol=1e-14)


def test_bicubic_reproduces_quadratic_inside():
    X, Z = _nodes()
    q = lambda x, z: 0.6 + 0.01 * x - 0.004 * z + 1e-4 * x * x + 2e-4 * x * z - 5e-5 * z * z
    s = q(X, Z)
    rng = np.random.default_rng(0)
    x = rng.uniform(-20 + 2.5, -20 + 2.5 * 14, 200)
    z = rng.uniform(33.0, 30.0 + 3 * 12, 200)
    assert np.allclose(path.bicubic(s, GRID, x, z), q(x, z), rtol=0, atol=1e-13)


def test_homogeneous_gives_length_times_slowness():
    s = np.full((15, 17), 0.66)
    rng = np.random.default_rng(1)
    ax, az = rng.uniform(-15, 15, 30), rng.uniform(32, 50, 30)
    px, pz = rng.uniform(-15, 15, 30), rng.uniform(40, 70, 30)
    l2 = np.hypot(px - ax, pz - az)
    t = path.medium_time(s, GRID, ax, az, px, pz, l2, 32)
    assert np.allclose(t, l2 * 0.66, rtol=1e-14)


def test_linear_field_trapezoid_exact():
    X, Z = _nodes()
    lin = lambda x, z: 0.65 + 0.002 * x - 0.001 * z
    s = lin(X, Z)
    ax, az, px, pz = -10.0, 36.0, 12.0, 62.0
    l2 = np.hypot(px - ax, pz - az)
    t = path.medium_time(s, GRID, np.array([ax]), np.array([az]), np.array([px]), np.array([pz]),
                         np.array([l2]), 7)
    assert abs(t[0] - l2 * 0.5 * (lin(ax, az) + lin(px, pz))) < 1e-13


def test_quadratic_field_trapezoid_closed_form():
    # for q quadratic in the ray parameter t in [0,1], the N-segment trapezoid sum equals
    # int_0^1 q dt + q''/(12 N^2)
    X, Z = _nodes()
    q = lambda x, z: 0.6 + 1e-4 * x * x - 5e-5 * z * z + 2e-4 * x * z
    s = q(X, Z)
    ax, az, px, pz = -12.0, 35.0, 10.0, 60.0
    dx_, dz_ = px - ax, pz - az
    # q(t) = q(a + t d): second derivative in t
    q2 = 2 * (1e-4 * dx_ * dx_ - 5e-5 * dz_ * dz_ + 2e-4 * dx_ * dz_)
    tt = np.linspace(0, 1, 20001)
    integ = np.trapezoid(q(ax + tt * dx_, az + tt * dz_), tt) - q2 / (12 * 20000 ** 2)
    for n in (4, 16, 32):
        got = path.medium_time(s, GRID, np.array([ax]), np.array([az]), np.array([px]),
                               np.array([pz]), np.array([1.0]), n)[0]
        assert abs(got - (integ + q2 / (12 * n * n))) < 1e-12


def test_convergence_second_order():
    X, Z = _nodes()
    f = lambda x, z: 0.65 + 0.02 * np.sin(x / 7.0) * np.cos(z / 9.0)
    s = f(X, Z)
    a = (np.array([-9.0]), np.array([34.0]), np.array([11.0]), np.array([63.0]), np.array([1.0]))
    ref = path.medium_time(s, GRID, *a[:4], a[4], 4096)[0]
    e16 = abs(path.medium_time(s, GRID, *a[:4], a[4], 16)[0] - ref)
    e64 = abs(path.medium_time(s, GRID, *a[:4], a[4], 64)[0] - ref)
    assert e64 < e16 / 10.0  # ~16x for a second-order rule


def test_adjoint_dot_product():
    rng = np.random.default_rng(4)
    n = 40
    ax, az = rng.uniform(-15, 15, n), rng.uniform(31, 40, n)
    px, pz = rng.uniform(-19, 19, n), rng.uniform(40, 71, n)
    px[0], pz[0] = -19.9, 30.1  # near the corner: exercises index clamping
    l2 = np.hypot(px - ax, pz - az)
    ds = rng.standard_normal((15, 17))
    gbar = rng.standard_normal(n)
    lhs = np.sum(gbar * path.medium_time(ds, GRID, ax, az, px, pz, l2, 32))
    rhs = np.sum(ds * path.medium_time_adjoint(gbar, GRID, ax, az, px, pz, l2, 32))
    assert abs(lhs - rhs) < 1e-11 * max(1.0, abs(lhs))
