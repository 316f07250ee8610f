"""Pins of the oracle's deadzone regularisers (Eqs. 10-11) against closed forms."""
import numpy as np

from oracle import reg


def _grid(nz=6, nx=7, dx=2.0, dz=3.0):
    X, Z = np.meshgrid(dx * np.arange(nx), dz * np.arange(nz))
    return X, Z, dx, dz


def test_linear_speed_closed_form():
    X, Z, dx, dz = _grid()
    bx, bz = 0.02, -0.005
    c = 1.5 + bx * X + bz * Z
    kx1, kz1 = 0.01, 0.001
    tv, sv = reg.reg_terms(1.0 / c, dx, dz, kx1, kz1, 1e-3, 1e-3)
    nz, nx = c.shape
    exp = (nz * (nx - 1) * max(0, abs(bx) - kx1) + (nz - 1) * nx * max(0, abs(bz) - kz1)) / c.size
    assert abs(tv - exp) < 1e-12
    assert abs(sv) < 1e-12


def test_quadratic_speed_closed_form():
    X, Z, dx, dz = _grid()
    q = 1e-3
    c = 1.5 + q * X * X
    tv, sv = reg.reg_terms(1.0 / c, dx, dz, 0.0, 0.0, 1e-4, 1e-4)
    nz, nx = c.shape
    # d_x c between nodes j, j+1 = q (x_j + x_{j+1}); d_xx c = 2q everywhere inside
    xs = dx * np.arange(nx)
    exp_tv = nz * np.sum(np.abs(q * (xs[1:] + xs[:-1]))) / c.size
    exp_sv = nz * (nx - 2) * (2 * q - 1e-4) / c.size
    assert abs(tv - exp_tv) < 1e-12
    assert abs(sv - exp_sv) < 1e-12


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    X, Z, dx, dz = _grid()
    s = 1.0 / (1.5 + 0.05 * rng.standard_normal(X.shape))
    k = (0.01, 0.005, 0.002, 0.003)
    w1, w2 = 3.0, 5.0
    g = reg.reg_grad(s, dx, dz, *k, w1, w2)
    f = lambda ss: w1 * reg.reg_terms(ss, dx, dz, *k)[0] + w2 * reg.reg_terms(ss, dx, dz, *k)[1]
    eps = 1e-7
    for idx in [(0, 0), (2, 3), (5, 6), (3, 1)]:
        sp = s.copy(); sp[idx] += eps
        sm = s.copy(); sm[idx] -= eps
        assert abs((f(sp) - f(sm)) / (2 * eps) - g[idx]) < 1e-5
