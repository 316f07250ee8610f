"""Pins of the oracle's CMPE reading, speckle brightness and coherence factor."""
import math

import numpy as np

from oracle import cmpe


def _wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def test_known_phases():
    rng = np.random.default_rng(0)
    ns, n_pix, M = 5, 6, 9
    phase = rng.uniform(-np.pi, np.pi, (ns, ns, n_pix))
    amp = rng.uniform(0.5, 2.0, (n_pix, M))
    bsub = (amp[None, None] * np.exp(1j * phase)[..., None]).reshape(ns, ns, n_pix * M)
    loss, nv, cmap, d = cmpe.cmpe_loss(bsub, M, 0.9)
    # every pair is perfectly correlated (rho = 1): error = |wrapped phase difference|
    exp = np.abs(_wrap(phase[:-1, 1:] - phase[1:, :-1]))
    assert nv == (ns - 1) ** 2 * n_pix
    assert np.allclose(d["rho"], 1.0)
    assert np.allclose(d["err"], exp, atol=1e-12)
    assert abs(loss - exp.mean()) < 1e-12
    assert np.allclose(cmap, exp.mean(axis=(0, 1)))


def test_threshold_and_zero_energy():
    rng = np.random.default_rng(1)
    ns, n_pix, M = 3, 4, 9
    bsub = rng.standard_normal((ns, ns, n_pix * M)) + 1j * rng.standard_normal((ns, ns, n_pix * M))
    bsub[0, 1, :M] = 0.0  # X of pair (0,0) is empty for pixel 0
    _, nv, _, d = cmpe.cmpe_loss(bsub, M, 0.0)
    assert not d["valid"][0, 0, 0]
    assert nv == (ns - 1) ** 2 * n_pix - 1
    _, nv_hi, _, d = cmpe.cmpe_loss(bsub, M, 0.9)
    assert np.all(d["valid"] == (d["rho"] >= 0.9) & (d["ex"] > 0) & (d["ey"] > 0))
    # energies too small for FP32 (|C|^2 underflows) count as empty
    tiny = bsub * 1e-18
    assert cmpe.cmpe_loss(tiny, M, 0.0)[1] == 0
    assert cmpe.cmpe_loss(np.zeros_like(bsub), M, 0.5)[0] == 0.0


def test_subaperture_sum_and_adjoint():
    rng = np.random.default_rng(2)
    nb, P = 5, 18
    bblk = rng.standard_normal((nb, nb, P)) + 1j * rng.standard_normal((nb, nb, P))
    bsub = cmpe.subaperture_images(bblk)
    assert np.allclose(bsub[1, 2], bblk[1, 2] + bblk[2, 2] + bblk[1, 3] + bblk[2, 3])
    y = rng.standard_normal(bsub.shape) + 1j * rng.standard_normal(bsub.shape)
    lhs = np.real(np.vdot(y, bsub))
    rhs = np.real(np.vdot(cmpe.subaperture_images_adjoint(y), bblk))
    assert abs(lhs - rhs) < 1e-11


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    ns, n_pix, M = 4, 5, 9
    base = rng.standard_normal((n_pix * M)) + 1j * rng.standard_normal((n_pix * M))
    bsub = base[None, None] * np.exp(1j * rng.uniform(-1, 1, (ns, ns, 1))) + \
        0.2 * (rng.standard_normal((ns, ns, n_pix * M)) + 1j * rng.standard_normal((ns, ns, n_pix * M)))
    g = cmpe.cmpe_loss_grad(bsub, M, 0.5)
    _, _, _, d0 = cmpe.cmpe_loss(bsub, M, 0.5)
    eps = 1e-6
    for idx in [(0, 1, 3), (2, 1, 17), (3, 3, 44), (1, 0, 9)]:
        for unit in (1.0, 1j):
            bp = bsub.copy(); bp[idx] += eps * unit
            bm = bsub.copy(); bm[idx] -= eps * unit
            assert np.array_equal(cmpe.cmpe_loss(bp, M, 0.5)[3]["valid"], d0["valid"])
            fd = (cmpe.cmpe_loss(bp, M, 0.5)[0] - cmpe.cmpe_loss(bm, M, 0.5)[0]) / (2 * eps)
            an = g[idx].real if unit == 1.0 else g[idx].imag
            assert abs(fd - an) < 1e-7


def test_speckle_brightness_and_cf():
    rng = np.random.default_rng(4)
    nb, n_pix, M = 3, 7, 9
    bblk = rng.standard_normal((nb, nb, n_pix * M)) + 1j * rng.standard_normal((nb, nb, n_pix * M))
    full = bblk.sum(axis=(0, 1)).reshape(n_pix, M)[:, 4]
    assert abs(cmpe.speckle_brightness(bblk, M) - np.mean(np.abs(full) ** 2)) < 1e-12
    g = cmpe.speckle_brightness_grad(bblk, M)
    eps = 1e-6
    bp = bblk.copy(); bp[1, 2, 3 * M + 4] += eps
    bm = bblk.copy(); bm[1, 2, 3 * M + 4] -= eps
    fd = (cmpe.speckle_brightness(bp, M) - cmpe.speckle_brightness(bm, M)) / (2 * eps)
    assert abs(fd - g[1, 2, 3 * M + 4].real) < 1e-7
    cf = cmpe.coherence_factor(bblk, M)
    assert np.all((cf >= 0) & (cf <= 1 + 1e-12))
    same = np.broadcast_to(bblk[:1, :1], bblk.shape).copy()
    assert np.allclose(cmpe.coherence_factor(same, M), 1.0)


def test_cmcc_map_closed_forms():
    """rho = 1 for pairs that differ by a complex factor, rho = |<u, v>| / (|u||v|)
    for an explicit pair, pixels with no energy give 0 and the threshold plays no
    part."""
    rng = np.random.default_rng(5)
    ns, n_pix, M = 4, 3, 9
    u = rng.standard_normal((n_pix, M)) + 1j * rng.standard_normal((n_pix, M))
    gains = rng.uniform(0.5, 2.0, (ns, ns, 1, 1)) * np.exp(1j * rng.uniform(-3, 3, (ns, ns, 1, 1)))
    bsub = (gains * u[None, None]).reshape(ns, ns, n_pix * M)
    assert np.allclose(cmpe.cmcc_map(bsub, M), 1.0)
    # one explicit pair: ns = 2 has the single pair X = B_{0,1}, Y = B_{1,0}
    x = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    b2 = np.zeros((2, 2, M), dtype=complex)
    b2[0, 1], b2[1, 0] = x, y
    exp = abs(np.sum(x * np.conj(y))) / (np.linalg.norm(x) * np.linalg.norm(y))
    assert abs(cmpe.cmcc_map(b2, M)[0] - exp) < 1e-12
    b2[1, 0] = 0.0
    assert cmpe.cmcc_map(b2, M)[0] == 0.0
