"""Pins of the oracle's delay-and-sum (Eq. 5): impulse closed form, linearity,
reciprocity, point-target focusing and the adjoint against finite differences."""
import math

import numpy as np

import afsynth
from oracle import das, fermat, geometry, path, simulate

KW = dict(t0=0.3, fs=12.0, fd=3.0, t_ttp=0.05, block=2)


def _rand_T(n, P, seed, lo=5.0, hi=30.0):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, (n, P))


def test_impulse_closed_form():
    n, ns, P = 4, 800, 50
    T = _rand_T(n, P, 0)
    h = np.ones((n, P), dtype=bool)
    h[1, ::3] = False
    t_, r_, n0 = 2, 1, 0
    u = (T[t_] + T[r_] + KW["t_ttp"] - KW["t0"]) * KW["fs"]
    n0 = int(np.median(np.floor(u)))
    iq = np.zeros((n, n, ns), dtype=np.complex128)
    iq[t_, r_, n0] = 1.0 + 0.5j
    b = das.das_blocks(iq, T, h, **KW)
    tau = T[t_] + T[r_] + KW["t_ttp"]
    k = np.floor(u)
    f = u - k
    wgt = np.where(k == n0, 1 - f, 0.0) + np.where(k + 1 == n0, f, 0.0)
    expect = wgt * (1.0 + 0.5j) * np.exp(2j * math.pi * KW["fd"] * tau) * (h[t_] & h[r_])
    assert np.allclose(b[t_ // 2, r_ // 2], expect, atol=1e-14)
    others = np.abs(b).sum() - np.abs(b[t_ // 2, r_ // 2]).sum()
    assert others == 0.0


def test_out_of_record_is_zero_and_last_sample():
    n, ns = 2, 10
    iq = np.ones((n, n, ns), dtype=np.complex128)
    h = np.ones((n, 3), dtype=bool)
    kw = dict(KW, t0=0.0, t_ttp=0.0, fd=0.0, block=1)
    # u = -0.1, exactly ns-1, and beyond
    T = np.array([[-0.1 / 24, (ns - 1) / 24.0, (ns - 0.9) / 24.0]] * n)
    b = das.das_blocks(iq, T, h, **kw)
    assert b[0, 0, 0] == 0 and abs(b[0, 0, 1] - 1.0) < 1e-15 and b[0, 0, 2] == 0


def test_linearity_and_reciprocity():
    rng = np.random.default_rng(2)
    n, ns, P = 4, 700, 30
    T = _rand_T(n, P, 1)
    h = rng.uniform(size=(n, P)) > 0.2
    a = rng.standard_normal((n, n, ns)) + 1j * rng.standard_normal((n, n, ns))
    b = rng.standard_normal((n, n, ns)) + 1j * rng.standard_normal((n, n, ns))
    ba = das.das_blocks(a, T, h, **KW)
    bb = das.das_blocks(b, T, h, **KW)
    bab = das.das_blocks(2.0 * a - 3j * b, T, h, **KW)
    assert np.allclose(bab, 2.0 * ba - 3j * bb, atol=1e-12)
    sym = a + a.transpose(1, 0, 2)
    bs = das.das_blocks(sym, T, h, **KW)
    assert np.allclose(bs, bs.transpose(1, 0, 2), atol=1e-12)


def test_adjoint_matches_finite_differences():
    rng = np.random.default_rng(5)
    n, ns, P = 4, 800, 20
    T = _rand_T(n, P, 3)
    h = rng.uniform(size=(n, P)) > 0.1
    iq = rng.standard_normal((n, n, ns)) + 1j * rng.standard_normal((n, n, ns))
    G = rng.standard_normal((2, 2, P)) + 1j * rng.standard_normal((2, 2, P))
    g = das.das_blocks_adjoint_T(iq, T, h, G, **KW)
    L = lambda TT: np.real(np.sum(np.conj(G) * das.das_blocks(iq, TT, h, **KW)))
    eps = 1e-7
    for (a, p) in [(0, 0), (1, 3), (3, 7), (2, 19)]:
        Tp = T.copy(); Tp[a, p] += eps
        Tm = T.copy(); Tm[a, p] -= eps
        fd = (L(Tp) - L(Tm)) / (2 * eps)
        assert abs(fd - g[a, p]) < 1e-5 * max(1.0, abs(fd))


def test_point_target_focuses_at_true_speed():
    # one scatterer in a homogeneous medium, simulated and beamformed with the same model
    arr = afsynth.ArrayCfg(16, 30.0, 0.5, 0.8, 1.0)
    elem = afsynth.element_positions(arr)
    c = 1.54
    rl = 30.8
    scat = np.array([[1.0, rl + 15.0]])
    grid = (-15.0, 25.0, 1.0, 1.0, 31, 40)
    s = np.full((40, 31), 1.0 / c)
    fc, fs, ns = 3.0, 12.0, 512
    iq = simulate.simulate(elem, arr.d_lens, arr.c_lens, 0.0, s, grid, 32, scat, np.array([1.0]),
                           t0=0.0, fs=fs, fd=fc, ns=ns, fc=fc, frac_bw=0.7)
    sp = c / (2 * fc) / 2
    xs = scat[0, 0] + sp * np.arange(-6, 7)
    zs = scat[0, 1] + sp * np.arange(-6, 7)
    X, Z = np.meshgrid(xs, zs)
    pts = np.stack([X.ravel(), Z.ravel()], 1)
    r = fermat.refract(elem, arr.d_lens, arr.c_lens, c, pts)
    px = np.broadcast_to(pts[None, :, 0], r["l2"].shape)
    pz = np.broadcast_to(pts[None, :, 1], r["l2"].shape)
    T = r["l1"] / arr.c_lens + path.medium_time(s, grid, r["ref_x"], r["ref_z"], px, pz, r["l2"], 32)
    th = geometry.element_orientation(elem)
    h = np.ones_like(T, dtype=bool)
    b = das.das_blocks(iq, T, h, t0=0.0, fs=fs, fd=fc, t_ttp=0.0, block=4).sum(axis=(0, 1))
    pk = int(np.argmax(np.abs(b)))
    assert np.hypot(*(pts[pk] - scat[0])) <= sp * 1.01
    centre = 6 * 13 + 6
    # at the scatterer every sample is phase-aligned: the image is real and positive
    assert abs(np.angle(b[centre])) < 1e-3
