"""End-to-end pins of the oracle: gradient vs finite differences, sweep minimum at the
true speed, Adam vs the torch library routine, and the simulator's closed forms."""
import math

import numpy as np
import pytest

import afsynth
import problems
from oracle import adam, model, simulate, sweep

SMALL = afsynth.configs.MICRO.with_(
    img=afsynth.ImgCfg(n_depth=6, n_angle=5, depth_min=6.0, depth_max=24.0),
    method=afsynth.MethodCfg(block=4, fnum=0.5, n_seg=12, nx=4, nz=5, w1=10.0, w2=100.0,
                             kx1=0.01, kz1=0.01, kx2=0.001, kz2=0.001, rho_thresh=0.3),
)


# the same on a linear array with a flat lens
SMALL_LINEAR = afsynth.configs.MICRO_LINEAR.with_(
    img=afsynth.ImgCfg(n_depth=5, n_angle=5, depth_min=3.0, depth_max=12.0),
    method=SMALL.method,
)


def _small(cfg):
    med = afsynth.medium_for(cfg)
    iq = problems.simulate_iq(cfg, med, n_seg=64)
    prob = problems.problem(cfg, iq)
    s_true = problems.true_slowness(cfg, med, prob)
    return prob, s_true


@pytest.fixture(scope="module")
def small_problem():
    return _small(SMALL)


@pytest.mark.parametrize("which", ["arc", "linear"])
def test_gradient_matches_finite_differences(small_problem, which):
    prob, s_true = small_problem if which == "arc" else _small(SMALL_LINEAR)
    rng = np.random.default_rng(0)
    s = s_true * (1.0 + 0.01 * rng.standard_normal(s_true.shape))
    lp = problems.loss_params(SMALL, sb_ref=50.0)
    lp.w_sb = 0.05
    cm = model.c_mean(s)
    f0, g = model.loss_and_grad(prob, s, lp, c_med=cm)
    assert f0["n_valid"] > 0
    eps = 1e-7
    worst = 0.0
    dirs = [rng.standard_normal(s.shape) for _ in range(3)]
    for k in range(s.size):
        e = np.zeros(s.size); e[k] = 1.0
        dirs.append(e.reshape(s.shape))
    for d in dirs:
        fp = model.forward(prob, s + eps * d, lp, c_med=cm)
        fm = model.forward(prob, s - eps * d, lp, c_med=cm)
        if fp["n_valid"] != f0["n_valid"] or fm["n_valid"] != f0["n_valid"]:
            continue
        fd = (fp["total"] - fm["total"]) / (2 * eps)
        an = float(np.sum(g * d))
        worst = max(worst, abs(fd - an) / max(np.linalg.norm(g) * np.linalg.norm(d), 1e-12))
    assert worst < 1e-4


@pytest.mark.parametrize("c_true", [1.500, 1.560])
def test_sweep_minimum_at_true_speed(c_true):
    # the tiny case's aperture (32 elements, 8 blocks -> 36 pairs per patch) in a
    # homogeneous medium: the dynamic-grid sweep minimum is within one 10 m/s step
    cfg = afsynth.configs.C1.with_(
        img=afsynth.ImgCfg(n_depth=10, n_angle=8, depth_min=10.0, depth_max=50.0),
        n_scat_random=1500)
    med = afsynth.medium_for(cfg)
    med.layer_c = np.array([c_true, c_true])
    iq = problems.simulate_iq(cfg, med, n_seg=16)
    prob = problems.problem(cfg, iq, depth_scale_max=1.62 / 1.54)
    lp = problems.loss_params(cfg)
    speeds = np.arange(c_true - 0.06, c_true + 0.0601, 0.01)
    _, vals, best = sweep.sweep(prob, lp, cfg.acq.fc, speeds=speeds)
    assert abs(best - c_true) <= 0.010 + 1e-9


def test_static_grid_is_the_dynamic_grid_of_its_own_speed(small_problem):
    # the static grid is laid out once for 1500 m/s: at that speed both sweeps see the
    # same pixels and kernel spacing, at any other speed the static one does not move
    prob, _ = small_problem
    lp = problems.loss_params(SMALL)
    speeds = np.array([1.47, 1.50])
    _, vd, _ = sweep.sweep(prob, lp, SMALL.acq.fc, speeds=speeds)
    _, vs, _ = sweep.sweep(prob, lp, SMALL.acq.fc, speeds=speeds, dynamic=False)
    assert vd[1] == vs[1]
    assert vd[0] != vs[0]


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    s = rng.standard_normal(20)
    p = torch.tensor(s.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(20)
    v = np.zeros(20)
    for step in range(1, 6):
        g = rng.standard_normal(20)
        p.grad = torch.tensor(g)
        opt.step()
        s, m, v = adam.adam_step(s, m, v, g, step, 0.01)
    assert np.allclose(s, p.detach().numpy(), rtol=0, atol=1e-13)


def test_simulator_single_scatterer_closed_form():
    arr = afsynth.ArrayCfg(4, 30.0, 0.5, 1e-12, 1.0)
    elem = afsynth.element_positions(arr)
    c = 1.54
    scat = np.array([[2.0, 60.0]])
    grid = (-10.0, 25.0, 1.0, 1.0, 21, 45)
    s = np.full((45, 21), 1.0 / c)
    fc, fs, ns, bw = 3.0, 48.0, 8192, 0.7
    iq = simulate.simulate(elem, 0.0, 1.0, 0.1, s, grid, 16, scat, np.array([2.0]),
                           t0=0.0, fs=fs, fd=fc, ns=ns, fc=fc, frac_bw=bw)
    t, r = 0, 3
    tau = (np.hypot(*(scat[0] - elem[t])) + np.hypot(*(scat[0] - elem[r]))) / c + 0.1
    n = int(np.argmax(np.abs(iq[t, r])))
    assert abs(n / fs - tau) <= 0.5 / fs
    sig = simulate.pulse_sigma(fc, bw)
    tn = np.arange(ns) / fs
    expect = 2.0 * np.exp(-(tn - tau) ** 2 / (2 * sig * sig)) * np.exp(-2j * np.pi * fc * tau)
    expect[np.abs(tn - tau) > 6 * sig] = 0
    assert np.allclose(iq[t, r], expect, atol=1e-12)
    # -6 dB fractional bandwidth of the modulated pulse equals frac_bw
    tt = np.arange(-4096, 4096) / 400.0
    pulse = np.exp(-tt ** 2 / (2 * sig * sig)) * np.cos(2 * np.pi * fc * tt)
    spec = np.abs(np.fft.rfft(pulse))
    f = np.fft.rfftfreq(tt.size, 1 / 400.0)
    above = f[spec >= 0.5 * spec.max()]
    assert abs((above.max() - above.min()) / fc - bw) < 0.02
