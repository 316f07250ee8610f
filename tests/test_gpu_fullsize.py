"""Parity at full size in the launch configuration the benchmark times: the whole
clinical (128 elements, 2560 samples, 256 x 256 pixels x 3 x 3 points, 32 x 32
grid), largest (192 elements, 4096 samples, 512 x 512 pixels, 64 x 64 grid) and
linear-array (128 elements at 0.2 mm, flat lens, 1536 samples, 128 x 128 pixels,
16 x 16 grid) geometries are set up exactly as in the benchmark, and sampled outputs are
compared with the FP64 oracle computed for those pixels alone:

* travel times of every element to every point of 40 random pixels (1e-6);
* block images and the coherence-factor map at those pixels (1e-4);
* loss and gradient of a context holding only the sampled pixels (same array,
  channel data and grid) against the oracle (1e-4 / 1e-3), the loss on the noise
  data and on coherent echoes the oracle simulates, the gradient on the echoes;
* at full size, the gradient along a smooth direction against a central
  difference of the library's own loss (a property that holds at any size).

The channel data of the oracle comparisons are seeded circular Gaussian noise
(afsynth.random_iq) or echoes of seeded scatterers simulated by the oracle:
oracle inputs never come from the library.  The directional
check compares the library with itself and runs on echoes the library simulates
through the seeded medium."""
import os

import numpy as np
import pytest

import afsynth
import gpu_setup as G
import problems
from oracle import model

pytestmark = pytest.mark.gpu

N_SAMPLE_PIX = 40
DEPTH_SCALE = 1.740 / 1.540     # the grid covers every speed of the dynamic-grid sweep


def _slowness(grid, seed):
    """Smooth seeded slowness around 1/1540 us/mm on the node grid."""
    return problems.smooth_slowness(grid, seed)


def _lp(cfg):
    lp = problems.loss_params(cfg)
    return model.LossParams(**{**lp.__dict__, "rho_thresh": 0.5})


@pytest.fixture(scope="module", params=["c2_clinical", "c5_largest", "l1_linear"])
def full(request):
    import torch
    from paper_2608_06853_amd import autofocus as af, workloads
    G.ensure_built()
    cfg = afsynth.config_by_name(request.param)
    print("full-size case", cfg.name, flush=True)
    acqd, imgd, grid, cover = workloads.geometry(cfg)
    prob = problems.problem(cfg, depth_scale_max=DEPTH_SCALE)
    assert np.allclose(prob.grid[:4], (grid.x0, grid.z0, grid.dx, grid.dz))
    iq = afsynth.random_iq(cfg.array.n_elem, cfg.acq.n_samples, seed=cfg.seed)
    s = _slowness(prob.grid, cfg.seed)
    bf = af.Beamformer(acqd, imgd, grid)
    iq_d = torch.from_numpy(iq).cuda().reshape(-1)
    bf.set_slowness(torch.from_numpy(s).cuda())
    rng = np.random.default_rng(cfg.seed + 101)
    sel = np.sort(rng.choice(prob.centres.shape[0], N_SAMPLE_PIX, replace=False))
    sub = model.Problem(**{**prob.__dict__, "centres": prob.centres[sel], "_cache": {},
                           "iq": iq.astype(np.complex128)})
    yield cfg, bf, iq_d, s, sel, sub, acqd, imgd, grid
    del bf
    torch.cuda.empty_cache()


def _point_index(sel, M):
    return (sel[:, None] * M + np.arange(M)[None, :]).reshape(-1)


def test_travel_times_sampled(full):
    import torch
    cfg, bf, iq_d, s, sel, sub, *_ = full
    M = sub.n_patch
    idx = torch.from_numpy(_point_index(sel, M)).cuda()
    T = bf.travel_times().index_select(1, idx).cpu().numpy().astype(np.float64)
    To = model.travel_times(sub, s.astype(np.float64))
    h = sub.apod()
    assert np.array_equal(np.isfinite(T), h)
    err = np.abs(T[h] - To[h]) / To[h]
    print(cfg.name, "sampled T max rel err", err.max(), "rays", int(h.sum()), flush=True)
    assert err.max() < 1e-6


def test_block_images_sampled(full):
    import torch
    cfg, bf, iq_d, s, sel, sub, *_ = full
    M = sub.n_patch
    lp = _lp(cfg)
    bf.ctx.loss_and_grad(iq_d, G.lib_params(lp), bf.empty_terms(), None)
    img, maps, blk = bf.beamform(iq_d, blocks=True)
    nb = bf.n_blk
    idx = torch.from_numpy(_point_index(sel, M)).cuda()
    bg = blk.view(nb * nb, -1).index_select(1, idx).cpu().numpy().reshape(nb, nb, -1)
    del blk
    f = model.forward(sub, s.astype(np.float64), lp, keep=True)
    e_blk = G.rel(bg, f["bblk"])
    cf = maps.view(3, -1)[1].cpu().numpy()[sel]
    cmcc = maps.view(3, -1)[2].cpu().numpy()[sel]
    e_cf = G.rel(cf, f["cf"])
    e_cc = G.rel(cmcc, f["cmcc"])
    print(cfg.name, "sampled blocks rel", e_blk, "cf rel", e_cf, "cmcc rel", e_cc, flush=True)
    assert e_blk < 1e-4 and e_cf < 1e-4 and e_cc < 1e-4


N_SCAT_COHERENT = 600


@pytest.fixture(scope="module")
def coherent(full):
    """Channel data the oracle simulates (64 ray segments) from the configuration's
    medium with 600 seeded point scatterers: coherent echoes, computed on the host."""
    cfg = full[0]
    c = cfg.with_(n_scat_random=N_SCAT_COHERENT)
    return problems.simulate_iq_parallel(c, afsynth.medium_for(c), 64)


def _sampled_loss_and_grad(full, iq):
    """Library and oracle loss terms and gradient of a context holding only the
    sampled pixels, on channel data ``iq`` [N][N][Ns]; asserts the terms."""
    import torch
    from dataclasses import replace
    from paper_2608_06853_amd import autofocus as af
    cfg, bf, _, s, sel, sub, acqd, imgd, grid = full
    lp = _lp(cfg)
    sub = model.Problem(**{**sub.__dict__, "_cache": {}, "iq": iq.astype(np.complex128)})
    bs = af.Beamformer(acqd, replace(imgd, centres=imgd.centres[sel]), grid)
    iq_d = torch.from_numpy(np.ascontiguousarray(iq, dtype=np.complex64)).cuda().reshape(-1)
    terms, grad = bs.loss_and_grad(iq_d, G.lib_params(lp), torch.from_numpy(s).cuda())
    t = terms.cpu().numpy()
    fo, go = model.loss_and_grad(sub, s.astype(np.float64), lp)
    print(cfg.name, "sampled-pixel loss gpu", t[:6], "oracle", fo["cmpe"], fo["total"],
          fo["n_valid"], flush=True)
    assert fo["n_valid"] > 50
    # valid counts may differ only by pairs within 1e-4 of the threshold, each of
    # which moves the CMPE mean by at most pi / n_valid
    from oracle import cmpe as ocmpe
    d = ocmpe.cmpe(fo["bsub"], sub.n_patch, lp.rho_thresh)
    pos = (d["ex"] > ocmpe.MIN_ENERGY) & (d["ey"] > ocmpe.MIN_ENERGY)
    n_near = int(np.sum(pos & (np.abs(d["rho"] - lp.rho_thresh) < 1e-4)))
    dn = abs(t[5] - fo["n_valid"])
    assert dn <= n_near
    assert abs(t[4] - fo["total"]) <= 1e-4 * abs(fo["total"]) + np.pi * dn / fo["n_valid"]
    return grad.cpu().numpy(), go, dn


def test_loss_sampled_pixels_noise(full):
    """Loss terms on the seeded noise data."""
    cfg = full[0]
    iq = afsynth.random_iq(cfg.array.n_elem, cfg.acq.n_samples, seed=cfg.seed)
    _sampled_loss_and_grad(full, iq)


def test_loss_and_gradient_sampled_pixels(full, coherent):
    """Loss terms and gradient on coherent echoes.  (On noise data the gradient at
    deep points of the linear array is a sum of terms of random sign that cancel to
    about 1e-4 of their magnitude, so FP32 rounding alone moves it by about 1e-3;
    the terms above are compared on noise data as well.)"""
    cfg = full[0]
    g, go, dn = _sampled_loss_and_grad(full, coherent)
    eg = G.rel(g, go)
    print(cfg.name, "sampled-pixel grad rel err (coherent echoes)", eg, "valid-count difference",
          dn, flush=True)
    assert eg < 1e-3


def test_full_size_gradient_directional(full):
    """Central difference of the library's own loss along a smooth direction that
    keeps mean(1/s) (hence c_med and the refraction points, which the gradient
    holds constant) fixed to first order.  The channel data are simulated through
    the seeded medium (coherent echoes: a property check of the library against
    itself); on noise data the directional derivative is a sum of random-sign
    terms and the kinks of |arg C| at 0 and +-pi set its noise floor.
    rho_thresh = 0 keeps every pair valid, so no validity mask flips inside the
    step; the step is scaled by 1/f_c (the same phase excursion at every centre
    frequency), and the adjoint is taken along the step realised in float32."""
    import torch
    from paper_2608_06853_amd import workloads
    cfg, bf, _, s, *_ = full
    med = afsynth.medium_for(cfg)
    iq_d = workloads.simulate(bf, cfg, med, workloads.geometry(cfg)[3])
    lp = G.lib_params(model.LossParams(**{**_lp(cfg).__dict__, "rho_thresh": 0.0}))
    s_d = torch.from_numpy(s).cuda()
    terms, grad = bf.loss_and_grad(iq_d, lp, s_d)
    t = terms.cpu().numpy()
    assert np.isfinite(t).all() and torch.isfinite(grad).all()
    assert t[5] > 1000
    nz, nx = s.shape
    X, Z = np.meshgrid(np.linspace(-1, 1, nx), np.linspace(-1, 1, nz))
    d = Z + 0.3 * X                       # a depth ramp with a lateral tilt
    w = 1.0 / s.astype(np.float64) ** 2
    d -= (d * w).sum() / (w * w).sum() * w
    d *= 2e-5 * (3.5 / cfg.acq.fc) * float(s.mean()) / np.abs(d).max()
    lv, sides = [], []
    for sgn in (1.0, -1.0):
        side = (s + sgn * d).astype(np.float32)
        sides.append(side.astype(np.float64))
        tt, _ = bf.loss_and_grad(iq_d, lp, torch.from_numpy(side).cuda(), want_grad=False)
        lv.append(float(tt[4].item()))
    fd = (lv[0] - lv[1]) / 2.0
    d_real = (sides[0] - sides[1]) / 2.0  # the step realised in float32
    g = grad.cpu().numpy().astype(np.float64)
    an = float((g * d_real).sum())
    err = abs(fd - an) / (np.linalg.norm(g) * np.linalg.norm(d_real))
    print(cfg.name, "directional derivative fd", fd, "adjoint", an, "normalised err", err,
          "relative err", abs(fd - an) / abs(an), flush=True)
    assert err < 1e-2


def test_gradient_bitwise_reproducible(full):
    """In deterministic mode every reduction of the loss and gradient runs in a
    fixed order (no floating-point atomics), so two evaluations at the same
    slowness agree bit for bit, also with an evaluation at another slowness in
    between; the default mode (atomic transmit-role sums) agrees with it to
    rounding."""
    import torch
    cfg, bf, iq_d, s, *_ = full
    lp = G.lib_params(_lp(cfg))
    s_d = torch.from_numpy(s).cuda()
    t0, g0 = bf.loss_and_grad(iq_d, lp, s_d)
    t0, g0 = t0.clone(), g0.clone()
    bf.ctx.set_deterministic(True)
    try:
        t1, g1 = bf.loss_and_grad(iq_d, lp, s_d)
        t1, g1 = t1.clone(), g1.clone()
        bf.loss_and_grad(iq_d, lp, torch.from_numpy((s * 1.01).astype(np.float32)).cuda())
        t2, g2 = bf.loss_and_grad(iq_d, lp, s_d)
        torch.cuda.synchronize()
    finally:
        bf.ctx.set_deterministic(False)
    assert torch.isfinite(g1).all() and float(g1.abs().max()) > 0
    assert torch.equal(t1, t2)
    assert torch.equal(g1, g2)
    assert torch.equal(t0, t1)  # the forward pass is the same in both modes
    e = G.rel(g0.cpu().numpy(), g1.cpu().numpy())
    print(cfg.name, "default vs deterministic gradient rel", e, flush=True)
    assert e < 1e-5


def _launch(cfg):
    """The benchmark's launch configuration of ``cfg`` (geometry, lens, slowness grid)
    and the oracle problem of the same geometry."""
    from paper_2608_06853_amd import autofocus as af, workloads
    acqd, imgd, grid, cover = workloads.geometry(cfg)
    prob = problems.problem(cfg, depth_scale_max=DEPTH_SCALE)
    assert np.allclose(prob.grid[:4], (grid.x0, grid.z0, grid.dx, grid.dz))
    return af.Beamformer(acqd, imgd, grid), prob


@pytest.mark.parametrize("name", ["c1_tiny", "c3_plain_loop"])
def test_full_launch_gradient_against_oracle(name):
    """The whole small workload (32 elements, 64 x 64 pixels x 3 x 3 points, 144
    tiles) at the configured loss parameters (CMPE threshold 0.9; the plain loop's
    speckle-brightness weight for c3_plain_loop) on echoes the oracle simulates:
    terms and the gradient of every grid node against the FP64 oracle."""
    import torch
    G.ensure_built()
    cfg = afsynth.config_by_name(name)
    print("full launch", name, flush=True)
    bf, prob = _launch(cfg)
    med = afsynth.medium_for(cfg)
    iq = problems.simulate_iq(cfg, med, n_seg=64).astype(np.complex64)
    prob.iq = iq.astype(np.complex128)
    s = problems.smooth_slowness(prob.grid, cfg.seed)
    lp = problems.loss_params(cfg, sb_ref=float(np.mean(np.abs(iq)) ** 2 * 50.0))
    terms, grad = bf.loss_and_grad(torch.from_numpy(iq).cuda().reshape(-1), G.lib_params(lp),
                                   torch.from_numpy(s).cuda())
    t = terms.cpu().numpy()
    f, go = model.loss_and_grad(prob, s.astype(np.float64), lp)
    g = grad.cpu().numpy().astype(np.float64)
    print(name, "tiles", bf.ctx.query(6), "gpu", t[:6], "oracle", f["cmpe"], f["total"],
          f["n_valid"], flush=True)
    assert t[5] == f["n_valid"] and f["n_valid"] > 1000
    for k, key in enumerate(["cmpe", "tv", "sv", "sb", "total"]):
        assert abs(t[k] - f[key]) <= 1e-4 * max(abs(f[key]), 1e-6), key
    e_norm = G.rel(g, go)
    e_max = float(np.max(np.abs(g - go)) / np.max(np.abs(go)))
    print(name, "gradient rel err (norm)", e_norm, "(max entry / max |g|)", e_max, flush=True)
    assert e_norm < 1e-3 and e_max < 1e-3


GOLDEN_C2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "c2_clinical_loss_grad.json")


def test_c2_full_launch_against_oracle_golden():
    """The whole clinical workload in the benchmark's launch configuration (2,341
    tiles) against the FP64 oracle's loss and gradient of every grid node, computed
    on the host in pixel chunks by tests/golden/make_c2_golden.py.  The inputs are
    rebuilt here exactly as that script builds them: channel data the oracle
    simulates from the seeded clinical medium with 2000 scatterers (about half a
    minute on the host cores), the perturbed true slowness and the configured loss
    parameters.  The valid-pair counts may differ only by pairs within 1e-4 of the
    threshold (counted by the oracle)."""
    import importlib.util
    import json
    import torch
    G.ensure_built()
    with open(GOLDEN_C2) as fh:
        gold = json.load(fh)
    spec = importlib.util.spec_from_file_location(
        "make_c2_golden", os.path.join(os.path.dirname(GOLDEN_C2), "make_c2_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    print("c2 full launch: simulating the channel data with the oracle", flush=True)
    cfg, prob, s, lp = mk.inputs()
    assert cfg.name == gold["config"] and lp.rho_thresh == gold["rho_thresh"]
    bf, prob_l = _launch(cfg)
    assert np.allclose(prob_l.grid, prob.grid)
    iq = prob.iq
    terms, grad = bf.loss_and_grad(torch.from_numpy(iq).cuda().reshape(-1), G.lib_params(lp),
                                   torch.from_numpy(s).cuda())
    t = terms.cpu().numpy()
    go = np.array(gold["grad"])
    gt = gold["terms"]
    dn = abs(t[5] - gt["n_valid"])
    print("c2 full launch: gpu", t[:6], "oracle", gt, "near-threshold pairs", gold["n_near"],
          flush=True)
    assert dn <= gold["n_near"]
    slack = np.pi * dn / gt["n_valid"]
    for k, key in enumerate(["cmpe", "tv", "sv", "sb", "total"]):
        tol = 1e-4 * max(abs(gt[key]), 1e-6) + (slack if key in ("cmpe", "total") else 0.0)
        assert abs(t[k] - gt[key]) <= tol, key
    g = grad.cpu().numpy().astype(np.float64)
    e_norm = G.rel(g, go)
    e_max = float(np.max(np.abs(g - go)) / np.max(np.abs(go)))
    print("c2 gradient rel err (norm)", e_norm, "(max entry / max |g|)", e_max, flush=True)
    assert e_norm < 1e-3 and e_max < 1e-3
