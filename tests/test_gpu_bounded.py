"""Bounded-memory mode (af_set_memory_budget): the hot path over chunks of tiles,
with the travel-time table and block images recomputed in the gradient pass,
against the same calls without a budget (and, on the small full launch, against
the FP64 oracle).  The loss terms, images and travel times are formed per tile in
both modes and summed in the same fixed order, so they agree bit for bit; the
gradient's sums over tiles are grouped by chunk, so it agrees to rounding."""
import numpy as np
import pytest

import afsynth
import gpu_setup as G

pytestmark = pytest.mark.gpu


def _pair(name, budget):
    """(cfg, unbounded beamformer, bounded beamformer, channel data, loss params) of
    the benchmark's launch configuration of ``name``."""
    import torch
    from paper_2608_06853_amd import autofocus as af, workloads
    G.ensure_built()
    cfg = afsynth.config_by_name(name)
    bf, iq, med = workloads.build(cfg)
    acqd, imgd, grid, cover = workloads.geometry(cfg)
    bb = af.Beamformer(acqd, imgd, grid, memory_budget=budget)
    s0 = torch.full(grid.shape, 1.0 / cfg.img.c_ref, device=bf.device)
    bb.set_slowness(s0)
    return cfg, bf, bb, iq, workloads.loss_params(cfg)


def _slowness(grid, seed):
    import problems
    return problems.smooth_slowness((grid.x0, grid.z0, grid.dx, grid.dz, grid.nx, grid.nz), seed)


@pytest.mark.parametrize("name,budget", [("c1_tiny", 24 << 20), ("c3_plain_loop", 16 << 20)])
def test_bounded_matches_unbounded(name, budget):
    import torch
    from paper_2608_06853_amd import _lib
    cfg, bf, bb, iq, lp = _pair(name, budget)
    k = bb.ctx.query(_lib.Q_CHUNKS)
    mem_u, mem_b = bf.ctx.query(_lib.Q_DEVICE_BYTES), bb.ctx.query(_lib.Q_DEVICE_BYTES)
    print(name, "chunks", k, "device bytes unbounded", mem_u, "bounded", mem_b, flush=True)
    assert k >= 3 and mem_b < mem_u
    s = torch.from_numpy(_slowness(bf.grid, cfg.seed)).cuda()
    tu, gu = bf.loss_and_grad(iq, lp, s)
    tb, gb = bb.loss_and_grad(iq, lp, s)
    torch.cuda.synchronize()
    assert torch.equal(tu, tb)
    e = G.rel(gb.cpu().numpy(), gu.cpu().numpy())
    print(name, "gradient rel", e, flush=True)
    assert e < 1e-5
    iu, mu, bu = bf.beamform(iq, blocks=True)
    ib, mb, bl = bb.beamform(iq, blocks=True)
    assert torch.equal(iu, ib) and torch.equal(mu, mb) and torch.equal(bu, bl)
    Tu, Tb = bf.travel_times(), bb.travel_times()  # NaN marks masked entries
    assert torch.equal(torch.isnan(Tu), torch.isnan(Tb))
    assert torch.equal(torch.nan_to_num(Tu), torch.nan_to_num(Tb))
    # the autograd wrapper forms the same gradient in both modes
    from paper_2608_06853_amd import autofocus as af
    for b, ref in ((bf, gu), (bb, gb)):
        x = s.clone().requires_grad_(True)
        tot, _ = af.cmpe_loss(x, b, iq, lp)
        tot.backward()
        assert G.rel(x.grad.cpu().numpy(), ref.cpu().numpy()) < 1e-5


def test_bounded_autofocus_steps_and_sweep():
    import torch
    from paper_2608_06853_amd import _lib, autofocus as af
    cfg, bf, bb, iq, lp = _pair("c1_tiny", 24 << 20)
    ap = _lib.adam_params(lr=cfg.method.lr)
    su, hu = af.plain_autofocus(bf, iq, lp, ap, 4)
    sb, hb = af.plain_autofocus(bb, iq, lp, ap, 4)
    for a, b in zip(hu.terms, hb.terms):
        assert abs(a[_lib.TERM_TOTAL] - b[_lib.TERM_TOTAL]) <= 1e-5 * abs(a[_lib.TERM_TOTAL])
    assert G.rel(sb.cpu().numpy(), su.cpu().numpy()) < 1e-6
    _, vu, best_u = af.sweep(bf, iq, lp, cfg.acq.fc)
    _, vb, best_b = af.sweep(bb, iq, lp, cfg.acq.fc)
    assert np.array_equal(vu, vb) and best_u == best_b


def test_bounded_refuses_whole_point_calls():
    import torch
    from paper_2608_06853_amd import _lib
    cfg, bf, bb, iq, lp = _pair("c1_tiny", 24 << 20)
    terms = bb.empty_terms()
    gblk = torch.empty(bb.ctx.query(_lib.Q_GBLK_ELEMS), device=bb.device, dtype=torch.complex64)
    with pytest.raises(_lib.AfError) as e:
        bb.ctx.forward(iq, lp, terms, gblk)
    assert e.value.status == _lib.AF_ERR_STATE
    with pytest.raises(_lib.AfError) as e:
        bb.channel_images(iq)
    assert e.value.status == _lib.AF_ERR_STATE
    # lifting the budget restores them
    bb.ctx.set_memory_budget(0)
    assert bb.ctx.query(_lib.Q_CHUNKS) == 1
    bb.ctx.forward(iq, lp, terms, gblk)
    bb.channel_images(iq)


def test_bounded_c1_against_oracle():
    """The whole small workload in bounded mode (at least 3 chunks) against the FP64
    oracle, as the unbounded full-launch test does it."""
    import torch
    import problems
    from oracle import model
    from paper_2608_06853_amd import _lib
    from test_gpu_fullsize import _launch
    G.ensure_built()
    cfg = afsynth.config_by_name("c1_tiny")
    bf, prob = _launch(cfg)
    bf.ctx.set_memory_budget(24 << 20)
    assert bf.ctx.query(_lib.Q_CHUNKS) >= 3
    med = afsynth.medium_for(cfg)
    iq = problems.simulate_iq(cfg, med, n_seg=64).astype(np.complex64)
    prob.iq = iq.astype(np.complex128)
    s = problems.smooth_slowness(prob.grid, cfg.seed)
    lp = problems.loss_params(cfg, sb_ref=float(np.mean(np.abs(iq)) ** 2 * 50.0))
    terms, grad = bf.loss_and_grad(torch.from_numpy(iq).cuda().reshape(-1), G.lib_params(lp),
                                   torch.from_numpy(s).cuda())
    t = terms.cpu().numpy()
    f, go = model.loss_and_grad(prob, s.astype(np.float64), lp)
    assert t[5] == f["n_valid"]
    assert abs(t[4] - f["total"]) <= 1e-4 * abs(f["total"])
    e = G.rel(grad.cpu().numpy().astype(np.float64), go)
    print("c1 bounded: chunks", bf.ctx.query(_lib.Q_CHUNKS), "gradient rel err vs oracle", e,
          flush=True)
    assert e < 1e-3


def test_bounded_clinical_full_size():
    """The clinical workload under a 512 MB budget: the same terms, the gradient to
    rounding, less device memory; prints both footprints and step times."""
    import time
    import torch
    from paper_2608_06853_amd import _lib
    cfg, bf, bb, iq, lp = _pair("c2_clinical", 512 << 20)
    k = bb.ctx.query(_lib.Q_CHUNKS)
    s = torch.from_numpy(_slowness(bf.grid, cfg.seed)).cuda()
    out = {}
    for tag, b in (("unbounded", bf), ("bounded", bb)):
        b.set_slowness(s)
        terms, grad = b.loss_and_grad(iq, lp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            b.ctx.loss_and_grad(iq, lp, terms, grad)
        torch.cuda.synchronize()
        out[tag] = (terms.clone(), grad.clone(), (time.perf_counter() - t0) / 5 * 1e3,
                    b.ctx.query(_lib.Q_DEVICE_BYTES))
    print("c2 chunks", k, {t: (round(v[2], 3), v[3]) for t, v in out.items()},
          "(ms per loss_and_grad, device bytes)", flush=True)
    assert k >= 4 and out["bounded"][3] < out["unbounded"][3]
    assert torch.equal(out["unbounded"][0], out["bounded"][0])
    assert G.rel(out["bounded"][1].cpu().numpy(), out["unbounded"][1].cpu().numpy()) < 1e-5
