#!/usr/bin/env python3
"""Throughput of the differentiable beamformer's hot path on one MI355X.

One step = one ``af_loss_and_grad`` call on the clinical-size workload (128-element
curvilinear array, 128 transmits, 2560 complex samples, 256 x 256 pixels with 3 x 3
patches to 160 mm, 32 x 32 slowness grid): bent-ray travel-time table, DAS over
transmit x receive x point, CMPE + regularisers, DAS adjoint, path adjoint and the
gradient on the grid.  Channel data are simulated on the GPU from a seeded random
liver-like medium before timing and stay resident in HBM.

Prints one JSON line: metric/value (nominal tx*rx*point samples per second of the
forward+adjoint pass), the roofline of the dominant kernel (timed with HIP events
on the library stream) and the FP64 oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DAS fwd+bwd Gsamples/s (tx·rx·pix); autofocus s-to-target CMP error, learned vs plain"
UNIT = "Gsamples/s"

# MI355X published peaks
PEAK_FP32_TFLOPS = 157.3        # 256 CU x 2.4 GHz x 256 FP32 flop/clk/CU (packed FP32)
# The library is built without packed FP32 instructions (they have given wrong
# results on these boxes), so one FMA per lane per issue is the attainable vector
# ceiling: 256 CU x 2.4 GHz x 128 flop/clk/CU.
PEAK_FP32_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
PEAK_BF16_TFLOPS = 2500.0       # dense MFMA, no sparsity

# Algorithmic FP32 operations per unit of each kernel (counted from the arithmetic
# the step needs, not from the compiled code).
FLOPS_PER_UNIT = {
    "das_fwd": 14.0,     # per active (t, r, point) sample: interpolate (6) + rotate-accumulate (8)
    "das_adj": 22.0,     # per active sample: interpolate + derivative (12) + rotate (6) + Re/acc (4)
    "table": 64.0,       # per ray point: bicubic weights (20) + 16 taps (40) + position (4)
    "path_adj": 60.0,    # per ray point: weights (20) + 16 scatter products (20) + the 16
                         # additions into the grid (16) + position (4)
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2_clinical")
    ap.add_argument("--cpu-pixels", type=int, default=1024,
                    help="pixels of the bounded oracle sample (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter scale)")
    ap.add_argument("--no-autofocus", action="store_true",
                    help="skip the plain-loop report and the learned-vs-plain s-to-target runs")
    ap.add_argument("--reports", default="all",
                    help="comma-separated report names to run after the timed steps (default all)")
    return ap.parse_args()


def workload(cfg, device=0):
    from paper_2608_06853_amd import workloads
    return workloads.build(cfg, device=device)


_cpu = {}


def _cpu_init():
    from threadpoolctl import threadpool_limits
    _cpu["limits"] = threadpool_limits(limits=1)   # one thread per process


def _cpu_chunk(sel):
    from oracle import model
    prob, s, lp = _cpu["prob"], _cpu["s"], _cpu["lp"]
    sub = model.Problem(**{**prob.__dict__, "centres": prob.centres[sel], "_cache": {}})
    return model.loss_and_grad_parts(sub, s, lp)


def cpu_baseline(cfg, n_pix_sample: int):
    """The FP64 oracle as it stands, on the host's cores (one process per core, at
    most 16), on a bounded sample of the same workload: the full array and
    channel-data shape, every k-th pixel of the image (n_pix_sample of them), dealt
    round-robin into one chunk per process so that every chunk spans all depths;
    the chunks' sums are combined as the whole loss_and_grad would combine them
    (oracle.model.combine_parts)."""
    import multiprocessing as mp
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import afsynth
    import problems
    from oracle import model

    prob = problems.problem(cfg, depth_scale_max=1.74 / 1.54)
    n_all = prob.centres.shape[0]
    stride = max(1, n_all // n_pix_sample)
    sel = np.arange(0, n_all, stride)[:n_pix_sample]
    prob.iq = afsynth.random_iq(cfg.array.n_elem, cfg.acq.n_samples, seed=cfg.seed)
    x0, z0, dx, dz, nx, nz = prob.grid
    s = np.full((nz, nx), 1.0 / 1.54)
    lp = problems.loss_params(cfg)
    _cpu.update(prob=prob, s=s, lp=lp)
    workers = max(1, min(16, os.cpu_count() or 1, len(sel)))
    chunks = [sel[w::workers] for w in range(workers)]
    with mp.get_context("fork").Pool(workers, initializer=_cpu_init) as pool:
        t0 = time.perf_counter()
        parts = pool.map(_cpu_chunk, chunks, chunksize=1)
        model.combine_parts(parts, s, lp, prob.grid)
        dt = time.perf_counter() - t0
    samples = cfg.array.n_elem ** 2 * len(sel) * prob.n_patch
    return dict(value=samples / dt / 1e9, unit=UNIT, cores=workers, kind="oracle",
                sample=f"{len(sel)} of {n_all} pixels (x{prob.n_patch} points: every "
                       f"{stride}th pixel of the image), full "
                       f"{cfg.array.n_elem}x{cfg.array.n_elem}x{cfg.acq.n_samples} channel "
                       f"data, loss and gradient in one chunk per process on {workers} "
                       f"processes: {dt:.1f} s; scaled per sample, the whole image would take "
                       f"about {dt * n_all / len(sel):.0f} s")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_clinical_hbm_traffic.txt")


def measured_traffic(cfg_name: str, family: str):
    """HBM bytes per launch of ``family`` from the committed rocprofv3 counter summary,
    or None when there is none for this workload or the kernel's sources changed since."""
    from paper_2608_06853_amd import profsummary
    if cfg_name != "c2_clinical" or not os.path.exists(TRAFFIC_FILE):
        return None
    rec = profsummary.read_traffic(TRAFFIC_FILE).get(family)
    if rec is None or rec[0] != profsummary.source_hash(family):
        return None
    return rec[1]


COUNTERS_FILE = os.path.join(ROOT, "profiles", "c2_clinical_valu_counters.txt")


def measured_issue(cfg_name: str, family: str, units: float):
    """VALU instructions per CU per ns, active-lane share and VALU lane-instructions
    per algorithmic unit of ``family`` from the committed SQ counter summary, or None
    when there is none for this workload or the kernel's sources changed since."""
    from paper_2608_06853_amd import profsummary
    if cfg_name != "c2_clinical" or not os.path.exists(COUNTERS_FILE):
        return None
    rec = profsummary.read_counters(COUNTERS_FILE).get(family)
    if rec is None or rec[0] != profsummary.source_hash(family):
        return None
    lane_instr = rec[3] * 64.0 * rec[2]
    return {"valu_instr_per_cu_per_ns": rec[1], "active_lane_share": rec[2],
            "valu_lane_instr_per_unit": round(lane_instr / units, 2) if units > 0 else None}


def memory_report():
    """Device memory the context holds and time per autofocus step (forward, adjoint,
    Adam) without a memory budget and under budgets (af_set_memory_budget: the
    gradient pass recomputes each chunk's table and block images), on the
    clinical and the largest workload.  The caller's channel data are not
    counted."""
    import torch
    import afsynth
    from paper_2608_06853_amd import _lib, workloads
    out = {}
    for name, budgets in (("c2_clinical", (0, 1 << 30, 512 << 20)),
                          ("c5_largest", (0, 4 << 30, 2 << 30))):
        cfg = afsynth.config_by_name(name)
        bf, iq, med = workloads.build(cfg)
        lp = workloads.loss_params(cfg)
        ap = _lib.adam_params(lr=cfg.method.lr)
        rows = []
        for b in budgets:
            bf.ctx.set_memory_budget(b)
            s = torch.full(bf.grid.shape, 1.0 / cfg.img.c_ref, device=bf.device)
            m, v = torch.zeros_like(s), torch.zeros_like(s)
            terms = bf.empty_terms()
            bf.ctx.autofocus_step(iq, lp, ap, 1, s, m, v, terms)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for it in range(2, 7):
                bf.ctx.autofocus_step(iq, lp, ap, it, s, m, v, terms)
            torch.cuda.synchronize()
            rows.append({"budget_bytes": b, "chunks": bf.ctx.query(_lib.Q_CHUNKS),
                         "device_bytes": bf.ctx.query(_lib.Q_DEVICE_BYTES),
                         "ms_per_autofocus_step": round((time.perf_counter() - t0) / 5 * 1e3, 3)})
        out[name] = rows
        del bf, iq
        torch.cuda.empty_cache()
    return out


def plain_loop_report():
    """The full plain method (sweep + Adam with CMPE and speckle brightness) on the
    two-layer medium with a cyst: speed errors and image quality before and after."""
    import torch
    import afsynth
    from paper_2608_06853_amd import metrics, warmstart, workloads
    cfg = afsynth.configs.C3
    bf, iq, med = workloads.build(cfg)
    base = bf.img
    c_true = workloads.true_speed_nodes(cfg, med, bf.grid)
    npx = base.centres.shape[0]
    M = base.patch * base.patch

    depth = np.linspace(cfg.img.depth_min, cfg.img.depth_max, cfg.img.n_depth)

    def image_quality(s):
        bf.set_imaging(base)
        img, maps, _ = bf.beamform(iq, s=s)
        env = img.abs().view(npx, M)[:, M // 2].cpu().numpy()
        q = metrics.contrast_cnr(env, base.centres, med.cyst_xz[0], float(med.cyst_r[0]))
        mp = maps.view(3, -1).cpu().numpy()
        g = {"speckle_brightness": float((img.abs() ** 2).mean().item()),
             "coherence_factor": float(mp[1].mean()), "cmcc": float(mp[2].mean()),
             "cmpe_map_mean": float(mp[0].mean()),
             "lag_one_coherence": float(bf.lag_one_coherence(iq).mean().item())}
        return q, g, env.reshape(cfg.img.n_depth, cfg.img.n_angle)

    # the nine point targets of the medium: 15/30/45 mm deep at -1/3, 0, +1/3 of the
    # half-span; lateral -6 dB width along the image row (arc length)
    th0, th1 = afsynth.element_span(cfg.array)
    ang = np.linspace(th0, th1, cfg.img.n_angle)
    arc = (afsynth.lens_radius(cfg.array) + depth)[:, None] * ang[None, :]

    def target_width(env2):
        w = [metrics.point_width(env2, arc, int(np.argmin(np.abs(depth - dp))),
                                 int(np.argmin(np.abs(ang - f * 0.5 * (th1 - th0)))))
             for dp in (15.0, 30.0, 45.0) for f in (-1.0 / 3.0, 0.0, 1.0 / 3.0)]
        return float(np.nanmean(w))

    s_hom = torch.full(bf.grid.shape, 1.0 / cfg.img.c_ref, device=bf.device)
    q0, g0, env0 = image_quality(s_hom)
    torch.cuda.synchronize()
    s, cm, times, t_sweep, best = warmstart.run_plain(bf, iq, cfg, cfg.method.n_iter)
    q1, g1, env1 = image_quality(s)
    e_hom = metrics.speed_errors(s_hom.cpu().numpy(), c_true)
    e_swp = metrics.speed_errors(np.full(bf.grid.shape, 1.0 / best), c_true)
    e_fin = metrics.speed_errors(s.cpu().numpy(), c_true)
    return {"config": cfg.name, "iterations": len(cm), "seconds": round(times[-1], 3),
            "sweep_seconds": round(t_sweep, 3), "sweep_best_speed": best,
            "cmpe_first": cm[0], "cmpe_final": cm[-1],
            "rmse_mps": {"homogeneous_1540": e_hom["rmse_mps"], "sweep": e_swp["rmse_mps"],
                         "final": e_fin["rmse_mps"]},
            "mae_mps": {"homogeneous_1540": e_hom["mae_mps"], "sweep": e_swp["mae_mps"],
                        "final": e_fin["mae_mps"]},
            "cyst_contrast_db": {"homogeneous_1540": q0["contrast_db"], "final": q1["contrast_db"]},
            "cyst_cnr": {"homogeneous_1540": q0["cnr"], "final": q1["cnr"]},
            "cyst_gcnr": {"homogeneous_1540": q0["gcnr"], "final": q1["gcnr"]},
            "global_metrics": {"homogeneous_1540": g0, "final": g1,
                               "change_pct": {k: 100.0 * (g1[k] / g0[k] - 1.0) for k in g0
                                              if g0[k] != 0}},
            "tenengrad_change_pct": metrics.tenengrad_change(env0, env1, depth),
            "point_target_width_mm": {"homogeneous_1540": target_width(env0),
                                      "final": target_width(env1)}}


def lens_model_report():
    """The paper's lens ablation on the plain loop's medium: channel data simulated
    through the lens (bent rays), then the plain method (sweep + Adam) run with
    each lens model of the beamformer; global speed and map errors against the
    true medium."""
    import afsynth
    from paper_2608_06853_amd import metrics, warmstart, workloads
    cfg = afsynth.configs.C3
    out = {}
    for model in workloads.LENS_MODELS:
        bf, iq, med = workloads.build(cfg, lens_model=model)
        s, cm, times, t_sweep, best = warmstart.run_plain(bf, iq, cfg, cfg.method.n_iter)
        c_true = workloads.true_speed_nodes(cfg, med, bf.grid)
        e = metrics.speed_errors(s.cpu().numpy(), c_true)
        e_sweep = metrics.speed_errors(np.full(bf.grid.shape, 1.0 / best), c_true)
        out[model] = {"sweep_best_speed": best, "sweep_mae_mps": e_sweep["mae_mps"],
                      "final_mae_mps": e["mae_mps"], "final_rmse_mps": e["rmse_mps"],
                      "cmpe_final": cm[-1]}
    return out


def linear_array_report(seeds=(30, 31, 32)):
    """Linear array with a flat lens (128 elements at 0.2 mm, the Table I lens) on
    seeded bi-layer phantoms (1575 m/s over 1490/1516/1540 m/s): the plain method
    (sweep + Adam) with each lens model of the beamformer, sound-speed MAE over the
    imaged depths against the true medium, and the time of one loss_and_grad."""
    import torch
    import afsynth
    from paper_2608_06853_amd import _lib, metrics, warmstart, workloads
    cfg = afsynth.configs.L1
    z_lo = cfg.array.d_lens + cfg.img.depth_min
    z_hi = cfg.array.d_lens + cfg.img.depth_max
    rows, timing = [], None
    for sd in seeds:
        row = {"seed": sd}
        for model in workloads.LENS_MODELS:
            bf, iq, med = workloads.build(cfg, seed=sd, lens_model=model)
            row["phantom_speed"] = float(med.layer_c[-1])
            if timing is None:
                lp = workloads.loss_params(cfg)
                terms = bf.empty_terms()
                grad = torch.empty(bf.grid.shape, device=bf.device)
                bf.ctx.loss_and_grad(iq, lp, terms, grad)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(10):
                    bf.ctx.loss_and_grad(iq, lp, terms, grad)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) / 10 * 1e3
                n, P = cfg.array.n_elem, bf.n_points
                timing = {"ms_per_loss_and_grad": round(ms, 3),
                          "nominal_Gsamples_per_s": round(n * n * P / ms / 1e6, 1)}
            s, cm, times, t_sweep, best = warmstart.run_plain(bf, iq, cfg, cfg.method.n_iter)
            c_true = workloads.true_speed_nodes(cfg, med, bf.grid)
            zs = bf.grid.z0 + bf.grid.dz * np.arange(bf.grid.nz)
            keep = (zs >= z_lo) & (zs <= z_hi)
            e = metrics.speed_errors(s.cpu().numpy()[keep], c_true[keep])
            e_sw = metrics.speed_errors(np.full((int(keep.sum()), bf.grid.nx), 1.0 / best),
                                        c_true[keep])
            row[model] = {"sweep_best_speed": best, "sweep_mae_mps": round(e_sw["mae_mps"], 2),
                          "final_mae_mps": round(e["mae_mps"], 2), "cmpe_final": cm[-1],
                          "seconds": round(times[-1], 3)}
            del bf, iq
        rows.append(row)
    summ = {m: {"sweep_mae_mps": round(float(np.mean([r[m]["sweep_mae_mps"] for r in rows])), 2),
                "final_mae_mps": round(float(np.mean([r[m]["final_mae_mps"] for r in rows])), 2)}
            for m in workloads.LENS_MODELS}
    return {"timing": timing, "summary": summ, "media": rows}


def grid_init_report(seeds=range(9000, 9008)):
    """Model initialisation on the static grid (laid out once for 1500 m/s) against
    the dynamic grid (moved with every swept speed): the speed each selects against
    the mean true speed of the grid nodes, on held-out random two-layer media of
    the tiny array and on the clinical medium, and how often a choice falls on an
    end of the sweep range.  The sweep curves of the clinical medium are kept."""
    import afsynth
    from paper_2608_06853_amd import autofocus as af, workloads
    speeds = af.sweep_speeds()
    ends = (float(speeds[0]), float(speeds[-1]))
    rows, curves = [], {}
    cases = [(afsynth.configs.C4, int(sd)) for sd in seeds] + [(afsynth.configs.C2, None)]
    for cfg, sd in cases:
        bf, iq, med = workloads.build(cfg, seed=sd)
        base = bf.img
        lp = workloads.loss_params(cfg)
        c_true = float(workloads.true_speed_nodes(cfg, med, bf.grid).mean())
        row = {"config": cfg.name, "seed": sd, "c_mean_true": round(c_true, 5)}
        for mode in ("dynamic", "static"):
            bf.set_imaging(base, keep_slowness=False)
            _, vals, best = af.sweep(bf, iq, lp, cfg.acq.fc, dynamic=(mode == "dynamic"))
            row[f"{mode}_best"] = best
            row[f"{mode}_err_mps"] = round(1000.0 * abs(best - c_true), 2)
            row[f"{mode}_at_range_end"] = best in ends
            if sd is None:
                curves[mode] = [round(float(v), 5) for v in vals]
        rows.append(row)
        del bf, iq
    summ = {}
    for mode in ("dynamic", "static"):
        summ[f"{mode}_mean_err_mps"] = round(float(np.mean([r[f"{mode}_err_mps"] for r in rows])), 2)
        summ[f"{mode}_range_end_picks"] = int(sum(r[f"{mode}_at_range_end"] for r in rows))
    return {"summary": summ, "media": rows, "speeds": [round(float(c), 3) for c in speeds],
            "clinical_curves": curves}


def refraction_search_report(ns=(8, 32, 128), reps: int = 5):
    """The discrete N_search refraction search against the continuous root on the
    clinical geometry: deviation of the travel times, of the loss, and the time of
    one loss_and_grad."""
    import torch
    import afsynth
    from paper_2608_06853_amd import _lib, workloads
    cfg = afsynth.configs.C2
    bf, iq, med = workloads.build(cfg)
    lp = workloads.loss_params(cfg)
    terms = bf.empty_terms()
    grad = torch.empty(bf.grid.shape, device=bf.device)

    def run(n):
        bf.ctx.set_refraction_search(n)
        bf.ctx.loss_and_grad(iq, lp, terms, grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            bf.ctx.loss_and_grad(iq, lp, terms, grad)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / reps * 1e3
        return ms, float(terms[_lib.TERM_CMPE].item()), bf.travel_times()

    ms0, cm0, T0 = run(0)
    ok = torch.isfinite(T0)
    out = {"continuous": {"ms_per_loss_and_grad": round(ms0, 3), "cmpe": cm0}}
    for n in ns:
        ms, cm, T = run(n)
        rel = ((T - T0).abs() / T0)[ok]
        out[f"n_search_{n}"] = {"ms_per_loss_and_grad": round(ms, 3), "cmpe": cm,
                                "T_rel_dev_median": float(rel.median().item()),
                                "T_rel_dev_max": float(rel.max().item())}
        del T, rel
    bf.ctx.set_refraction_search(0)
    return out


def s_to_target_report(n_heldout: int = 8):
    """Wall-clock to the plain method's final CMPE, learned warm start vs plain
    initialisation, on held-out media of the network's training distribution and
    on the largest workload; plus the initial-map RMSE of both networks."""
    import afsynth
    from paper_2608_06853_amd import warmstart
    nets = {k: warmstart.load_network(k) for k in ("plain", "true")}
    keep = ("target_cmpe", "plain_seconds", "plain_iters", "plain_best_speed", "learned_seconds",
            "learned_iters", "learned_reached", "learned_start", "learned_speeds_evaluated",
            "learned_cmpe_map", "learned_cmpe_local", "speedup", "plain_rmse_mps",
            "learned_rmse_mps")
    out = {}
    rows = [warmstart.s_to_target(afsynth.configs.C4, nets["plain"], seed=9000 + k)
            for k in range(n_heldout)]
    tp = sum(r["plain_seconds"] for r in rows)
    tl = sum(r["learned_seconds"] for r in rows)
    out["c4_heldout_summary"] = {
        "media": n_heldout, "plain_seconds_total": tp, "learned_seconds_total": tl,
        "speedup_total": tp / tl if tl > 0 else None,
        "reached": sum(bool(r["learned_reached"]) for r in rows),
        "starts": {k: sum(r["learned_start"] == k for r in rows) for k in ("map", "local_sweep", "sweep")}}
    out["c4_heldout"] = [{k: r[k] for k in keep} for r in rows]
    r = warmstart.s_to_target(afsynth.configs.C5, nets["plain"])
    out["c5_largest"] = {k: r[k] for k in keep}
    out["c4_heldout_initial_rmse_mps"] = warmstart.evaluate_init(nets, range(9000, 9008))
    return out


def conv_counts(B: int):
    """Algorithmic FLOPs and compulsory HBM bytes per call family of one forward
    and one backward over a batch of B feature maps, from the layer shapes
    (unpadded K = 9 Cin; BF16 activations, FP32 network output)."""
    from paper_2608_06853_amd import cnn
    fl = {"conv_fwd": 0.0, "conv_bwd_data": 0.0, "conv_bwd_weight": 0.0}
    by = dict(fl)
    h, w = cnn.FEAT_H, cnn.FEAT_W
    for li, (ci, co, st, relu) in enumerate(cnn.LAYERS):
        ho, wo = cnn.out_size(h, st), cnn.out_size(w, st)
        mac = 2.0 * B * ho * wo * co * 9 * ci
        x_b, y_b = 2.0 * B * h * w * ci, (2.0 if relu else 4.0) * B * ho * wo * co
        g_b = 2.0 * B * ho * wo * co
        fl["conv_fwd"] += mac
        by["conv_fwd"] += x_b + y_b
        fl["conv_bwd_weight"] += mac
        by["conv_bwd_weight"] += x_b + g_b
        if li > 0:       # input gradient: read dout and the ReLU mask, write din
            fl["conv_bwd_data"] += mac
            by["conv_bwd_data"] += g_b + 2 * x_b
        h, w = ho, wo
    return fl, by


def cnn_report(reps: int = 20):
    """The learned warm start's BF16 MFMA convolutions on random inputs of the
    feature shape: inference (forward) at batch 256 and a training step (forward,
    loss, backward, Adam) at the training batch of 32 and at 256.  Per call family:
    time per pass from HIP events, achieved TFLOP/s and GB/s, and the fraction of
    the bound that applies (HBM: the layers carry 40 FLOP per compulsory byte,
    below the BF16 ridge of 312)."""
    import torch
    from paper_2608_06853_amd import _lib, cnn
    ctx = _lib.Context(0)
    net = cnn.WarmStartNet(ctx, seed=0)
    g = torch.Generator(device="cuda").manual_seed(0)
    out = {}
    for mode, B in (("forward", 256), ("train_step", 32), ("train_step", 256)):
        x = torch.randn((B, cnn.FEAT_H, cnn.FEAT_W, 2), device="cuda",
                        generator=g).to(torch.bfloat16)
        lab = 0.1 * torch.randn((B, cnn.OUT_H, cnn.OUT_W), device="cuda", generator=g)
        step = (lambda: net.forward(x, B)) if mode == "forward" else \
            (lambda: net.train_step(x, lab, B, 1e-4))
        for _ in range(3):
            step()
        torch.cuda.synchronize()
        ctx.set_profiling(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        prof = ctx.profile_read()
        ctx.set_profiling(False)
        fl, by = conv_counts(B)
        fam = {}
        for k in fl:
            if k not in prof:
                continue
            t = prof[k][0] / reps / 1e3
            tf, gb = fl[k] / t / 1e12, by[k] / t / 1e9
            fam[k] = {"ms": round(t * 1e3, 4), "launches": prof[k][1] // reps,
                      "TFLOP_per_s": round(tf, 2), "GB_per_s": round(gb, 1),
                      "hbm_frac": round(gb / PEAK_HBM_GBS, 3),
                      "bf16_mfma_frac": round(tf / PEAK_BF16_TFLOPS, 4)}
        out[f"{mode}_b{B}"] = {"ms_per_pass": round(wall * 1e3, 4),
                               "samples_per_s": round(B / wall, 1), "families": fam}
        del x, lab
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library drives a single GPU "
              f"(--gpus {args.gpus} requested; the path would shard by points)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n}))
        return
    import afsynth
    from paper_2608_06853_amd import _lib

    cfg = afsynth.config_by_name(args.config)
    met = cfg.method
    bf, iq, med = workload(cfg)
    lp = _lib.loss_params(met.w1, met.kx1, met.kz1, met.w2, met.kx2, met.kz2, met.rho_thresh,
                          met.w_sb, 1.0)
    terms = bf.empty_terms()
    grad = torch.empty((met.nz, met.nx), device="cuda")
    for _ in range(args.warmup):
        bf.ctx.loss_and_grad(iq, lp, terms, grad)
    torch.cuda.synchronize()
    bf.ctx.set_profiling(True)
    bf.ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bf.ctx.loss_and_grad(iq, lp, terms, grad)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = bf.ctx.profile_read()
    bf.ctx.set_profiling(False)
    tv = terms.cpu().numpy()
    if not np.isfinite(tv[_lib.TERM_TOTAL]) or not torch.isfinite(grad).all():
        raise SystemExit("non-finite loss or gradient")

    n = cfg.array.n_elem
    P = bf.n_points
    nominal = float(n * n * P)
    active_samples = float(bf.ctx.query(_lib.Q_ACTIVE_SAMPLES))
    active_rays = float(bf.ctx.query(_lib.Q_ACTIVE_PAIRS))
    value = nominal * args.steps / dt / 1e9

    # dominant kernel and its roofline (per-launch average from HIP events)
    dom = max(prof, key=lambda k: prof[k][0])
    ms_tot, calls = prof[dom]
    avg_s = ms_tot / calls / 1e3
    units = {"das_fwd": active_samples, "das_adj": active_samples,
             "table": active_rays * (met.n_seg + 1), "path_adj": active_rays * (met.n_seg + 1)}
    roof = None
    if dom in FLOPS_PER_UNIT:
        ach = FLOPS_PER_UNIT[dom] * units[dom] / avg_s / 1e12
        tr = measured_traffic(cfg.name, dom)
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                "peak_nonpacked": PEAK_FP32_NONPACKED_TFLOPS,
                "frac_nonpacked": round(ach / PEAK_FP32_NONPACKED_TFLOPS, 4),
                "flop_per_unit": FLOPS_PER_UNIT[dom], "units_per_launch": units[dom],
                "traffic": tr, "traffic_unit": "bytes per launch",
                "avg_launch_ms": round(avg_s * 1e3, 4),
                "valu_issue": measured_issue(cfg.name, dom, units[dom])}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated FSA data of a seeded random "
                + ("bi-layer phantom)" if afsynth.is_linear(cfg.array) else "liver-like medium)"),
        "config": {"workload": f"{cfg.name}: {n} el "
                               + (f"linear pitch {cfg.array.pitch} mm, flat lens, "
                                  if afsynth.is_linear(cfg.array)
                                  else f"curvilinear R {cfg.array.radius} mm, ")
                               + f"{n} tx, "
                               f"{cfg.acq.n_samples} IQ samples, {cfg.img.n_depth}x{cfg.img.n_angle} px "
                               f"x 3x3 patch to {cfg.img.depth_max} mm, {met.nx}x{met.nz} slowness grid, "
                               f"one loss_and_grad per step",
                   "nominal_samples": nominal, "active_samples": active_samples,
                   "active_rays": active_rays, "tiles": bf.ctx.query(_lib.Q_TILES),
                   "tile_active_elements_max": bf.ctx.query(_lib.Q_NA_MAX),
                   "tile_active_blocks_max": bf.ctx.query(_lib.Q_NBA_MAX),
                   "active_Gsamples_per_s":
                       round(active_samples * args.steps / dt / 1e9, 2)},
        "roofline": roof,
        "kernels_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in sorted(prof.items())},
        "loss_terms": [float(x) for x in tv[:7]],
    }
    del bf, iq
    torch.cuda.empty_cache()
    if not args.no_autofocus:
        t0 = time.perf_counter()
        for key, fn in (("plain_loop", plain_loop_report), ("memory", memory_report),
                        ("lens_models", lens_model_report),
                        ("linear_array", linear_array_report),
                        ("grid_init", grid_init_report),
                        ("refraction_search", refraction_search_report),
                        ("cnn_kernels", cnn_report),
                        ("s_to_target", s_to_target_report)):
            if args.reports != "all" and key not in args.reports.split(","):
                continue
            print(f"report {key}", file=sys.stderr, flush=True)
            out[key] = fn()
        out["autofocus_report_seconds"] = round(time.perf_counter() - t0, 1)
    if args.cpu_pixels > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_pixels)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
