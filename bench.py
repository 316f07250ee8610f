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
PEAK_FP32_TFLOPS = 157.3        # 256 CU x 2.4 GHz x 256 FP32 flop/clk/CU
PEAK_HBM_GBS = 8000.0

# Algorithmic FP32 operations per unit (Measurement).
FLOPS_PER_UNIT = {
    "das_fwd": 14.0,     # per active (t, r, point) sample: interpolate (6) + rotate-accumulate (8)
    "das_adj": 22.0,     # per active sample: interpolate + derivative (12) + rotate (6) + Re/acc (4)
    "table": 64.0,       # per ray point: bicubic weights (20) + 16 taps (40) + position (4)
    "path_adj": 44.0,    # per ray point: weights (20) + 16 scatter products (20) + position (4)
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2_clinical")
    ap.add_argument("--cpu-pixels", type=int, default=192,
                    help="pixels of the bounded oracle sample (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (HBM counter scale)")
    return ap.parse_args()


def workload(cfg, device=0):
    from paper_2608_06853_amd import workloads
    return workloads.build(cfg, device=device)


def cpu_baseline(cfg, n_pix_sample: int):
    """The FP64 oracle as it stands on a bounded sample of the same workload: the
    full array and channel-data shape, ``n_pix_sample`` pixels spread over the image."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import afsynth
    import problems
    from oracle import model

    prob = problems.problem(cfg, depth_scale_max=1.74 / 1.54)
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(prob.centres.shape[0], n_pix_sample, replace=False))
    prob = model.Problem(**{**prob.__dict__, "centres": prob.centres[sel], "_cache": {}})
    prob.iq = afsynth.random_iq(cfg.array.n_elem, cfg.acq.n_samples, seed=cfg.seed)
    x0, z0, dx, dz, nx, nz = prob.grid
    s = np.full((nz, nx), 1.0 / 1.54)
    lp = problems.loss_params(cfg)
    t0 = time.perf_counter()
    model.loss_and_grad(prob, s, lp)
    dt = time.perf_counter() - t0
    samples = cfg.array.n_elem ** 2 * n_pix_sample * prob.n_patch
    return dict(value=samples / dt / 1e9, unit=UNIT, cores=1, kind="oracle",
                sample=f"{n_pix_sample} of {cfg.img.n_depth * cfg.img.n_angle} pixels "
                       f"(x{prob.n_patch} points), full {cfg.array.n_elem}x{cfg.array.n_elem}"
                       f"x{cfg.acq.n_samples} channel data, one loss_and_grad in "
                       f"{dt:.1f} s (numpy single thread)")


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build is single-GPU by design "
              f"(--gpus {args.gpus} requested; see DESIGN.md for how the path shards)",
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
        roof = {"bound": "alu", "kernel": dom, "achieved": round(ach, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                "traffic": None, "avg_launch_ms": round(avg_s * 1e3, 4)}

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (GPU-simulated FSA data of a seeded random liver-like medium)",
        "config": {"workload": f"{cfg.name}: {n} el curvilinear R {cfg.array.radius} mm, {n} tx, "
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
    if args.cpu_pixels > 0:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_pixels)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
