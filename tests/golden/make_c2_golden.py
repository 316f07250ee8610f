"""Writes ``c2_clinical_loss_grad.json``: the FP64 oracle's loss terms and slowness
gradient of the whole clinical workload in the benchmark's launch configuration
(128 elements, 128 transmits, 2560 samples, 256 x 256 pixels x 3 x 3 points to
160 mm, 32 x 32 grid covering every speed of the dynamic-grid sweep).

Inputs: seeded circular Gaussian channel data (afsynth.random_iq, seed of the
configuration) and a seeded smooth slowness (problems.smooth_slowness), CMPE
threshold 0.5 (noise data have few pairs above the configured 0.9).  The
oracle evaluates disjoint chunks of pixels in parallel processes on every host
core (oracle.model.loss_and_grad_parts) and combines them
(oracle.model.combine_parts).  Nothing here calls the GPU library.

    python tests/golden/make_c2_golden.py [--workers N] [--chunk PIXELS]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.join(ROOT, "tests")):
    if p not in sys.path:
        sys.path.insert(0, p)

import afsynth  # noqa: E402
import problems  # noqa: E402
from oracle import model  # noqa: E402

OUT = os.path.join(HERE, "c2_clinical_loss_grad.json")
CONFIG = "c2_clinical"
DEPTH_SCALE = 1.740 / 1.540
RHO = 0.5
RHO_BAND = 1e-4

_state = {}


def setup():
    cfg = afsynth.config_by_name(CONFIG)
    prob = problems.problem(cfg, depth_scale_max=DEPTH_SCALE)
    prob.iq = afsynth.random_iq(cfg.array.n_elem, cfg.acq.n_samples, seed=cfg.seed)
    s = problems.smooth_slowness(prob.grid, cfg.seed)
    lp = problems.loss_params(cfg)
    lp = model.LossParams(**{**lp.__dict__, "rho_thresh": RHO})
    return cfg, prob, s, lp


def _init():
    from threadpoolctl import threadpool_limits
    _state["limits"] = threadpool_limits(limits=1)   # one thread per process


def _work(bounds):
    prob, s, lp = _state["prob"], _state["s"], _state["lp"]
    q0, q1 = bounds
    sub = model.Problem(**{**prob.__dict__, "centres": prob.centres[q0:q1], "_cache": {}})
    return model.loss_and_grad_parts(sub, s.astype(np.float64), lp, rho_band=RHO_BAND)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    ap.add_argument("--chunk", type=int, default=256)
    args = ap.parse_args()
    cfg, prob, s, lp = setup()
    _state.update(prob=prob, s=s, lp=lp)
    n_pix = prob.centres.shape[0]
    chunks = [(q, min(q + args.chunk, n_pix)) for q in range(0, n_pix, args.chunk)]
    t0 = time.perf_counter()
    parts = []
    with mp.get_context("fork").Pool(args.workers, initializer=_init) as pool:
        for k, part in enumerate(pool.imap(_work, chunks)):
            parts.append(part)
            if (k + 1) % 16 == 0:
                print(f"  {k + 1}/{len(chunks)} chunks, {time.perf_counter() - t0:.0f} s",
                      flush=True)
    terms, g = model.combine_parts(parts, s, lp, prob.grid)
    out = {"config": CONFIG, "iq": f"afsynth.random_iq(seed={cfg.seed})",
           "slowness": f"problems.smooth_slowness(seed={cfg.seed})", "rho_thresh": RHO,
           "rho_band": RHO_BAND, "n_near": int(sum(p["n_near"] for p in parts)),
           "n_pix": n_pix, "terms": {k: float(v) for k, v in terms.items()},
           "grad": [[float(v) for v in row] for row in g],
           "seconds": round(time.perf_counter() - t0, 1), "workers": args.workers}
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, terms, f"{out['seconds']} s on {args.workers} processes", flush=True)


if __name__ == "__main__":
    main()
