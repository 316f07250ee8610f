"""Writes ``c2_clinical_loss_grad.json``: the FP64 oracle's loss terms and slowness
gradient of the whole clinical workload in the benchmark's launch configuration
(128 elements, 128 transmits, 2560 samples, 256 x 256 pixels x 3 x 3 points to
160 mm, 32 x 32 grid covering every speed of the dynamic-grid sweep).

Inputs: channel data the oracle simulates (oracle.simulate, 64 ray segments)
from the clinical medium with 2000 point scatterers (the configuration's seed;
fewer than its speckle density, so that the simulation takes seconds), the true
slowness of that medium on the grid perturbed by 1 % seeded noise, and the
configured loss parameters (CMPE threshold 0.9).  Coherent echoes keep the
gradient a coherent sum over the valid pairs; on noise data every pair adds a
term of random sign, and the few pairs whose validity FP32 and FP64 judge
differently then move it by about sqrt(flips / n_valid).  The oracle evaluates
disjoint chunks of pixels in parallel processes on every host core
(oracle.model.loss_and_grad_parts) and combines them
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
N_SCAT = 2000
SIM_NSEG = 64
DEPTH_SCALE = 1.740 / 1.540
RHO_BAND = 1e-4


def inputs(workers=None):
    """(cfg, oracle problem with its channel data, slowness, loss parameters) of the
    comparison; the GPU test builds the same inputs."""
    cfg = afsynth.config_by_name(CONFIG).with_(n_scat_random=N_SCAT)
    med = afsynth.medium_for(cfg)
    prob = problems.problem(cfg, depth_scale_max=DEPTH_SCALE)
    prob.iq = problems.simulate_iq_parallel(cfg, med, SIM_NSEG, workers)
    s_true = problems.true_slowness(cfg, med, prob)
    rng = np.random.default_rng(cfg.seed + 11)
    s = (s_true * (1.0 + 0.01 * rng.standard_normal(s_true.shape))).astype(np.float32)
    lp = problems.loss_params(cfg)
    return cfg, prob, s, lp


_state = {}


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
    cfg, prob, s, lp = inputs(args.workers)
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
    out = {"config": CONFIG, "n_scat": N_SCAT, "sim_nseg": SIM_NSEG,
           "iq": "oracle.simulate of afsynth.medium_for(c2_clinical, n_scat_random=2000)",
           "slowness": "true slowness x (1 + 0.01 N(0,1)), seed + 11",
           "rho_thresh": float(lp.rho_thresh),
           "rho_band": RHO_BAND, "n_near": int(sum(p["n_near"] for p in parts)),
           "n_pix": n_pix, "terms": {k: float(v) for k, v in terms.items()},
           "grad": [[float(v) for v in row] for row in g],
           "seconds": round(time.perf_counter() - t0, 1), "workers": args.workers}
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote", OUT, terms, f"{out['seconds']} s on {args.workers} processes", flush=True)


if __name__ == "__main__":
    main()
