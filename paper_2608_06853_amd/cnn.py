"""Learned warm start of the slowness map.

A four-layer 3x3 CNN maps two feature maps of a homogeneous 1540 m/s beamform
(integrated CMPE and coherence factor on a 128 x 128 polar pixel grid) to a
32 x 32 polar map of the slowness deviation from 1/1540 us/mm.  Every
convolution, its gradients, the loss and the Adam update run in libaf.so on the
BF16 matrix cores (FP32 accumulate); this module holds parameters and buffers
(torch tensors) and sequences the library calls.

Two networks of this shape are trained on the same features: one on the true
slowness of each medium (how close the initial map is to the truth) and one on
the plain method's converged solution (what the objective prefers, used as the
warm start).  The prediction is resampled onto the slowness grid and checked
against the homogeneous initial guess: if its loss is higher, the plain
adaptive-grid initialisation is used instead.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

import afsynth
from . import _lib, autofocus as af, workloads

LAYERS = [(2, 32, 1, True), (32, 32, 2, True), (32, 32, 2, True), (32, 1, 1, False)]
FEAT_H = FEAT_W = 128
OUT_H = OUT_W = 32
DS_SCALE = 0.03          # us/mm per unit of network output
S_BASE = 1.0 / 1.540
SPEED_MIN, SPEED_MAX = 1.340, 1.740   # mm/us, the global sweep's range


def out_size(n, stride):
    return (n - 1) // stride + 1


class WarmStartNet:
    """Parameters, packed BF16 operands, Adam state and per-batch buffers."""

    def __init__(self, ctx: _lib.Context, seed: int = 0, device: int = 0):
        self.ctx = ctx
        self.dev = torch.device("cuda", device)
        rng = np.random.default_rng(seed)
        self.w, self.b, self.wp, self.wtp = [], [], [], []
        for ci, co, _, _ in LAYERS:
            std = math.sqrt(2.0 / (9 * ci))
            self.w.append(torch.from_numpy((rng.standard_normal((co, 9 * ci)) * std)
                                           .astype(np.float32)).to(self.dev))
            self.b.append(torch.zeros(co, device=self.dev))
            kp, ktp = ctx.conv_shapes(ci, co)
            self.wp.append(torch.empty(32 * kp, device=self.dev, dtype=torch.bfloat16))
            self.wtp.append(torch.empty(32 * ktp, device=self.dev, dtype=torch.bfloat16))
        self.params = self.w + self.b
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.step_count = 0
        self._B = None
        self.pack()

    # --- parameters --------------------------------------------------------------------
    def pack(self):
        for (ci, co, _, _), w, wp, wtp in zip(LAYERS, self.w, self.wp, self.wtp):
            self.ctx.conv3x3_pack(ci, co, w, wp, wtp)

    def state(self) -> dict:
        return {f"w{i}": w.cpu().numpy() for i, w in enumerate(self.w)} | \
               {f"b{i}": b.cpu().numpy() for i, b in enumerate(self.b)}

    def load(self, st: dict):
        for i in range(len(LAYERS)):
            self.w[i].copy_(torch.from_numpy(np.asarray(st[f"w{i}"], dtype=np.float32)))
            self.b[i].copy_(torch.from_numpy(np.asarray(st[f"b{i}"], dtype=np.float32)))
        self.pack()

    # --- buffers -------------------------------------------------------------------------
    def _alloc(self, B: int):
        if self._B == B:
            return
        self._B = B
        h, w = FEAT_H, FEAT_W
        self.shapes = []           # (H, W) of each layer input
        self.acts = []             # layer outputs (BF16), last layer FP32
        for li, (ci, co, st, relu) in enumerate(LAYERS):
            self.shapes.append((h, w))
            h, w = out_size(h, st), out_size(w, st)
            if relu:
                self.acts.append(torch.empty(B * h * w * co, device=self.dev, dtype=torch.bfloat16))
        self.out = torch.empty(B * h * w, device=self.dev)
        self.gouts = []            # d loss / d pre-activation of each layer (BF16)
        for li, (ci, co, st, relu) in enumerate(LAYERS):
            hh, ww = self.shapes[li]
            self.gouts.append(torch.empty(B * out_size(hh, st) * out_size(ww, st) * co,
                                          device=self.dev, dtype=torch.bfloat16))
        self.loss_parts = torch.empty((B * h * w + 255) // 256, device=self.dev)

    # --- forward / backward ----------------------------------------------------------------
    def forward(self, x: torch.Tensor, B: int) -> torch.Tensor:
        """x: [B][128][128][2] BF16.  Returns the [B][32][32] FP32 output."""
        self._alloc(B)
        inp = x
        for li, (ci, co, st, relu) in enumerate(LAYERS):
            H, W = self.shapes[li]
            if relu:
                self.ctx.conv3x3_fwd(B, H, W, ci, co, st, True, inp, self.wp[li], self.b[li],
                                     out=self.acts[li])
                inp = self.acts[li]
            else:
                self.ctx.conv3x3_fwd(B, H, W, ci, co, st, False, inp, self.wp[li], self.b[li],
                                     outf=self.out)
        self._x = x
        return self.out.view(B, OUT_H, OUT_W)

    def backward(self, B: int):
        """Gradients of the last ``loss`` call into self.grads."""
        n = len(LAYERS)
        for li in reversed(range(n)):
            ci, co, st, relu = LAYERS[li]
            H, W = self.shapes[li]
            x_in = self._x if li == 0 else self.acts[li - 1]
            self.ctx.conv3x3_bwd_weight(B, H, W, ci, co, st, x_in, self.gouts[li], self.grads[li],
                                        self.grads[n + li])
            if li > 0:
                self.ctx.conv3x3_bwd_data(B, H, W, ci, co, st, self.gouts[li], self.wtp[li],
                                          self.acts[li - 1], self.gouts[li - 1])

    def loss(self, label: torch.Tensor, B: int) -> torch.Tensor:
        """Mean squared error of the last forward against ``label`` [B][32][32]; sets the
        output gradient.  Returns the loss as a device scalar."""
        n = B * OUT_H * OUT_W
        self.ctx.mse_loss(self.out, label.reshape(-1), 1.0 / n, self.loss_parts, self.gouts[-1])
        return self.loss_parts.sum()

    def adam(self, lr: float):
        self.step_count += 1
        ap = _lib.adam_params(lr=lr)
        for p, m, v, g in zip(self.params, self.m, self.v, self.grads):
            self.ctx.adam_update(ap, self.step_count, p, m, v, g)
        self.pack()

    def train_step(self, x, label, B, lr) -> torch.Tensor:
        self.forward(x, B)
        loss = self.loss(label, B)
        self.backward(B)
        self.adam(lr)
        return loss


# --- features, labels and the output grid ----------------------------------------------------
@dataclass
class OutGrid:
    """Polar 32 x 32 output grid: rows are radii r0 + a dr, columns angles t0 + b dt."""
    r0: float
    dr: float
    t0: float
    dt: float

    @staticmethod
    def for_config(cfg) -> "OutGrid":
        arr, img = cfg.array, cfg.img
        rl = afsynth.lens_radius(arr)
        th0, th1 = afsynth.element_span(arr)
        dr = (img.depth_max - img.depth_min) / OUT_H
        dt = (th1 - th0) / OUT_W
        return OutGrid(r0=rl + img.depth_min + 0.5 * dr, dr=dr, t0=th0 + 0.5 * dt, dt=dt)


def feature_config(cfg):
    """The configuration's array and acquisition with a 128 x 128 pixel grid."""
    from dataclasses import replace
    return cfg.with_(img=replace(cfg.img, n_depth=FEAT_H, n_angle=FEAT_W))


class FeatureMaker:
    """Beamformer at a homogeneous 1540 m/s on the 128 x 128 feature grid."""

    def __init__(self, cfg, device: int = 0):
        self.cfg = feature_config(cfg)
        acqd, imgd, grid, cover = workloads.geometry(self.cfg)
        self.cover = cover
        self.bf = af.Beamformer(acqd, imgd, grid, device)
        self.bf.set_slowness(torch.full(grid.shape, S_BASE, device=self.bf.device))
        self.shift = torch.tensor([0.6, 0.3], device=self.bf.device)
        self.scale = torch.tensor([2.0, 3.0], device=self.bf.device)

    def features(self, iq: torch.Tensor, out: torch.Tensor):
        """out: [128 * 128 * 2] BF16 (NHWC of one sample)."""
        _, maps, _ = self.bf.beamform(iq, blocks=False, maps=True)
        n = maps.numel() // 3  # channels: CMPE map, coherence factor (CMCC unused)
        self.bf.ctx.features(maps[:2 * n], self.shift, self.scale, out)


def label_map(cfg, med, og: OutGrid, sub: int = 4) -> np.ndarray:
    """Mean true slowness deviation over each output bin, in network units [32][32]."""
    fa = (np.arange(sub) + 0.5) / sub - 0.5
    r = og.r0 + og.dr * (np.arange(OUT_H)[:, None] + fa[None, :])        # [32][sub]
    t = og.t0 + og.dt * (np.arange(OUT_W)[:, None] + fa[None, :])
    R = r[:, None, :, None]
    T = t[None, :, None, :]
    x = R * np.sin(T)
    z = R * np.cos(T)
    c = afsynth.sample_speed(med, x, z)
    s = (1.0 / c).mean(axis=(2, 3))
    return ((s - S_BASE) / DS_SCALE).astype(np.float32)


def grid_to_polar(s_grid: np.ndarray, grid: af.Grid, og: OutGrid) -> np.ndarray:
    """Slowness given on the node grid, sampled bilinearly (clamped to the node range)
    at the centres of the polar output bins, in network units [32][32]."""
    r = og.r0 + og.dr * np.arange(OUT_H)[:, None]
    t = og.t0 + og.dt * np.arange(OUT_W)[None, :]
    u = np.clip((r * np.sin(t) - grid.x0) / grid.dx, 0.0, grid.nx - 1.0)
    v = np.clip((r * np.cos(t) - grid.z0) / grid.dz, 0.0, grid.nz - 1.0)
    j0 = np.minimum(u.astype(int), grid.nx - 2)
    i0 = np.minimum(v.astype(int), grid.nz - 2)
    fu, fv = u - j0, v - i0
    sg = np.asarray(s_grid, dtype=np.float64)
    val = ((1 - fv) * ((1 - fu) * sg[i0, j0] + fu * sg[i0, j0 + 1])
           + fv * ((1 - fu) * sg[i0 + 1, j0] + fu * sg[i0 + 1, j0 + 1]))
    return ((val - S_BASE) / DS_SCALE).astype(np.float32)


def make_dataset(cfg, seeds, device: int = 0, progress: bool = False, plain_iters: int = 0):
    """Features [n][128][128][2] BF16 and labels [n][32][32] FP32, on the device.

    Returns (X, Y_true, Y_plain): Y_true is the true slowness of each medium;
    Y_plain (None unless ``plain_iters`` > 0) is the plain method's solution on
    the configuration's own grid (adaptive-grid sweep, then ``plain_iters`` Adam
    steps), both as deviations from 1/1540 in network units."""
    fm = FeatureMaker(cfg, device)
    og = OutGrid.for_config(cfg)
    n = len(seeds)
    X = torch.empty(n, FEAT_H * FEAT_W * 2, device=fm.bf.device, dtype=torch.bfloat16)
    Y = torch.empty(n, OUT_H, OUT_W, device=fm.bf.device)
    Yp = None
    if plain_iters > 0:
        Yp = torch.empty(n, OUT_H, OUT_W, device=fm.bf.device)
        acqd, imgd, grid, _ = workloads.geometry(cfg)
        bfp = af.Beamformer(acqd, imgd, grid, device)
        lp = workloads.loss_params(cfg)
        ap = _lib.adam_params(lr=cfg.method.lr)
    t0 = time.perf_counter()
    for i, sd in enumerate(seeds):
        med = afsynth.medium_for(fm.cfg, int(sd))
        iq = workloads.simulate(fm.bf, fm.cfg, med, fm.cover)
        fm.features(iq, X[i])
        Y[i] = torch.from_numpy(label_map(fm.cfg, med, og)).to(fm.bf.device)
        if plain_iters > 0:
            bfp.set_imaging(imgd)
            af.sweep(bfp, iq, lp, cfg.acq.fc)
            s, _ = af.plain_autofocus(bfp, iq, lp, ap, plain_iters, record_every=0)
            Yp[i] = torch.from_numpy(grid_to_polar(s.cpu().numpy(), grid, og)).to(fm.bf.device)
        if progress and (i + 1) % 256 == 0:
            torch.cuda.synchronize()
            print(f"  dataset {i + 1}/{n}  {time.perf_counter() - t0:.1f} s", flush=True)
    return X.view(n, FEAT_H, FEAT_W, 2), Y, Yp


def train(net: WarmStartNet, X, Y, epochs: int, batch: int = 32, lr: float = 1e-3, seed: int = 0,
          progress: bool = False) -> list:
    """Mini-batch Adam on (X, Y).  Returns the mean loss of every epoch."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(X.device)
        tot = torch.zeros((), device=X.device)
        nb = 0
        for s0 in range(0, n - batch + 1, batch):
            idx = perm[s0:s0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            tot += net.train_step(xb, yb, batch, lr)
            nb += 1
        hist.append(float(tot.item()) / max(nb, 1))
        if progress:
            print(f"  epoch {ep + 1}/{epochs} loss {hist[-1]:.4f}", flush=True)
    return hist


def predict_slowness(net: WarmStartNet, fm: FeatureMaker, iq, cfg, grid: af.Grid) -> torch.Tensor:
    """Warm-start slowness on ``grid`` from channel data ``iq`` of configuration ``cfg``."""
    x = torch.empty(FEAT_H * FEAT_W * 2, device=fm.bf.device, dtype=torch.bfloat16)
    fm.features(iq, x)
    out = net.forward(x.view(1, FEAT_H, FEAT_W, 2), 1)
    og = OutGrid.for_config(cfg)
    s = torch.empty(grid.shape, device=fm.bf.device)
    # the prediction is kept inside the sweep's speed range (1340-1740 m/s)
    fm.bf.ctx.polar_to_grid(out.reshape(-1), OUT_H, OUT_W, og.r0, og.dr, og.t0, og.dt, grid.nx,
                            grid.nz, grid.x0, grid.z0, grid.dx, grid.dz, S_BASE, DS_SCALE,
                            1.0 / SPEED_MAX, 1.0 / SPEED_MIN, s)
    return s
