"""FP64 reference of the warm-start network (test infrastructure only).

Network (the learned initialisation of the slowness map; not in the paper):
conv3x3(2 -> 32, stride 1) + ReLU, conv3x3(32 -> 32, stride 2) + ReLU,
conv3x3(32 -> 32, stride 2) + ReLU, conv3x3(32 -> 1, stride 1); zero padding 1,
tensors NHWC, weights [Cout][3][3][Cin].  Training loss: scale * sum (out - label)^2.

Each convolution is the definition written out: for output pixel (y, x) and
tap (ky, kx), the padded input at (y * stride + ky, x * stride + kx) times
w[:, ky, kx, :]; the backward pass is its chain rule.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(2, 32, 1, True), (32, 32, 2, True), (32, 32, 2, True), (32, 1, 1, False)]


def out_size(n: int, stride: int) -> int:
    return (n - 1) // stride + 1


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    B, H, W, Ci = x.shape
    Co = w.shape[0]
    Ho, Wo = out_size(H, stride), out_size(W, stride)
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1] = x
    out = np.broadcast_to(b, (B, Ho, Wo, Co)).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            patch = xp[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride]
            out += patch @ w[:, ky, kx, :].T
    return out


def conv3x3_backward(x: np.ndarray, w: np.ndarray, stride: int, dout: np.ndarray):
    """(dx, dw, db) of sum(dout * conv3x3(x, w, b))."""
    B, H, W, Ci = x.shape
    Ho, Wo = dout.shape[1], dout.shape[2]
    xp = np.zeros((B, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for ky in range(3):
        for kx in range(3):
            sl = (slice(None), slice(ky, ky + stride * (Ho - 1) + 1, stride),
                  slice(kx, kx + stride * (Wo - 1) + 1, stride))
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwi->oi", dout, xp[sl])
            dxp[sl] += dout @ w[:, ky, kx, :]
    return dxp[:, 1:-1, 1:-1], dw, dout.sum(axis=(0, 1, 2))


def forward(params, x):
    """params: list of (w, b) per layer.  Returns (output, activations per layer input)."""
    acts = [x]
    h = x
    for (w, b), (_, _, stride, relu) in zip(params, LAYERS):
        z = conv3x3(h, w, b, stride)
        h = np.maximum(z, 0.0) if relu else z
        acts.append(h)
    return h, acts


def backward(params, acts, dout):
    """Gradients [(dw, db)] for every layer given d loss / d output."""
    grads = [None] * len(params)
    g = dout
    for li in reversed(range(len(params))):
        w, _ = params[li]
        _, _, stride, _ = LAYERS[li]
        dx, dw, db = conv3x3_backward(acts[li], w, stride, g)
        grads[li] = (dw, db)
        if li > 0:
            g = dx * (acts[li] > 0)  # ReLU of the layer below
    return grads


def mse(out, label, scale):
    d = out - label
    return float(scale * np.sum(d * d)), 2.0 * scale * d
