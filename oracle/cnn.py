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


# --- the glue around the network: its input features and its output resampling ---------------
# (the learned warm start is an extension; the paper has no learned part)

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Nearest BF16 value of every entry (ties to even), returned in float64.

    BF16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of an
    IEEE single; the value is first rounded to single precision and its low 16
    bits then rounded away to nearest even."""
    b = np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(maps: np.ndarray, shift: np.ndarray, scale: np.ndarray) -> np.ndarray:
    """Network input from channel-major feature maps [C][n]: the entries
    (maps[c][i] - shift[c]) * scale[c] in pixel-major order [n][C] (not rounded)."""
    maps = np.asarray(maps, dtype=np.float64)
    return ((maps - shift[:, None]) * scale[:, None]).T.copy()


def polar_to_grid(pmap: np.ndarray, r0: float, dr: float, t0: float, dt: float, nx: int,
                  nz: int, x0: float, z0: float, dx: float, dz: float, s_base: float,
                  scale: float, s_lo: float, s_hi: float) -> np.ndarray:
    """Slowness on the node grid [nz][nx] from a polar map [nr][nt] whose rows are
    radii r0 + a dr and columns polar angles t0 + b dt (angle from the z axis
    towards x).  At node (x0 + j dx, z0 + i dz): the fractional map indices of its
    radius and angle, each clamped to the map; bilinear interpolation between the
    four surrounding map entries; s_base + scale * value, clamped to [s_lo, s_hi]."""
    pmap = np.asarray(pmap, dtype=np.float64)
    nr, nt = pmap.shape
    out = np.empty((nz, nx))
    for i in range(nz):
        for j in range(nx):
            x, z = x0 + j * dx, z0 + i * dz
            u = min(max((np.hypot(x, z) - r0) / dr, 0.0), nr - 1.0)
            v = min(max((np.arctan2(x, z) - t0) / dt, 0.0), nt - 1.0)
            a, b = min(int(u), nr - 2), min(int(v), nt - 2)
            fu, fv = u - a, v - b
            val = ((1 - fu) * ((1 - fv) * pmap[a, b] + fv * pmap[a, b + 1])
                   + fu * ((1 - fv) * pmap[a + 1, b] + fv * pmap[a + 1, b + 1]))
            out[i, j] = min(max(s_base + scale * val, s_lo), s_hi)
    return out
