"""Common-midpoint phase error, speckle brightness and coherence factor.

Paper: Objective Function subsection (CMPE as the focusing loss, taken over
from Simson et al.), Model Implementation subsection (3x3 patch at lambda/2 per
evaluation pixel), the correlation-based filtering threshold of the
hyperparameter table, and the integrated CMPE image of the in-vivo results.
Speckle brightness and coherence factor are the image-quality metrics of the
Model Evaluation subsection.

The exact CMPE definition lives in the cited Simson et al. paper, which is not
at hand, so this module implements a reading of the translating-aperture idea:

* subaperture i spans blocks {i, i+1} (2S elements, stride S), so the image of
  transmit subaperture i and receive subaperture j is the sum of four block-pair
  images;
* the two images of a common-midpoint neighbour pair are X = B_{i,j+1} and
  Y = B_{i+1,j} (both have midpoint (i + j + 1)/2), i, j = 0..Nsub-2;
* per patch q: C = sum_m X_m conj(Y_m), rho = |C| / sqrt(sum|X|^2 sum|Y|^2);
  the pair is valid when both energies exceed MIN_ENERGY = 1e-30 (the smallest
  energy whose pair phase is still differentiable in FP32, where |C|^2 would
  otherwise underflow; any image of physical size is far above it) and
  rho >= rho_thresh;
  its phase error is |arg C| (radians);
* L_CMPE = mean of |arg C| over valid (patch, pair) entries (0 if none);
* the integrated CMPE map is the per-patch mean over its valid pairs;
* validity masks are constants for the gradient; d|x|/dx at 0 is taken as 0.

Points are stored pixel-major: point p = q * M + m for patch point m of pixel q.
"""
from __future__ import annotations

import numpy as np

MIN_ENERGY = 1e-30


def subaperture_images(bblk: np.ndarray) -> np.ndarray:
    """B_{i,j} = sum over blocks {i,i+1} x {j,j+1}; shape [Nb-1][Nb-1][P]."""
    return bblk[:-1, :-1] + bblk[1:, :-1] + bblk[:-1, 1:] + bblk[1:, 1:]


def subaperture_images_adjoint(gsub: np.ndarray) -> np.ndarray:
    """Adjoint of ``subaperture_images`` (block gradient from subaperture gradient)."""
    ns = gsub.shape[0]
    out = np.zeros((ns + 1, ns + 1) + gsub.shape[2:], dtype=gsub.dtype)
    out[:-1, :-1] += gsub
    out[1:, :-1] += gsub
    out[:-1, 1:] += gsub
    out[1:, 1:] += gsub
    return out


def cm_pairs(bsub: np.ndarray, n_patch: int):
    """X, Y of every common-midpoint neighbour pair: arrays [Ns-1][Ns-1][n_pix][M]."""
    ns = bsub.shape[0]
    P = bsub.shape[2]
    X = bsub[0:ns - 1, 1:ns].reshape(ns - 1, ns - 1, P // n_patch, n_patch)
    Y = bsub[1:ns, 0:ns - 1].reshape(ns - 1, ns - 1, P // n_patch, n_patch)
    return X, Y


def cmpe(bsub: np.ndarray, n_patch: int, rho_thresh: float):
    """Per-pair quantities.  Returns dict(C, ex, ey, rho, valid, err) with
    shapes [Ns-1][Ns-1][n_pix]."""
    X, Y = cm_pairs(bsub, n_patch)
    C = np.sum(X * np.conj(Y), axis=-1)
    ex = np.sum(np.abs(X) ** 2, axis=-1)
    ey = np.sum(np.abs(Y) ** 2, axis=-1)
    pos = (ex > MIN_ENERGY) & (ey > MIN_ENERGY)
    rho = np.where(pos, np.abs(C) / np.sqrt(np.where(pos, ex * ey, 1.0)), 0.0)
    valid = pos & (rho >= rho_thresh)
    err = np.abs(np.angle(C))
    return dict(C=C, ex=ex, ey=ey, rho=rho, valid=valid, err=err)


def cmpe_loss(bsub: np.ndarray, n_patch: int, rho_thresh: float):
    """(L_CMPE, n_valid, per-pixel map, per-pair dict)."""
    d = cmpe(bsub, n_patch, rho_thresh)
    nv = int(np.sum(d["valid"]))
    tot = float(np.sum(np.where(d["valid"], d["err"], 0.0)))
    loss = tot / nv if nv > 0 else 0.0
    cnt = np.sum(d["valid"], axis=(0, 1))
    sm = np.sum(np.where(d["valid"], d["err"], 0.0), axis=(0, 1))
    cmap = np.where(cnt > 0, sm / np.maximum(cnt, 1), 0.0)
    return loss, nv, cmap, d


def cmpe_loss_grad(bsub: np.ndarray, n_patch: int, rho_thresh: float) -> np.ndarray:
    """dL_CMPE/dB_sub as G = dL/dRe + j dL/dIm, shape of ``bsub``.

    d|arg C|/dC = sign(arg C) * j C / |C|^2; with C = sum X conj(Y) the pair
    contributes G_C Y to X and conj(G_C) X to Y.  Scaled by 1/n_valid.
    """
    X, Y = cm_pairs(bsub, n_patch)
    loss, nv, _, d = cmpe_loss(bsub, n_patch, rho_thresh)
    gsub = np.zeros_like(bsub)
    if nv == 0:
        return gsub
    C = d["C"]
    mag2 = np.abs(C) ** 2
    gC = np.where(d["valid"], np.sign(np.angle(C)) * 1j * C / np.where(mag2 > 0, mag2, 1.0), 0.0)
    gC = gC / nv
    gX = gC[..., None] * Y
    gY = np.conj(gC)[..., None] * X
    ns = bsub.shape[0]
    P = bsub.shape[2]
    gsub[0:ns - 1, 1:ns] += gX.reshape(ns - 1, ns - 1, P)
    gsub[1:ns, 0:ns - 1] += gY.reshape(ns - 1, ns - 1, P)
    return gsub


def full_image(bblk: np.ndarray) -> np.ndarray:
    """Full-aperture image: sum of every block pair."""
    return np.sum(bblk, axis=(0, 1))


def speckle_brightness(bblk: np.ndarray, n_patch: int) -> float:
    """Reading: mean over patch centres of |B|^2 of the full-aperture image
    (un-normalised; the loss divides by a reference value)."""
    b = full_image(bblk)
    centres = b.reshape(-1, n_patch)[:, n_patch // 2]
    return float(np.mean(np.abs(centres) ** 2))


def speckle_brightness_grad(bblk: np.ndarray, n_patch: int) -> np.ndarray:
    """d SB / d B^blk (G convention): 2 B(q) / n_pix at each centre point, every block."""
    b = full_image(bblk)
    n_pix = b.shape[0] // n_patch
    g = np.zeros(b.shape, dtype=np.complex128)
    idx = np.arange(n_pix) * n_patch + n_patch // 2
    g[idx] = 2.0 * b[idx] / n_pix
    return np.broadcast_to(g, bblk.shape).copy()


def cmcc_map(bsub: np.ndarray, n_patch: int) -> np.ndarray:
    """Per-pixel common-midpoint correlation coefficient: the mean of rho over the
    pixel's common-midpoint pairs whose two energies exceed MIN_ENERGY, before any
    rho threshold (0 when there is none).  One of the global image-quality
    metrics of the Model Evaluation subsection; its exact formula is in the cited
    work, which is not at hand, so this is the reading that matches the CMPE
    reading above."""
    d = cmpe(bsub, n_patch, 0.0)
    pos = (d["ex"] > MIN_ENERGY) & (d["ey"] > MIN_ENERGY)
    n = np.sum(pos, axis=(0, 1))
    tot = np.sum(np.where(pos, d["rho"], 0.0), axis=(0, 1))
    return np.where(n > 0, tot / np.maximum(n, 1), 0.0)


def coherence_factor(bblk: np.ndarray, n_patch: int) -> np.ndarray:
    """Per-pixel coherence factor at the patch centre:
    |sum_ij B^blk_ij|^2 / (Nb^2 sum_ij |B^blk_ij|^2) (0 when there is no energy)."""
    nb = bblk.shape[0]
    c = bblk.reshape(nb, nb, -1, n_patch)[..., n_patch // 2]
    num = np.abs(np.sum(c, axis=(0, 1))) ** 2
    den = nb * nb * np.sum(np.abs(c) ** 2, axis=(0, 1))
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
