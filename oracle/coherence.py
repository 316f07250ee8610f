"""Receive-channel images and lag-one coherence (test infrastructure only).

Paper: Model Evaluation subsection -- lag-one coherence is one of the global
image-quality metrics (after Long et al., defined in the cited Frey et al.,
which is not at hand).

Readings:
* the focused signal of receive element r at point p is Eq. 5 with the whole
  array as transmit aperture and {r} as receive aperture,
      X_r(p) = sum_t h_t h_r Psi_{t,r}(tau) exp(j 2 pi f_d tau);
* the coherence of adjacent elements r, r+1 at pixel q is the real part of their
  normalised correlation over the pixel's patch points m (the IQ form of the
  zero-lag correlation of RF signals),
      rho_r = Re(sum_m X_r conj X_{r+1}) / sqrt(E_r E_{r+1}),  E_r = sum_m |X_r|^2,
  taken over pairs whose energies both exceed MIN_ENERGY (a channel outside the
  apodisation has none);
* LOC(q) is the mean of rho_r over those pairs, 0 if there are none.
"""
from __future__ import annotations

import numpy as np

from . import das
from .model import Problem, travel_times

MIN_ENERGY = 1e-30


def channel_images(prob: Problem, s: np.ndarray, c_med: float | None = None) -> np.ndarray:
    """X [N][P] complex128 at slowness ``s``: the transmit sum of the block-pair
    images of single-element blocks."""
    h = prob.apod()
    T = np.where(h, travel_times(prob, s, h, c_med), 0.0)
    b1 = das.das_blocks(prob.iq, T, h, t0=prob.t0, fs=prob.fs, fd=prob.fd, t_ttp=prob.tau_offset,
                        block=1)
    return b1.sum(axis=0)


def lag_one_coherence(X: np.ndarray, n_patch: int) -> np.ndarray:
    """LOC per pixel from channel images X [N][n_pix * n_patch]."""
    n = X.shape[0]
    Xp = X.reshape(n, -1, n_patch)
    E = np.sum(np.abs(Xp) ** 2, axis=2)                          # [N][n_pix]
    C = np.sum(Xp[:-1] * np.conj(Xp[1:]), axis=2).real          # [N-1][n_pix]
    ok = (E[:-1] > MIN_ENERGY) & (E[1:] > MIN_ENERGY)
    rho = np.where(ok, C / np.sqrt(np.where(ok, E[:-1] * E[1:], 1.0)), 0.0)
    cnt = ok.sum(axis=0)
    return np.where(cnt > 0, rho.sum(axis=0) / np.maximum(cnt, 1), 0.0)
