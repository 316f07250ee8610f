"""Forward simulator of demodulated FSA channel data from point scatterers.

Synthetic stand-in for the paper's k-Wave simulations and in-vivo data (which
are not available): the echo of scatterer k on transmit t / receive r is a
baseband Gaussian envelope at the bent-ray round-trip time,

    Psi[t][r][n] = sum_k A_k g(t_n - tau_trk) exp(-j 2 pi f_d tau_trk),
    g(t) = exp(-t^2 / (2 sigma^2)) for |t| <= 6 sigma, else 0,

with t_n = t0 + n/fs, tau_trk = T[t,k] + T[r,k] + t_ttp and T from the same
bent-ray model as the beamformer (refraction at the node-mean speed of the
true map, then the bicubic path integral on the true map with ``n_seg``
segments) -- an "inverse crime" by construction.  sigma follows from the -6 dB
fractional bandwidth B: sigma = sqrt(2 ln 2) / (pi B f_c).  No spreading loss,
no directivity.
"""
from __future__ import annotations

import math

import numpy as np

from . import fermat, path


def pulse_sigma(fc: float, frac_bw: float) -> float:
    return math.sqrt(2.0 * math.log(2.0)) / (math.pi * frac_bw * fc)


def scatterer_times(elem_xz, d_lens, c_lens, s_true, grid, n_seg, scat_xz):
    """[N][K] one-way bent-ray times from every element to every scatterer."""
    c_med = float(np.mean(1.0 / s_true))
    r = fermat.refract(elem_xz, d_lens, c_lens, c_med, scat_xz)
    px = np.broadcast_to(scat_xz[None, :, 0], r["l2"].shape)
    pz = np.broadcast_to(scat_xz[None, :, 1], r["l2"].shape)
    tm = path.medium_time(s_true, grid, r["ref_x"], r["ref_z"], px, pz, r["l2"], n_seg)
    return r["l1"] / c_lens + tm


def synthesize(T: np.ndarray, amp: np.ndarray, *, t_ttp, t0, fs, fd, ns, fc, frac_bw,
               rows=None):
    """Channel data [N][N][Ns] complex128 from one-way times T [N][K]; with ``rows``
    (transmit indices) only those records, [len(rows)][N][Ns]."""
    n = T.shape[0]
    rows = range(n) if rows is None else list(rows)
    sig = pulse_sigma(fc, frac_bw)
    half = 6.0 * sig
    width = int(math.floor(2.0 * half * fs)) + 2
    out = np.zeros((len(rows), n, ns), dtype=np.complex128)
    offs = np.arange(width)
    for i, t in enumerate(rows):
        for r in range(n):
            tau = T[t] + T[r] + t_ttp
            n0 = np.ceil((tau - half - t0) * fs).astype(np.int64)
            idx = n0[:, None] + offs[None, :]
            tn = t0 + idx / fs
            dt = tn - tau[:, None]
            ok = (np.abs(dt) <= half) & (idx >= 0) & (idx < ns)
            val = amp[:, None] * np.exp(-dt * dt / (2.0 * sig * sig)) * \
                np.exp(-2j * np.pi * fd * tau)[:, None]
            val = np.where(ok, val, 0.0)
            ii = np.where(ok, idx, 0).ravel()
            out[i, r] += np.bincount(ii, weights=val.real.ravel(), minlength=ns) + \
                1j * np.bincount(ii, weights=val.imag.ravel(), minlength=ns)
    return out


def simulate(elem_xz, d_lens, c_lens, t_ttp, s_true, grid, n_seg, scat_xz, scat_amp, *,
             t0, fs, fd, ns, fc, frac_bw):
    T = scatterer_times(elem_xz, d_lens, c_lens, s_true, grid, n_seg, scat_xz)
    return synthesize(T, scat_amp, t_ttp=t_ttp, t0=t0, fs=fs, fd=fd, ns=ns, fc=fc,
                      frac_bw=frac_bw)
