"""Synthetic-aperture delay-and-sum with phase rotation over subaperture blocks.

Paper: round-trip time tau = t_d(t -> p) + t_d(p -> r) (Section II-A), plus the
time-to-peak offset of the bent-ray model (Eq. 7); beamforming Eq. 5:
    B_{T,R}(p) = sum_{t in T} sum_{r in R} Psi_{t,r}(tau) exp(j 2 pi f_d tau) h_t h_r .

Readings:
* Psi_{t,r}(tau) is linear interpolation of I and Q between the two samples
  around u = (tau - t0) fs, zero outside 0 <= u <= Ns - 1 (at u = Ns - 1 the
  last interval is used);
* the exponent sign +j assumes demodulation by exp(-j 2 pi f_d t);
* the channel data layout is [Nt][Nr][Ns] (the paper writes Ns x Nt x Nr);
* elements are grouped in contiguous blocks of S; the oracle returns the
  block-pair images B^blk[i][j](p), from which subaperture images are sums.
"""
from __future__ import annotations

import numpy as np


def sample_index(tau, t0, fs, ns):
    """(valid, k, f) for fractional sample u = (tau - t0) fs."""
    u = (tau - t0) * fs
    valid = (u >= 0.0) & (u <= ns - 1)
    k = np.floor(np.where(valid, u, 0.0)).astype(np.int64)
    k = np.where(k >= ns - 1, ns - 2, k)
    f = np.where(valid, u - k, 0.0)
    return valid, k, f


def das_blocks(iq: np.ndarray, T: np.ndarray, h: np.ndarray, *, t0: float, fs: float,
               fd: float, t_ttp: float, block: int) -> np.ndarray:
    """Block-pair images B^blk[i][j][p] (complex128).

    iq: [N][N][Ns] complex; T: [N][P] one-way times (us); h: [N][P] apodisation.
    """
    n, _, ns = iq.shape
    nb = n // block
    P = T.shape[1]
    out = np.zeros((nb, nb, P), dtype=np.complex128)
    for t in range(n):
        for r in range(n):
            w = h[t] & h[r]
            if not np.any(w):
                continue
            tau = T[t] + T[r] + t_ttp
            valid, k, f = sample_index(tau, t0, fs, ns)
            trace = iq[t, r].astype(np.complex128)
            v = (1.0 - f) * trace[k] + f * trace[k + 1]
            contrib = np.where(valid & w, v * np.exp(2j * np.pi * fd * tau), 0.0)
            out[t // block, r // block] += contrib
    return out


def das_blocks_adjoint_T(iq: np.ndarray, T: np.ndarray, h: np.ndarray, G: np.ndarray, *,
                         t0: float, fs: float, fd: float, t_ttp: float, block: int) -> np.ndarray:
    """dL/dT[a][p] given G = dL/dRe B^blk + j dL/dIm B^blk ([Nb][Nb][P]).

    By the chain rule of Eq. 5: for each sample, d/dtau [v(tau) e^{j w tau}] =
    (v'(tau) + j w v(tau)) e^{j w tau} with v' = fs (Psi[k+1] - Psi[k]); the
    sample adds Re(conj(G) * that) * h_t h_r to g[t] (transmit leg) and to g[r]
    (receive leg).  Apodisation and the validity window are constants.
    """
    n, _, ns = iq.shape
    P = T.shape[1]
    g = np.zeros((n, P))
    w_d = 2.0 * np.pi * fd
    for t in range(n):
        for r in range(n):
            w = h[t] & h[r]
            if not np.any(w):
                continue
            tau = T[t] + T[r] + t_ttp
            valid, k, f = sample_index(tau, t0, fs, ns)
            trace = iq[t, r].astype(np.complex128)
            a0 = trace[k]
            a1 = trace[k + 1]
            v = (1.0 - f) * a0 + f * a1
            dv = fs * (a1 - a0)
            rot = np.exp(1j * w_d * tau)
            d = np.real(np.conj(G[t // block, r // block]) * (dv + 1j * w_d * v) * rot)
            d = np.where(valid & w, d, 0.0)
            g[t] += d
            g[r] += d
    return g
