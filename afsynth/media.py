"""Seeded random media: sound-speed maps and scatterer lists.

A medium is a set of concentric layers (radii measured from the centre of
curvature, so every layer follows the lens surface) or, for a linear array,
horizontal layers (bounded by depths z), optional Gaussian speed blobs,
optional anechoic cysts (no scatterers, same speed) and a list of point
scatterers with real amplitudes.  Speeds are in mm/us.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .configs import Config
from .geometry import element_span, element_x, is_linear, lens_radius


@dataclass
class Medium:
    layer_r: np.ndarray            # [L] outer radius of each layer but the last (mm, increasing)
    layer_c: np.ndarray            # [L+1] speed of each layer, innermost first (mm/us)
    blob_xz: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    blob_sigma: np.ndarray = field(default_factory=lambda: np.zeros(0))
    blob_amp: np.ndarray = field(default_factory=lambda: np.zeros(0))
    cyst_xz: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    cyst_r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    scat_xz: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    scat_amp: np.ndarray = field(default_factory=lambda: np.zeros(0))
    layer_axis: str = "radial"     # "radial": layer_r are radii; "depth": they are depths z

    @property
    def n_scat(self) -> int:
        return int(self.scat_amp.shape[0])


def sample_speed(med: Medium, x: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Speed (mm/us) of ``med`` at points (x, z)."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    rho = np.hypot(x, z) if med.layer_axis == "radial" else z
    idx = np.searchsorted(med.layer_r, rho, side="right")
    c = med.layer_c[idx].astype(np.float64)
    for (bx, bz), sg, am in zip(med.blob_xz, med.blob_sigma, med.blob_amp):
        c = c + am * np.exp(-((x - bx) ** 2 + (z - bz) ** 2) / (2.0 * sg * sg))
    return c


def speed_on_grid(med: Medium, x0: float, z0: float, dx: float, dz: float,
                  nx: int, nz: int) -> np.ndarray:
    """[nz][nx] speed at the nodes x0 + j dx, z0 + i dz."""
    xs = x0 + dx * np.arange(nx)
    zs = z0 + dz * np.arange(nz)
    X, Z = np.meshgrid(xs, zs)
    return sample_speed(med, X, Z)


def _sector_uniform(rng, n, rho0, rho1, th0, th1):
    rho = np.sqrt(rng.uniform(rho0 * rho0, rho1 * rho1, n))
    th = rng.uniform(th0, th1, n)
    return np.stack([rho * np.sin(th), rho * np.cos(th)], axis=1)


def _drop_in_cysts(xz, amp, cyst_xz, cyst_r):
    keep = np.ones(xz.shape[0], dtype=bool)
    for (cx, cz), r in zip(cyst_xz, cyst_r):
        keep &= (xz[:, 0] - cx) ** 2 + (xz[:, 1] - cz) ** 2 > r * r
    return xz[keep], amp[keep]


def _polar(rho, th):
    return np.array([rho * math.sin(th), rho * math.cos(th)])


def _linear_medium(cfg: Config, rng, seed: int) -> Medium:
    """Bi-layer phantom under a linear array: a layer at 1575 m/s (the paper's chicken
    breast) of thickness U(6, 12) mm on the lens over a phantom at 1490, 1516 or
    1540 m/s (seed mod 3), one anechoic cyst, nine point targets and random
    scatterers."""
    arr, img = cfg.array, cfg.img
    xe = element_x(arr)
    x0, x1 = float(xe[0]), float(xe[-1])
    z_lo, z_hi = arr.d_lens + img.depth_min, arr.d_lens + img.depth_max
    top = arr.d_lens + rng.uniform(6.0, 12.0)
    layer_r = np.array([top])
    layer_c = np.array([1.575, (1.490, 1.516, 1.540)[seed % 3]])
    span = x1 - x0
    cyst_xz = np.array([[x0 + rng.uniform(0.35, 0.65) * span,
                         rng.uniform(top + 6.0, max(top + 7.0, z_hi - 8.0))]])
    cyst_r = np.array([rng.uniform(2.0, 3.5)])
    area = (x1 - x0) * (z_hi - z_lo)
    n_rand = cfg.n_scat_random if cfg.n_scat_random > 0 else int(round(cfg.scat_density * area))
    rand_xz = np.stack([rng.uniform(x0, x1, n_rand), rng.uniform(z_lo, z_hi, n_rand)], axis=1)
    rand_amp = rng.standard_normal(n_rand)
    dep = (z_lo + 0.25 * (z_hi - z_lo), z_lo + 0.5 * (z_hi - z_lo), z_lo + 0.75 * (z_hi - z_lo))
    tg = np.array([[x0 + f * span, d] for d in dep for f in (0.25, 0.5, 0.75)])
    scat_xz = np.concatenate([tg, rand_xz])
    scat_amp = np.concatenate([np.full(9, 10.0), rand_amp])
    scat_xz, scat_amp = _drop_in_cysts(scat_xz, scat_amp, cyst_xz, cyst_r)
    return Medium(layer_r=layer_r, layer_c=layer_c, cyst_xz=cyst_xz, cyst_r=cyst_r,
                  scat_xz=scat_xz, scat_amp=scat_amp, layer_axis="depth")


def medium_for(cfg: Config, seed: int | None = None) -> Medium:
    """Draw the medium named by ``cfg.medium`` from ``seed`` (default ``cfg.seed``)."""
    seed = cfg.seed if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    if cfg.medium == "linear_bilayer":
        return _linear_medium(cfg, rng, seed)
    arr, img = cfg.array, cfg.img
    rl = lens_radius(arr)
    th0, th1 = element_span(arr)
    half = 0.5 * (th1 - th0)
    rho_lo, rho_hi = rl + img.depth_min, rl + img.depth_max
    kind = cfg.medium

    cyst_xz = np.zeros((0, 2))
    cyst_r = np.zeros(0)
    blob_xz = np.zeros((0, 2))
    blob_sigma = np.zeros(0)
    blob_amp = np.zeros(0)

    if kind in ("c1_two_layer", "c1_two_layer_cyst"):
        layer_r = np.array([rl + 10.0])
        layer_c = np.array([1.450, 1.570])
        if kind == "c1_two_layer_cyst":
            cyst_xz = _polar(rl + 35.0, 0.0)[None, :]
            cyst_r = np.array([4.0])
    elif kind == "c1_random":
        thick = rng.uniform(5.0, 15.0)
        layer_r = np.array([rl + thick])
        layer_c = np.array([rng.uniform(1.420, 1.500), rng.uniform(1.540, 1.600)])
    elif kind in ("liver_wall", "liver_wall_deep"):
        n_wall = 3 if kind == "liver_wall" else int(rng.integers(3, 5))
        thick = rng.uniform(5.0, 25.0, n_wall)
        layer_r = rl + np.cumsum(thick)
        wall_c = rng.uniform(1.420, 1.600, n_wall)
        liver_c = rng.uniform(1.540, 1.580)
        layer_c = np.concatenate([wall_c, [liver_c]])
        liver_top = layer_r[-1]
        n_blob = int(rng.integers(3, 6))
        blob_sigma = rng.uniform(5.0, 15.0, n_blob)
        blob_amp = rng.uniform(-0.020, 0.020, n_blob)
        blob_xz = np.stack([_polar(rng.uniform(liver_top, rho_hi), rng.uniform(th0, th1))
                            for _ in range(n_blob)])
        n_cyst = int(rng.integers(2, 4))
        cyst_r = rng.uniform(3.0, 8.0, n_cyst)
        cyst_xz = np.stack([_polar(rng.uniform(liver_top + 8.0, max(liver_top + 9.0, rho_hi - 20.0)),
                                   rng.uniform(th0 + 0.25 * (th1 - th0), th1 - 0.25 * (th1 - th0)))
                            for _ in range(n_cyst)])
    else:
        raise KeyError(kind)

    # scatterers
    if cfg.n_scat_random > 0:
        n_rand = cfg.n_scat_random
    else:
        area = 0.5 * (rho_hi ** 2 - rho_lo ** 2) * (th1 - th0)
        n_rand = int(round(cfg.scat_density * area))
    rand_xz = _sector_uniform(rng, n_rand, rho_lo, rho_hi, th0, th1)
    rand_amp = rng.standard_normal(n_rand)
    pts = [rand_xz]
    amps = [rand_amp]
    if kind.startswith("c1"):
        # nine bright point targets on a 3x3 lattice (depth 15/30/45 mm x angle -1/3, 0, +1/3 half-span)
        tg = [_polar(rl + d, f * half) for d in (15.0, 30.0, 45.0) for f in (-1 / 3, 0.0, 1 / 3)]
        pts.insert(0, np.stack(tg))
        amps.insert(0, np.full(9, 10.0))
    scat_xz = np.concatenate(pts)
    scat_amp = np.concatenate(amps)
    scat_xz, scat_amp = _drop_in_cysts(scat_xz, scat_amp, cyst_xz, cyst_r)
    return Medium(layer_r=layer_r, layer_c=layer_c, blob_xz=blob_xz, blob_sigma=blob_sigma,
                  blob_amp=blob_amp, cyst_xz=cyst_xz, cyst_r=cyst_r,
                  scat_xz=scat_xz, scat_amp=scat_amp)


def random_iq(n_elem: int, n_samples: int, seed: int, dtype=np.complex64) -> np.ndarray:
    """[Nt][Nr][Ns] circular complex Gaussian channel data (unit variance)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (n_elem, n_elem, n_samples)
    re = rng.standard_normal(shape, dtype=np.float32)
    im = rng.standard_normal(shape, dtype=np.float32)
    out = np.empty(shape, dtype=dtype)
    out.real = re * np.float32(math.sqrt(0.5))
    out.imag = im * np.float32(math.sqrt(0.5))
    return out
