"""Workload configurations.

Each configuration fixes the array, the acquisition, the pixel grid, the
slowness-grid size and the method's hyperparameters.  Lens constants follow
the paper's calibration table (Table I) only where a configuration names them;
the regulariser, threshold, F and N_segments defaults are the C5-2v phantom and
in-vivo columns of the paper's hyperparameter table (Table II).  The learning
rate is an Adam step on the slowness in us/mm, whose scale the paper does not
fix: 0.003 for the 32-element configurations and 0.001 for the 128/192-element
ones (0.05, the in-vivo value read in these units, diverges).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class ArrayCfg:
    n_elem: int          # number of elements (= transmits = receives, FSA)
    radius: float        # mm, radius of curvature of the element arc (inf: linear array)
    pitch: float         # mm, arc length between neighbouring elements
    d_lens: float        # mm, lens thickness (elements sit this far behind the lens arc)
    c_lens: float        # mm/us, lens sound speed
    t_ttp: float = 0.0   # us, time-to-peak offset of the received envelope


@dataclass(frozen=True)
class AcqCfg:
    fc: float            # MHz, centre (= demodulation) frequency
    fs: float            # MHz, sampling rate of the demodulated data
    n_samples: int       # samples per channel
    t0: float = 0.0      # us, time of sample 0
    frac_bw: float = 0.70  # -6 dB fractional bandwidth of the Gaussian pulse


@dataclass(frozen=True)
class ImgCfg:
    n_depth: int         # pixel rows (depth)
    n_angle: int         # pixel columns (polar angle, across the element span)
    depth_min: float     # mm below the lens surface
    depth_max: float     # mm below the lens surface
    patch: int = 3       # points per side of the evaluation patch (3 -> 3x3)
    c_ref: float = 1.540  # mm/us, speed that sets the patch spacing lambda/2


@dataclass(frozen=True)
class MethodCfg:
    block: int           # S, elements per block; subapertures are 2 blocks wide
    fnum: float          # F of the apodisation |x'| <= (F/2) z'
    n_seg: int           # ray segments after leaving the lens
    nx: int              # slowness grid nodes, lateral
    nz: int              # slowness grid nodes, axial
    lr: float = 0.003
    w1: float = 10.0
    kx1: float = 0.01
    kz1: float = 0.01
    w2: float = 100.0
    kx2: float = 0.001
    kz2: float = 0.001
    rho_thresh: float = 0.9
    w_sb: float = 0.0
    n_iter: int = 5


@dataclass(frozen=True)
class Config:
    name: str
    array: ArrayCfg
    acq: AcqCfg
    img: ImgCfg
    method: MethodCfg
    medium: str          # name of the medium generator (see media.py)
    seed: int
    n_scat_random: int = 0     # 0 -> density based
    scat_density: float = 1.5  # scatterers per mm^2 when n_scat_random == 0
    sim_spacing: float = 0.5   # mm, node spacing of the simulator's true-speed grid
    sim_nseg: int = 256        # ray segments used by the simulator
    notes: str = ""

    def with_(self, **kw):
        return replace(self, **kw)


# Tiny plain-method case (32 elements, 64 x 64 pixels, 8 x 8 grid).
C1 = Config(
    name="c1_tiny",
    array=ArrayCfg(n_elem=32, radius=40.0, pitch=0.4, d_lens=1.0, c_lens=1.000),
    acq=AcqCfg(fc=3.0, fs=12.0, n_samples=1024),
    img=ImgCfg(n_depth=64, n_angle=64, depth_min=1.0, depth_max=60.0),
    method=MethodCfg(block=4, fnum=0.5, n_seg=32, nx=8, nz=8, n_iter=5),
    medium="c1_two_layer", seed=0, n_scat_random=2000,
)

# Clinical-size forward + adjoint (128 elements, 256 x 256 pixels): the benchmarked workload.
C2 = Config(
    name="c2_clinical",
    array=ArrayCfg(n_elem=128, radius=60.0, pitch=0.37, d_lens=1.2, c_lens=1.000),
    acq=AcqCfg(fc=3.5, fs=14.0, n_samples=2560),
    img=ImgCfg(n_depth=256, n_angle=256, depth_min=1.0, depth_max=160.0),
    method=MethodCfg(block=8, fnum=0.4, n_seg=32, nx=32, nz=32, lr=0.001,
                     w1=100.0, kx2=0.002, kz2=0.002, n_iter=1),
    medium="liver_wall", seed=2, sim_spacing=1.0,
)

# Full plain autofocus loop on the tiny case's medium plus one cyst, CMPE + SB.
C3 = C1.with_(
    name="c3_plain_loop",
    method=replace(C1.method, n_iter=200, w_sb=0.1),
    medium="c1_two_layer_cyst",
)

# Learned warm-start training media: randomised two-layer media on the tiny case's array.
C4 = C1.with_(name="c4_train", medium="c1_random", seed=1000,
              method=replace(C1.method, n_iter=200))

# Largest: 192 elements, 4096 samples, 512 x 512 pixels, 64 x 64 grid.
C5 = Config(
    name="c5_largest",
    array=ArrayCfg(n_elem=192, radius=60.0, pitch=0.37, d_lens=1.2, c_lens=1.000),
    acq=AcqCfg(fc=3.5, fs=14.0, n_samples=4096),
    img=ImgCfg(n_depth=512, n_angle=512, depth_min=1.0, depth_max=200.0),
    method=MethodCfg(block=8, fnum=0.4, n_seg=64, nx=64, nz=64, lr=0.001,
                     w1=100.0, kx2=0.002, kz2=0.002, n_iter=200),
    medium="liver_wall_deep", seed=5, sim_spacing=1.0,
)

# A very small case for unit tests (seconds in the oracle, several GPU tiles).
MICRO = Config(
    name="micro",
    array=ArrayCfg(n_elem=16, radius=30.0, pitch=0.5, d_lens=0.8, c_lens=1.000,
                   t_ttp=0.0),
    acq=AcqCfg(fc=3.0, fs=12.0, n_samples=512),
    img=ImgCfg(n_depth=20, n_angle=17, depth_min=2.0, depth_max=28.0),
    method=MethodCfg(block=4, fnum=0.5, n_seg=16, nx=6, nz=7, n_iter=3),
    medium="c1_two_layer", seed=7, n_scat_random=300,
)

# Linear array with a flat lens: the paper's L12-3v (0.2 mm pitch, Table I lens
# 1049.4 m/s, 0.67 mm, t_ttp 578.3 ns; 128 captured elements, 7.35 MHz) and its
# phantom hyperparameters (Table II: F 0.75, 32 segments, w1 7, no second-order
# term), on a bi-layer phantom (1575 m/s layer over 1490/1516/1540 m/s), imaged
# to 36 mm, about the depth the 1536-sample record reaches at 1490 m/s.
L1 = Config(
    name="l1_linear",
    array=ArrayCfg(n_elem=128, radius=math.inf, pitch=0.2, d_lens=0.67, c_lens=1.0494,
                   t_ttp=0.5783),
    acq=AcqCfg(fc=7.35, fs=29.4, n_samples=1536),
    img=ImgCfg(n_depth=128, n_angle=128, depth_min=2.0, depth_max=36.0),
    method=MethodCfg(block=8, fnum=0.75, n_seg=32, nx=16, nz=16, lr=0.003, w1=7.0,
                     kx1=0.001, kz1=0.02, w2=0.0, kx2=0.0, kz2=0.0, n_iter=200),
    medium="linear_bilayer", seed=31, scat_density=6.0, sim_spacing=0.25,
)

# Small linear-array case for the oracle (16 elements, 12 x 10 pixels).
MICRO_LINEAR = Config(
    name="micro_linear",
    array=ArrayCfg(n_elem=16, radius=math.inf, pitch=0.3, d_lens=0.67, c_lens=1.0494,
                   t_ttp=0.0),
    acq=AcqCfg(fc=5.0, fs=20.0, n_samples=512),
    img=ImgCfg(n_depth=12, n_angle=10, depth_min=2.0, depth_max=14.0),
    method=MethodCfg(block=4, fnum=0.75, n_seg=16, nx=6, nz=7, n_iter=3),
    medium="linear_bilayer", seed=5, n_scat_random=300,
)

CONFIGS = [C1, C2, C3, C4, C5, L1]


def config_by_name(name: str) -> Config:
    for c in CONFIGS + [MICRO, MICRO_LINEAR]:
        if c.name == name:
            return c
    raise KeyError(name)
