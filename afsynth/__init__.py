"""Seeded synthetic inputs for lens-aware autofocusing.

This module makes the *inputs* of the method and nothing else: array element
positions, polar pixel grids, the box of the slowness grid, random media
(sound-speed maps and scatterer lists) and random channel data.  It holds no
step of the method itself (no element orientation, apodisation, refraction,
travel time, interpolation, delay-and-sum, loss or gradient), so the FP64 CPU
oracle and the GPU library can both consume what it makes without sharing any
of the method's arithmetic.

Units throughout: lengths in mm, times in microseconds, frequencies in MHz,
sound speed in mm/us (= km/s), slowness in us/mm.  The origin is the centre of
curvature of the curvilinear array; x is lateral and z points into the body.
"""
from .configs import (ArrayCfg, AcqCfg, ImgCfg, MethodCfg, Config, CONFIGS,
                      config_by_name)
from .geometry import (element_positions, element_span, pixel_centres,
                       patch_spacing, slowness_box, sim_box, lens_radius,
                       is_linear)
from .media import (Medium, medium_for, sample_speed, speed_on_grid,
                    random_iq)

__all__ = [
    "ArrayCfg", "AcqCfg", "ImgCfg", "MethodCfg", "Config", "CONFIGS",
    "config_by_name", "element_positions", "element_span", "pixel_centres",
    "patch_spacing", "slowness_box", "sim_box", "lens_radius", "is_linear", "Medium",
    "medium_for", "sample_speed", "speed_on_grid", "random_iq",
]
