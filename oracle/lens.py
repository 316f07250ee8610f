"""Lens models of the round-trip delay.

Paper: Section II-B.  Two ways of accounting for the transducer lens are
compared there:

* the conventional model (Eq. 6): the straight-ray round trip from the
  element positions through the medium, plus a scalar lens-correction offset
  and the scalar time-to-peak offset of the received envelope;
* the bent-ray model (Eqs. 7-8): the lens is a layer of thickness d_lens and
  speed c_lens, crossed by rays that refract at its surface (``fermat``), plus
  the time-to-peak offset.

The paper names a third case in its comparisons, the model without lens
correction: straight rays from the elements and no lens term.

Reading of the conventional offset: the paper says only that it is a scalar,
usually derived under the homogeneous 1540 m/s assumption.  Here it is the
round-trip excess time of crossing the lens twice along the element normal at
the lens speed instead of the reference speed,

    tau_lenscor = 2 d_lens (1 / c_lens - 1 / c_ref),   c_ref = 1.540 mm/us .

For a ray along the element normal in a medium of speed c_ref the conventional
round trip then equals the bent-ray round trip exactly (the pin of this
reading).
"""
from __future__ import annotations

MODELS = ("bent", "conventional", "none")
C_REF = 1.540


def conventional_offset(d_lens: float, c_lens: float, c_ref: float = C_REF) -> float:
    """Scalar lens-correction offset of the conventional model (Eq. 6), in us."""
    return 2.0 * d_lens * (1.0 / c_lens - 1.0 / c_ref)


def ray_lens_thickness(model: str, d_lens: float) -> float:
    """Lens thickness the rays of ``model`` refract through: the bent-ray model
    traces the lens (Eqs. 7-8); the other two start straight rays at the elements."""
    if model not in MODELS:
        raise ValueError(f"lens model must be one of {MODELS}")
    return d_lens if model == "bent" else 0.0


def round_trip_offset(model: str, d_lens: float, c_lens: float, t_ttp: float,
                      c_ref: float = C_REF) -> float:
    """Scalar added to every round trip T_t + T_r: the time-to-peak offset (Eqs. 6
    and 7), plus the lens-correction offset for the conventional model (Eq. 6)."""
    if model not in MODELS:
        raise ValueError(f"lens model must be one of {MODELS}")
    extra = conventional_offset(d_lens, c_lens, c_ref) if model == "conventional" else 0.0
    return t_ttp + extra
