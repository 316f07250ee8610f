"""Plain FP64 CPU oracle of lens-aware differentiable beamforming.

TEST INFRASTRUCTURE ONLY.  This package is the parity reference for the GPU
library: only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark import it.  The product path (the HIP library and its Python
binding) never imports, calls or links anything here, and this package imports
nothing from the product; the only code both sides share is the seeded input
generator ``afsynth``, which holds none of the method's arithmetic.

Every function follows one passage of the paper (cited in its docstring) and is
written for checking by eye: no blocking, fusion or reordering beyond what the
definition states.  Where the paper is silent or ambiguous the function states
the reading it takes.

Units: mm, us, MHz; speed in mm/us, slowness in us/mm.
"""
from . import geometry, fermat, lens, path, das, cmpe, reg, model, adam, sweep, simulate  # noqa: F401
