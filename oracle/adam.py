"""Adam update of the slowness grid.

The paper's update rule is plain gradient descent on the sound speed (Eq. 9);
the plain-method loop here uses Adam (Kingma and Ba, 2015) on the slowness,
with bias correction.  ``descent_step`` is Eq. 9 itself, for reference.
"""
from __future__ import annotations

import numpy as np


def adam_step(s, m, v, g, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam step (``step`` is 1-based).  Returns (s, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return s - lr * mhat / (np.sqrt(vhat) + eps), m, v


def descent_step(c, grad_c, gamma: float):
    """Eq. 9: c <- c - gamma dL/dc."""
    return c - gamma * grad_c
