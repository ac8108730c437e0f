"""Wendland phi_{3,1} (Section 5): phi(r) = (1 - r)_+^4 (4 r + 1).

Positive definite on R^d for d <= 3 and C^2 at r = 1 (a (1-r)^3 zero of the
derivative). Used here in the unit-peak form phi(||x - y|| / delta), the paper's
Phi_delta of eq. (kernelscaling) without the delta^-d prefactor.
"""
from __future__ import annotations

import numpy as np


def phi31(r) -> np.ndarray:
    """phi_{3,1}(r) for r >= 0, exactly zero for r >= 1."""
    r = np.asarray(r, dtype=np.float64)
    t = np.maximum(1.0 - r, 0.0)
    t2 = t * t
    return t2 * t2 * (4.0 * r + 1.0)
