"""Angle quadrature of the oracle: Gauss-Legendre nodes on (0, 1) per
hemisphere (double-Gauss), weights summing to one.

Test infrastructure only (see the package docstring)."""
from __future__ import annotations

import numpy as np


def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule mapped from [-1, 1] to (0, 1).

    Returns (mu, w) ascending in mu with sum(w) == 1 up to rounding.  A rule
    with n points integrates polynomials of degree 2n-1 exactly."""
    if n < 1:
        raise ValueError("n must be >= 1")
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w
