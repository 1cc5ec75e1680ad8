"""Independent periodic B-spline machinery for the pins, built on scipy's BSpline.

Test helper only: it touches neither the oracle nor the HIP library.  Periodic
splines on the uniform grid x_j = j dx are represented as non-periodic scipy
splines on an extended knot vector, with coefficients repeated periodically,
so that positions a few cells outside [0, L) evaluate correctly.
"""
from __future__ import annotations

import numpy as np
from scipy.interpolate import BSpline

PAD = 3  # extra periods of cells on each side


def _knots(M: int, dx: float, deg: int) -> np.ndarray:
    # basis element i has support [t_i, t_{i+deg+1}) with t_i = (i - deg - PAD) dx
    return (np.arange(M + 2 * deg + 2 * PAD + 1) - deg - PAD) * dx


def periodic_spline(coef: np.ndarray, dx: float, deg: int) -> BSpline:
    """The spline sum_j coef_j N^deg_j(x) with periodic index j (mod M)."""
    M = len(coef)
    t = _knots(M, dx, deg)
    ncoef = len(t) - deg - 1
    idx = (np.arange(ncoef) - deg - PAD) % M     # element i <-> basis index j = i - deg - PAD
    return BSpline(t, np.asarray(coef, dtype=np.float64)[idx], deg, extrapolate=False)


def basis_integrals(M: int, dx: float, deg: int, x0: float, x1: float) -> np.ndarray:
    """Vector over j (mod M) of int_{x0}^{x1} N^deg_j (signed, path may be unwrapped)."""
    out = np.zeros(M)
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        out[j] = periodic_spline(e, dx, deg).integrate(x0, x1)
    return out


def basis_values(M: int, dx: float, deg: int, x: float) -> np.ndarray:
    out = np.zeros(M)
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        out[j] = periodic_spline(e, dx, deg)(x)
    return out


def basis_derivs(M: int, dx: float, deg: int, x: float) -> np.ndarray:
    """Vector over j (mod M) of dN^deg_j/dx at x (scipy's own derivative)."""
    out = np.zeros(M)
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        out[j] = periodic_spline(e, dx, deg).derivative()(x)
    return out
