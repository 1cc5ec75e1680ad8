"""Linear dispersion relation of the circularly polarised pump in the reduced 1D
model (Section 2.1, spin off), derived here from the model's equations with a
fluid closure.  Test helper only: the paper compares its growth rates with the
analytic rates of another reference, which its text does not reproduce, so the
relation used here is this derivation (stated in full so it can be checked).

Model (normalised units of Section 2.1, ions a fixed background):
    d_t^2 A = d_x^2 A - (n / gamma) A,       A = A_y + i A_z,
    d_t n + d_x (n v) = 0,   v = p / gamma,
    (d_t + v d_x) p = E_x - d_x |A|^2 / (2 gamma),   d_x E_x = n - 1,
    gamma = sqrt(1 + p^2 + |A|^2).
Pump: n = 1, p = 0, A = a0 exp(i(k0 x - w0 t)); |A| is uniform, so there is no
ponderomotive force; gamma0 = sqrt(1 + a0^2) and w0^2 = k0^2 + 1/gamma0.

Perturb A = (a0 + psi) exp(i theta0), n = 1 + N, p = P.  To first order
gamma = gamma0 + a0 Re(psi) / gamma0, and
    [(d_t - i w0)^2 - (d_x + i k0)^2 + 1/gamma0] psi + a0 (N / gamma0 - a0 Re(psi) / gamma0^3) = 0,
    (d_t^2 + wL^2) N = (a0 / gamma0^2) d_x^2 Re(psi),
where wL^2 = 1/gamma0 + 3 k^2 T / gamma0^2 adds the 1D adiabatic pressure of a
Maxwellian of momentum temperature T (velocity spread sqrt(T) / gamma0).  With
N = n~ exp(i(k x - w t)) + c.c. and psi = alpha exp(i(k x - w t)) + conj(beta)
exp(-i(k x - conj(w) t)), the two sidebands obey
    D+ alpha = D- beta = Q,   D+- = (k +- k0)^2 - (w +- w0)^2 + 1/gamma0,
    Q = (a0^2 / (2 gamma0^3)) (alpha + beta) [1 - k^2 / (w^2 - wL^2)],
so that nontrivial solutions need
    (D+ + D-) (w^2 - wL^2 - k^2) = (2 gamma0^3 / a0^2) (w^2 - wL^2) D+ D-,
a polynomial of degree 6 in w with real coefficients.  The growth rate of
wavenumber k is the largest Im w of its roots.  The relation is invariant under
(w, k) -> (-w, -k), so +-k grow alike.
"""
from __future__ import annotations

import math

import numpy as np


def dispersion_polynomial(a0: float, k0: float, T: float, k: float) -> np.polynomial.Polynomial:
    g0 = math.sqrt(1.0 + a0 * a0)
    w0 = math.sqrt(k0 * k0 + 1.0 / g0)
    wl2 = 1.0 / g0 + 3.0 * k * k * T / (g0 * g0)
    w = np.polynomial.Polynomial([0.0, 1.0])
    Dp = (k + k0) ** 2 - (w + w0) ** 2 + 1.0 / g0
    Dm = (k - k0) ** 2 - (w - w0) ** 2 + 1.0 / g0
    return (Dp + Dm) * (w * w - wl2 - k * k) - (2.0 * g0 ** 3 / (a0 * a0)) * (w * w - wl2) * Dp * Dm


def roots(a0: float, k0: float, T: float, k: float) -> np.ndarray:
    return dispersion_polynomial(a0, k0, T, k).roots()


def growth_rate(a0: float, k0: float, T: float, k: float) -> float:
    """Largest Im w over the roots (0 if every root is real)."""
    return max(0.0, float(np.max(roots(a0, k0, T, k).imag)))
