"""Pins of the derived dispersion relation of the circularly polarised pump
(tests/_dispersion.py) against what fixes it independently of its algebra:
* weak pump: as a0 -> 0 the roots become the uncoupled linear modes of the
  model (the Langmuir branch w^2 = wL^2 and the two electromagnetic sidebands
  D+- = 0 of the transverse wave equation), all real;
* k = 0 is neutral (a uniform perturbation of the pump does not grow);
* +-k grow alike (the relation's symmetry under (w, k) -> (-w, -k));
* the polynomial against a direct time integration of the linearised sideband
  equations it was assembled from (growth rate of their solution).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from tests._dispersion import growth_rate, roots

K0 = 1.0 / math.sqrt(2.0)
T = 3.0 / 511.0


def test_weak_pump_gives_the_uncoupled_modes():
    a0, k = 1e-4, 1.3
    g0 = math.sqrt(1 + a0 * a0)
    w0 = math.sqrt(K0 * K0 + 1 / g0)
    wl = math.sqrt(1 / g0 + 3 * k * k * T / g0 ** 2)
    expect = [wl, -wl]
    for s in (+1, -1):   # D+- = 0: (w +- w0)^2 = (k +- k0)^2 + 1/gamma0
        r = math.sqrt((k + s * K0) ** 2 + 1 / g0)
        expect += [-s * w0 + r, -s * w0 - r]
    got = np.sort_complex(roots(a0, K0, T, k))
    assert np.abs(got.imag).max() < 1e-6
    np.testing.assert_allclose(np.sort(got.real), np.sort(expect), atol=1e-6)


def test_uniform_perturbation_is_neutral():
    for a0 in (0.3, math.sqrt(3.0), 4.0):
        assert growth_rate(a0, K0, T, 0.0) == 0.0


@pytest.mark.parametrize("k", [0.4, 1.4142135623730951, 2.1])
def test_both_directions_grow_alike(k):
    a0 = math.sqrt(3.0)
    assert abs(growth_rate(a0, K0, T, k) - growth_rate(a0, K0, T, -k)) <= 1e-9


def test_polynomial_against_the_sideband_equations():
    """Integrate the linearised equations for (alpha, beta, n~) at one k,
        alpha'' = 2 i w0 alpha' + [w0^2 - (k + k0)^2 - 1/g0] alpha - a0 (n/g0 - a0 S/(2 g0^3)),
        beta''  = -2 i w0 beta' + [w0^2 - (k - k0)^2 - 1/g0] beta - a0 (n/g0 - a0 S/(2 g0^3)),
        n''     = -wL^2 n - (a0 k^2 / (2 g0^2)) S,      S = alpha + beta,
    (the Fourier components e^{-iwt} of D+ alpha = D- beta = Q), and compare the growth
    of the solution with the largest Im w of the polynomial."""
    a0, k = math.sqrt(3.0), math.sqrt(2.0)
    g0 = math.sqrt(1 + a0 * a0)
    w0 = math.sqrt(K0 * K0 + 1 / g0)
    wl2 = 1 / g0 + 3 * k * k * T / g0 ** 2

    def rhs(t, y):
        al, alp, be, bep, n, np_ = y[0] + 1j * y[1], y[2] + 1j * y[3], y[4] + 1j * y[5], y[6] + 1j * y[7], \
            y[8] + 1j * y[9], y[10] + 1j * y[11]
        S = al + be
        Q = a0 * (n / g0 - a0 * S / (2 * g0 ** 3))
        alpp = 2j * w0 * alp + (w0 ** 2 - (k + K0) ** 2 - 1 / g0) * al - Q
        bepp = -2j * w0 * bep + (w0 ** 2 - (k - K0) ** 2 - 1 / g0) * be - Q
        npp = -wl2 * n - a0 * k * k / (2 * g0 ** 2) * S
        out = [alp, alpp, bep, bepp, np_, npp]
        return [v for z in out for v in (z.real, z.imag)]

    y0 = np.zeros(12)
    y0[8] = 1e-6
    sol = solve_ivp(rhs, (0.0, 60.0), y0, rtol=1e-10, atol=1e-30, dense_output=True)
    t = np.linspace(30.0, 60.0, 301)
    n = np.abs(sol.sol(t)[8] + 1j * sol.sol(t)[9])
    slope = np.polyfit(t, np.log(n), 1)[0]
    assert abs(slope - growth_rate(a0, K0, T, k)) <= 2e-3 * growth_rate(a0, K0, T, k)
