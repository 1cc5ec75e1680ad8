"""Pins of the 2D oracle's spin terms (hbar != 0; Sections 2.2 and 4.3) against what
the paper and the mathematics fix, evaluated independently of the oracle where it
matters:

* the Zeeman energy hbar sum_a w s_a . B_h(x_a), B_h = (dA_z/dx2, -dA_z/dx1, B_z),
  with B_h from scipy's B-splines and their own derivatives;
* the spin sources as gradients of that energy: for any a_z and b_z,
  a_z . G*^T Lambda1*^T W S_xy and b_z . Lambda2^T W S_z are its xy and z parts;
* the spin force of Subsystem I as the printed divided differences of s . B_h along
  the two legs (point values from scipy);
* Subsystem II's spin rotation against scipy's ODE solver;
* energy conservation of every substep and of Lie steps with the Zeeman term (a
  wrong sign in any spin term breaks it), the Gauss law, and hbar = 0 reducing to
  the plain functions.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.twod import Oracle2D, initial_state2d
from tests._splines import basis_derivs, basis_values
from workloads.twod import generate2d, get2d


def setup(name, n=200, **kw):
    w = get2d(name).scaled(n_particles=n)
    o = Oracle2D.from_workload(w, **kw)
    return w, o, initial_state2d(o, generate2d(w))


def scipy_B(o, s, x1, x2):
    """B_h at a point from scipy: (dA/dx2, -dA/dx1, B_z)."""
    c, p = o.cfg, o.cfg.p
    A = np.asarray(s["az"]).reshape(c.M1, c.M2)
    Bz = np.asarray(s["bz"]).reshape(c.M1, c.M2)
    h1, h2 = c.L1 / c.M1, c.L2 / c.M2
    v1, v2 = basis_values(c.M1, h1, p, x1 % c.L1), basis_values(c.M2, h2, p, x2 % c.L2)
    d1, d2 = basis_derivs(c.M1, h1, p, x1 % c.L1), basis_derivs(c.M2, h2, p, x2 % c.L2)
    w1, w2 = basis_values(c.M1, h1, p - 1, x1 % c.L1), basis_values(c.M2, h2, p - 1, x2 % c.L2)
    return np.array([v1 @ A @ d2, -(d1 @ A @ v2), w1 @ Bz @ w2])


def zeeman_density(o, s, a, x1, x2):
    B = scipy_B(o, s, x1, x2)
    return s["sx"][a] * B[0] + s["sy"][a] * B[1] + s["sz"][a] * B[2]


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_zeeman_energy_against_scipy(name):
    w, o, s = setup(name, n=40)
    z = sum(o.cfg.w * zeeman_density(o, s, a, s["x1"][a], s["x2"][a]) for a in range(40))
    H = o.energy_s(s)
    assert abs(H[5] - o.hbar * z) < 1e-13 * abs(o.hbar * z)
    assert abs(H[6] - (o.energy(s)[5] + H[5])) < 1e-13 * H[6]


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_spin_sources_are_gradients_of_the_zeeman_energy(name):
    """The Zeeman energy is linear in a_z and in b_z: for random fields its xy part
    is a_z . sxy and its z part b_z . dz (B_h from scipy at the particles)."""
    w, o, s = setup(name, n=30)
    sxy, dz = o.spin_sources(s)
    rng = np.random.default_rng(7)
    t = dict(s)
    t["az"], t["bz"] = rng.normal(size=o.N), rng.normal(size=o.N)
    zxy = zz = 0.0
    for a in range(30):
        B = scipy_B(o, t, s["x1"][a], s["x2"][a])
        zxy += o.cfg.w * (s["sx"][a] * B[0] + s["sy"][a] * B[1])
        zz += o.cfg.w * s["sz"][a] * B[2]
    assert abs(t["az"] @ sxy - zxy) < 1e-12 * max(1.0, abs(zxy))
    assert abs(t["bz"] @ dz - zz) < 1e-12 * max(1.0, abs(zz))


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_spin_force_is_the_printed_divided_difference(name):
    """With the same increment and field, the map with spin minus the map without
    changes p by -dt hbar (DD1, DD2) of S = s . B_h: DD1 = (S(b1, b2) - S(a1, b2))/d1
    and DD2 = (S(a1, b2) - S(a1, a2))/d2, point values from scipy (legs of a third
    of a cell, so no cancellation)."""
    w, o, s = setup(name, n=12)
    rng = np.random.default_rng(3)
    ebar = s["e"]
    ga = o.G(s["az"])
    for a in range(12):
        x = np.array([s["x1"][a], s["x2"][a]])
        p = np.array([s["p1"][a], s["p2"][a]])
        d = rng.uniform(0.2, 0.4, 2) * np.array([w.dx1, w.dx2]) * rng.choice([-1.0, 1.0], 2)
        pn_s, _ = o.particle_map_s(s, a, x, p, d, ebar)
        pn_0, _ = o.particle_map(x, p, d, ebar, s["az"], ga)
        b = x + d
        S = lambda u1, u2: zeeman_density(o, s, a, u1, u2)   # noqa: E731
        dd = np.array([(S(b[0], b[1]) - S(x[0], b[1])) / d[0], (S(x[0], b[1]) - S(x[0], x[1])) / d[1]])
        np.testing.assert_allclose(pn_s - pn_0, -o.cfg.dt * o.hbar * dd, rtol=1e-9, atol=1e-14)


def test_subsystem_II_spin_rotation_against_ode_solver():
    """ds/dt = s x B_h(x) at fixed x (B_h from scipy), and p as without spin."""
    w, o, s = setup("twod16s", n=10)
    t = {k: v.copy() for k, v in s.items()}
    o.substep_II_s(t, 0.7)
    u = {k: v.copy() for k, v in s.items()}
    o.substep_II(u, 0.7)
    np.testing.assert_array_equal(t["p1"], u["p1"])
    np.testing.assert_array_equal(t["p2"], u["p2"])
    for a in range(10):
        B = scipy_B(o, s, s["x1"][a], s["x2"][a])
        s0 = np.array([s["sx"][a], s["sy"][a], s["sz"][a]])
        sol = solve_ivp(lambda _, y: np.cross(y, B), (0.0, 0.7), s0, rtol=1e-12, atol=1e-14)
        got = np.array([t["sx"][a], t["sy"][a], t["sz"][a]])
        np.testing.assert_allclose(got, sol.y[:, -1], atol=1e-10)
        assert abs(np.linalg.norm(got) - 1.0) < 1e-14
        assert abs(got @ B - s0 @ B) < 1e-14


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_substeps_with_spin_conserve_energy_and_gauss(name):
    w, o, s = setup(name, n=300)
    H0 = o.energy_s(s)
    moved = 0.0
    for call in (o.substep_I_s, o.substep_II_s, o.substep_III_s, o.substep_IV_s):
        r = call(s)
        assert r is None or r[0] == 0
        H = o.energy_s(s)
        assert abs(H[6] - H0[6]) < 2e-14 * H0[6], (call.__name__, H, H0)
        moved = max(moved, abs(H[5] - H0[5]))
        H0 = H
    assert moved > 1e-4 * abs(H0[6])   # the Zeeman term does exchange energy
    assert o.gauss_residual(s) < 1e-13


def test_lie_steps_with_spin_conserve_energy():
    w, o, s = setup("twod16s", n=400)
    H0 = o.energy_s(s)[6]
    st, kI, kIII = o.step_s(s, 3)
    assert st == 0
    assert abs(o.energy_s(s)[6] - H0) < 1e-13 * H0
    assert o.gauss_residual(s) < 1e-13
    assert np.abs(np.sqrt(s["sx"] ** 2 + s["sy"] ** 2 + s["sz"] ** 2) - 1.0).max() < 1e-14


def test_zero_hbar_reduces_to_the_plain_scheme():
    """hbar = 0: particles and fields follow the plain functions exactly (spins still
    precess in Subsystem II, which does not involve hbar)."""
    w, o, s = setup("twod16s", n=200, hbar=0.0)
    t = {k: v.copy() for k, v in s.items()}
    assert o.step_s(s, 2)[0] == 0
    assert o.step(t, 2)[0] == 0
    for k in ("x1", "x2", "p1", "p2", "e", "bz", "ez", "az"):
        np.testing.assert_array_equal(s[k], t[k])
