"""Pins of the oracle's spin terms (hbar != 0, Sections 2.1 and 4.2).

The spin enters through the Zeeman energy of the discrete Hamiltonian,
hbar sum_a w (s_y dA_z/dx - s_z dA_y/dx)(x_a), in three places: a force in
Subsystem I (a divided difference of dA/dx along the step), a constant source in
Subsystem II, and Subsystem III, which rotates each spin exactly. Pins:
* Subsystem III against an independent route to the same exact flow, scipy's
  matrix exponential of the printed generator with dA/dx from scipy splines.
  Also its invariants (|s|, s.r and the energy) and its group property;
* the divided difference of dA/dx as line means of the degree p-2 splines,
  against the plain difference quotient of scipy's spline derivative, and the
  second derivative at a zero-length step;
* brute force: Newton's method on the Subsystem I equations with the spin force
  written from scipy splines;
* energy conservation (to the Picard tolerance) and the Gauss law over runs with
  spin, for both splittings. Subsystem II alone conserves energy with its
  source, and Subsystem III alone leaves it unchanged;
* hbar = 0 decouples: positions, momenta and fields equal the run without spins
  bit for bit, while the spins still precess.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

import workloads
from oracle import Oracle, initial_state
from tests._splines import basis_integrals, periodic_spline
from tests.test_oracle_pins import eulerian


def _state(w, seidel=1, tol=1e-14, **kw):
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel, tol=tol, **kw)
    return o, initial_state(o, arr)


def _copy(s):
    return {k: v.copy() for k, v in s.items()}


def _small(n=40, hbar=0.3, seed=11, **kw):
    args = dict(M=12, L=3.0, n=n, dt=0.06, amplitude=0.4, sigma=0.5, seed=seed, hbar=hbar, spin="sphere")
    args.update(kw)
    return workloads.small(**args)


# --------------------------------------------------------------------------
# Subsystem III: the exact rotation (eq. spin_rodrigue)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("h", [0.02, 0.7])
def test_subsystem_III_is_the_matrix_exponential(h):
    """s^{n+1} = exp(h rhat) s^n with rhat = [[0, Y, Z], [-Y, 0, 0], [-Z, 0, 0]] and
    Y, Z = dA_y/dx, dA_z/dx at the particle (scipy spline derivatives here)."""
    w = _small(n=30, amplitude=1.3)
    o, s = _state(w)
    s0 = _copy(s)
    o.substep_III(s, h)
    Ay = periodic_spline(s0["ay"], w.dx, w.degree).derivative()
    Az = periodic_spline(s0["az"], w.dx, w.degree).derivative()
    for a in range(w.n_particles):
        Y, Z = float(Ay(s0["x"][a])), float(Az(s0["x"][a]))
        R = np.array([[0.0, Y, Z], [-Y, 0.0, 0.0], [-Z, 0.0, 0.0]])
        ref = expm(h * R) @ np.array([s0["sx"][a], s0["sy"][a], s0["sz"][a]])
        got = np.array([s["sx"][a], s["sy"][a], s["sz"][a]])
        np.testing.assert_allclose(got, ref, atol=2e-15)
    for k in ("x", "p", "ex", "ey", "ez", "ay", "az"):   # nothing else moves
        np.testing.assert_array_equal(s[k], s0[k])


def test_subsystem_III_invariants_and_group_property():
    """A rotation about r = (0, Z, -Y) keeps |s| and s.r. The Zeeman energy is
    hbar w s.r, so the energy is unchanged. It is an exact flow, so
    III(h1) III(h2) = III(h1 + h2)."""
    w = _small(n=50, amplitude=1.1)
    o, s = _state(w)
    H0 = o.energy(s)[4]
    a = _copy(s)
    o.substep_III(a, 0.9)
    n0 = np.sqrt(s["sx"] ** 2 + s["sy"] ** 2 + s["sz"] ** 2)
    n1 = np.sqrt(a["sx"] ** 2 + a["sy"] ** 2 + a["sz"] ** 2)
    np.testing.assert_allclose(n1, n0, atol=4e-16)
    assert abs(o.energy(a)[4] - H0) <= 1e-15 * abs(H0)
    assert np.abs(a["sx"] - s["sx"]).max() > 1e-3    # it turned
    b = _copy(s)
    o.substep_III(b, 0.35)
    o.substep_III(b, 0.55)
    for k in ("sx", "sy", "sz"):
        np.testing.assert_allclose(b[k], a[k], atol=3e-15)


def test_subsystem_III_without_field_derivative_is_the_identity():
    """Uniform transverse potential: dA/dx = 0, r = 0, the spins stay."""
    w = _small(n=20)
    o, s = _state(w)
    s["ay"][:] = 0.3
    s["az"][:] = -0.2
    s0 = _copy(s)
    o.substep_III(s, 1.0)
    for k in ("sx", "sy", "sz"):
        np.testing.assert_allclose(s[k], s0[k], atol=1e-15)


# --------------------------------------------------------------------------
# The divided difference of dA/dx (Subsystem I spin force)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3, 5])
def test_line_mean2_gives_the_divided_difference_of_the_derivative(p):
    """sum_j (G G a)_j mean_j(Lambda2) over [x0, x1] equals (A'(x1) - A'(x0))/(x1 - x0)
    for separated points. It equals A''(x0) for x1 = x0. Same on a step across a knot."""
    M, L = 10, 2.5
    dx = L / M
    o = Oracle(L=L, M=M, p=p, n=1)
    rng = np.random.default_rng(p)
    a = rng.normal(0.0, 1.0, M)
    hh = o.G(o.G(a))
    d1 = periodic_spline(a, dx, p).derivative()
    d2 = d1.derivative()
    for x0, x1 in [(0.31, 0.77), (1.01, 0.52), (2.24, 2.26), (0.9, 1.6)]:
        jlo, m2 = o.line_mean2(x0, x1)
        got = sum(m2[k] * hh[(jlo + k) % M] for k in range(len(m2)))
        ref = (float(d1(x1)) - float(d1(x0))) / (x1 - x0)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (x0, x1, got, ref)
    if p >= 3:   # A'' is continuous
        x0 = 0.83
        jlo, m2 = o.line_mean2(x0, x0)
        got = sum(m2[k] * hh[(jlo + k) % M] for k in range(len(m2)))
        assert abs(got - float(d2(x0))) <= 1e-12 * max(1.0, abs(float(d2(x0))))


def _newton_spin_I(L, M, p, dt, w, hbar, x0, p0, sy_, sz_, ex, ay, az):
    """Newton's method on the Subsystem I scheme with spin (Section 4.2), written with
    scipy splines: literal difference quotients of A and of dA/dx, basis integrals,
    M1 from its Eulerian row."""
    dx = L / M
    n = len(x0)
    Sy, Sz = periodic_spline(ay, dx, p), periodic_spline(az, dx, p)
    Dy, Dz = Sy.derivative(), Sz.derivative()
    d = 2 * (p - 1) + 1
    row = np.array([eulerian(d, k) for k in range(d)], float) / math.factorial(d) * dx
    M1 = np.zeros((M, M))
    for i in range(M):
        for k in range(-(p - 1), p):
            M1[i, (i + k) % M] += row[k + p - 1]

    def force(a, xa, xb, ebar):
        A0 = np.array([Sy(xa), Sz(xa)]); A1 = np.array([Sy(xb), Sz(xb)])
        g00 = math.sqrt(1 + p0[a] ** 2 + A0 @ A0)
        g01 = math.sqrt(1 + p0[a] ** 2 + A1 @ A1)
        f = ebar.integrate(xa, xb) / (xb - xa) - (A0 + A1) @ ((A1 - A0) / (xb - xa)) / (g00 + g01)
        f += hbar * (sz_[a] * (Dy(xb) - Dy(xa)) - sy_[a] * (Dz(xb) - Dz(xa))) / (xb - xa)
        return f, A1

    def resid(u):
        delta, e = u[:n], u[n:]
        ebar = periodic_spline(0.5 * (ex + e), dx, p - 1)
        R = np.zeros(n + M)
        cur = np.zeros(M)
        for a in range(n):
            xa, xb = x0[a], x0[a] + delta[a]
            f, A1 = force(a, xa, xb, ebar)
            p1 = p0[a] + dt * f
            g01 = math.sqrt(1 + p0[a] ** 2 + A1 @ A1)
            g11 = math.sqrt(1 + p1 ** 2 + A1 @ A1)
            R[a] = delta[a] - dt * (p0[a] + p1) / (g01 + g11)
            cur += w * basis_integrals(M, dx, p - 1, xa, xb)
        R[n:] = M1 @ (e - ex) + cur
        return R

    u = np.concatenate([dt * p0 / np.sqrt(1 + p0 ** 2), ex])
    for _ in range(30):
        R = resid(u)
        if np.abs(R).max() < 1e-16:
            break
        J = np.zeros((len(u), len(u)))
        for i in range(len(u)):
            st = 1e-7 * max(1.0, abs(u[i]))
            up, um = u.copy(), u.copy()
            up[i] += st; um[i] -= st
            J[:, i] = (resid(up) - resid(um)) / (2 * st)
        u = u - np.linalg.solve(J, R)
    delta, e = u[:n], u[n:]
    ebar = periodic_spline(0.5 * (ex + e), dx, p - 1)
    p1 = np.array([p0[a] + dt * force(a, x0[a], x0[a] + delta[a], ebar)[0] for a in range(n)])
    return delta, p1, e


@pytest.mark.parametrize("seidel", [0, 1])
@pytest.mark.parametrize("n", [1, 3])
def test_spin_picard_matches_newton(n, seidel):
    w_ = workloads.small(M=8, L=2.0, n=n, dt=0.08, amplitude=0.6, sigma=0.6, seed=40 + n, hbar=0.5,
                         spin="sphere")
    o, s = _state(w_, seidel=seidel)
    x0, p0, ex0 = s["x"].copy(), s["p"].copy(), s["ex"].copy()
    st, k, r = o.substep_I(s)
    assert st == 0 and k >= 2
    delta, p1, e = _newton_spin_I(w_.L, w_.M, w_.degree, w_.dt, w_.weight, w_.hbar, x0, p0, s["sy"], s["sz"],
                                  ex0, s["ay"], s["az"])
    got = np.mod(s["x"] - x0 + w_.L / 2, w_.L) - w_.L / 2
    np.testing.assert_allclose(got, delta, atol=1e-13)
    np.testing.assert_allclose(s["p"], p1, atol=1e-12)
    np.testing.assert_allclose(s["ex"], e, atol=1e-12)
    # the spin force is really there: without it the momenta differ
    w0 = w_.scaled(hbar=0.0)
    o0, s0 = _state(w0, seidel=seidel)
    o0.substep_I(s0)
    assert np.abs(s0["p"] - s["p"]).max() > 1e-6


# --------------------------------------------------------------------------
# Invariants over substeps and runs
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sub", ["I", "I_adjoint", "II"])
def test_substeps_with_spin_conserve_energy(sub):
    """Every substep is a discrete gradient of the Hamiltonian with its Zeeman term, so
    H is kept to the iteration tolerance (Subsystem II keeps it whatever the source,
    which is linear in a)."""
    w = _small(n=60, hbar=0.8, amplitude=0.9, dt=0.08)
    o, s = _state(w, tol=1e-15)
    H0 = o.energy(s)[4]
    z0 = o.last_zeeman
    st = getattr(o, "substep_" + sub)(s)[0]
    assert st == 0
    H1 = o.energy(s)[4]
    assert abs(o.last_zeeman - z0) > 1e-6 * abs(H0)    # the Zeeman part changed
    assert abs(H1 - H0) <= 2e-14 * abs(H0)


@pytest.mark.parametrize("splitting", [0, 1])
def test_spin_runs_conserve_energy_and_gauss(splitting):
    """paper52 (Section 5.2 setup) with 1500 particles: energy to the tolerance, Gauss's
    law to round-off, |s| = 1, and the spin moment S_z leaves 1."""
    w = workloads.get("paper52").scaled(n_particles=1500)
    o, s = _state(w, tol=1e-13, splitting=splitting)
    st, kI, kII, E = o.step(s, 25, energies=True)
    assert st == 0
    H = E[:, 4]
    assert np.abs(H - H[0]).max() <= 1e-12 * H[0]
    assert o.gauss_residual(s["x"], s["ex"]) <= 1e-13
    nrm = np.sqrt(s["sx"] ** 2 + s["sy"] ** 2 + s["sz"] ** 2)
    np.testing.assert_allclose(nrm, 1.0, atol=1e-14)
    assert s["sz"].mean() < 0.999


def test_zero_hbar_decouples_the_spins():
    """With hbar = 0 the spins precess but act on nothing: the particles and fields of
    a run with spins equal those of the run without, bit for bit."""
    w = workloads.get("paper52").scaled(n_particles=800, hbar=0.0)
    o, s = _state(w, tol=1e-13)
    o2 = Oracle.from_workload(w, seidel=1, tol=1e-13)
    s2 = {k: v.copy() for k, v in s.items() if k not in ("sx", "sy", "sz")}
    assert o.step(s, 6)[0] == 0 and o2.step(s2, 6)[0] == 0
    for k in s2:
        np.testing.assert_array_equal(s[k], s2[k])
    assert np.abs(s["sz"] - 1.0).max() > 1e-6


def test_symmetric_splitting_with_spin_is_second_order():
    """Richardson ratios |u_h - u_{h/2}| / |u_{h/2} - u_{h/4}| over a fixed time: 4 for the
    symmetric composition I(h/2) III(h/2) II(h) III(h/2) I*(h/2) with spin (Subsystems II
    and III are self-adjoint), 2 for Lie-Trotter I, II, III."""
    w = workloads.small("ord", M=16, L=2 * math.pi, n=64, dt=0.05, amplitude=0.3, sigma=0.3, seed=3,
                        hbar=0.3, spin="sphere")
    arr = workloads.generate(w)
    T = 0.8

    def run(ns, splitting):
        o = Oracle(L=w.L, M=w.M, p=w.degree, n=w.n_particles, dt=T / ns, tol=1e-14, seidel=1,
                   splitting=splitting, kmax=100, hbar=w.hbar)
        s = initial_state(o, arr)
        assert o.step(s, ns)[0] == 0
        return s

    def dist(a, b):
        d = np.mod(a["x"] - b["x"] + w.L / 2, w.L) - w.L / 2
        return max([np.abs(d).max()] + [np.abs(a[k] - b[k]).max()
                                         for k in ("p", "sx", "sy", "sz", "ex", "ey", "ez", "ay", "az")])

    ratios = {}
    for splitting in (0, 1):
        runs = [run(ns, splitting) for ns in (16, 32, 64, 128)]
        d = [dist(runs[i], runs[i + 1]) for i in range(3)]
        ratios[splitting] = [d[0] / d[1], d[1] / d[2]]
    assert all(3.6 <= r <= 4.4 for r in ratios[1]), ratios
    assert ratios[0][1] <= 2.6, ratios
