"""Pins of the oracle's adjoint Subsystem I scheme, the symmetric splitting built
from it, the previous-step start and the V1 field evaluation.

The adjoint scheme takes the discrete gradient of Section 4.1 with the two
particle coordinates varied in the other order (p first at x^n, then x at
p^{n+1}) in place of the order of the Subsystem I scheme of Section 4.2.  Pins:
* it is the adjoint: the scheme run backwards (step -h) undoes it, a property of
  the pair that a wrong sign, a swapped gamma or a wrong end point breaks;
* brute force: an independent Newton solve of its equations, written with scipy
  splines, gives the same state;
* closed forms: free streaming, and the exact relativistic motion in a uniform
  E_x that any discrete gradient of this form reproduces;
* invariants: the Gauss law and the energy held by the substep;
* the symmetric composition I(dt/2), II(dt), adjoint I(dt/2) is second order
  (Richardson ratios of 4 per halving of dt), Lie-Trotter first order.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import Oracle, initial_state
from tests._splines import basis_integrals, periodic_spline
from tests.test_oracle_pins import _zero_field_state, eulerian


def _state(w, seidel=1, tol=1e-14, **kw):
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel, tol=tol, **kw)
    return o, initial_state(o, arr)


def _copy(s):
    return {k: v.copy() for k, v in s.items()}


def _dist(a, b, L):
    d = np.mod(a["x"] - b["x"] + L / 2, L) - L / 2
    return max([np.abs(d).max()] + [np.abs(a[k] - b[k]).max() for k in ("p", "ex", "ey", "ez", "ay", "az")])


# --------------------------------------------------------------------------
# the adjoint Subsystem I scheme
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seidel", [0, 1])
@pytest.mark.parametrize("h", [0.05, 0.11])
def test_adjoint_is_undone_by_the_scheme_run_backwards(h, seidel):
    """Phi*_h = (Phi_{-h})^{-1} defines the adjoint of a one-step map: the Subsystem I
    scheme over -h, applied to the adjoint's result, returns the initial state (to the
    Picard tolerance).  A Jacobi or Seidel iteration of the backward step reaches the
    same fixed point, so both are checked."""
    w = workloads.small(M=12, L=3.0, n=40, dt=h, amplitude=0.4, sigma=0.5, seed=8)
    o, s0 = _state(w, seidel=seidel, tol=1e-15)
    s = _copy(s0)
    st, k, r = o.substep_I_adjoint(s, h)
    assert st == 0 and k >= 3
    assert _dist(s, s0, w.L) > 1e-3          # it moved
    st, k, r = o.substep_I(s, -h)
    assert st == 0
    assert _dist(s, s0, w.L) <= 2e-14


def test_scheme_is_undone_by_the_adjoint_run_backwards():
    """The same relation read the other way: Phi*_{-h} o Phi_h = identity."""
    w = workloads.small(M=12, L=3.0, n=40, dt=0.07, amplitude=0.4, sigma=0.5, seed=9)
    o, s0 = _state(w, tol=1e-15)
    s = _copy(s0)
    assert o.substep_I(s, 0.07)[0] == 0
    assert o.substep_I_adjoint(s, -0.07)[0] == 0
    assert _dist(s, s0, w.L) <= 2e-14


def _newton_adjoint_I(L, M, p, h, w, x0, p0, ex, ay, az):
    """Solve the adjoint scheme for (delta, p1, e) with Newton's method; residuals written
    from the discrete gradients with scipy splines (difference quotients of gamma, exact
    basis integrals, M1 from its Eulerian row)."""
    dx = L / M
    n = len(x0)
    sy, sz = periodic_spline(ay, dx, p), periodic_spline(az, dx, p)
    d = 2 * (p - 1) + 1
    row = np.array([eulerian(d, k) for k in range(d)], float) / math.factorial(d) * dx
    M1 = np.zeros((M, M))
    for i in range(M):
        for k in range(-(p - 1), p):
            M1[i, (i + k) % M] += row[k + p - 1]

    def gamma(x, pp):
        return math.sqrt(1 + pp * pp + sy(x) ** 2 + sz(x) ** 2)

    def resid(u):
        delta, p1, e = u[:n], u[n:2 * n], u[2 * n:]
        ebar = periodic_spline(0.5 * (ex + e), dx, p - 1)
        R = np.zeros(2 * n + M)
        cur = np.zeros(M)
        for a in range(n):
            xa, xb = x0[a], x0[a] + delta[a]
            grad_p = (gamma(xa, p1[a]) - gamma(xa, p0[a])) / (p1[a] - p0[a])
            grad_x = (gamma(xb, p1[a]) - gamma(xa, p1[a])) / (xb - xa)
            R[a] = delta[a] - h * grad_p
            R[n + a] = p1[a] - p0[a] - h * (ebar.integrate(xa, xb) / (xb - xa) - grad_x)
            cur += w * basis_integrals(M, dx, p - 1, xa, xb)
        R[2 * n:] = M1 @ (e - ex) + cur
        return R

    u = np.concatenate([h * p0 / np.sqrt(1 + p0 ** 2), p0 + 1e-3, ex])
    for _ in range(40):
        R = resid(u)
        if np.abs(R).max() < 1e-15:
            break
        J = np.zeros((len(u), len(u)))
        for i in range(len(u)):
            st = 1e-7 * max(1.0, abs(u[i]))
            up, um = u.copy(), u.copy()
            up[i] += st; um[i] -= st
            J[:, i] = (resid(up) - resid(um)) / (2 * st)
        u = u - np.linalg.solve(J, R)
    return u[:n], u[n:2 * n], u[2 * n:]


@pytest.mark.parametrize("n", [1, 3])
def test_adjoint_picard_matches_newton(n):
    w_ = workloads.small(M=8, L=2.0, n=n, dt=0.08, amplitude=0.4, sigma=0.6, seed=30 + n)
    o, s = _state(w_)
    x0, p0, ex0 = s["x"].copy(), s["p"].copy(), s["ex"].copy()
    st, k, r = o.substep_I_adjoint(s)
    assert st == 0 and k >= 2
    delta, p1, e = _newton_adjoint_I(w_.L, w_.M, w_.degree, w_.dt, w_.weight, x0, p0, ex0, s["ay"], s["az"])
    got = np.mod(s["x"] - x0 + w_.L / 2, w_.L) - w_.L / 2
    np.testing.assert_allclose(got, delta, atol=1e-13)
    np.testing.assert_allclose(s["p"], p1, atol=1e-12)
    np.testing.assert_allclose(s["ex"], e, atol=1e-12)


def test_adjoint_free_streaming_and_uniform_field():
    """No transverse field gradient and w = 0: the adjoint step is the exact relativistic
    motion, p+ = p + h E, displacement (gamma(p+) - gamma(p)) / E, and free streaming
    dx = h p / sqrt(1 + p^2 + c^2) under a uniform a_y = c."""
    M, L, h = 16, 4.0, 0.05
    rng = np.random.default_rng(5)
    x = rng.uniform(0, L, 30)
    p = rng.normal(0, 0.6, 30)
    for c in (0.0, 0.7):
        o = Oracle(L=L, M=M, p=3, n=len(x), w=0.0, dt=h, tol=1e-15)
        s = _zero_field_state(o, x, p, ay=np.full(M, c))
        assert o.substep_I_adjoint(s)[0] == 0
        np.testing.assert_array_equal(s["p"], p)
        np.testing.assert_allclose(s["x"], np.mod(x + h * p / np.sqrt(1 + p * p + c * c), L), atol=1e-14)
    E = 0.37
    o = Oracle(L=L, M=M, p=3, n=len(x), w=0.0, dt=h, tol=1e-15)
    s = _zero_field_state(o, x, p, ex=np.full(M, E))
    assert o.substep_I_adjoint(s)[0] == 0
    p1 = p + h * E
    np.testing.assert_allclose(s["p"], p1, rtol=1e-14, atol=1e-15)
    disp = (np.sqrt(1 + p1 ** 2) - np.sqrt(1 + p ** 2)) / E
    np.testing.assert_allclose(np.mod(s["x"] - x + L / 2, L) - L / 2, disp, atol=1e-14)


@pytest.mark.parametrize("name,n", [("langmuir64", 4000), ("paper51", 4000)])
def test_adjoint_holds_gauss_and_energy(name, n):
    """Second remark of Section 4.2 (the deposit and the position come from one
    increment) and the discrete-gradient identity of Section 4.1 for the adjoint."""
    w_ = workloads.get(name)
    arr = workloads.generate(w_, n=n)
    o = Oracle.from_workload(w_, n=n, seidel=1)
    s = initial_state(o, arr)
    g0, r0 = o.gauss_residual(s["x"], s["ex"], vec=True)
    H0 = o.energy(s)[4]
    for _ in range(3):
        st, k, r = o.substep_I_adjoint(s)
        assert st == 0
    g1, r1 = o.gauss_residual(s["x"], s["ex"], vec=True)
    assert np.abs(r1 - r0).max() <= 1e-14
    assert abs(o.energy(s)[4] - H0) / H0 <= 5e-13


def test_adjoint_map_agrees_with_its_own_fixed_point():
    """At the committed state the map reproduces the committed momentum and increment
    (the fixed point the Picard test stopped at), particle by particle."""
    w_ = workloads.small(M=10, L=2.5, n=25, dt=0.06, amplitude=0.4, sigma=0.5, seed=12)
    o, s0 = _state(w_)
    s = _copy(s0)
    assert o.substep_I_adjoint(s)[0] == 0
    gy, gz = o.G(s0["ay"]), o.G(s0["az"])
    ebar = 0.5 * (s0["ex"] + s["ex"])
    for a in range(w_.n_particles):
        delta = np.mod(s["x"][a] - s0["x"][a] + w_.L / 2, w_.L) - w_.L / 2
        d_of_P, Pn, dn = o.particle_map_adjoint(s0["x"][a], s0["p"][a], s["p"][a], s0["ay"], s0["az"], gy, gz, ebar)
        assert abs(d_of_P - delta) <= 1e-15
        assert abs(Pn - s["p"][a]) <= 1e-13
        assert abs(dn - delta) <= 1e-13


# --------------------------------------------------------------------------
# splitting order
# --------------------------------------------------------------------------

def test_symmetric_splitting_is_second_order_lie_trotter_first():
    """Richardson ratios |u_h - u_{h/2}| / |u_{h/2} - u_{h/4}| over a fixed time T: 4 for
    the symmetric composition I(dt/2) o II(dt) o adjoint I(dt/2) (a symmetric method built
    from a map and its adjoint around a symmetric one), 2 for Lie-Trotter."""
    w = workloads.small("ord", M=16, L=2 * math.pi, n=64, dt=0.05, amplitude=0.3, sigma=0.3, seed=3)
    arr = workloads.generate(w)
    T = 0.8

    def run(ns, splitting):
        o = Oracle(L=w.L, M=w.M, p=w.degree, n=w.n_particles, dt=T / ns, tol=1e-14, seidel=1,
                   splitting=splitting, kmax=100)
        s = initial_state(o, arr)
        st, kI, kII, _ = o.step(s, ns)
        assert st == 0
        if splitting:
            assert (o.last_sweeps_I2 > 0).all()
        return s

    ratios, last = {}, {}
    for splitting in (0, 1):
        runs = [run(ns, splitting) for ns in (16, 32, 64, 128)]
        d = [_dist(runs[i], runs[i + 1], w.L) for i in range(3)]
        ratios[splitting] = [d[0] / d[1], d[1] / d[2]]
        last[splitting] = d[2]
    assert all(3.6 <= r <= 4.4 for r in ratios[1]), ratios
    assert ratios[0][1] <= 2.6, ratios
    assert last[1] <= 0.5 * last[0]


def test_symmetric_step_conserves_energy_and_gauss():
    w_ = workloads.get("langmuir64")
    arr = workloads.generate(w_, n=3000)
    o = Oracle.from_workload(w_, n=3000, seidel=1, splitting=1)
    s = initial_state(o, arr)
    g0, r0 = o.gauss_residual(s["x"], s["ex"], vec=True)
    st, kI, kII, E = o.step(s, 20, energies=True)
    assert st == 0
    assert np.abs(E[:, 4] - E[0, 4]).max() / E[0, 4] <= 1e-12
    g1, r1 = o.gauss_residual(s["x"], s["ex"], vec=True)
    assert np.abs(r1 - r0).max() <= 1e-14


# --------------------------------------------------------------------------
# previous-step start
# --------------------------------------------------------------------------

def test_previous_step_start_reaches_the_same_fixed_point():
    """Starting each Subsystem I iteration from the last committed increments changes only
    the iterates, not the fixed point: ten steps agree with the explicit start to within
    the Picard tolerance's effect."""
    w_ = workloads.get("langmuir64")
    arr = workloads.generate(w_, n=2000)
    out = []
    for warm in (False, True):
        o = Oracle.from_workload(w_, n=2000, seidel=1, warm_previous=warm)
        s = initial_state(o, arr)
        st, kI, kII, _ = o.step(s, 10)
        assert st == 0
        out.append((s, kI))
    assert _dist(out[0][0], out[1][0], w_.L) <= 1e-11
    assert out[0][1][0] == out[1][1][0]   # the first step has no previous increments


def test_committed_increments_are_returned():
    w_ = workloads.small(M=8, L=2.0, n=20, dt=0.05, amplitude=0.3, sigma=0.4, seed=4)
    for adjoint in (False, True):
        o, s0 = _state(w_)
        s = _copy(s0)
        dc = np.zeros(w_.n_particles)
        st = (o.substep_I_adjoint(s, dcommit=dc) if adjoint else o.substep_I(s, dcommit=dc))[0]
        assert st == 0
        np.testing.assert_allclose(np.mod(s0["x"] + dc, w_.L), s["x"], atol=1e-15)


# --------------------------------------------------------------------------
# V1 field evaluation (Section 3.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3, 5])
def test_field1_partition_of_unity_and_derivative_of_field0(p):
    """sum_j Lambda1_j = 1, and d/dx sum_j c_j Lambda0_j = sum_j (G c)_j Lambda1_j (the
    derivative relation of Section 3.1), the latter against a central difference of the
    V0 field."""
    M, L = 12, 3.0
    o = Oracle(L=L, M=M, p=p, n=1)
    rng = np.random.default_rng(p)
    c = rng.normal(size=M)
    gc = o.G(c)
    for x in rng.uniform(0, L, 25):
        assert o.field1(np.ones(M), x) == pytest.approx(1.0, abs=1e-14)
        h = 1e-5
        fd = (o.field0(c, x + h) - o.field0(c, x - h)) / (2 * h)
        assert o.field1(gc, x) == pytest.approx(fd, abs=1e-7)
