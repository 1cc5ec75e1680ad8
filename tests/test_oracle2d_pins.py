"""Pins of the 2D FP64 oracle (Sections 2.2, 3.2, 4.3) against what the paper and
mathematics fix, never against a re-typing of the oracle's own formulas:

* tensor-product fields against scipy's B-splines (tests/_splines.py);
* the de Rham relations of the spaces: grad of a V0 field is the V1 field G a,
  curl of a V1 field is the V2 field C e (finite differences of point values),
  C G = 0, mass matrices against brute-force quadrature of point values;
* path means against brute-force sampling, the divided-difference identity, and
  charge continuity G^T J = Lambda0(x^{n+1}) - Lambda0(x^n);
* reduction to the (separately pinned) 1D oracle for data that do not vary in x2;
* the committed Subsystem I state against the printed scheme, evaluated
  independently (divided differences as printed, path means by sampling);
* Subsystem II against scipy's ODE solver, Subsystem IV against the exact
  travelling wave of Maxwell's equations (convergence), energy and Gauss laws.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import Oracle, initial_state
from oracle.twod import Oracle2D, initial_state2d
from tests._splines import basis_values
from workloads.twod import generate2d, get2d, small2d


def scipy_eval(o, coef, d1, d2, x1, x2):
    c = o.cfg
    v1 = basis_values(c.M1, c.L1 / c.M1, d1, x1 % c.L1)
    v2 = basis_values(c.M2, c.L2 / c.M2, d2, x2 % c.L2)
    return v1 @ np.asarray(coef).reshape(c.M1, c.M2) @ v2


def small_oracle(p=3, M1=6, M2=5, n=1, L1=3.0, L2=2.5, **kw):
    return Oracle2D(L1=L1, L2=L2, M1=M1, M2=M2, p=p, n=n, **kw)


# --------------------------------------------------------------------------
# Section 3.2: spaces and operators
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3, 4])
def test_tensor_fields_match_scipy(p):
    o = small_oracle(p=p)
    rng = np.random.default_rng(p)
    for d1, d2 in [(p, p), (p - 1, p), (p, p - 1), (p - 1, p - 1)]:
        coef = rng.normal(size=o.N)
        for x1, x2 in rng.uniform([0, 0], [3.0, 2.5], (6, 2)):
            assert o.eval(coef, d1, d2, x1, x2) == pytest.approx(scipy_eval(o, coef, d1, d2, x1, x2),
                                                                   rel=1e-13, abs=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_gradient_and_curl_are_exact(p):
    """d/dx_k of the V0 field equals the V1 field G a component k; the curl
    d1 E2 - d2 E1 of a V1 field equals the V2 field C e (central differences of
    point values, step 1e-5); C G = 0."""
    o = small_oracle(p=p)
    rng = np.random.default_rng(10 + p)
    a = rng.normal(size=o.N)
    e = rng.normal(size=2 * o.N)
    g, ce = o.G(a), o.C(e)
    N, h = o.N, 1e-5
    for x1, x2 in rng.uniform([0, 0], [3.0, 2.5], (6, 2)):
        d1 = (o.eval(a, p, p, x1 + h, x2) - o.eval(a, p, p, x1 - h, x2)) / (2 * h)
        d2 = (o.eval(a, p, p, x1, x2 + h) - o.eval(a, p, p, x1, x2 - h)) / (2 * h)
        assert d1 == pytest.approx(o.eval(g[:N], p - 1, p, x1, x2), abs=1e-8)
        assert d2 == pytest.approx(o.eval(g[N:], p, p - 1, x1, x2), abs=1e-8)
        dE2 = (o.eval(e[N:], p, p - 1, x1 + h, x2) - o.eval(e[N:], p, p - 1, x1 - h, x2)) / (2 * h)
        dE1 = (o.eval(e[:N], p - 1, p, x1, x2 + h) - o.eval(e[:N], p - 1, p, x1, x2 - h)) / (2 * h)
        assert dE2 - dE1 == pytest.approx(o.eval(ce, p - 1, p - 1, x1, x2), abs=1e-7)
    assert np.abs(o.C(g)).max() <= 1e-12 * np.abs(g).max()


def test_transposes_are_adjoints():
    o = small_oracle(p=3)
    rng = np.random.default_rng(3)
    a, u, b = rng.normal(size=o.N), rng.normal(size=2 * o.N), rng.normal(size=o.N)
    assert o.G(a) @ u == pytest.approx(a @ o.GT(u), rel=1e-13)
    assert o.C(u) @ b == pytest.approx(u @ o.CT(b), rel=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_mass_matrices_against_quadrature(p):
    """x^T M y = int X Y over the domain, by tensor Gauss-Legendre on every cell
    (10 points per direction, exact for these degrees) of point values."""
    o = small_oracle(p=p, M1=4, M2=3, L1=2.0, L2=1.5)
    rng = np.random.default_rng(20 + p)
    gx, gw = np.polynomial.legendre.leggauss(10)
    c = o.cfg
    h1, h2 = c.L1 / c.M1, c.L2 / c.M2
    pts1 = np.concatenate([(i + 0.5 + 0.5 * gx) * h1 for i in range(c.M1)])
    pts2 = np.concatenate([(i + 0.5 + 0.5 * gx) * h2 for i in range(c.M2)])
    w1 = np.tile(0.5 * gw * h1, c.M1)
    w2 = np.tile(0.5 * gw * h2, c.M2)

    def integral(f, g, d1, d2):
        s = 0.0
        for a, wa in zip(pts1, w1):
            for b, wb in zip(pts2, w2):
                s += wa * wb * o.eval(f, d1, d2, a, b) * o.eval(g, d1, d2, a, b)
        return s

    x, y = rng.normal(size=o.N), rng.normal(size=o.N)
    assert x @ o.M0(y) == pytest.approx(integral(x, y, p, p), rel=1e-12)
    assert x @ o.M2(y) == pytest.approx(integral(x, y, p - 1, p - 1), rel=1e-12)
    u, v = rng.normal(size=2 * o.N), rng.normal(size=2 * o.N)
    N = o.N
    expect = integral(u[:N], v[:N], p - 1, p) + integral(u[N:], v[N:], p, p - 1)
    assert u @ o.M1(v) == pytest.approx(expect, rel=1e-12)
    # M0 1 = dx1 dx2 1 (partition of unity); K 1 = 0
    np.testing.assert_allclose(o.M0(np.ones(N)), h1 * h2, rtol=1e-14)
    assert np.abs(o.K(np.ones(N))).max() < 1e-12


# --------------------------------------------------------------------------
# Section 4.3, Subsystem I: path means and charge continuity
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seg", [((0.3, 0.4), (0.9, 1.3)), ((2.9, 0.1), (3.3, -0.4)), ((1.0, 1.0), (1.0, 1.7)),
                                 ((0.75, 0.5), (0.75, 0.5))])
def test_path_mean_against_sampling(seg):
    """Mean of a tensor-product field along a straight segment (crossing grid lines
    in both directions, wrapping the domain, axis-parallel, zero length) against
    the composite midpoint rule with 20000 points."""
    o = small_oracle(p=3)
    rng = np.random.default_rng(4)
    coef = rng.normal(size=o.N)
    a, b = np.array(seg[0]), np.array(seg[1])
    s = (np.arange(20000) + 0.5) / 20000
    for d1, d2 in [(3, 3), (2, 3), (3, 2)]:
        brute = np.mean([o.eval(coef, d1, d2, *(a + t * (b - a))) for t in s])
        assert o.line_mean(coef, d1, d2, a, b) == pytest.approx(brute, abs=2e-8)


def test_leg_means_are_divided_differences():
    """Mean of dA/dx2 along a vertical leg and of dA/dx1 along a horizontal leg equal
    the divided differences of A printed in the Subsystem I discrete gradient."""
    o = small_oracle(p=3)
    rng = np.random.default_rng(5)
    a = rng.normal(size=o.N)
    g = o.G(a)
    N = o.N
    x1, x2, y1, y2 = 0.4, 1.1, 1.35, 0.2
    d2 = o.line_mean(g[N:], 3, 2, (x1, x2), (x1, y2))
    d1 = o.line_mean(g[:N], 2, 3, (x1, y2), (y1, y2))
    assert d2 == pytest.approx((o.eval(a, 3, 3, x1, y2) - o.eval(a, 3, 3, x1, x2)) / (y2 - x2), rel=1e-12)
    assert d1 == pytest.approx((o.eval(a, 3, 3, y1, y2) - o.eval(a, 3, 3, x1, y2)) / (y1 - x1), rel=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_charge_continuity_of_the_path_current(p):
    """G^T (sum_a path mean of Lambda1 times the increment) = Lambda0(X^{n+1}) -
    Lambda0(X^n): the identity behind the exact discrete Gauss law of Subsystem I."""
    o = small_oracle(p=p)
    rng = np.random.default_rng(6 + p)
    N = o.N
    J = np.zeros(2 * N)
    rho0, rho1 = np.zeros(N), np.zeros(N)
    for _ in range(5):
        a = rng.uniform([0, 0], [3.0, 2.5])
        b = a + rng.uniform(-0.6, 0.6, 2)
        d = b - a
        o.line_deposit(p - 1, p, a, b, d[0], J[:N])
        o.line_deposit(p, p - 1, a, b, d[1], J[N:])
        o.line_deposit(p, p, a, a, 1.0, rho0)
        o.line_deposit(p, p, b, b, 1.0, rho1)
    np.testing.assert_allclose(o.GT(J), rho1 - rho0, atol=1e-14)


# --------------------------------------------------------------------------
# Reduction to the 1D oracle (x2-independent data)
# --------------------------------------------------------------------------

def _reduced_pair(p=3, n1=40, M1=12, M2=4, seed=8, tol=1e-14):
    """A 1D state (A_y = 0, e_y = 0) and the 2D state that repeats it along x2: each
    1D particle copied to x2 = (j + theta) dx2, j < M2, with weight w1D dx2 and p2 = 0;
    coefficients repeated along i2."""
    rng = np.random.default_rng(seed)
    L1, L2 = 4.0, 2.0
    dx2 = L2 / M2
    x = rng.uniform(0, L1, n1)
    p_ = rng.normal(0, 0.3, n1)
    g = (np.arange(M1) + 0.5 * (p + 1)) * L1 / M1
    az1 = 0.4 * np.cos(2 * math.pi * g / L1) + 0.1 * rng.normal(size=M1)
    ez1 = 0.3 * np.sin(2 * math.pi * g / L1)
    o1 = Oracle(L=L1, M=M1, p=p, n=n1, dt=0.05, tol=tol)
    s1 = initial_state(o1, {"x": x, "p": p_, "ey": np.zeros(M1), "ez": ez1, "ay": np.zeros(M1), "az": az1})
    theta = rng.uniform(0, 1, n1)
    x1 = np.repeat(x, M2)
    x2 = ((np.tile(np.arange(M2), n1) + np.repeat(theta, M2)) * dx2) % L2
    o2 = Oracle2D(L1=L1, L2=L2, M1=M1, M2=M2, p=p, n=n1 * M2, w=(L1 / n1) * dx2, dt=0.05, tol=tol)
    rep = lambda v: np.repeat(v, M2)   # noqa: E731  (i1 M2 + i2 layout)
    s2 = {"x1": x1, "x2": x2, "p1": np.repeat(p_, M2), "p2": np.zeros(n1 * M2),
          "e": np.concatenate([rep(s1["ex"]), np.zeros(M1 * M2)]), "bz": np.zeros(M1 * M2),
          "ez": rep(ez1), "az": rep(az1)}
    return o1, s1, o2, s2


def test_subsystem_I_reduces_to_1d():
    o1, s1, o2, s2 = _reduced_pair()
    assert o2.gauss_residual(s2) < 1e-13
    st1, k1, _ = o1.substep_I(s1)
    st2, k2, _ = o2.substep_I(s2)
    assert st1 == st2 == 0 and k1 == k2
    M2 = o2.cfg.M2
    np.testing.assert_allclose(s2["x1"].reshape(-1, M2), np.repeat(s1["x"][:, None], M2, 1), atol=1e-14)
    np.testing.assert_allclose(s2["p1"].reshape(-1, M2), np.repeat(s1["p"][:, None], M2, 1), atol=1e-14)
    assert np.abs(s2["p2"]).max() == 0.0
    N = o2.N
    np.testing.assert_allclose(s2["e"][:N].reshape(-1, M2), np.repeat(s1["ex"][:, None], M2, 1), atol=1e-14)
    assert np.abs(s2["e"][N:]).max() < 1e-15


def test_subsystem_III_reduces_to_1d():
    # tolerance well above round-off so that both stop on the same iterate
    o1, s1, o2, s2 = _reduced_pair(seed=9, tol=1e-12)
    st1, k1, _ = o1.substep_II(s1)
    st2, k2, _ = o2.substep_III(s2)
    assert st1 == st2 == 0 and k1 == k2
    M2 = o2.cfg.M2
    np.testing.assert_allclose(s2["ez"].reshape(-1, M2), np.repeat(s1["ez"][:, None], M2, 1), atol=1e-14)
    np.testing.assert_allclose(s2["az"].reshape(-1, M2), np.repeat(s1["az"][:, None], M2, 1), atol=1e-14)


# --------------------------------------------------------------------------
# Subsystem I in 2D: the printed scheme, energy, Gauss
# --------------------------------------------------------------------------

def test_subsystem_I_commit_satisfies_the_printed_scheme():
    """After the Picard iteration the committed (x^{n+1}, p^{n+1}, e^{n+1}) satisfy the
    printed Subsystem I scheme, every term evaluated independently: point values by
    scipy, the divided differences of A_z as printed (x2 varied first at x1^n), the
    path means of Lambda1^T (e^n + e^{n+1})/2 by 4000-point sampling, and the field
    update through the oracle's own M1 applied to the sampled path means."""
    w = small2d(n=4, M1=5, M2=4, L1=2.5, L2=2.0, degree=3, tol=1e-14)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, generate2d(w))
    s0 = {k: v.copy() for k, v in s.items()}
    assert o.substep_I(s)[0] == 0
    c, N, dt = o.cfg, o.N, o.cfg.dt
    ebar = 0.5 * (s0["e"] + s["e"])
    tt = (np.arange(4000) + 0.5) / 4000
    J = np.zeros(2 * N)
    for a in range(c.n):
        xa = np.array([s0["x1"][a], s0["x2"][a]])
        pa = np.array([s0["p1"][a], s0["p2"][a]])
        pb = np.array([s["p1"][a], s["p2"][a]])
        d = np.array([s["x1"][a] - xa[0], s["x2"][a] - xa[1]])
        d = (d + np.array([c.L1, c.L2]) / 2) % np.array([c.L1, c.L2]) - np.array([c.L1, c.L2]) / 2
        xb = xa + d
        A = lambda u1, u2: scipy_eval(o, s0["az"], 3, 3, u1, u2)   # noqa: E731
        Aa, Ab = A(*xa), A(*xb)
        D1 = (A(xb[0], xb[1]) - A(xa[0], xb[1])) / d[0]
        D2 = (A(xa[0], xb[1]) - A(xa[0], xa[1])) / d[1]
        gam = lambda p_, A_: math.sqrt(1 + p_ @ p_ + A_ * A_)   # noqa: E731
        ga, gb, gc = gam(pa, Aa), gam(pa, Ab), gam(pb, Ab)
        # x update
        np.testing.assert_allclose(d / dt, (pa + pb) / (gb + gc), atol=1e-11)
        # p update: path mean of E by sampling
        E1 = np.mean([o.eval(ebar[:N], 2, 3, *(xa + t * d)) for t in tt])
        E2 = np.mean([o.eval(ebar[N:], 3, 2, *(xa + t * d)) for t in tt])
        F = -(Aa + Ab) / (ga + gb) * np.array([D1, D2])
        np.testing.assert_allclose((pb - pa) / dt, np.array([E1, E2]) + F, atol=5e-8)
        # current of this particle by sampling the basis along the path
        for t in tt:
            o.line_deposit(2, 3, xa + t * d, xa + t * d, c.w * d[0] / len(tt), J[:N])
            o.line_deposit(3, 2, xa + t * d, xa + t * d, c.w * d[1] / len(tt), J[N:])
    np.testing.assert_allclose(o.M1(s["e"] - s0["e"]), -J, atol=5e-8)


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_substeps_conserve_energy_and_gauss(name):
    w = get2d(name).scaled(n_particles=300)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, generate2d(w))
    assert o.gauss_residual(s) < 1e-13
    H = o.energy(s)[5]
    for sub in ("substep_I", "substep_II", "substep_III", "substep_IV"):
        out = getattr(o, sub)(s)
        if out is not None:
            assert out[0] == 0
        H1 = o.energy(s)[5]
        assert abs(H1 - H) <= 1e-13 * H, sub
        assert o.gauss_residual(s) < 1e-13, sub
        H = H1


def test_subsystem_I_empty_and_single_particle():
    w = small2d(n=1)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, generate2d(w))
    H = o.energy(s)[5]
    assert o.substep_I(s)[0] == 0
    assert abs(o.energy(s)[5] - H) < 1e-13 * H
    o0 = Oracle2D(L1=2, L2=2, M1=4, M2=4, p=2, n=0, w=0.0)
    s0 = {k: np.zeros(2 * 16 if k == "e" else (0 if k in ("x1", "x2", "p1", "p2") else 16)) for k in
          ("x1", "x2", "p1", "p2", "e", "bz", "ez", "az")}
    s0["e"][:16] = 0.1
    st, k, r = o0.substep_I(s0)
    assert st == 0 and k == 1 and np.all(s0["e"][:16] == 0.1)


# --------------------------------------------------------------------------
# Subsystem II: rotation by B_z
# --------------------------------------------------------------------------

def test_subsystem_II_against_ode_solver():
    w = small2d(n=5, degree=3, M1=5, M2=6)
    o = Oracle2D.from_workload(w, dt=0.4)
    s = initial_state2d(o, generate2d(w))
    s["bz"] += 0.7
    s0 = {k: v.copy() for k, v in s.items()}
    o.substep_II(s)
    for a in range(5):
        B = scipy_eval(o, s0["bz"], 2, 2, s0["x1"][a], s0["x2"][a])
        A = scipy_eval(o, s0["az"], 3, 3, s0["x1"][a], s0["x2"][a])

        def rhs(t, y):
            g = math.sqrt(1 + y[0] ** 2 + y[1] ** 2 + A * A)
            return [y[1] * B / g, -y[0] * B / g]
        sol = solve_ivp(rhs, (0, 0.4), [s0["p1"][a], s0["p2"][a]], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose([s["p1"][a], s["p2"][a]], sol.y[:, -1], atol=1e-10)
    assert np.all(s["x1"] == s0["x1"]) and np.all(s["e"] == s0["e"])


# --------------------------------------------------------------------------
# Subsystem III: a_z, e_z
# --------------------------------------------------------------------------

def test_subsystem_III_scheme_relations():
    """(a^{n+1} - a^n)/dt = -(e^n + e^{n+1})/2 exactly, and the e_z equation with the
    particle term evaluated by scipy at the particles (residual at the tolerance)."""
    w = get2d("twod16").scaled(n_particles=50)
    o = Oracle2D.from_workload(w, tol=1e-14)
    s = initial_state2d(o, generate2d(w))
    s0 = {k: v.copy() for k, v in s.items()}
    assert o.substep_III(s)[0] == 0
    dt, N, p = o.cfg.dt, o.N, 3
    np.testing.assert_allclose((s["az"] - s0["az"]) / dt, -0.5 * (s0["ez"] + s["ez"]), atol=1e-13)
    S = np.zeros(N)
    for a in range(o.cfg.n):
        x = (s0["x1"][a], s0["x2"][a])
        An, A1 = scipy_eval(o, s0["az"], p, p, *x), scipy_eval(o, s["az"], p, p, *x)
        g = lambda A: math.sqrt(1 + s0["p1"][a] ** 2 + s0["p2"][a] ** 2 + A * A)   # noqa: E731
        o.line_deposit(p, p, x, x, o.cfg.w * (An + A1) / (g(An) + g(A1)), S)
    lhs = o.M0(s["ez"] - s0["ez"]) / dt
    rhs = o.K(0.5 * (s0["az"] + s["az"])) + S
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


# --------------------------------------------------------------------------
# Subsystem IV: Maxwell
# --------------------------------------------------------------------------

def _te_wave(M, p, t):
    """Exact vacuum TE wave along x2 on [0, 2 pi)^2: B_z = E_x... with k = 1, w = 1:
    B_z = cos(x2 - t), E_x = -cos(x2 - t); coefficients interpolate at Greville points
    (quasi-interpolant), e_y = 0."""
    L = 2 * math.pi
    h = L / M
    g1 = (np.arange(M) + 0.5 * p) * h
    gz = (np.arange(M) + 0.5 * (p + 1)) * h
    bz = np.cos(np.add.outer(np.zeros(M), g1) - t).ravel()
    e1 = -np.cos(np.add.outer(np.zeros(M), gz) - t).ravel()
    return bz, np.concatenate([e1, np.zeros(M * M)])


def test_subsystem_IV_conserves_and_is_reversible():
    w = get2d("twod8x16")
    o = Oracle2D.from_workload(w, n=1)
    rng = np.random.default_rng(12)
    e, b = rng.normal(size=2 * o.N), rng.normal(size=o.N)
    s = {"e": e.copy(), "bz": b.copy()}
    W = lambda s: 0.5 * s["e"] @ o.M1(s["e"]) + 0.5 * s["bz"] @ o.M2(s["bz"])   # noqa: E731
    W0, g0 = W(s), o.GT(o.M1(s["e"]))
    o.substep_IV(s, 0.3)
    assert abs(W(s) - W0) < 1e-13 * W0
    np.testing.assert_allclose(o.GT(o.M1(s["e"])), g0, atol=1e-12)
    o.substep_IV(s, -0.3)
    np.testing.assert_allclose(s["e"], e, atol=1e-12)
    np.testing.assert_allclose(s["bz"], b, atol=1e-12)


def test_subsystem_IV_converges_to_the_travelling_wave():
    """B_z at a probe point after t = 1 against cos(x2 - t): the error falls by about
    4 (second order) as dx and dt halve."""
    errs = []
    for M in (8, 16, 32):
        p = 3
        o = Oracle2D(L1=2 * math.pi, L2=2 * math.pi, M1=M, M2=M, p=p, n=1)
        bz, e = _te_wave(M, p, 0.0)
        s = {"e": e, "bz": bz}
        steps = M // 2
        for _ in range(steps):
            o.substep_IV(s, 1.0 / steps)
        probe = [o.eval(s["bz"], p - 1, p - 1, 1.0, x2) - math.cos(x2 - 1.0) for x2 in np.linspace(0, 6, 13)]
        errs.append(np.abs(probe).max())
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


# --------------------------------------------------------------------------
# Whole Lie-Trotter steps
# --------------------------------------------------------------------------

def test_lie_steps_conserve_energy_and_gauss():
    w = get2d("twod16").scaled(n_particles=200)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, generate2d(w))
    H0 = o.energy(s)[5]
    st, kI, kIII = o.step(s, 3)
    assert st == 0 and (kI > 1).all() and (kIII >= 1).all()
    assert abs(o.energy(s)[5] - H0) <= 3e-13 * H0
    assert o.gauss_residual(s) < 1e-13


def test_gauss_law_is_exact_at_a_loose_tolerance():
    """The discrete Gauss law holds to round-off whatever the Picard tolerance (the
    paper's remark on Subsystem I): the committed positions are those whose current
    was deposited, so a stop at tol = 1e-5 still leaves r at round-off."""
    w = get2d("twod16").scaled(n_particles=300)
    o = Oracle2D.from_workload(w, tol=1e-5)
    s = initial_state2d(o, generate2d(w))
    st, k, r = o.substep_I(s)
    assert st == 0 and k <= 6 and r > 1e-10
    assert o.gauss_residual(s) < 1e-14


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_linear_solves_reach_their_solution(p):
    """Every linear system of the 2D scheme is solved, at every degree (the quintic mass
    matrices are the worst conditioned): M1 x = b, the Gauss correction (residual at
    round-off), Subsystem IV (energy kept, reversible) and Subsystem III's midpoint
    relation."""
    o = Oracle2D(L1=4 * math.pi, L2=2 * math.pi, M1=16, M2=8, p=p, n=1)
    rng = np.random.default_rng(40 + p)
    b = rng.normal(size=2 * o.N)
    assert np.abs(o.M1(o.solve_M1(b)) - b).max() <= 1e-12 * np.abs(b).max()
    w = get2d("twod16").scaled(degree=p, n_particles=200, M2=8, L2=2 * math.pi)
    o2 = Oracle2D.from_workload(w)
    s = initial_state2d(o2, generate2d(w))
    assert o2.gauss_residual(s) < 1e-13
    W = lambda s: 0.5 * s["e"] @ o2.M1(s["e"]) + 0.5 * s["bz"] @ o2.M2(s["bz"])   # noqa: E731
    e0, b0, W0 = s["e"].copy(), s["bz"].copy(), W(s)
    o2.substep_IV(s, 0.3)
    assert abs(W(s) - W0) < 1e-13 * W0
    o2.substep_IV(s, -0.3)
    np.testing.assert_allclose(s["e"], e0, atol=1e-12)
    np.testing.assert_allclose(s["bz"], b0, atol=1e-12)
    a0, ez0 = s["az"].copy(), s["ez"].copy()
    assert o2.substep_III(s)[0] == 0
    np.testing.assert_allclose((s["az"] - a0) / w.dt, -0.5 * (ez0 + s["ez"]), atol=1e-12)
