"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it pins.  None of them re-types the oracle's own
formula: values come from closed forms (Eulerian numbers, exact relativistic
motion, Fourier symbols), from an independent library route (scipy's B-spline
evaluation and integration), from invariants (Gauss law, energy, mirror
symmetry) or from a brute-force Newton solve of the implicit scheme.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import Oracle, initial_state
from tests._splines import basis_integrals, basis_values, periodic_spline

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def eulerian(n, k):
    """Closed form A(n, k) = sum_{j=0}^{k} (-1)^j C(n+1, j) (k+1-j)^n."""
    return sum((-1) ** j * math.comb(n + 1, j) * (k + 1 - j) ** n for j in range(k + 1))


# --------------------------------------------------------------------------
# Section 3.1: bases, derivative relation, mass and stiffness matrices
# --------------------------------------------------------------------------

def test_eulerian_fixture_matches_closed_form():
    data = json.load(open(os.path.join(GOLDEN, "eulerian.json")))["A"]
    for n, row in data.items():
        n = int(n)
        assert [eulerian(n, k) for k in range(n)] == row
        assert sum(row) == math.factorial(n)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_bspline_knot_values_are_eulerian(d):
    for k in range(d):
        assert Oracle.bspline(d, k + 1.0) == pytest.approx(eulerian(d, k) / math.factorial(d), rel=1e-15, abs=1e-16)


@pytest.mark.parametrize("p", [1, 2, 3, 5])
def test_bases_match_scipy_and_partition_of_unity(p):
    M, L = 9, 3.7
    o = Oracle(L=L, M=M, p=p, n=1)
    rng = np.random.default_rng(p)
    for x in rng.uniform(0.0, L, 25):
        v0 = np.zeros(M)
        v1 = np.zeros(M)
        for j in range(-p - 2, M + 2):
            v0[j % M] += o.lambda0(j, x)
            if p >= 1:
                v1[j % M] += o.lambda1(j, x)
        assert v0.sum() == pytest.approx(1.0, abs=2e-15)
        assert v1.sum() == pytest.approx(1.0, abs=2e-15)
        np.testing.assert_allclose(v0, basis_values(M, L / M, p, x), atol=2e-15)
        if p >= 2:
            np.testing.assert_allclose(v1, basis_values(M, L / M, p - 1, x), atol=2e-15)


@pytest.mark.parametrize("p", [2, 3, 5])
def test_derivative_relation(p):
    """d/dx Lambda0_j = (Lambda1_j - Lambda1_{j+1}) / dx (Section 3.1).

    A five-point central difference is exact for polynomials of degree <= 4, so
    for p <= 4 and points away from knots it reproduces the derivative up to
    rounding; p = 5 carries an O(h^4) truncation term."""
    M, L = 10, 2.5
    dx = L / M
    o = Oracle(L=L, M=M, p=p, n=1)
    h = 1e-3 * dx
    rng = np.random.default_rng(11)
    for _ in range(20):
        cell = rng.integers(0, M)
        x = (cell + rng.uniform(0.1, 0.9)) * dx
        for j in range(cell - p, cell + 1):
            f = lambda y: o.lambda0(j, y)
            d5 = (-f(x + 2 * h) + 8 * f(x + h) - 8 * f(x - h) + f(x - 2 * h)) / (12 * h)
            rel = (o.lambda1(j, x) - o.lambda1(j + 1, x)) / dx
            assert d5 == pytest.approx(rel, abs=1e-8)


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_mass_rows_are_eulerian(d):
    row = Oracle.mass_row(d)
    n = 2 * d + 1
    expect = np.array([eulerian(n, k) for k in range(n)], dtype=float) / math.factorial(n)
    np.testing.assert_allclose(row, expect, rtol=1e-14, atol=1e-17)


def test_stiffness_row_p3():
    g = json.load(open(os.path.join(GOLDEN, "stiffness_p3.json")))
    M, L = 16, 4.0
    dx = L / M
    o = Oracle(L=L, M=M, p=3, n=1)
    e0 = np.zeros(M)
    e0[0] = 1.0
    col = o.K(e0)
    expect = np.array(g["row"], dtype=float) / g["denominator"] / dx
    got = np.array([col[k % M] for k in range(-3, 4)])
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=1e-15)
    assert abs(col.sum()) < 1e-13


def test_mass_condition_numbers():
    """Circulant spectra: cond(M1, degree 2) = 7.5 and cond(M0, degree 3) = 272/5040 inverse."""
    M = 64
    th = 2 * np.pi * np.arange(M) / M
    for d, cond in ((2, 7.5), (3, 5040.0 / 272.0)):
        row = Oracle.mass_row(d)
        lam = sum(row[k + d] * np.cos(k * th) for k in range(-d, d + 1))
        assert lam.max() / lam.min() == pytest.approx(cond, rel=1e-12)


@pytest.mark.parametrize("p,dt", [(3, 0.05), (5, 0.01)])
def test_solvers_match_dense_numpy(p, dt):
    M, L = 24, 3.0
    o = Oracle(L=L, M=M, p=p, n=1, dt=dt)
    I = np.eye(M)
    A1 = np.column_stack([o.M1(I[:, i]) for i in range(M)])
    Acn = np.column_stack([o.cn_plus(I[:, i]) for i in range(M)])
    A0 = np.column_stack([o.M0(I[:, i]) for i in range(M)])
    assert np.abs(A1 - A1.T).max() < 1e-15 and np.abs(Acn - Acn.T).max() < 1e-15
    rng = np.random.default_rng(3)
    for _ in range(3):
        b = rng.normal(size=M)
        np.testing.assert_allclose(o.solve_M1(b), np.linalg.solve(A1, b), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(o.solve_cn(b), np.linalg.solve(Acn, b), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(o.solve_M0(b), np.linalg.solve(A0, b), rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------
# Subsystem I scheme: line integrals and the 0/0-free divided difference
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3, 5])
def test_line_integrals(p):
    """sum_j I_j = x1 - x0 and (G^T I)_j = Lambda0_j(x1) - Lambda0_j(x0) (second remark of
    Section 4.2), and I_j agrees with scipy's exact B-spline integral."""
    M, L = 8, 2.0
    dx = L / M
    o = Oracle(L=L, M=M, p=p, n=1)
    rng = np.random.default_rng(5 + p)
    cases = [(0.3, 0.31), (0.249, 0.251), (1.999, 2.0004), (0.0001, -0.0003), (0.77, 0.77)]
    cases += [tuple(v) for v in rng.uniform(0, L, (10, 2)) * [1, 0] + [[0, 0]] * 10]
    for x0, x1 in cases:
        if x1 == 0.0:
            x1 = x0 + rng.uniform(-0.9, 0.9) * dx
        jlo, lbar = o.line_mean(x0, x1)
        I = np.zeros(M)
        for k, v in enumerate(lbar):
            I[(jlo + k) % M] += (x1 - x0) * v
        assert I.sum() == pytest.approx(x1 - x0, abs=1e-16)
        ref = basis_integrals(M, dx, p - 1, x0, x1) if p >= 2 else None
        np.testing.assert_allclose(I, ref, atol=5e-17)
        GT_I = np.array([(I[j] - I[(j + 1) % M]) / dx for j in range(M)])
        dL0 = basis_values(M, dx, p, x1) - basis_values(M, dx, p, x0)
        np.testing.assert_allclose(GT_I, dL0, atol=2e-15)
        if x0 == x1:
            np.testing.assert_allclose(lbar.sum(), 1.0, atol=1e-15)


def test_divided_difference_identity():
    """(A(x1)-A(x0))/(x1-x0) = sum_j (G a)_j lbar_j for any V0 field (the 0/0-free form used
    for the difference quotients of Subsystem I); at x1 = x0 it is A'(x0)."""
    M, L, p = 12, 3.0, 3
    o = Oracle(L=L, M=M, p=p, n=1)
    rng = np.random.default_rng(9)
    a = rng.normal(size=M)
    g = o.G(a)
    spl = periodic_spline(a, L / M, p)
    for _ in range(30):
        x0 = rng.uniform(0, L)
        x1 = x0 + rng.uniform(-0.2, 0.2)
        jlo, lbar = o.line_mean(x0, x1)
        lhs = (spl(x1) - spl(x0)) / (x1 - x0)
        rhs = sum(g[(jlo + k) % M] * v for k, v in enumerate(lbar))
        assert rhs == pytest.approx(lhs, rel=1e-11, abs=1e-12)
    x0 = 1.234
    jlo, lbar = o.line_mean(x0, x0)
    rhs = sum(g[(jlo + k) % M] * v for k, v in enumerate(lbar))
    assert rhs == pytest.approx(spl.derivative()(x0), rel=1e-13)


# --------------------------------------------------------------------------
# Subsystem I: closed-form special cases
# --------------------------------------------------------------------------

def _zero_field_state(o, x, p, ex=None, ay=None):
    M = o.cfg.M
    return {"x": np.array(x, float), "p": np.array(p, float),
            "ex": np.zeros(M) if ex is None else np.array(ex, float),
            "ey": np.zeros(M), "ez": np.zeros(M),
            "ay": np.zeros(M) if ay is None else np.array(ay, float), "az": np.zeros(M)}


@pytest.mark.parametrize("seidel", [0, 1])
def test_free_streaming(seidel):
    """a_perp = 0, e_x = 0, test particles (w = 0): p unchanged, dx = dt p / sqrt(1 + p^2);
    with a uniform a_y = c the divided differences vanish and dx = dt p / sqrt(1 + p^2 + c^2)."""
    M, L, dt = 16, 4.0, 0.05
    rng = np.random.default_rng(1)
    x = rng.uniform(0, L, 40)
    p = rng.normal(0, 0.8, 40)
    for c in (0.0, 0.7):
        o = Oracle(L=L, M=M, p=3, n=len(x), w=0.0, dt=dt, tol=1e-14, seidel=seidel)
        s = _zero_field_state(o, x, p, ay=np.full(M, c))
        st, k, r = o.substep_I(s)
        assert st == 0
        np.testing.assert_array_equal(s["p"], p)
        expect = np.mod(x + dt * p / np.sqrt(1 + p * p + c * c), L)
        np.testing.assert_allclose(s["x"], expect, rtol=0, atol=1e-14)
        np.testing.assert_array_equal(s["ex"], 0.0)


@pytest.mark.parametrize("seidel", [0, 1])
def test_uniform_electric_field_is_exact(seidel):
    """Uniform E_x (all e_j = E), a_perp = 0, w = 0: p+ = p + dt E and the step equals the exact
    relativistic displacement (gamma(p+) - gamma(p)) / E."""
    M, L, dt, E = 16, 4.0, 0.05, 0.37
    rng = np.random.default_rng(2)
    x = rng.uniform(0, L, 30)
    p = rng.normal(0, 0.5, 30)
    o = Oracle(L=L, M=M, p=3, n=len(x), w=0.0, dt=dt, tol=1e-15, seidel=seidel)
    s = _zero_field_state(o, x, p, ex=np.full(M, E))
    st, k, r = o.substep_I(s)
    assert st == 0
    p1 = p + dt * E
    np.testing.assert_allclose(s["p"], p1, rtol=1e-14, atol=1e-15)
    disp = (np.sqrt(1 + p1 ** 2) - np.sqrt(1 + p ** 2)) / E
    np.testing.assert_allclose(np.mod(s["x"] - x + L / 2, L) - L / 2, disp, atol=1e-14)


@pytest.mark.parametrize("seidel", [0, 1])
def test_work_theorem_single_test_particle(seidel):
    """Discrete gradient property (Section 4.1) for one particle in frozen fields (w = 0):
    gamma(x1, p1) - gamma(x0, p0) equals the work int_{x0}^{x1} E_x dx of the midpoint field."""
    M, L, dt, p = 10, 2.5, 0.05, 3
    rng = np.random.default_rng(4)
    ay, az, ex = rng.normal(0, 0.4, M), rng.normal(0, 0.4, M), rng.normal(0, 0.3, M)
    dx = L / M
    sy, sz, se = periodic_spline(ay, dx, p), periodic_spline(az, dx, p), periodic_spline(ex, dx, p - 1)
    for x0, p0 in [(0.31, 0.4), (1.0 - 1e-9, 0.9), (2.49, 0.7), (0.12, -0.6)]:
        o = Oracle(L=L, M=M, p=p, n=1, w=0.0, dt=dt, tol=1e-15, seidel=seidel)
        s = _zero_field_state(o, [x0], [p0], ex=ex)
        s["ay"], s["az"] = ay.copy(), az.copy()
        st, k, r = o.substep_I(s)
        assert st == 0
        x1 = x0 + (np.mod(s["x"][0] - x0 + L / 2, L) - L / 2)
        p1 = s["p"][0]
        g0 = math.sqrt(1 + p0 ** 2 + sy(x0) ** 2 + sz(x0) ** 2)
        g1 = math.sqrt(1 + p1 ** 2 + sy(x1) ** 2 + sz(x1) ** 2)
        assert g1 - g0 == pytest.approx(se.integrate(x0, x1), abs=2e-14)


# --------------------------------------------------------------------------
# Brute force: Newton on the full implicit Subsystem I system (few particles)
# --------------------------------------------------------------------------

def _newton_subsystem_I(L, M, p, dt, w, x0, p0, ex, ay, az):
    """Solve the Subsystem I scheme (Section 4.2, no spin) with Newton's method.  The
    residual is written from the scheme with scipy splines: literal difference quotients,
    time-averaged basis as exact integrals, M1 from its Eulerian row."""
    dx = L / M
    n = len(x0)
    sy, sz = periodic_spline(ay, dx, p), periodic_spline(az, dx, p)
    d = 2 * (p - 1) + 1
    row = np.array([eulerian(d, k) for k in range(d)], float) / math.factorial(d) * dx
    M1 = np.zeros((M, M))
    for i in range(M):
        for k in range(-(p - 1), p):
            M1[i, (i + k) % M] += row[k + p - 1]

    def resid(u):
        delta, e = u[:n], u[n:]
        ebar = periodic_spline(0.5 * (ex + e), dx, p - 1)
        R = np.zeros(n + M)
        cur = np.zeros(M)
        for a in range(n):
            xa, xb = x0[a], x0[a] + delta[a]
            A0 = np.array([sy(xa), sz(xa)]); A1 = np.array([sy(xb), sz(xb)])
            g00 = math.sqrt(1 + p0[a] ** 2 + A0 @ A0)
            g01 = math.sqrt(1 + p0[a] ** 2 + A1 @ A1)
            force = ebar.integrate(xa, xb) / (xb - xa) - (A0 + A1) @ ((A1 - A0) / (xb - xa)) / (g00 + g01)
            p1 = p0[a] + dt * force
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
            h = 1e-7 * max(1.0, abs(u[i]))
            up, um = u.copy(), u.copy()
            up[i] += h; um[i] -= h
            J[:, i] = (resid(up) - resid(um)) / (2 * h)
        u = u - np.linalg.solve(J, R)
    delta, e = u[:n], u[n:]
    # momentum at the solution
    ebar = periodic_spline(0.5 * (ex + e), dx, p - 1)
    p1 = np.zeros(n)
    for a in range(n):
        xa, xb = x0[a], x0[a] + delta[a]
        A0 = np.array([sy(xa), sz(xa)]); A1 = np.array([sy(xb), sz(xb)])
        g00 = math.sqrt(1 + p0[a] ** 2 + A0 @ A0); g01 = math.sqrt(1 + p0[a] ** 2 + A1 @ A1)
        p1[a] = p0[a] + dt * (ebar.integrate(xa, xb) / (xb - xa)
                              - (A0 + A1) @ ((A1 - A0) / (xb - xa)) / (g00 + g01))
    return delta, p1, e


@pytest.mark.parametrize("seidel", [0, 1])
@pytest.mark.parametrize("n", [1, 3])
def test_picard_matches_newton(n, seidel):
    w_ = workloads.small(M=8, L=2.0, n=n, dt=0.08, amplitude=0.4, sigma=0.6, seed=20 + n)
    arr = workloads.generate(w_)
    o = Oracle.from_workload(w_, seidel=seidel, tol=1e-14)
    s = initial_state(o, arr)
    x0, p0, ex0 = s["x"].copy(), s["p"].copy(), s["ex"].copy()
    st, k, r = o.substep_I(s)
    assert st == 0 and k >= 2
    delta, p1, e = _newton_subsystem_I(w_.L, w_.M, w_.degree, w_.dt, w_.weight, x0, p0, ex0,
                                       s["ay"], s["az"])
    got = np.mod(s["x"] - x0 + w_.L / 2, w_.L) - w_.L / 2
    np.testing.assert_allclose(got, delta, atol=1e-13)
    np.testing.assert_allclose(s["p"], p1, atol=1e-12)
    np.testing.assert_allclose(s["ex"], e, atol=1e-12)


# --------------------------------------------------------------------------
# Invariants: Gauss law (second remark, Section 4.2) and energy (Section 4.1)
# --------------------------------------------------------------------------

def test_solve_gauss_satisfies_discrete_poisson():
    w_ = workloads.get("langmuir64")
    arr = workloads.generate(w_, n=2000)
    o = Oracle.from_workload(w_, n=2000)
    ex = o.solve_gauss(arr["x"])
    rho = o.deposit_charge(arr["x"])
    assert rho.sum() == pytest.approx(w_.L, rel=1e-14)
    res = o.GT(o.M1(ex)) + rho - w_.dx
    assert np.abs(res).max() < 1e-14
    assert abs(ex.mean()) < 1e-15
    assert o.gauss_residual(arr["x"], ex) < 1e-14
    # charge deposit against scipy's basis
    dx = w_.dx
    rho_ref = sum(o.cfg.w * basis_values(w_.M, dx, 3, xx) for xx in arr["x"][:50])
    o50 = Oracle(L=w_.L, M=w_.M, p=3, n=50, w=o.cfg.w)
    np.testing.assert_allclose(o50.deposit_charge(arr["x"][:50]), rho_ref, atol=1e-15)


@pytest.mark.parametrize("seidel,kmax,force", [(0, 50, False), (1, 50, False), (0, 1, True), (1, 2, True)])
def test_gauss_law_held_every_step(seidel, kmax, force):
    """G^T M1 e_x + Lambda0(X)^T W 1 is invariant, converged or not."""
    w_ = workloads.get("langmuir64").scaled(M=16, L=2 * math.pi, n_particles=600)
    arr = workloads.generate(w_)
    o = Oracle.from_workload(w_, seidel=seidel, kmax=kmax, commit_unconverged=force)
    s = initial_state(o, arr)
    r0 = o.gauss_residual(s["x"], s["ex"], vec=True)[1]
    for _ in range(15):
        st, k, r = o.substep_I(s)
        assert st == (0 if not force else st)
        rn = o.gauss_residual(s["x"], s["ex"], vec=True)[1]
        assert np.abs(rn - r0).max() < 2e-15


@pytest.mark.parametrize("name,steps,n", [("langmuir64", 30, 10_000), ("paper51", 60, 4000)])
@pytest.mark.parametrize("seidel", [0, 1])
def test_energy_conserved_to_tolerance(name, steps, n, seidel):
    w_ = workloads.get(name)
    arr = workloads.generate(w_, n=n)
    o = Oracle.from_workload(w_, n=n, seidel=seidel)
    s = initial_state(o, arr)
    st, kI, kII, E = o.step(s, steps, energies=True)
    assert st == 0
    H = E[:, 4]
    drift = np.abs(H - H[0]) / H[0]
    assert drift.max() < 50 * w_.tol
    assert o.gauss_residual(s["x"], s["ex"]) < 1e-13


def test_mirror_symmetry_preserved():
    """A configuration symmetric under x -> L - x, p -> -p (a_perp even, e_x odd) stays symmetric."""
    M, L, p, dt = 16, 4.0, 3, 0.05
    rng = np.random.default_rng(8)
    xh = rng.uniform(0.05, L / 2 - 0.05, 40)
    ph = rng.normal(0, 0.3, 40)
    x = np.concatenate([xh, L - xh])
    pp = np.concatenate([ph, -ph])
    # even V0 coefficients: a_j = a_{M-p-1-j}; odd V1 coefficients: e_j = -e_{M-p-j}
    ay = rng.normal(0, 0.2, M); ay = 0.5 * (ay + ay[(M - p - 1 - np.arange(M)) % M])
    az = rng.normal(0, 0.2, M); az = 0.5 * (az + az[(M - p - 1 - np.arange(M)) % M])
    o = Oracle(L=L, M=M, p=p, n=len(x), dt=dt, tol=1e-14)
    s = _zero_field_state(o, x, pp)
    s["ay"], s["az"] = ay, az
    s["ex"] = o.solve_gauss(s["x"])
    s["ey"] = 0.5 * (ay + 0.0)
    s["ez"] = az.copy()
    assert np.abs(s["ex"] + s["ex"][(M - p - np.arange(M)) % M]).max() < 1e-14
    for _ in range(5):
        st, kI, kII, _ = o.step(s, 1)
        assert st == 0
    n2 = len(xh)
    ssum = np.mod(s["x"][:n2] + s["x"][n2:], L)
    np.testing.assert_allclose(np.minimum(ssum, L - ssum), 0.0, atol=1e-13)
    np.testing.assert_allclose(s["p"][:n2], -s["p"][n2:], atol=1e-14)
    np.testing.assert_allclose(s["ex"], -s["ex"][(M - p - np.arange(M)) % M], atol=1e-14)
    np.testing.assert_allclose(s["ay"], s["ay"][(M - p - 1 - np.arange(M)) % M], atol=1e-14)


# --------------------------------------------------------------------------
# Subsystem II: closed form without particles
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p,dt,mode", [(3, 0.05, 3), (3, 0.3, 5), (5, 0.02, 2)])
def test_subsystem_II_vacuum_is_a_rotation(p, dt, mode):
    """With no particles the scheme of Subsystem II is the implicit midpoint rule of a linear
    wave system; per Fourier mode it rotates (sqrt(lam_M0) e, sqrt(lam_K) a) by
    2 atan(dt/2 sqrt(lam_K / lam_M0)) and conserves the quadratic energy exactly."""
    M, L = 16, 4.0
    dx = L / M
    th = 2 * np.pi * mode / M
    d0 = 2 * p + 1
    m0 = np.array([eulerian(d0, k) for k in range(d0)], float) / math.factorial(d0)
    d1 = 2 * p - 1
    m1 = np.array([eulerian(d1, k) for k in range(d1)], float) / math.factorial(d1)
    lamM0 = dx * sum(m0[k + p] * math.cos(k * th) for k in range(-p, p + 1))
    lamM1 = dx * sum(m1[k + p - 1] * math.cos(k * th) for k in range(-(p - 1), p))
    lamK = lamM1 * (2 - 2 * math.cos(th)) / dx ** 2
    phi = 2 * math.atan(0.5 * dt * math.sqrt(lamK / lamM0))
    j = np.arange(M)
    for basis in (np.cos(th * j), np.sin(th * j)):
        e0, a0 = 0.7 * basis, -0.4 * basis
        o = Oracle(L=L, M=M, p=p, n=0, w=0.0, dt=dt, tol=1e-15)
        s = {"x": np.zeros(0), "p": np.zeros(0), "ey": e0.copy(), "ez": np.zeros(M),
             "ay": a0.copy(), "az": np.zeros(M)}
        st, k, r = o.substep_II(s)
        assert st == 0
        u0, v0 = math.sqrt(lamM0) * 0.7, math.sqrt(lamK) * -0.4
        u1 = math.cos(phi) * u0 + math.sin(phi) * v0
        v1 = -math.sin(phi) * u0 + math.cos(phi) * v0
        np.testing.assert_allclose(s["ey"], u1 / math.sqrt(lamM0) * basis, atol=1e-13)
        np.testing.assert_allclose(s["ay"], v1 / math.sqrt(lamK) * basis, atol=1e-13)


def test_subsystem_II_conserves_energy_with_particles():
    w_ = workloads.get("paper51")
    arr = workloads.generate(w_, n=1000)
    o = Oracle.from_workload(w_, n=1000)
    s = initial_state(o, arr)
    H0 = o.energy(s)[4]
    for _ in range(5):
        st, k, r = o.substep_II(s)
        assert st == 0
    assert abs(o.energy(s)[4] - H0) / H0 < 10 * w_.tol


def test_paper51_setup_and_pump_dispersion():
    """The Section 5.1 pump is an exact relativistic circularly polarised wave: gamma0 =
    sqrt(1 + E0^2) = 2 and w^2 = k^2 + 1/gamma0 = 1, so E_perp = -dA_perp/dt at t = 0."""
    g = json.load(open(os.path.join(GOLDEN, "paper51_setup.json")))
    w_ = workloads.get("paper51")
    assert w_.tol == g["tolerance"] and w_.degree == g["degree_V0"]
    assert w_.sigma ** 2 == pytest.approx(g["T"], rel=1e-15)
    assert w_.amplitude ** 2 == pytest.approx(g["E0_squared"])
    k = 2 * math.pi / w_.L
    assert k * k == pytest.approx(g["k_squared"])
    assert (w_.M, w_.n_particles, w_.dt) == (g["cells"], g["particles"], g["dt"])
    gamma0 = math.sqrt(1 + g["E0_squared"])
    assert gamma0 == 2.0 and k * k + 1 / gamma0 == pytest.approx(1.0)
