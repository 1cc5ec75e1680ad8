"""GPU parity of the 2D path (include/ecpic2d.h) against the 2D FP64 oracle.

Every test calls the HIP library through the C-ABI binding and compares with the
oracle on the same seeded inputs: element by element at sizes the oracle
finishes in seconds (several tiles per row, both spline degrees the small
workloads use, a rectangular grid), and at the 512 x 512, 2^24-particle size of
the bench on sampled particles and on properties that hold at any size.

Tolerances: both sides stop their fixed points at the same absolute tolerance
(1e-13 small, 1e-12 large) on the same maps, so states agree to a few times the
tolerance; the linear substeps (II, IV) agree to rounding (1e-13 relative).
"""
import math

import numpy as np
import pytest

import paper_2203_06513_amd as ec
from oracle.twod import Oracle2D, initial_state2d
from workloads.twod import generate2d, get2d

pytestmark = pytest.mark.gpu


def setup(name, n=None, **kw):
    w = get2d(name)
    if n is not None:
        w = w.scaled(n_particles=n)
    w = w.scaled(**kw) if kw else w
    arr = generate2d(w)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    ctx = ec.Context2D.from_workload(w)
    ctx.load(arr)
    return w, o, s, ctx


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


def compare(w, g, s, bar):
    """Max relative differences of every state array (positions modulo the period)."""
    out = {}
    for k, L in (("x1", w.L1), ("x2", w.L2)):
        d = np.mod(g[k] - s[k] + L / 2, L) - L / 2
        out[k] = np.abs(d).max() / L
    for k in ("p1", "p2", "e", "bz", "ez", "az"):
        out[k] = rel(g[k], s[k]) if np.abs(s[k]).max() > 0 else np.abs(g[k]).max()
    bad = {k: v for k, v in out.items() if not v <= bar}
    assert not bad, (bad, out)
    return out


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_gauss_solve_and_charge_match_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        g = ctx.state()
        assert rel(g["e"], s["e"]) < 1e-13
        assert rel(ctx.deposit_charge(), o.deposit_charge(s)) < 1e-14
        m, r = ctx.gauss_residual(vec=True)
        assert m < 1e-13
        mo, ro = o.gauss_residual(s, vec=True)
        assert np.abs(r - ro).max() < 1e-13


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_substep_I_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        kg, rg = ctx.substep_I()
        st, ko, ro = o.substep_I(s)
        assert st == 0 and abs(kg - ko) <= 1, (kg, ko)
        compare(w, ctx.state(), s, 1e-11)
        assert ctx.gauss_residual() < 1e-13


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_substep_II_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        ctx.substep_II()
        o.substep_II(s)
        compare(w, ctx.state(), s, 1e-13)


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_substep_III_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        kg, _ = ctx.substep_III()
        st, ko, _ = o.substep_III(s)
        assert st == 0 and abs(kg - ko) <= 1, (kg, ko)
        compare(w, ctx.state(), s, 1e-12)


@pytest.mark.parametrize("name", ["twod16", "twod8x16"])
def test_substep_IV_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        ctx.substep_IV()
        o.substep_IV(s)
        compare(w, ctx.state(), s, 1e-13)
        assert ctx.gauss_residual() < 1e-13


def _min_image(d, L):
    return np.mod(d + L / 2, L) - L / 2


@pytest.mark.parametrize("M1,M2,degree", [(32, 64, 2), (128, 256, 3), (256, 8, 3)])
def test_spectral_solves_at_other_transform_lengths(M1, M2, degree):
    """Grids whose FFT lengths take the radix-8 stages with a radix-4 or radix-2
    last stage (32, 128, 256) and a single block of columns (M2 = 8).  The
    oracle's own solves take minutes here, so the GPU state is checked against
    the scheme's relations through the oracle's operators: the Gauss law after
    the load, M1 (e^{n+1} - e^n) = -J(path) after Subsystem I, the Subsystem III
    pair (a and e_z, particle term evaluated at the particles), the implicit
    midpoint pair of Subsystem IV."""
    w = get2d("twod16").scaled(M1=M1, M2=M2, degree=degree, n_particles=600, L1=0.6 * M1, L2=0.6 * M2)
    o = Oracle2D.from_workload(w)
    p, N, dt, wt = degree, o.N, w.dt, o.cfg.w
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(generate2d(w))
        s0 = ctx.state()
        assert o.gauss_residual(s0) < 1e-12 * w.dx1 * w.dx2
        ctx.substep_I()
        s1 = ctx.state()
        J = np.zeros(2 * N)
        for a in range(w.n_particles):
            xa = np.array([s0["x1"][a], s0["x2"][a]])
            d = np.array([_min_image(s1["x1"][a] - xa[0], w.L1), _min_image(s1["x2"][a] - xa[1], w.L2)])
            o.line_deposit(p - 1, p, xa, xa + d, wt * d[0], J[:N])
            o.line_deposit(p, p - 1, xa, xa + d, wt * d[1], J[N:])
        assert np.abs(o.M1(s1["e"] - s0["e"]) + J).max() < 1e-11 * np.abs(J).max()
        ctx.substep_II()
        s2 = ctx.state()
        ctx.substep_III()
        s3 = ctx.state()
        assert rel((s3["az"] - s2["az"]) / dt, -0.5 * (s2["ez"] + s3["ez"])) < 1e-12
        S = np.zeros(N)
        for a in range(w.n_particles):
            x = (s2["x1"][a], s2["x2"][a])
            An, A1 = o.eval(s2["az"], p, p, *x), o.eval(s3["az"], p, p, *x)
            q2 = 1 + s2["p1"][a] ** 2 + s2["p2"][a] ** 2
            o.line_deposit(p, p, x, x, wt * (An + A1) / (math.sqrt(q2 + An * An) + math.sqrt(q2 + A1 * A1)), S)
        assert rel(o.M0(s3["ez"] - s2["ez"]) / dt, o.K(0.5 * (s2["az"] + s3["az"])) + S) < 1e-11
        ctx.substep_IV()
        s4 = ctx.state()
        assert rel(o.M1(s4["e"] - s3["e"]) / dt, o.CT(o.M2(0.5 * (s3["bz"] + s4["bz"])))) < 1e-11
        assert rel((s4["bz"] - s3["bz"]) / dt, -o.C(0.5 * (s3["e"] + s4["e"]))) < 1e-11
        assert o.gauss_residual(s4) < 1e-12 * w.dx1 * w.dx2


def test_lie_steps_match_oracle_and_conserve():
    w, o, s, ctx = setup("twod16", n=1500)
    with ctx:
        H0 = ctx.energy()
        np.testing.assert_allclose(H0[:6], o.energy(s), rtol=1e-13, atol=1e-15)
        kg, kIIIg = ctx.step(3)
        st, ko, kIIIo = o.step(s, 3)
        assert st == 0
        assert np.abs(kg - ko).max() <= 1 and np.abs(kIIIg - kIIIo).max() <= 1
        compare(w, ctx.state(), s, 3e-11)
        H1 = ctx.energy()
        np.testing.assert_allclose(H1[:6], o.energy(s), rtol=1e-11, atol=1e-14)
        assert abs(H1[5] - H0[5]) <= 1e-12 * H0[5]
        assert ctx.gauss_residual() < 1e-13


def test_dense_tiles_take_the_direct_resort():
    """About 10^4 particles per tile (8 x 16 cells, one 16-cell tile per row):
    more than the re-sort keeps in LDS, so every tile is written by the direct
    path; one Lie step against the oracle and the tile order afterwards."""
    w, o, s, ctx = setup("twod8x16", n=80000)
    with ctx:
        kg, kIIIg = ctx.step(1)
        st, ko, kIIIo = o.step(s, 1)
        assert st == 0 and np.abs(kg - ko).max() <= 1 and np.abs(kIIIg - kIIIo).max() <= 1
        compare(w, ctx.state(), s, 1e-11)
        assert ctx.gauss_residual() < 1e-13


def test_nonfinite_field_is_reported_and_state_restorable():
    """A NaN coefficient of e (Subsystem I) or of a_z (Subsystem III) stops the
    fixed point with ECPIC_ENONFINITE and commits nothing; with the fields set
    again the run matches the oracle."""
    w, o, s, ctx = setup("twod16", n=1500)
    with ctx:
        good = ctx.get_fields()
        parts = ctx.get_particles()
        for name, call in (("e", ctx.substep_I), ("az", ctx.substep_III)):
            bad = {k: v.copy() for k, v in good.items()}
            bad[name][17] = np.nan
            ctx.set_fields(**bad)
            with pytest.raises(ec.EcpicError) as e:
                call()
            assert e.value.status == ec.ENONFINITE, name
            after, fields = ctx.get_particles(), ctx.get_fields()
            for k in parts:
                np.testing.assert_array_equal(after[k], parts[k])
            for k in good:
                np.testing.assert_array_equal(fields[k], bad[k])
        ctx.set_fields(**good)
        kg, kIIIg = ctx.step(2)
        st, ko, kIIIo = o.step(s, 2)
        assert st == 0 and np.abs(kg - ko).max() <= 1 and np.abs(kIIIg - kIIIo).max() <= 1
        compare(w, ctx.state(), s, 3e-11)


def test_edge_positions_and_order():
    """Particles on and just inside the domain boundary, negative and beyond-L
    positions (wrapped), returned in input order."""
    w = get2d("twod8x16").scaled(n_particles=8)
    arr = generate2d(w)
    eps = 1e-15
    arr["x1"][:4] = [0.0, w.L1 - eps, -0.25 * w.L1, 1.5 * w.L1]
    arr["x2"][:4] = [w.L2 - eps, 0.0, 2.25 * w.L2, -eps]
    o = Oracle2D.from_workload(w)
    wrapped = dict(arr)
    wrapped["x1"] = np.mod(arr["x1"], w.L1)
    wrapped["x2"] = np.mod(arr["x2"], w.L2)
    s = initial_state2d(o, wrapped)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        g = ctx.get_particles()
        for k, L in (("x1", w.L1), ("x2", w.L2)):
            assert np.all((g[k] >= 0) & (g[k] < L))
            d = np.mod(g[k] - s[k] + L / 2, L) - L / 2
            assert np.abs(d).max() < 1e-12 * L
        np.testing.assert_array_equal(g["p1"], arr["p1"])
        ctx.substep_I()
        o.substep_I(s)
        compare(w, ctx.state(), s, 1e-11)


def test_grid_lines_corners_and_tiny_steps():
    """Degenerate steps: particles exactly on interior grid lines and on cell
    corners, with momenta zero, +-1e-300 and +-1e-16, and steps that start just
    off a cell corner and cross both grid lines next to it; one substep I and one
    Lie step against the oracle."""
    w = get2d("twod16").scaled(n_particles=64)
    arr = generate2d(w)
    dx1, dx2 = w.L1 / w.M1, w.L2 / w.M2
    rng = np.random.default_rng(5)
    c1 = rng.integers(0, w.M1, 64)
    c2 = rng.integers(0, w.M2, 64)
    mom = np.array([0.0, 1e-300, -1e-300, 1e-16, -1e-16, 0.05, -0.05, 0.02])
    arr["x1"] = c1 * dx1
    arr["x2"] = c2 * dx2
    arr["x2"][::3] += 0.5 * dx2          # on an x1 grid line only
    arr["p1"] = mom[np.arange(64) % 8]
    arr["p2"] = mom[(np.arange(64) // 8) % 8]
    # steps from just below and left of a corner across both of its grid lines
    arr["x1"][56:] = c1[56:] * dx1 - 1e-4 * dx1
    arr["x2"][56:] = c2[56:] * dx2 - 1e-4 * dx2
    arr["p1"][56:] = 0.05
    arr["p2"][56:] = 0.05 * dx2 / dx1
    arr["x1"] = np.mod(arr["x1"], w.L1)
    arr["x2"] = np.mod(arr["x2"], w.L2)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        ctx.substep_I()
        assert o.substep_I(s)[0] == 0
        compare(w, ctx.state(), s, 1e-11)
        ctx.step(1)
        assert o.step(s, 1)[0] == 0
        g = ctx.state()
    for k in g:
        assert np.all(np.isfinite(g[k])), k
    compare(w, g, s, 1e-11)


def test_no_particles_and_rollback():
    w = get2d("twod16")
    arr = generate2d(w, n=0)
    with ec.Context2D.from_workload(w, n=0) as ctx:
        ctx.load(arr)
        k, _ = ctx.substep_I()
        assert k == 1
        ctx.step(2)
        # without particles nothing neutralises the background: r = -dx1 dx2 everywhere
        m, r = ctx.gauss_residual(vec=True)
        assert np.abs(r + w.dx1 * w.dx2).max() < 1e-13
    w, o, s, ctx = setup("twod16", n=500)
    ctx.close()
    with ec.Context2D.from_workload(w, kmax=1) as ctx:
        ctx.load(generate2d(w))
        before = ctx.state()
        with pytest.raises(ec.EcpicError) as e:
            ctx.substep_I()
        assert e.value.status == ec.ENOTCONV
        after = ctx.state()
        for k in before:
            np.testing.assert_array_equal(after[k], before[k])
        with pytest.raises(ec.EcpicError) as e:
            ctx.substep_III()
        assert e.value.status == ec.ENOTCONV
        after = ctx.state()
        for k in before:
            np.testing.assert_array_equal(after[k], before[k])


# --------------------------------------------------------------------------
# Full size (512 x 512 cells, 2^24 particles): sampled particles and invariants
# --------------------------------------------------------------------------

def test_full_size_step_properties():
    w = get2d("twod512")
    arr = generate2d(w)
    o = Oracle2D.from_workload(w)
    rng = np.random.default_rng(3)
    idx = rng.choice(w.n_particles, 64, replace=False)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        assert ctx.gauss_residual() < 1e-12
        s0 = ctx.state()
        H0 = ctx.energy()[5]
        # Subsystem I: the committed state satisfies the scheme at sampled particles
        k, r = ctx.substep_I()
        s1 = ctx.state()
        H1 = ctx.energy()[5]
        assert abs(H1 - H0) <= 1e-12 * H0
        assert ctx.gauss_residual() < 1e-12
        ebar = 0.5 * (s0["e"] + s1["e"])
        ga = o.G(s0["az"])
        for a in idx:
            x = (s0["x1"][a], s0["x2"][a])
            d = [np.mod(s1[k_][a] - s0[k_][a] + L / 2, L) - L / 2 for k_, L in (("x1", w.L1), ("x2", w.L2))]
            pn, dn = o.particle_map(x, (s0["p1"][a], s0["p2"][a]), d, ebar, s0["az"], ga)
            assert abs(pn[0] - s1["p1"][a]) < 1e-10 and abs(pn[1] - s1["p2"][a]) < 1e-10
            assert abs(dn[0] - d[0]) < 1e-10 and abs(dn[1] - d[1]) < 1e-10
        # Subsystem II: sampled particles against the oracle's rotation of the same particles
        ctx.substep_II()
        s2 = ctx.state()
        osub = Oracle2D.from_workload(w, n=len(idx))
        sub = {"x1": s1["x1"][idx].copy(), "x2": s1["x2"][idx].copy(), "p1": s1["p1"][idx].copy(),
               "p2": s1["p2"][idx].copy(), "bz": s1["bz"], "az": s1["az"]}
        osub.substep_II(sub)
        assert rel(s2["p1"][idx], sub["p1"]) < 1e-13 and rel(s2["p2"][idx], sub["p2"]) < 1e-13
        H2 = ctx.energy()[5]
        assert abs(H2 - H1) <= 1e-13 * H1
        # Subsystem III: midpoint relation on the grid, energy
        ctx.substep_III()
        s3 = ctx.state()
        np.testing.assert_allclose((s3["az"] - s2["az"]) / w.dt, -0.5 * (s2["ez"] + s3["ez"]), atol=1e-12)
        H3 = ctx.energy()[5]
        assert abs(H3 - H2) <= 1e-12 * H2
        # Subsystem IV: energy, Gauss, reversibility
        ctx.substep_IV()
        H4 = ctx.energy()[5]
        assert abs(H4 - H3) <= 1e-13 * H3
        assert ctx.gauss_residual() < 1e-12
        ctx.substep_IV(-w.dt)
        s5 = ctx.state()
        assert rel(s5["e"], s3["e"]) < 1e-12 and rel(s5["bz"], s3["bz"]) < 1e-12
        assert k >= 2 and math.isfinite(r)


def test_fresh_context_after_destroyed_one():
    """A context created right after another was destroyed (its allocations may reuse
    memory holding the old context's values): the per-tile counters of the sort start
    from zero, so the first Subsystem I commit still matches the oracle."""
    w = get2d("twod8x16")
    arr = generate2d(w)
    with ec.Context2D.from_workload(w) as old:
        old.load(arr)
        old.step(3)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        ctx.substep_I()
        assert o.substep_I(s)[0] == 0
        compare(w, ctx.state(), s, 1e-11)


@pytest.mark.parametrize("degree", [4, 5])
def test_high_degree_substeps_and_step(degree):
    """Degrees 4 and 5 (the sweep at its register limits): Subsystem I and a whole Lie
    step against the oracle element by element."""
    w = get2d("twod16").scaled(degree=degree, n_particles=1200 if degree == 4 else 500)
    arr = generate2d(w)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        assert rel(ctx.state()["e"], s["e"]) < 1e-12
        kg, _ = ctx.substep_I()
        st, ko, _ = o.substep_I(s)
        assert st == 0 and abs(kg - ko) <= 1
        compare(w, ctx.state(), s, 1e-11)
        ctx.substep_II()
        o.substep_II(s)
        ctx.substep_III()
        assert o.substep_III(s)[0] == 0
        ctx.substep_IV()
        o.substep_IV(s)
        ctx.step(1)
        assert o.step(s, 1)[0] == 0
        compare(w, ctx.state(), s, 3e-11)
        assert ctx.gauss_residual() < 1e-13
