"""GPU parity of the 2D path with spin (include/ecpic2d.h, cfg.spin = 1; Sections
2.2 and 4.3, the hbar terms) against the 2D oracle's spin functions.

Every test calls the HIP library through the C-ABI binding and compares with the
oracle on the same seeded inputs: every substep element by element (spins
included) on the two small plasmas with spin, Lie steps with the Zeeman energy,
hbar = 0 against the run without spin, and properties at 512 x 512 with 2^24
particles.  Bars as without spin: 1e-11 relative for I (both sides stop their
fixed points at the same tolerance), 1e-12 for III, 1e-13 for II and IV.
"""
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
    out = {}
    for k, L in (("x1", w.L1), ("x2", w.L2)):
        d = np.mod(g[k] - s[k] + L / 2, L) - L / 2
        out[k] = np.abs(d).max() / L
    for k in ("p1", "p2", "sx", "sy", "sz", "e", "bz", "ez", "az"):
        out[k] = rel(g[k], s[k]) if np.abs(s[k]).max() > 0 else np.abs(g[k]).max()
    bad = {k: v for k, v in out.items() if not v <= bar}
    assert not bad, (bad, out)
    return out


def test_spins_round_trip_and_reset():
    w, o, s, ctx = setup("twod16s", n=700)
    with ctx:
        g = ctx.get_spins()
        for k in ("sx", "sy", "sz"):
            np.testing.assert_array_equal(g[k], s[k])
        ctx.set_particles(s["x1"], s["x2"], s["p1"], s["p2"])
        assert all(np.all(v == 0.0) for v in ctx.get_spins().values())
    with ec.Context2D.from_workload(get2d("twod16").scaled(n_particles=10)) as plain:
        with pytest.raises(ec.EcpicError) as e:
            plain.get_spins()
        assert e.value.status == ec.EINVAL


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_energy_with_zeeman_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        g = ctx.energy()
        h = o.energy_s(s)
        assert abs(g[6] - h[5]) < 1e-13 * abs(h[5])
        assert abs(g[5] - h[6]) < 1e-13 * h[6]


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_substep_I_with_spin_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        kg, _ = ctx.substep_I()
        st, ko, _ = o.substep_I_s(s)
        assert st == 0 and abs(kg - ko) <= 1, (kg, ko)
        compare(w, ctx.state(), s, 1e-11)
        assert ctx.gauss_residual() < 1e-13


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_substep_II_with_spin_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        ctx.substep_II()
        o.substep_II_s(s)
        compare(w, ctx.state(), s, 1e-13)


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_substep_III_with_spin_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        kg, _ = ctx.substep_III()
        st, ko, _ = o.substep_III_s(s)
        assert st == 0 and abs(kg - ko) <= 1, (kg, ko)
        compare(w, ctx.state(), s, 1e-12)


@pytest.mark.parametrize("name", ["twod16s", "twod8x16s"])
def test_substep_IV_with_spin_matches_oracle(name):
    w, o, s, ctx = setup(name)
    with ctx:
        ctx.substep_IV()
        o.substep_IV_s(s)
        compare(w, ctx.state(), s, 1e-13)
        assert ctx.gauss_residual() < 1e-13


def test_lie_steps_with_spin_match_oracle_and_conserve():
    w, o, s, ctx = setup("twod16s", n=1500)
    with ctx:
        H0 = ctx.energy()[5]
        kg, kIIIg = ctx.step(3)
        st, ko, kIIIo = o.step_s(s, 3)
        assert st == 0
        assert np.abs(kg - ko).max() <= 1 and np.abs(kIIIg - kIIIo).max() <= 1
        compare(w, ctx.state(), s, 3e-11)
        H1 = ctx.energy()
        assert abs(H1[5] - o.energy_s(s)[6]) < 1e-11 * H1[5]
        assert abs(H1[5] - H0) <= 1e-12 * H0
        assert ctx.gauss_residual() < 1e-13


def test_zero_hbar_follows_the_run_without_spin():
    """cfg.spin = 1 with hbar = 0: particles and fields as without spin (the spins
    precess but act on nothing)."""
    w = get2d("twod16s").scaled(n_particles=800, hbar=0.0)
    arr = generate2d(w)
    with ec.Context2D.from_workload(w) as a, ec.Context2D.from_workload(w.scaled(spin="none")) as b:
        a.load(arr)
        b.load(arr)
        a.step(2)
        b.step(2)
        ga, gb = a.state(), b.state()
        for k in ("x1", "x2", "p1", "p2", "e", "bz", "ez", "az"):
            assert rel(ga[k], gb[k]) < 1e-13, k


def test_full_size_spin_step_properties():
    """512 x 512, 2^24 particles with spin: two Lie steps conserve the energy with the
    Zeeman term to the tolerance, hold Gauss's law, keep |s| = 1, and the Zeeman
    term does exchange energy."""
    w = get2d("twod512s")
    arr = generate2d(w)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        del arr
        H0 = ctx.energy()
        ctx.step(2)
        H1 = ctx.energy()
        assert abs(H1[5] - H0[5]) < 1e-12 * H0[5]
        assert abs(H1[6] - H0[6]) > 0.0
        assert ctx.gauss_residual() < 1e-13
        sp = ctx.get_spins()
        assert np.abs(np.sqrt(sp["sx"] ** 2 + sp["sy"] ** 2 + sp["sz"] ** 2) - 1.0).max() < 1e-13


@pytest.mark.parametrize("degree", [2, 4, 5])
def test_other_degrees_with_spin(degree):
    """Degrees 2 (the derivative fields of the spin force on degree 0), 4 and 5 (the
    spin sweep at its register limits): Subsystem I and a whole Lie step with spin
    against the oracle element by element."""
    w = get2d("twod16s").scaled(degree=degree, n_particles=900 if degree < 5 else 250)
    arr = generate2d(w)
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        kg, _ = ctx.substep_I()
        st, ko, _ = o.substep_I_s(s)
        assert st == 0 and abs(kg - ko) <= 1
        compare(w, ctx.state(), s, 1e-11)
        ctx.step(1)
        assert o.step_s(s, 1)[0] == 0
        compare(w, ctx.state(), s, 3e-11)
        assert ctx.gauss_residual() < 1e-13


def test_dense_tiles_move_the_spins():
    """About 10^4 particles per tile (more than the re-sort keeps in LDS): the direct
    re-sort path carries the spins with their particles; one Lie step with spin
    against the oracle."""
    w, o, s, ctx = setup("twod8x16s", n=80000)
    with ctx:
        kg, kIIIg = ctx.step(1)
        st, ko, kIIIo = o.step_s(s, 1)
        assert st == 0 and np.abs(kg - ko).max() <= 1 and np.abs(kIIIg - kIIIo).max() <= 1
        compare(w, ctx.state(), s, 1e-11)


def test_degenerate_steps_and_spins():
    """Particles on grid lines and cell corners with momenta 0, +-1e-300, +-1e-16,
    steps across both grid lines next to a corner, and spins along each axis and
    zero: one Lie step with spin against the oracle."""
    w = get2d("twod16s").scaled(n_particles=64)
    arr = generate2d(w)
    dx1, dx2 = w.L1 / w.M1, w.L2 / w.M2
    rng = np.random.default_rng(6)
    c1 = rng.integers(0, w.M1, 64)
    c2 = rng.integers(0, w.M2, 64)
    mom = np.array([0.0, 1e-300, -1e-300, 1e-16, -1e-16, 0.05, -0.05, 0.02])
    arr["x1"] = c1 * dx1
    arr["x2"] = c2 * dx2
    arr["x2"][::3] += 0.5 * dx2
    arr["p1"] = mom[np.arange(64) % 8]
    arr["p2"] = mom[(np.arange(64) // 8) % 8]
    arr["x1"][56:] = c1[56:] * dx1 - 1e-4 * dx1
    arr["x2"][56:] = c2[56:] * dx2 - 1e-4 * dx2
    arr["p1"][56:] = 0.05
    arr["p2"][56:] = 0.05 * dx2 / dx1
    arr["x1"] = np.mod(arr["x1"], w.L1)
    arr["x2"] = np.mod(arr["x2"], w.L2)
    axes = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [0.0, 0.0, 0.0]])
    sp = axes[np.arange(64) % 5]
    arr["sx"], arr["sy"], arr["sz"] = sp[:, 0].copy(), sp[:, 1].copy(), sp[:, 2].copy()
    o = Oracle2D.from_workload(w)
    s = initial_state2d(o, arr)
    with ec.Context2D.from_workload(w) as ctx:
        ctx.load(arr)
        ctx.step(1)
        assert o.step_s(s, 1)[0] == 0
        g = ctx.state()
    for k in g:
        assert np.all(np.isfinite(g[k])), k
    assert np.all(g["sx"][4::5] == 0.0) and np.all(g["sz"][4::5] == 0.0)   # a zero spin stays zero
    compare(w, g, s, 3e-11)
