"""Parity of the HIP path (through the C-ABI) with the FP64 CPU oracle.

Same seeded inputs on both sides; every comparison is element by element with
the bar ||gpu - oracle||_inf / ||oracle||_inf <= 1e-12 per array (positions
compared on the circle, relative to L), and equal Picard sweep counts.
"""
import math

import numpy as np
import pytest

import paper_2203_06513_amd as ec
import workloads
from oracle import Oracle, initial_state

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)


def xrel(a, b, L):
    d = np.mod(np.asarray(a) - np.asarray(b) + L / 2, L) - L / 2
    return np.abs(d).max(initial=0.0) / L


def assert_state_close(g, s, L, tol=TOL, keys=("ex", "ey", "ez", "ay", "az")):
    errs = {"x": xrel(g["x"], s["x"], L), "p": rel(g["p"], s["p"])}
    for k in keys:
        errs[k] = rel(g[k], s[k]) if np.abs(s[k]).max() > 0 else np.abs(g[k]).max()
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"parity above {tol}: {bad} (all: {errs})"
    return errs


def gpu_ctx(w, n=None, **kw):
    return ec.Context.from_workload(w, n=n, **kw)


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_deposit_current_segments(p):
    """Line integrals of Lambda1 along straight segments, including knot crossings,
    periodic wrap and zero-length steps."""
    M, L = 16, 3.0
    dx = L / M
    rng = np.random.default_rng(p)
    n = 4000
    x0 = rng.uniform(0, L, n)
    x0[:10] = np.arange(10) * dx                 # exactly on knots
    x1 = x0 + rng.uniform(-0.95, 0.95, n) * dx
    x1[10:20] = x0[10:20]                        # zero length
    x0[20:25] = L - 1e-14; x1[20:25] = L + 0.3 * dx      # wrap right
    x0[25:30] = 1e-14; x1[25:30] = -0.4 * dx             # wrap left
    o = Oracle(L=L, M=M, p=p, n=n, w=0.37, dt=0.01)
    with ec.Context(L=L, M=M, degree=p, n_particles=0, dt=0.01, tol=1e-12, weight=0.37) as c:
        J = c.deposit_current(x0, x1)
    Jo = o.deposit_current(x0, x1)
    assert rel(J, Jo) <= 1e-13
    assert abs(J.sum() - 0.37 * (x1 - x0).sum()) <= 1e-12


@pytest.mark.parametrize("name,n", [("langmuir64", None), ("paper51", None), ("pump2048", 200_000)])
def test_sort_charge_poisson_energy(name, n):
    w = workloads.get(name)
    arr = workloads.generate(w, n=n)
    nn = len(arr["x"])
    o = Oracle.from_workload(w, n=nn)
    s = initial_state(o, arr)
    with gpu_ctx(w, n=nn) as c:
        c.load(arr)
        g = c.state()
        rho = c.deposit_charge()
        E = c.energy()
        gmax = c.gauss_residual()
    # round trip of the particles through the cell sort
    np.testing.assert_array_equal(g["p"], arr["p"])
    assert xrel(g["x"], arr["x"], w.L) <= 1e-15
    assert rel(rho, o.deposit_charge(s["x"])) <= 1e-13
    assert rel(g["ex"], s["ex"]) <= TOL
    assert rel(E, o.energy(s)) <= 1e-13
    assert gmax <= 1e-13


# --------------------------------------------------------------------------
# Subsystem I and II, one call from an identical state
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seidel", [0, 1])
@pytest.mark.parametrize("name,n", [("langmuir64", None), ("paper51", None)])
def test_subsystem_I_one_call(name, n, seidel):
    w = workloads.get(name)
    arr = workloads.generate(w, n=n)
    o = Oracle.from_workload(w, n=n, seidel=seidel)
    s = initial_state(o, arr)
    st, k_o, r_o = o.substep_I(s)
    assert st == 0
    with gpu_ctx(w, n=n, map=seidel) as c:
        c.load(arr)
        k_g, r_g = c.substep_particles()
        g = c.state()
    assert k_g == k_o
    assert_state_close(g, s, w.L)


@pytest.mark.parametrize("name", ["langmuir64", "paper51"])
def test_subsystem_II_one_call(name):
    w = workloads.get(name)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w)
    s = initial_state(o, arr)
    st, k_o, r_o = o.substep_II(s)
    assert st == 0
    with gpu_ctx(w) as c:
        c.load(arr)
        k_g, r_g = c.substep_fields()
        g = c.state()
    assert k_g == k_o
    assert_state_close(g, s, w.L)


@pytest.mark.parametrize("seidel", [0, 1])
@pytest.mark.parametrize("p", [2, 4, 5])
def test_other_degrees_one_step(p, seidel):
    w = workloads.get("langmuir64").scaled(degree=p, n_particles=3000, M=32)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel)
    s = initial_state(o, arr)
    st, kI, kII, _ = o.step(s, 2)
    assert st == 0
    with gpu_ctx(w, map=seidel) as c:
        c.load(arr)
        rc, done, gI, gII, _ = c.step(2)
        g = c.state()
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L)


# --------------------------------------------------------------------------
# Lie-Trotter steps and run-level invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seidel", [0, 1])
def test_langmuir64_ten_steps(seidel):
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel)
    s = initial_state(o, arr)
    st, kI, kII, E = o.step(s, 10, energies=True)
    assert st == 0
    with gpu_ctx(w, map=seidel) as c:
        c.load(arr)
        H0 = c.energy()[4]
        rc, done, gI, gII, _ = c.step(10)
        g = c.state()
        H = c.energy()[4]
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L, tol=1e-11)
    assert abs(H - E[-1, 4]) / E[0, 4] <= 1e-12
    assert abs(H0 - E[0, 4]) / E[0, 4] <= 1e-13


def test_langmuir64_full_run_invariants():
    """The whole langmuir64 run (100 steps): energy drift and Gauss law held, and the energy
    history tracks the oracle's."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    st, kI, kII, E = o.step(s, w.steps, energies=True)
    assert st == 0
    Hs = []
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        g0 = c.gauss_residual()
        Hs.append(c.energy()[4])
        for _ in range(w.steps // 10):
            c.step(10)
            Hs.append(c.energy()[4])
        g1 = c.gauss_residual()
    Hs = np.array(Hs)
    assert np.abs(Hs - Hs[0]).max() / Hs[0] <= 1e-11
    assert np.abs(Hs - E[::10, 4]).max() / Hs[0] <= 1e-11
    assert g1 <= 1e-13 and g0 <= 1e-13


def test_paper51_run_invariants():
    w = workloads.get("paper51")
    arr = workloads.generate(w)
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        H0 = c.energy()[4]
        g0, r0 = c.gauss_residual(vec=True)
        rc, done, gI, gII, _ = c.step(400)
        H1 = c.energy()[4]
        g1, r1 = c.gauss_residual(vec=True)
    assert done == 400
    assert abs(H1 - H0) / H0 <= 1e-11
    assert np.abs(r1 - r0).max() <= 1e-13


# --------------------------------------------------------------------------
# full-size pump2048 in the bench launch configuration: sampled per-particle
# checks of the committed state against the oracle's scheme equations
# --------------------------------------------------------------------------

def test_pump2048_full_size_step_properties():
    w = workloads.get("pump2048")
    arr = workloads.generate(w)
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        s0 = c.state()
        H0 = c.energy()[4]
        gr0, r0 = c.gauss_residual(vec=True)
        k, res = c.substep_particles()
        s1 = c.state()
        gr1, r1 = c.gauss_residual(vec=True)
        c.substep_fields()
        s2 = c.state()
        H2 = c.energy()[4]
    assert res <= w.tol
    # Gauss law carried exactly through the substep (second remark, Section 4.2)
    assert np.abs(r1 - r0).max() <= 1e-13
    # energy through one full step
    assert abs(H2 - H0) / H0 <= 1e-12
    # sampled particles satisfy the Subsystem I equations with the committed fields
    o = Oracle.from_workload(w, n=1)
    gy, gz = o.G(s0["ay"]), o.G(s0["az"])
    ebar = 0.5 * (s0["ex"] + s1["ex"])
    rng = np.random.default_rng(0)
    idx = rng.choice(w.n_particles, 3000, replace=False)
    for a in idx:
        delta = np.mod(s1["x"][a] - s0["x"][a] + w.L / 2, w.L) - w.L / 2
        p1, dn, _, _ = o.particle_map(s0["x"][a], s0["p"][a], delta, s0["ay"], s0["az"], gy, gz, ebar)
        assert abs(p1 - s1["p"][a]) <= 1e-12
        assert abs(dn - delta) <= 5 * w.tol
    # oracle diagnostics of the GPU state agree with the GPU's own
    on = Oracle.from_workload(w)
    assert abs(on.energy(s2)[4] - H2) / H2 <= 1e-13
    assert on.gauss_residual(s1["x"], s1["ex"]) <= 1e-13


def test_pump2048_full_size_two_steps_elementwise():
    """Two Lie-Trotter steps of the full pump2048 workload (2e6 particles, 2048 cells) in
    the launch configuration the benchmark times (ecpic_step: steps enqueued as one batch,
    Seidel map, the first Subsystem II deposit formed by the commit, the join of a step's
    Subsystem II commit with the next step's start) against the oracle's two steps from the
    identical state: every particle and every field coefficient at 1e-12, equal sweep and
    iteration counts."""
    w = workloads.get("pump2048")
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    start = dict(arr, ex=s["ex"].copy())
    st, kI, kII, E = o.step(s, 2, energies=True)
    assert st == 0
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(start, solve_gauss=False)
        rc, done, gI, gII, _ = c.step(2)
        g = c.state()
        H = c.energy()[4]
    assert rc == 0 and done == 2
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L)
    assert abs(H - E[-1, 4]) / E[0, 4] <= 1e-12


@pytest.mark.parametrize("p,seidel", [(4, 1), (5, 0), (5, 1)])
def test_crossing_queue_elementwise(p, seidel):
    """From degree 4 on, a wave computes every row with the own-cell terms and queues the
    particles whose step crosses a cell boundary, redoing them with every term, 64 at a
    time, after its last row.  One wave per item and 1500 particles per cell give every
    wave more than 64 crossings (full and partial redo rows); two steps against the oracle
    element by element, in this launch shape and in the default one."""
    w = workloads.get("langmuir64").scaled(degree=p, M=32, n_particles=48000, sigma=0.5)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel)
    s = initial_state(o, arr)
    start = dict(arr, ex=s["ex"].copy())
    st, kI, kII, _ = o.step(s, 2)
    assert st == 0
    with gpu_ctx(w, map=seidel, waves_per_item=1) as c:
        c.load(start, solve_gauss=False)
        rc, done, gI, gII, _ = c.step(2)
        queued = c.last_queue_I.copy()
        g = c.state()
    assert queued.all(), queued
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L)
    with gpu_ctx(w, map=seidel) as c:   # four waves per item here
        c.load(start, solve_gauss=False)
        rc, done, gI, gII, _ = c.step(2)
        queued = c.last_queue_I.copy()
        g = c.state()
    assert queued.all(), queued
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L)


def test_stress16384_full_size_step_properties():
    """The quintic stress workload at full size (1.28e8 particles, 16384 cells): one step
    in the launch configuration the benchmark uses.  The oracle cannot sum over all
    particles in test time, so it checks sampled particles one by one and the field parts
    of the energy; the invariants hold at any size."""
    w = workloads.get("stress16384")
    arr = workloads.generate(w)
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        s0 = c.state()
        E0 = c.energy()
        gr0, r0 = c.gauss_residual(vec=True)
        k, res = c.substep_particles()
        s1 = c.state()
        gr1, r1 = c.gauss_residual(vec=True)
        kII, resII = c.substep_fields()
        s2 = c.state()
        E2 = c.energy()
    del arr
    assert res <= w.tol and resII <= w.tol
    assert np.abs(r1 - r0).max() <= 1e-13
    assert abs(E2[4] - E0[4]) / E0[4] <= 1e-12
    # Subsystem II leaves the particles alone
    assert np.array_equal(s2["x"], s1["x"]) and np.array_equal(s2["p"], s1["p"])
    o1 = Oracle.from_workload(w, n=1)
    for s, E in ((s0, E0), (s2, E2)):
        ref = o1.energy({"x": s["x"][:1], "p": s["p"][:1], **{f: s[f] for f in ("ex", "ey", "ez", "ay", "az")}})
        for j in (1, 2, 3):   # field parts: longitudinal, transverse electric, magnetic
            assert abs(E[j] - ref[j]) <= 1e-13 * max(abs(ref[j]), 1e-300), (j, E[j], ref[j])
    gy, gz = o1.G(s0["ay"]), o1.G(s0["az"])
    ebar = 0.5 * (s0["ex"] + s1["ex"])
    rng = np.random.default_rng(1)
    for a in rng.choice(w.n_particles, 1500, replace=False):
        delta = np.mod(s1["x"][a] - s0["x"][a] + w.L / 2, w.L) - w.L / 2
        p1, dn, _, _ = o1.particle_map(s0["x"][a], s0["p"][a], delta, s0["ay"], s0["az"], gy, gz, ebar)
        assert abs(p1 - s1["p"][a]) <= 1e-12 * max(1.0, abs(p1))
        assert abs(dn - delta) <= 5 * w.tol


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

def test_vacuum_no_particles():
    w = workloads.small(M=16, L=4.0, n=0, dt=0.05)
    arr = workloads.generate(w)
    o = Oracle(L=w.L, M=w.M, p=3, n=0, w=0.0, dt=w.dt, tol=w.tol)
    s = {k: np.array(v, float) for k, v in arr.items()}
    s["ex"] = np.zeros(w.M)
    st, kI, kII, _ = o.step(s, 3)
    assert st == 0
    with ec.Context(L=w.L, M=w.M, degree=3, n_particles=0, dt=w.dt, tol=w.tol) as c:
        c.set_particles(np.zeros(0), np.zeros(0))
        c.set_fields(None, arr["ey"], arr["ez"], arr["ay"], arr["az"])
        rc, done, gI, gII, _ = c.step(3)
        g = c.state()
    assert_state_close(g, s, w.L, keys=("ey", "ez", "ay", "az"))


@pytest.mark.parametrize("seidel", [0, 1])
def test_tiny_and_degenerate_particles(seidel):
    """Three particles with boundary positions, a particle exactly on a knot, p = 0, and an
    unsorted input order; followed over several steps."""
    w = workloads.small(M=8, L=2.0, n=6, dt=0.05, amplitude=0.4, sigma=0.5)
    L, dx = w.L, w.dx
    arr = workloads.generate(w)
    arr["x"] = np.array([L - 1e-15, 0.0, 3 * dx, 1.3, 0.2, 1.9999])
    arr["p"] = np.array([0.9, -0.7, 0.0, -0.2, 0.35, 0.6])
    o = Oracle.from_workload(w, seidel=seidel, tol=1e-14)
    s = initial_state(o, arr)
    st, kI, kII, _ = o.step(s, 5)
    assert st == 0
    with gpu_ctx(w, map=seidel, tol=1e-14) as c:
        c.load(arr)
        rc, done, gI, gII, _ = c.step(5)
        g = c.state()
    assert gI.tolist() == kI.tolist()
    assert_state_close(g, s, L)


def _items_per_step(o, s, w, nsteps, chunk=2048):
    """Work items (cells cut into pieces of at most `chunk` particles) along the oracle run."""
    counts = []
    for _ in range(nsteps + 1):
        n = np.bincount(np.floor(s["x"] / w.dx).astype(int) % w.M, minlength=w.M)
        counts.append(int(np.sum((n + chunk - 1) // chunk)))
        st, _, _, _ = o.step(s, 1)
        assert st == 0
    return counts


@pytest.mark.parametrize("case", ["sparse", "sparse-guess1", "dense", "edge", "edge-guess1"])
def test_item_count_changes_within_steps(case):
    """Steps during which the number of work items changes (particles entering empty cells;
    a cell's count crossing the item size): Subsystem II runs on the new order, whose item
    count is only known on the device, and must cover every item.  With one sweep enqueued
    ahead (-guess1) every batch fails its first test, so the commits of the steps behind it
    run gated on an order that no commit has written yet.  The edge cases start with one
    item per cell and cross the item size both ways (item counts 6, 7, 6, .. on 6 cells):
    batched, the commit's block 0 builds the lists with two items in a cell; with the steps
    finished one by one the host knows the current count and a separate kernel builds them."""
    if case.startswith("sparse"):
        w = workloads.small("sparse", M=64, L=8.0, n=48, dt=0.05, sigma=0.6, amplitude=0.3)
    elif case.startswith("edge"):
        w = workloads.small("edge", M=6, L=1.5, n=12000, dt=0.05, sigma=0.3, amplitude=0.3, seed=7)
    else:
        w = workloads.small("dense", M=8, L=2.0, n=16384, dt=0.05, sigma=0.3, amplitude=0.3)
    arr = workloads.generate(w)
    nsteps = 12
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    items = _items_per_step(o, {k: v.copy() for k, v in s.items()}, w, nsteps)
    assert max(items[1:]) > items[0] or len(set(items)) > 1, items   # the case is exercised
    if case.startswith("edge"):
        assert items[0] == w.M and max(items) > w.M and items.count(w.M) > 1, items
    st, kI, kII, E = o.step(s, nsteps, energies=True)
    assert st == 0
    kw = {"sweep_guess": 1} if case.endswith("guess1") else {}
    with gpu_ctx(w, map=ec.MAP_SEIDEL, item_particles=2048, **kw) as c:
        c.load(arr)
        H0 = c.energy()[4]
        rc, done, gI, gII, _ = c.step(nsteps)
        g = c.state()
        H = c.energy()[4]
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L, tol=1e-11)
    assert abs(H - H0) / H0 <= 1e-12


@pytest.mark.parametrize("case", ["dense", "sparse", "quintic"])
def test_fused_first_field_iterate_matches_separate_pass(case):
    """Inside ecpic_step the Subsystem I commit forms the particle deposit of the first
    Subsystem II iterate, each particle into the cell it lands in, and the first field
    kernel maps cells to it through the item list of the order before the commit; the
    substep calls run that iterate as a particle pass of its own over the new order.  Both
    give the same iteration counts and the same state to round-off: with one item per
    cell, on a sparse order with empty cells (the general item list), and at degree 5."""
    if case == "sparse":
        w = workloads.small("sparse", M=64, L=8.0, n=48, dt=0.05, sigma=0.6, amplitude=0.3)
    elif case == "quintic":
        w = workloads.get("langmuir64").scaled(degree=5, n_particles=3000, M=32)
    else:
        w = workloads.small("dense", M=8, L=2.0, n=16384, dt=0.05, sigma=0.3, amplitude=0.3)
    arr = workloads.generate(w)
    nsteps = 3
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        rc, done, gI, gII, _ = c.step(nsteps)
        fused = c.state()
    assert rc == 0 and done == nsteps
    kI, kII = [], []
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        for _ in range(nsteps):
            kI.append(c.substep_particles()[0])
            kII.append(c.substep_fields()[0])
        sep = c.state()
    assert gI.tolist() == kI and gII.tolist() == kII
    assert_state_close(fused, sep, w.L, tol=1e-12)


def test_not_converged_rolls_back():
    w = workloads.get("langmuir64").scaled(n_particles=2000, kmax=2)
    arr = workloads.generate(w)
    with gpu_ctx(w, max_iter=2) as c:
        c.load(arr)
        before = c.state()
        rc, done, gI, gII, _ = c.step(1, check=False)
        after = c.state()
    assert rc == -3 and done == 0
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])


def test_deterministic_and_resumable():
    """Two runs from one state are bitwise equal (no floating-point atomics in the step), and a
    run split in two through get/set of the state matches the uninterrupted one."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    outs = []
    for split in (False, False, True):
        with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
            c.load(arr)
            if split:
                c.step(3)
                mid = c.state()
            else:
                c.step(6)
                outs.append(c.state())
                continue
        with gpu_ctx(w, map=ec.MAP_SEIDEL) as c2:
            c2.set_particles(mid["x"], mid["p"])
            c2.set_fields(mid["ex"], mid["ey"], mid["ez"], mid["ay"], mid["az"])
            c2.step(3)
            outs.append(c2.state())
    for k in outs[0]:
        np.testing.assert_array_equal(outs[0][k], outs[1][k])
    assert_state_close(outs[2], outs[0], w.L, tol=1e-12)


@pytest.mark.parametrize("guess", [1, 3, 8])
def test_batched_steps_match_single_steps(guess):
    """Steps enqueued in batches (gated on the device, the host reading statuses once per
    batch) give bitwise the state and sweep counts of steps run one call at a time, whatever
    number of sweeps is enqueued ahead: too few sends a step through the lone-step path
    mid-batch, too many leaves sweeps that exit at once."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    n = 37   # crosses two batch boundaries and ends on a partial batch
    with gpu_ctx(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        ref = [c.step(1) for _ in range(n)]
        s_ref = c.state()
    kI_ref = [r[2][0] for r in ref]
    kII_ref = [r[3][0] for r in ref]
    with gpu_ctx(w, map=ec.MAP_SEIDEL, sweep_guess=guess) as c:
        c.load(arr)
        rc, done, kI, kII, _ = c.step(n)
        s = c.state()
    assert rc == 0 and done == n
    assert kI.tolist() == kI_ref and kII.tolist() == kII_ref
    for k in s_ref:
        np.testing.assert_array_equal(s[k], s_ref[k])
