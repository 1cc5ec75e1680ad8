"""The adjoint Subsystem I scheme and the symmetric splitting on the GPU against
the FP64 oracle: element by element at 1e-12 relative per array (1e-11 over
several steps), equal sweep counts in every substep."""
import numpy as np
import pytest

import paper_2203_06513_amd as ec
import workloads
from oracle import Oracle, initial_state

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)


def assert_state_close(g, s, L, tol=1e-12, keys=("ex", "ey", "ez", "ay", "az")):
    d = np.mod(np.asarray(g["x"]) - np.asarray(s["x"]) + L / 2, L) - L / 2
    errs = {"x": np.abs(d).max(initial=0.0) / L, "p": rel(g["p"], s["p"])}
    for k in keys:
        errs[k] = rel(g[k], s[k]) if np.abs(s[k]).max() > 0 else np.abs(g[k]).max()
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"parity above {tol}: {bad} (all: {errs})"


@pytest.mark.parametrize("name", ["langmuir64", "paper51"])
def test_adjoint_substep_one_call(name):
    w = workloads.get(name)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    start = dict(arr, ex=s["ex"].copy())
    st, k_o, _ = o.substep_I_adjoint(s)
    assert st == 0
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL) as c:
        c.load(start, solve_gauss=False)
        g0 = c.gauss_residual(vec=True)[1]
        k_g, _ = c.substep_particles_adjoint()
        g = c.state()
        g1 = c.gauss_residual(vec=True)[1]
    assert k_g == k_o
    assert_state_close(g, s, w.L)
    assert np.abs(g1 - g0).max() <= 1e-13


@pytest.mark.parametrize("p,wpi", [(2, 0), (4, 1), (5, 1), (5, 0)])
def test_adjoint_other_degrees_and_the_crossing_queue(p, wpi):
    """Degrees 2 to 5; with one wave per item and 1500 particles per cell the quintic and
    quartic sweeps redo their crossing particles through the queue."""
    w = workloads.get("langmuir64").scaled(degree=p, M=32, n_particles=48000 if wpi else 3000, sigma=0.5)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    start = dict(arr, ex=s["ex"].copy())
    ks = []
    for _ in range(2):
        st, k, _ = o.substep_I_adjoint(s)
        assert st == 0
        ks.append(k)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, waves_per_item=wpi) as c:
        c.load(start, solve_gauss=False)
        kg, queued = [], []
        for _ in range(2):
            kg.append(c.substep_particles_adjoint()[0])
            queued.append(c.last_stats_I[3])
        g = c.state()
    assert kg == ks
    if wpi:
        assert all(queued)
    assert_state_close(g, s, w.L)


@pytest.mark.parametrize("warm", [False, True])
def test_symmetric_steps_match_oracle(warm):
    """Ten steps of I(dt/2), II(dt), adjoint I(dt/2); with the previous-step start each
    opening substep starts from the increments the closing adjoint one committed."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1, splitting=1, warm_previous=warm)
    s = initial_state(o, arr)
    start = dict(arr, ex=s["ex"].copy())
    st, kI, kII, E = o.step(s, 10, energies=True)
    assert st == 0
    kI2 = o.last_sweeps_I2.copy()
    ws = ec.WS_PREVIOUS if warm else ec.WS_EXPLICIT
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, splitting=ec.SYMMETRIC, warmstart=ws) as c:
        c.load(start, solve_gauss=False)
        rc, done, gI, gII, _ = c.step(10)
        gI2 = c.last_sweeps_I2.copy()
        g = c.state()
        H = c.energy()[4]
    assert rc == 0 and done == 10
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist() and gI2.tolist() == kI2.tolist()
    assert_state_close(g, s, w.L, tol=1e-11)
    assert abs(H - E[-1, 4]) / E[0, 4] <= 1e-12


def test_symmetric_run_invariants():
    """200 symmetric steps of the paper's Section 5.1 setup: energy and Gauss law held."""
    w = workloads.get("paper51")
    arr = workloads.generate(w)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, splitting=ec.SYMMETRIC) as c:
        c.load(arr)
        H0 = c.energy()[4]
        g0, r0 = c.gauss_residual(vec=True)
        rc, done, gI, gII, _ = c.step(200)
        H1 = c.energy()[4]
        g1, r1 = c.gauss_residual(vec=True)
    assert done == 200
    assert abs(H1 - H0) / H0 <= 1e-11
    assert np.abs(r1 - r0).max() <= 1e-13


@pytest.mark.parametrize("kmax", [2, 4])
def test_symmetric_step_rolls_back(kmax):
    """A step whose opening substep (kmax 2) or Subsystem II (kmax 4: the langmuir64 step
    needs 4 sweeps and 5 iterations) does not converge leaves the state as it was, bit for
    bit (after a committed opening substep the step's start is put back)."""
    w = workloads.get("langmuir64").scaled(n_particles=3000)
    arr = workloads.generate(w)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, splitting=ec.SYMMETRIC, max_iter=kmax) as c:
        c.load(arr)
        before = c.state()
        rc, done, kI, _, _ = c.step(1, check=False)
        after = c.state()
    assert rc == ec.ENOTCONV and done == 0
    if kmax == 4:
        assert kI[0] == 4   # the opening substep converged and committed before the failure
    for k in before:
        np.testing.assert_array_equal(before[k], after[k])
