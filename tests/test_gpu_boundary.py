"""The C-ABI's conventions on the GPU: the time step of a substep call, the
previous-step start, device memory and a stream handed over by PyTorch, and the
error paths (a non-finite value in the state, a segment of a cell or more).

Parity is against the FP64 oracle, element by element, at the bar of the plain
path (1e-12 relative per array, equal sweep counts).
"""
import numpy as np
import pytest

import paper_2203_06513_amd as ec
import workloads
from oracle import Oracle, initial_state

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max(initial=0.0) / max(np.abs(b).max(initial=0.0), 1e-300)


def assert_state_close(g, s, L, tol=TOL, keys=("ex", "ey", "ez", "ay", "az")):
    d = np.mod(np.asarray(g["x"]) - np.asarray(s["x"]) + L / 2, L) - L / 2
    errs = {"x": np.abs(d).max(initial=0.0) / L, "p": rel(g["p"], s["p"])}
    for k in keys:
        errs[k] = rel(g[k], s[k]) if np.abs(s[k]).max() > 0 else np.abs(g[k]).max()
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"parity above {tol}: {bad} (all: {errs})"


# --------------------------------------------------------------------------
# the time step of a substep call
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seidel", [0, 1])
def test_substeps_with_their_own_time_step(seidel):
    """Two Subsystem I calls over dt/2 and a Subsystem II call over a time step the context
    was not created with (its matrix inverse computed on first use), then one over the
    configured dt again: same sweeps and state as the oracle's substeps over the same h."""
    w = workloads.get("langmuir64").scaled(n_particles=4000)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel)
    s = initial_state(o, arr)
    ko = [o.substep_I(s, 0.5 * w.dt)[1], o.substep_I(s, 0.5 * w.dt)[1],
          o.substep_II(s, 0.7 * w.dt)[1], o.substep_II(s)[1]]
    with ec.Context.from_workload(w, map=seidel) as c:
        c.load(arr)
        kg = [c.substep_particles(0.5 * w.dt)[0], c.substep_particles(0.5 * w.dt)[0],
              c.substep_fields(0.7 * w.dt)[0], c.substep_fields()[0]]
        g = c.state()
        with pytest.raises(ec.EcpicError) as e:
            c.substep_particles(w.dx)      # a step of a full cell is refused
        assert e.value.status == ec.EINVAL
        with pytest.raises(ec.EcpicError):
            c.substep_fields(-w.dt)
    assert kg == ko
    assert_state_close(g, s, w.L)


# --------------------------------------------------------------------------
# previous-step start (delta^(0) = the last committed increments)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seidel", [0, 1])
def test_previous_step_start_matches_oracle(seidel):
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=seidel, warm_previous=True)
    s = initial_state(o, arr)
    st, kI, kII, E = o.step(s, 12, energies=True)
    assert st == 0
    with ec.Context.from_workload(w, map=seidel, warmstart=ec.WS_PREVIOUS) as c:
        c.load(arr)
        rc, done, gI, gII, _ = c.step(12)
        g = c.state()
        H = c.energy()[4]
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L, tol=1e-11)
    assert abs(H - E[-1, 4]) / E[0, 4] <= 1e-12


def test_previous_step_start_in_single_steps_and_after_a_new_state():
    """Steps one call at a time equal the batched steps bit for bit; set_particles starts
    the next step from the explicit predictor again (its sweeps equal a fresh context's)."""
    w = workloads.get("langmuir64").scaled(n_particles=3000)
    arr = workloads.generate(w)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, warmstart=ec.WS_PREVIOUS) as c:
        c.load(arr)
        one = [c.step(1)[2][0] for _ in range(20)]
        s1 = c.state()
        c.load(arr)
        again = c.step(1)[2][0]
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, warmstart=ec.WS_PREVIOUS, sweep_guess=2) as c:
        c.load(arr)
        rc, done, kI, _, _ = c.step(20)
        s2 = c.state()
    assert kI.tolist() == one and again == one[0]
    for k in s1:
        np.testing.assert_array_equal(s1[k], s2[k])


@pytest.mark.parametrize("warm", ["explicit", "previous"])
def test_residual_history_matches_oracle(warm):
    """The residuals the step reports for its first FP64 sweeps equal the oracle's: the
    residual of sweep k is what a substep limited to k + 1 sweeps ends with (run on a copy
    of the state at the step's start, from the same starting increments)."""
    w = workloads.get("langmuir64").scaled(n_particles=4000)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    short = [Oracle.from_workload(w, seidel=1, kmax=k) for k in (1, 2, 3)]
    s = initial_state(o, arr)
    nsteps, ref, dprev = 5, [], None
    for j in range(nsteps):
        ds = dprev if warm == "previous" else None
        r = []
        for ok in short:
            s1 = {k: v.copy() for k, v in s.items()}
            r.append(ok.substep_I(s1, None, dstart=ds)[2])
        ref.append(r)
        dc = np.zeros(w.n_particles)
        assert o.substep_I(s, None, dstart=ds, dcommit=dc)[0] == 0
        assert o.substep_II(s)[0] == 0
        dprev = dc
    ref = np.array(ref)
    kw = {"warmstart": ec.WS_PREVIOUS} if warm == "previous" else {}
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, **kw) as c:
        c.load(arr)
        c.step(nsteps)
        got = c.last_res_hist_I
    assert ref.min() > 1e-11   # the three sweeps compared are far from the tolerance
    np.testing.assert_allclose(got[:, :3], ref, rtol=1e-6, atol=0)


# --------------------------------------------------------------------------
# device memory and a stream from PyTorch
# --------------------------------------------------------------------------

def test_torch_memory_and_stream():
    """The _dev calls take torch-allocated device tensors, the context runs on a torch
    stream, and the result equals the host path bit for bit."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible to torch")
    w = workloads.get("langmuir64")
    arr = workloads.generate(w)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        c.step(5)
        ref = c.state()
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(arr["x"]).to(dev)
    pt = torch.from_numpy(arr["p"]).to(dev)
    xo = torch.empty_like(xt)
    po = torch.empty_like(pt)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        with ec.Context.from_workload(w, map=ec.MAP_SEIDEL, stream=stream.cuda_stream) as c:
            c.set_particles_dev(xt.data_ptr(), pt.data_ptr())
            c.set_fields(None, arr["ey"], arr["ez"], arr["ay"], arr["az"])
            c.solve_gauss()
            c.step(5)
            c.get_particles_dev(xo.data_ptr(), po.data_ptr())
            f = c.get_fields()
        # ordered after the library's work on the same stream
        x_host = xo.cpu().numpy()
        p_host = po.cpu().numpy()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(x_host, ref["x"])
    np.testing.assert_array_equal(p_host, ref["p"])
    for k in ("ex", "ey", "ez", "ay", "az"):
        np.testing.assert_array_equal(f[k], ref[k])


# --------------------------------------------------------------------------
# error paths
# --------------------------------------------------------------------------

@pytest.mark.parametrize("where", ["ex", "ay"])
def test_nonfinite_field_is_reported_and_state_restorable(where):
    """A NaN in a field coefficient makes the step report ECPIC_ENONFINITE without
    committing; after the state is set again the run continues and matches the oracle."""
    w = workloads.get("langmuir64").scaled(n_particles=3000)
    arr = workloads.generate(w)
    o = Oracle.from_workload(w, seidel=1)
    s = initial_state(o, arr)
    st, kI, kII, _ = o.step(s, 3)
    assert st == 0
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        good = c.get_fields()
        bad = {k: v.copy() for k, v in good.items()}
        bad[where][5] = np.nan
        c.set_fields(bad["ex"], bad["ey"], bad["ez"], bad["ay"], bad["az"])
        rc, done, _, _, _ = c.step(2, check=False)
        assert rc == ec.ENONFINITE and done == 0
        k, r = c.substep_particles(check=False)
        assert c.last_stats_I[4] == ec.ENONFINITE
        c.set_particles(arr["x"], arr["p"])
        c.set_fields(good["ex"], good["ey"], good["ez"], good["ay"], good["az"])
        rc, done, gI, gII, _ = c.step(3)
        g = c.state()
    assert rc == 0 and done == 3
    assert gI.tolist() == kI.tolist() and gII.tolist() == kII.tolist()
    assert_state_close(g, s, w.L)


def test_segment_of_a_cell_or_more_is_ecfl():
    L, M = 3.0, 16
    dx = L / M
    x0 = np.array([0.1, 1.0, 2.0])
    x1 = x0 + np.array([0.3, 1.2, -0.2]) * dx
    with ec.Context(L=L, M=M, degree=3, n_particles=0, dt=0.01, tol=1e-12, weight=0.5) as c:
        J = c.deposit_current(x0, x1)
        assert np.isfinite(J).all()
        x1[1] = x0[1] + 2.5 * dx
        with pytest.raises(ec.EcpicError) as e:
            c.deposit_current(x0, x1)
        assert e.value.status == ec.ECFL
