"""The learned warm start against the FP64 reference network and the oracle.

* gradients of the training kernels against the FP64 backward pass
  (oracle/mlp.py, itself pinned by central differences);
* recorded training pairs against the oracle's features and converged step;
* the per-cell tables (BF16 matrix cores) against the FP64 forward pass at the
  same nodes;
* training on pairs the method produced, then the A/B: Picard sweeps with and
  without the network, the same converged state, the same invariants.
"""
import math

import numpy as np
import pytest

import paper_2203_06513_amd as ec
import workloads
from oracle import Oracle, initial_state
from oracle import mlp

pytestmark = pytest.mark.gpu


def random_net(D, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, scale, mlp.n_params(D)).astype(np.float32)
    mu = rng.normal(0.0, 0.1, D + 2).astype(np.float32)
    sd = rng.uniform(0.5, 2.0, D + 2).astype(np.float32)
    pr = np.array([-0.3, 0.3], np.float32)
    return theta, mu, sd, pr


def test_ws_gradient_vs_fp64_reference():
    w = workloads.get("langmuir64")
    D = mlp.n_features(w.degree)
    theta, mu, sd, pr = random_net(D, 3)
    rng = np.random.default_rng(4)
    X = rng.normal(0, 1, (100, D)).astype(np.float32)
    T = rng.normal(0, 1, (100, 2)).astype(np.float32)
    with ec.Context.from_workload(w, n=10) as c:
        c.ws_set_weights(np.concatenate([theta, mu, sd, pr]))
        g, loss = c.ws_grad(X, T)
    L, gr = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - L) <= 1e-5 * L
    assert np.abs(g - gr).max() <= 1e-4 * np.abs(gr).max()


def test_ws_records_match_oracle():
    w = workloads.get("langmuir64")
    n = 2000
    arr = workloads.generate(w, n=n)
    o = Oracle.from_workload(w, n=n, seidel=1)
    s = initial_state(o, arr)
    f_ref = mlp.features(o, s, range(n), w.degree)
    x0, p0 = s["x"].copy(), s["p"].copy()
    st, k, _ = o.substep_I(s)
    assert st == 0
    delta = np.mod(s["x"] - x0 + w.L / 2, w.L) - w.L / 2
    Ay = np.array([o.field0(arr["ay"], v) for v in x0]); Az = np.array([o.field0(arr["az"], v) for v in x0])
    g0 = np.sqrt(1 + p0 ** 2 + Ay ** 2 + Az ** 2)
    y_ref = np.stack([(delta - w.dt * p0 / g0) / w.dt ** 2, (s["p"] - p0) / w.dt], axis=1)
    with ec.Context.from_workload(w, n=n, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        c.ws_record(1, 4 * n)
        c.substep_particles()
        assert c.ws_records() == n
        f, t = c.ws_get_records()
    # slot = particle id for stride 1
    assert np.abs(f - f_ref).max() <= 2e-6 * max(1.0, np.abs(f_ref).max())
    scale = np.abs(y_ref).max(axis=0)
    assert np.all(np.abs(t - y_ref).max(axis=0) <= 1e-5 * scale)


def test_ws_tables_vs_fp64_forward():
    """Tables from the BF16 matrix-core evaluation against the FP64 forward pass of
    the same network at the same (t, p) nodes."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w, n=500)
    o = Oracle.from_workload(w, n=500)
    s = initial_state(o, arr)
    D = mlp.n_features(w.degree)
    theta, mu, sd, pr = random_net(D, 7, scale=0.15)
    with ec.Context.from_workload(w, n=500) as c:
        c.load(arr)
        c.ws_set_weights(np.concatenate([theta, mu, sd, pr]))
        tab = c.ws_table()
    P, M, dx = w.degree, w.M, w.dx
    ref = np.empty((M, 8, 8))
    for cell in range(M):
        win = [(cell + j) % M for j in range(-P, P + 2)]
        for it in range(8):
            t = it / 7.0
            x = (cell + t) * dx
            Ay, Az = o.field0(s["ay"], x), o.field0(s["az"], x)
            for ip in range(8):
                p = pr[0] + (pr[1] - pr[0]) * ip / 7.0
                g0 = math.sqrt(1 + p * p + Ay * Ay + Az * Az)
                f = np.concatenate([[t - 0.5, p, g0 - 1.0], s["ay"][win], s["az"][win], s["ex"][win]])
                xn = (f - mu[:D]) / sd[:D]
                y, _ = mlp.forward(theta.astype(np.float64), xn[None, :])
                ref[cell, it, ip] = mu[D] + sd[D] * y[0, 0]
    err = np.abs(tab - ref).max()
    spread = np.abs(ref - mu[D]).max()
    print(f"\ntable vs FP64 forward: max error {err:.3e}, output spread {spread:.3e}")
    # BF16 keeps 8 significant bits (unit roundoff 2^-9); the products of layer 2
    # round their inputs so, and the 64-term sums partly cancel the errors.  Measured
    # 3.6e-3 of the spread; the bar is three times that.
    assert err <= 1.2e-2 * spread


def test_ws_first_training_step_vs_fp64_reference():
    """One step of the GPU training (Glorot start, normalisation statistics, the
    sampled batch, forward and backward pass, Adam) against the FP64 reference doing
    the same from the definitions: the normalisation to FP32 rounding, the new
    weights to 2e-7 where the gradient is well above its FP32 error, and elsewhere
    a move of at most lr (the first Adam step has length lr).  Then a second step
    (ws_train starts again from the same initialisation), whose moments now mix
    two gradients, from the GPU's first-step weights."""
    w = workloads.get("langmuir64")
    D = mlp.n_features(w.degree)
    P = mlp.n_params(D)
    seed, B, lr = 11, 256, 1e-3
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL) as c:
        c.load(workloads.generate(w))
        c.ws_record(1, 4 * w.n_particles)
        c.step(2)
        feat, targ = c.ws_get_records()
        c.ws_record(0)
        c.ws_train(steps=1, batch=B, lr=lr, seed=seed)
        wts = c.ws_get_weights()
        c.ws_train(steps=2, batch=B, lr=lr, seed=seed)
        theta2 = c.ws_get_weights()[:P].astype(np.float64)
    n = len(feat)
    assert n == 2 * w.n_particles
    theta1 = wts[:P].astype(np.float64)
    mu, sd = wts[P:P + D + 2], wts[P + D + 2:P + 2 * (D + 2)]
    allv = np.concatenate([feat, targ], axis=1).astype(np.float64)
    m64, s64 = allv.mean(axis=0), allv.std(axis=0)
    s64[~(s64 > 1e-12 * np.maximum(1.0, np.abs(m64)))] = 1.0
    assert np.all(np.abs(mu - m64) <= 1e-6 * np.maximum(np.abs(m64), s64))
    assert np.all(np.abs(sd - s64) <= 1e-6 * s64)
    theta0 = mlp.glorot_init(seed, D)
    idx = mlp.batch_indices(seed, 0, B, n)
    X = (feat[idx].astype(np.float64) - mu[:D]) / sd[:D]
    T = (targ[idx].astype(np.float64) - mu[D:]) / sd[D:]
    _, g = mlp.loss_and_grad(theta0, X, T)
    ref, _, _ = mlp.adam_step(theta0, 0.0, 0.0, g, 1, lr)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    err = np.abs(theta1 - ref)
    print(f"\n{n} records, batch {B}: {big.sum()} of {P} gradients well resolved, max error there "
          f"{err[big].max():.2e}, elsewhere max move {np.abs(theta1 - theta0)[~big].max():.2e}")
    assert big.sum() > 0.8 * P   # the weights of features that are constant here have no gradient
    assert err[big].max() <= 2e-7
    assert np.all(np.abs(theta1 - theta0.astype(np.float32))[~big] <= lr * (1.0 + 1e-5) + 1e-7)
    # step 2 from the GPU's weights after step 1, the moments of step 1 from the FP64 gradient
    m1, v1 = 0.1 * g, 0.001 * g * g
    idx2 = mlp.batch_indices(seed, 1, B, n)
    X2 = (feat[idx2].astype(np.float64) - mu[:D]) / sd[:D]
    T2 = (targ[idx2].astype(np.float64) - mu[D:]) / sd[D:]
    _, g2 = mlp.loss_and_grad(theta1, X2, T2)
    ref2, _, _ = mlp.adam_step(theta1, m1, v1, g2, 2, lr)
    both = (np.abs(g) > 0.1 * np.abs(g).max()) & (np.abs(g2) > 0.1 * np.abs(g2).max())
    err2 = np.abs(theta2 - ref2)[both]
    print(f"step 2: {both.sum()} coordinates with both gradients resolved to 1e-3, max error {err2.max():.2e}")
    assert both.sum() >= 10
    assert err2.max() <= 2e-6
    # every coordinate: |m_hat| / sqrt(v_hat) <= 1.0014 at t = 2 (Cauchy-Schwarz on the two terms)
    assert np.all(np.abs(theta2 - theta1) <= 1.0015 * lr + 1e-7)


@pytest.fixture(scope="module")
def trained():
    """Pairs recorded over 12 steps of a 200k-particle pump workload, then trained."""
    w = workloads.get("pump2048").scaled(n_particles=200_000)
    arr = workloads.generate(w)
    c = ec.Context.from_workload(w, map=ec.MAP_SEIDEL)
    c.load(arr)
    c.ws_record(4, 1_000_000)
    c.step(12)
    nrec = c.ws_records()
    c.ws_record(0)
    loss = c.ws_train(steps=1500, batch=1024, lr=2e-3, seed=11)
    weights = c.ws_get_weights()
    state = c.state()
    c.close()
    return w, state, weights, loss, nrec


def test_ws_training_converges(trained):
    w, state, weights, loss, nrec = trained
    print(f"\n{nrec} pairs, final training loss {loss:.3e}")
    assert nrec == 12 * 50_000
    assert loss < 0.05
    assert np.all(np.isfinite(weights))


def test_ws_training_deterministic(trained):
    w, state, weights, loss, nrec = trained
    arr = workloads.generate(w)
    with ec.Context.from_workload(w, map=ec.MAP_SEIDEL) as c:
        c.load(arr)
        c.ws_record(4, 1_000_000)
        c.step(12)
        c.ws_record(0)
        loss2 = c.ws_train(steps=1500, batch=1024, lr=2e-3, seed=11)
        w2 = c.ws_get_weights()
    assert loss2 == loss
    assert np.array_equal(w2, weights)


def _run(w, state, weights, use_net, precision=ec.FP64, steps=8):
    c = ec.Context.from_workload(w, map=ec.MAP_SEIDEL, precision=precision)
    c.set_particles(state["x"], state["p"])
    c.set_fields(state["ex"], state["ey"], state["ez"], state["ay"], state["az"])
    if use_net:
        c.ws_set_weights(weights)
        c.ws_enable(True)
    H0 = c.energy()[4]
    g0, r0 = c.gauss_residual(vec=True)
    rc, done, kI, kII, k32 = c.step(1)
    s1 = c.state()
    rc, done2, kI2, _, _ = c.step(steps - 1)
    H1 = c.energy()[4]
    g1, r1 = c.gauss_residual(vec=True)
    c.close()
    return s1, np.concatenate([kI, kI2]), abs(H1 - H0) / H0, np.abs(r1 - r0).max()


def test_ws_ab_fewer_sweeps_same_state(trained):
    w, state, weights, loss, nrec = trained
    s_plain, k_plain, drift_plain, gauss_plain = _run(w, state, weights, False)
    s_net, k_net, drift_net, gauss_net = _run(w, state, weights, True)
    print(f"\nPicard sweeps per step: plain {k_plain.mean():.2f}, with the network {k_net.mean():.2f} "
          f"(plus one predictor pass); drift {drift_plain:.1e} / {drift_net:.1e}")
    assert k_net.mean() < k_plain.mean()
    for key in ("x", "p", "ex"):
        d = s_net[key] - s_plain[key]
        if key == "x":
            d = np.mod(d + w.L / 2, w.L) - w.L / 2
        assert np.abs(d).max() <= 10 * w.tol, key
    assert drift_net <= 1e-11 and gauss_net <= 1e-13


def test_ws_with_fp32_form(trained):
    w, state, weights, loss, nrec = trained
    s_plain, k_plain, _, _ = _run(w, state, weights, False, steps=3)
    s_mix, k_mix, drift, gauss = _run(w, state, weights, True, precision=ec.FP32_MIXED, steps=3)
    for key in ("x", "p", "ex"):
        d = s_mix[key] - s_plain[key]
        if key == "x":
            d = np.mod(d + w.L / 2, w.L) - w.L / 2
        assert np.abs(d).max() <= 10 * w.tol, key
    assert drift <= 1e-11 and gauss <= 1e-13
