"""Pins of the FP64 reference network of the learned warm start (oracle/mlp.py).

The activation is held against the exact GELU (x Phi(x), from math.erf) within
the known accuracy of its tanh form, and its derivative, the loss gradient and
the feature map against brute force (central differences, shifted inputs).
"""
import math

import numpy as np
import pytest

import workloads
from oracle import Oracle, initial_state
from oracle import mlp


def test_gelu_tanh_form_close_to_exact_gelu():
    z = np.linspace(-8, 8, 4001)
    exact = np.array([0.5 * v * (1.0 + math.erf(v / math.sqrt(2.0))) for v in z])
    err = np.abs(mlp.gelu(z) - exact)
    assert err.max() < 1e-3             # the tanh form is a ~1e-3 approximation
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    assert abs(mlp.gelu(np.array([-8.0]))[0]) < 1e-12


def test_gelu_grad_by_central_differences():
    z = np.linspace(-6, 6, 241)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(z)).max() < 1e-8


@pytest.mark.parametrize("seed", [0, 1])
def test_loss_gradient_by_central_differences(seed):
    rng = np.random.default_rng(seed)
    d, h = 27, 16
    theta = rng.normal(0, 0.4, mlp.n_params(d, h))
    X = rng.normal(0, 1, (9, d))
    T = rng.normal(0, 1, (9, 2))
    _, g = mlp.loss_and_grad(theta, X, T, h)
    idx = rng.choice(len(theta), 60, replace=False)
    eps = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += eps
        tm = theta.copy(); tm[i] -= eps
        fd = (mlp.loss(tp, X, T, h) - mlp.loss(tm, X, T, h)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_output_bias_gradient_closed_form():
    """With every weight zero the network outputs b3, and the mean squared error's
    gradient in b3 is 2 (b3 - mean(T)) / 2 per output."""
    d = 27
    theta = np.zeros(mlp.n_params(d))
    theta[-2:] = [0.3, -0.7]
    rng = np.random.default_rng(5)
    X = rng.normal(size=(11, d)); T = rng.normal(size=(11, 2))
    L, g = mlp.loss_and_grad(theta, X, T)
    assert np.allclose(g[-2:], (theta[-2:] - T.mean(axis=0)), atol=1e-15)
    assert np.all(g[:-2] == 0.0)
    assert abs(L - np.mean((theta[-2:] - T) ** 2)) < 1e-15


def test_features_translation_invariant():
    """Shifting the fields by one cell and the particle by one cell width leaves the
    features unchanged (they only see the particle's local window)."""
    w = workloads.get("langmuir64")
    arr = workloads.generate(w, n=50)
    o = Oracle.from_workload(w, n=50)
    s = initial_state(o, arr)
    f0 = mlp.features(o, s, range(50), w.degree)
    s2 = dict(s)
    for k in ("ay", "az", "ex"):
        s2[k] = np.roll(s[k], 1)
    s2["x"] = np.mod(s["x"] + w.dx, w.L)
    f1 = mlp.features(o, s2, range(50), w.degree)
    assert np.abs(f1 - f0).max() < 1e-12
    assert f0.shape == (50, mlp.n_features(w.degree))
    assert np.all(np.abs(f0[:, 0]) <= 0.5)


# -- training: the counter-based generator, the initialisation, Adam ---------
def test_splitmix64_published_sequence():
    """splitmix64 seeded with 0 gives e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f (its published first outputs); the state advances by the
    golden-ratio increment between calls."""
    gamma = 0x9E3779B97F4A7C15
    outs = [mlp.splitmix64((k * gamma) & ((1 << 64) - 1)) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_glorot_init_bounds_and_variance():
    """Weights lie in +-sqrt(6 / (fan_in + fan_out)) with the variance of that
    uniform law (bound^2 / 3); biases start at zero."""
    D = mlp.n_features(3)
    th = mlp.glorot_init(7, D)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(th, D)
    for W, (a, b) in ((W1, (D, 64)), (W2, (64, 64)), (W3, (64, 2))):
        L = math.sqrt(6.0 / (a + b))
        assert np.abs(W).max() <= L
        if W.size >= 1000:
            assert abs(W.var() / (L * L / 3.0) - 1.0) < 0.1
    assert not np.any(b1) and not np.any(b2) and not np.any(b3)
    assert np.array_equal(th, mlp.glorot_init(7, D)) and not np.array_equal(th, mlp.glorot_init(8, D))


def test_batch_indices_range_and_spread():
    idx = mlp.batch_indices(3, 5, 4096, 1000)
    assert idx.min() >= 0 and idx.max() < 1000
    counts = np.bincount(idx, minlength=1000)
    assert counts.max() < 20 and np.count_nonzero(counts) > 950


def test_adam_first_step_has_length_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so every coordinate with
    |g| >> eps moves by lr against the sign of its gradient, whatever |g| is."""
    rng = np.random.default_rng(1)
    g = rng.choice([-1.0, 1.0], 200) * 10.0 ** rng.uniform(-4, 4, 200)
    th, m, v = mlp.adam_step(np.zeros(200), np.zeros(200), np.zeros(200), g, 1, 1e-3)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-3, atol=0)


def test_adam_invariant_to_gradient_scale():
    """Rescaling every gradient by c > 0 leaves the iterates unchanged (up to eps)."""
    rng = np.random.default_rng(2)
    gs = rng.normal(0.0, 1.0, (6, 50))
    out = []
    for c in (1.0, 1000.0):
        th, m, v = np.zeros(50), np.zeros(50), np.zeros(50)
        for t, g in enumerate(gs, start=1):
            th, m, v = mlp.adam_step(th, m, v, c * g, t, 0.01)
        out.append(th)
    assert np.allclose(out[0], out[1], rtol=1e-6, atol=1e-9)


def test_adam_minimises_a_quadratic():
    """On f = sum a_i (x_i - c_i)^2 / 2 with curvatures over four decades Adam reaches the minimum."""
    a = np.logspace(-2, 2, 8)
    cst = np.linspace(-1.0, 1.0, 8)
    th, m, v = np.zeros(8), np.zeros(8), np.zeros(8)
    for t in range(1, 4001):
        lr = 0.05 if t <= 2000 else 0.005
        th, m, v = mlp.adam_step(th, m, v, a * (th - cst), t, lr)
    assert np.abs(th - cst).max() < 1e-2
