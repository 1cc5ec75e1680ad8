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
