"""FP64 reference of the learned warm start's network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: only tests/, the smoke check and the benchmark's CPU
leg may import this module; the HIP library never does.

The network maps a particle's local state to the Picard increment of Subsystem I
(Section 4.2): a multilayer perceptron 27 -> 64 -> 64 -> 2 with the tanh form
of GELU (Hendrycks and Gimpel, 2016) on both hidden layers and a linear output.
Plain NumPy in float64, written from the textbook definitions of the forward
pass, of the mean squared error and of its gradient by the chain rule; no
blocking or fusion.

Features of a particle at x in cell c (local coordinate t = x/dx - c), for
spline degree p, and its targets (the increments the method converges to):
    f = [t - 1/2, p, gamma0 - 1,
         a_y[c-p .. c+p+1], a_z[c-p .. c+p+1], e_x[c-p .. c+p+1]]      (3 + 6 (p+1))
    y = [(delta - dt p / gamma0) / dt^2,  (p^{n+1} - p) / dt]
with gamma0 = sqrt(1 + p^2 + |A_perp(x)|^2).  Parameters are one flat vector
[W1 (H x D, row-major), b1 (H), W2 (H x H), b2 (H), W3 (2 x H), b3 (2)].
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 64
N_OUT = 2
_C = math.sqrt(2.0 / math.pi)
_A = 0.044715


def n_features(degree: int) -> int:
    return 3 + 6 * (degree + 1)


def n_params(d_in: int, h: int = HIDDEN) -> int:
    return h * d_in + h + h * h + h + N_OUT * h + N_OUT


def unpack(theta: np.ndarray, d_in: int, h: int = HIDDEN):
    i = 0
    def take(n, shape):
        nonlocal i
        v = theta[i:i + n].reshape(shape)
        i += n
        return v
    W1 = take(h * d_in, (h, d_in)); b1 = take(h, (h,))
    W2 = take(h * h, (h, h)); b2 = take(h, (h,))
    W3 = take(N_OUT * h, (N_OUT, h)); b3 = take(N_OUT, (N_OUT,))
    assert i == len(theta)
    return W1, b1, W2, b2, W3, b3


def gelu(z):
    """0.5 z (1 + tanh(sqrt(2/pi) (z + 0.044715 z^3)))."""
    return 0.5 * z * (1.0 + np.tanh(_C * (z + _A * z ** 3)))


def gelu_grad(z):
    t = np.tanh(_C * (z + _A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * _C * (1.0 + 3.0 * _A * z * z)


def forward(theta, X, h: int = HIDDEN):
    """X: (n, d_in) normalised features.  Returns outputs (n, 2) and the cache."""
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, np.float64), X.shape[1], h)
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(theta, X, T, h: int = HIDDEN) -> float:
    """Mean over samples and outputs of the squared error."""
    Y, _ = forward(theta, X, h)
    return float(np.mean((Y - np.asarray(T, np.float64)) ** 2))


def loss_and_grad(theta, X, T, h: int = HIDDEN):
    """Loss and its gradient with respect to theta (chain rule, layer by layer)."""
    theta = np.asarray(theta, np.float64)
    T = np.asarray(T, np.float64)
    Y, (X, Z1, H1, Z2, H2) = forward(theta, X, h)
    W1, b1, W2, b2, W3, b3 = unpack(theta, X.shape[1], h)
    n = X.shape[0]
    dY = 2.0 * (Y - T) / (n * N_OUT)
    gW3 = dY.T @ H2
    gb3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * gelu_grad(Z2)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return float(np.mean((Y - T) ** 2)), g


def features(o, s, idx, degree: int):
    """Raw features of particles idx of state s (x, p, ay, az, ex) for oracle o."""
    dx = o.cfg.L / o.cfg.M
    M = o.cfg.M
    out = np.empty((len(idx), n_features(degree)))
    for r, a in enumerate(idx):
        x = s["x"][a]
        xi = x / dx
        c = int(math.floor(xi))
        if c >= M:
            c = M - 1
        t = xi - c
        Ay = o.field0(s["ay"], x)
        Az = o.field0(s["az"], x)
        g0 = math.sqrt(1.0 + s["p"][a] ** 2 + Ay * Ay + Az * Az)
        win = [(c + j) % M for j in range(-degree, degree + 2)]
        out[r, 0] = t - 0.5
        out[r, 1] = s["p"][a]
        out[r, 2] = g0 - 1.0
        out[r, 3:3 + 2 * (degree + 1)] = s["ay"][win]
        out[r, 3 + 2 * (degree + 1):3 + 4 * (degree + 1)] = s["az"][win]
        out[r, 3 + 4 * (degree + 1):] = s["ex"][win]
    return out
