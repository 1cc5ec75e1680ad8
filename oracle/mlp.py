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


# -- training: initialisation, sampling and the Adam update ------------------
_M64 = (1 << 64) - 1


def splitmix64(z: int) -> int:
    """The output function of splitmix64 (Steele, Lea and Flood, 2014) for state z:
    add the golden-ratio increment, then xor-shift-multiply twice and xor-shift."""
    z = (z + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def unit_uniform(seed: int, k: int) -> float:
    """The k-th draw of a counter-based stream: the top 53 bits of
    splitmix64(seed xor splitmix64(k)) as a double in [0, 1)."""
    return (splitmix64((seed ^ splitmix64(k)) & _M64) >> 11) * 2.0 ** -53


def glorot_init(seed: int, d_in: int, h: int = HIDDEN) -> np.ndarray:
    """Glorot-uniform weights (Glorot and Bengio, 2010), zero biases: parameter k of
    a weight matrix with fan-in a and fan-out b is (2 u_k - 1) sqrt(6 / (a + b))."""
    W1, b1, W2, b2, W3, b3 = unpack(np.arange(n_params(d_in, h), dtype=np.float64), d_in, h)
    theta = np.zeros(n_params(d_in, h))
    for block, (a, b) in ((W1, (d_in, h)), (W2, (h, h)), (W3, (h, N_OUT))):
        for k in block.ravel().astype(np.int64):
            theta[k] = (2.0 * unit_uniform(seed, int(k)) - 1.0) * math.sqrt(6.0 / (a + b))
    return theta


def batch_indices(seed: int, step: int, batch: int, n: int) -> np.ndarray:
    """Sample j of training step `step`: record splitmix64(seed xor splitmix64(step B + j)) mod n."""
    return np.array([splitmix64((seed ^ splitmix64(step * batch + j)) & _M64) % n for j in range(batch)],
                    dtype=np.int64)


def adam_step(theta, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1) at step t >= 1: the biased
    first and second moment estimates, their bias corrections by 1 - beta^t, and the
    step lr m_hat / (sqrt(v_hat) + eps).  Returns (theta, m, v)."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return np.asarray(theta, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
