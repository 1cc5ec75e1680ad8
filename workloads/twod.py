"""Seeded synthetic workloads of the reduced 2D model (Section 2.2).

Like the 1D module, this draws random numbers and samples closed-form initial
profiles only: no spline evaluation, no mass matrix, no solve.  Both the oracle
and the HIP library receive the arrays it returns, and each corrects e_xy by its
own discrete Poisson solve so that the discrete Gauss law holds.

The paper runs no 2D experiment, so these workloads are synthetic plasmas of
its 2D model (normalised units: plasma frequency 1, light speed 1):

* ``twod16``  -- 4 pi x 4 pi, 16 x 16 cells, cubic, 4000 particles, density
  ripple 5 % in both directions, an A_z wave (0.05, wave vector (1, 1) modes), a
  TE wave (B_z, E_x) along x2 (0.05, mode 1), sigma = 0.1, dt = 0.05;
* ``twod8x16`` -- 2 pi x 4 pi, 8 x 16 cells, quadratic, 3000 particles (a
  rectangular grid with unequal cells);
* ``twod512`` -- 16 pi x 16 pi, 512 x 512 cells (dx = 0.098, about one Debye
  length at sigma = 0.1), cubic, 2^24 particles (64 per cell), ripple 1 % at
  mode (8, 8), A_z wave 0.05 at modes (8, 4), TE wave 0.05 at mode 8, dt = 0.05,
  tolerance 1e-12;
* ``twod16s``, ``twod8x16s`` -- the two small plasmas with spin: hbar = 0.1 and
  spins uniform on the unit sphere (as the 1D spin workload at scale);
* ``twod512s`` -- ``twod512`` with the same spins.

Spins are drawn after every other array, so a workload without spin draws
exactly what it drew before spins existed.

Coefficients are sampled at the Greville abscissae of each tensor-product
basis, as in 1D.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np

__all__ = ["Workload2D", "WORKLOADS_2D", "get2d", "generate2d", "small2d"]


@dataclasses.dataclass(frozen=True)
class Workload2D:
    name: str
    L1: float
    L2: float
    M1: int
    M2: int
    degree: int
    n_particles: int
    dt: float
    steps: int
    tol: float
    sigma: float                         # Maxwellian width of p1 and p2
    ripple: float = 0.0                  # eps in (1 + eps cos k1 x1)(1 + eps cos k2 x2)
    ripple_mode: Tuple[int, int] = (1, 1)
    az_amp: float = 0.0                  # A_z = a cos(k . x), E_z = -a w sin(k . x), w^2 = |k|^2 + 1
    az_mode: Tuple[int, int] = (1, 1)
    te_amp: float = 0.0                  # B_z = b cos(k x2), E_x = -(b w / k) cos(k x2)
    te_mode: int = 1
    seed: int = 0
    kmax: int = 50
    hbar: float = 0.0                    # spin coupling (Section 2.2)
    spin: str = "none"                   # "none" | "sphere" (uniform on the unit sphere)

    @property
    def dx1(self) -> float:
        return self.L1 / self.M1

    @property
    def dx2(self) -> float:
        return self.L2 / self.M2

    @property
    def weight(self) -> float:
        return self.L1 * self.L2 / self.n_particles

    def scaled(self, **kw) -> "Workload2D":
        return dataclasses.replace(self, **kw)


WORKLOADS_2D: Dict[str, Workload2D] = {
    "twod16": Workload2D(name="twod16", L1=4 * math.pi, L2=4 * math.pi, M1=16, M2=16, degree=3,
                         n_particles=4000, dt=0.05, steps=10, tol=1e-13, sigma=0.1, ripple=0.05,
                         ripple_mode=(1, 1), az_amp=0.05, az_mode=(1, 1), te_amp=0.05, te_mode=1, seed=1601),
    "twod8x16": Workload2D(name="twod8x16", L1=2 * math.pi, L2=4 * math.pi, M1=8, M2=16, degree=2,
                           n_particles=3000, dt=0.05, steps=10, tol=1e-13, sigma=0.2, ripple=0.05,
                           ripple_mode=(1, 2), az_amp=0.1, az_mode=(1, 1), te_amp=0.05, te_mode=2, seed=816),
    "twod512": Workload2D(name="twod512", L1=16 * math.pi, L2=16 * math.pi, M1=512, M2=512, degree=3,
                          n_particles=1 << 24, dt=0.05, steps=100, tol=1e-12, sigma=0.1, ripple=0.01,
                          ripple_mode=(8, 8), az_amp=0.05, az_mode=(8, 4), te_amp=0.05, te_mode=8, seed=5120),
}
WORKLOADS_2D["twod16s"] = WORKLOADS_2D["twod16"].scaled(name="twod16s", hbar=0.1, spin="sphere")
WORKLOADS_2D["twod8x16s"] = WORKLOADS_2D["twod8x16"].scaled(name="twod8x16s", hbar=0.1, spin="sphere")
WORKLOADS_2D["twod512s"] = WORKLOADS_2D["twod512"].scaled(name="twod512s", hbar=0.1, spin="sphere")


def get2d(name: str) -> Workload2D:
    return WORKLOADS_2D[name]


def small2d(name: str = "tiny2d", *, L1: float = 2.0, L2: float = 2.0, M1: int = 4, M2: int = 4,
            degree: int = 2, n: int = 3, dt: float = 0.05, tol: float = 1e-13, sigma: float = 0.3,
            seed: int = 9, **kw) -> Workload2D:
    """A hand-sized 2D workload for brute-force and edge-case tests."""
    kw.setdefault("az_amp", 0.3)
    kw.setdefault("te_amp", 0.2)
    kw.setdefault("ripple", 0.1)
    return Workload2D(name=name, L1=L1, L2=L2, M1=M1, M2=M2, degree=degree, n_particles=n, dt=dt, steps=1,
                      tol=tol, sigma=sigma, seed=seed, **kw)


def _coordinate(u: np.ndarray, L: float, eps: float, mode: int) -> np.ndarray:
    """Inverse CDF of (1 + eps cos(k x)) / L on [0, L), k = 2 pi mode / L (Newton)."""
    if eps == 0.0:
        x = L * u
    else:
        k = 2.0 * math.pi * mode / L
        target = u * L
        x = target.copy()
        for _ in range(60):
            f = x + (eps / k) * np.sin(k * x) - target
            x = x - f / (1.0 + eps * np.cos(k * x))
            if np.abs(f).max(initial=0.0) <= 1e-15 * L:
                break
        x = np.mod(x, L)
    x[x >= L] = 0.0
    return x


def _grid(w: Workload2D, s1: float, s2: float):
    """Sample points (i1 + s1) dx1, (i2 + s2) dx2 as two (M1, M2) arrays."""
    g1 = (np.arange(w.M1) + s1) * w.dx1
    g2 = (np.arange(w.M2) + s2) * w.dx2
    return np.meshgrid(g1, g2, indexing="ij")


def generate2d(w: Workload2D, n: Optional[int] = None, seed: Optional[int] = None) -> dict:
    """Initial state arrays (float64, host): x1, x2, p1, p2 (length n); e (e1 then e2,
    2 M1 M2), bz, ez, az (M1 M2), row-major with index i1 M2 + i2; with spin also sx,
    sy, sz (length n)."""
    n = w.n_particles if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    x1 = _coordinate(rng.random(n), w.L1, w.ripple, w.ripple_mode[0])
    x2 = _coordinate(rng.random(n), w.L2, w.ripple, w.ripple_mode[1])
    p1 = rng.normal(0.0, w.sigma, n)
    p2 = rng.normal(0.0, w.sigma, n)
    p = w.degree
    # V0 (degree p, p) at (i + (p+1)/2) dx; V1 component 1 (p-1, p), component 2 (p, p-1); V2 (p-1, p-1)
    k1 = 2.0 * math.pi * w.az_mode[0] / w.L1
    k2 = 2.0 * math.pi * w.az_mode[1] / w.L2
    om = math.sqrt(k1 * k1 + k2 * k2 + 1.0)
    X1, X2 = _grid(w, 0.5 * (p + 1), 0.5 * (p + 1))
    az = w.az_amp * np.cos(k1 * X1 + k2 * X2)
    ez = -w.az_amp * om * np.sin(k1 * X1 + k2 * X2)
    kt = 2.0 * math.pi * w.te_mode / w.L2
    omt = math.sqrt(kt * kt + 1.0)
    _, Y2 = _grid(w, 0.5 * p, 0.5 * p)
    bz = w.te_amp * np.cos(kt * Y2)
    _, E2 = _grid(w, 0.5 * p, 0.5 * (p + 1))
    e1 = -(w.te_amp * omt / kt) * np.cos(kt * E2)
    e2 = np.zeros((w.M1, w.M2))
    out = {"x1": x1.astype(np.float64), "x2": x2.astype(np.float64), "p1": p1, "p2": p2,
           "e": np.concatenate([e1.ravel(), e2.ravel()]), "bz": bz.ravel().copy(),
           "ez": ez.ravel().copy(), "az": az.ravel().copy()}
    if w.spin == "sphere":   # drawn after every other array: a workload without spin draws what it did
        u = rng.uniform(-1.0, 1.0, n)
        phi = rng.uniform(0.0, 2.0 * math.pi, n)
        r = np.sqrt(1.0 - u * u)
        out.update(sx=r * np.cos(phi), sy=r * np.sin(phi), sz=u)
    return out
