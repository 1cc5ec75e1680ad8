"""Seeded synthetic workloads shared by the oracle, the GPU path, the tests and the bench.

This module only draws random numbers and samples closed-form initial profiles.
It holds none of the method's arithmetic: no spline evaluation, no mass matrix,
no solve.  Both the oracle and the HIP library receive the arrays it returns.

Workloads (the physics follows the reduced 1D model of Section 2.1 with the
spin term switched off, and the parametric-instability setup of Section 5.1):

* ``paper51`` -- the paper's own run (Section 5.1): L = 2*pi/k, k = 1/sqrt(2),
  128 cells, 4000 particles, Maxwellian T = 3/511, circularly polarised pump
  E0 = sqrt(3), dt = 0.02, tolerance 1e-13.
* ``langmuir64`` -- L = 4 pi, 64 cells, 1e4 particles, 1 % density ripple,
  sigma = 0.1, linear transverse wave a = 0.05, dt = 0.05, 100 steps, tol 1e-13.
* ``pump2048`` -- L = 64 pi, 2048 cells, 2e6 particles, sigma = 0.05,
  circularly polarised pump a0 = 0.1 at k0 = 1 plus 1e-4 coefficient noise,
  dt = 0.02, 2000 steps, tol 1e-12.
* ``langmuir4096`` -- the ``langmuir64`` physics at L = 128 pi, 4096 cells,
  1.6e7 particles (the FP32 precision form is run on it).
* ``stress16384`` -- L = 256 pi, 16384 cells, quintic splines, 1.28e8
  particles, pump a0 = 0.3 at k0 = 1, sigma = 0.1, dt = 0.01, tol 1e-12.
* ``paper52`` -- the paper's run with spin (Section 5.2): the ``paper51``
  setup with 1e4 particles, hbar = 0.1 and every spin (0, 0, 1).
* ``spin4096`` -- the spin model at scale: the ``paper51`` physics (pump
  E0 = sqrt 3 at k = 1/sqrt 2, T = 3/511) on 32 wavelengths, 4096 cells,
  1.6e7 particles, hbar = 0.1, spins uniform on the unit sphere, dt = 0.02,
  tol 1e-12.

Spins are drawn after every other array, so a workload without spin draws
exactly what it drew before spins existed.

Field coefficients are sampled at the Greville abscissae x_j + (p+1) dx / 2 of
the degree-p basis (Schoenberg's variation-diminishing quasi-interpolant); the
paper leaves its projector to another reference, and since both sides start
from the same arrays the choice does not enter parity.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

__all__ = ["Workload", "WORKLOADS", "get", "generate", "small"]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    L: float
    M: int
    degree: int
    n_particles: int
    dt: float
    steps: int
    tol: float
    sigma: float                 # Maxwellian width of p_x
    density_ripple: float = 0.0  # eps in 1 + eps cos(k_rip x)
    ripple_mode: int = 1
    wave: str = "none"           # "none" | "linear_y" | "cp"
    amplitude: float = 0.0       # a (linear) or a0 (circular) or E0 (paper)
    wave_mode: int = 1           # k = 2 pi mode / L
    coef_noise: float = 0.0      # std of N(0, s^2) added to a_y, a_z coefficients
    seed: int = 0
    kmax: int = 50
    hbar: float = 0.0            # spin coupling (Section 2.1)
    spin: str = "none"           # "none" | "z" (every spin (0, 0, 1)) | "sphere" (uniform)

    @property
    def dx(self) -> float:
        return self.L / self.M

    @property
    def weight(self) -> float:
        return self.L / self.n_particles

    def scaled(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def _paper51() -> Workload:
    k = 1.0 / math.sqrt(2.0)
    return Workload(name="paper51", L=2.0 * math.pi / k, M=128, degree=3, n_particles=4000,
                    dt=0.02, steps=4000, tol=1e-13, sigma=math.sqrt(3.0 / 511.0),
                    wave="paper", amplitude=math.sqrt(3.0), wave_mode=1, seed=511)


def _spin4096() -> Workload:
    k = 1.0 / math.sqrt(2.0)
    return Workload(name="spin4096", L=32 * 2.0 * math.pi / k, M=4096, degree=3, n_particles=16_000_000,
                    dt=0.02, steps=1000, tol=1e-12, sigma=math.sqrt(3.0 / 511.0), wave="paper",
                    amplitude=math.sqrt(3.0), wave_mode=32, seed=5232, hbar=0.1, spin="sphere")


WORKLOADS: Dict[str, Workload] = {
    "paper51": _paper51(),
    "paper52": dataclasses.replace(_paper51(), name="paper52", n_particles=10_000, steps=10_000, seed=512,
                                   hbar=0.1, spin="z"),
    "spin4096": _spin4096(),
    "langmuir64": Workload(name="langmuir64", L=4.0 * math.pi, M=64, degree=3, n_particles=10_000,
                           dt=0.05, steps=100, tol=1e-13, sigma=0.1, density_ripple=0.01,
                           ripple_mode=1, wave="linear_y", amplitude=0.05, wave_mode=1, seed=101),
    "pump2048": Workload(name="pump2048", L=64.0 * math.pi, M=2048, degree=3, n_particles=2_000_000,
                         dt=0.02, steps=2000, tol=1e-12, sigma=0.05, wave="cp", amplitude=0.1,
                         wave_mode=32, coef_noise=1e-4, seed=202),
    "langmuir4096": Workload(name="langmuir4096", L=128.0 * math.pi, M=4096, degree=3,
                             n_particles=16_000_000, dt=0.05, steps=100, tol=1e-13, sigma=0.1,
                             density_ripple=0.01, ripple_mode=32, wave="linear_y", amplitude=0.05,
                             wave_mode=32, seed=303),
    "stress16384": Workload(name="stress16384", L=256.0 * math.pi, M=16384, degree=5,
                            n_particles=128_000_000, dt=0.01, steps=10_000, tol=1e-12, sigma=0.1,
                            wave="cp", amplitude=0.3, wave_mode=128, coef_noise=1e-4, seed=505),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]


def small(name: str = "tiny", *, L: float = 2.0, M: int = 8, degree: int = 3, n: int = 3,
          dt: float = 0.05, tol: float = 1e-13, sigma: float = 0.2, wave: str = "cp",
          amplitude: float = 0.3, seed: int = 7, **kw) -> Workload:
    """A hand-sized workload for brute-force and edge-case tests."""
    return Workload(name=name, L=L, M=M, degree=degree, n_particles=n, dt=dt, steps=1, tol=tol,
                    sigma=sigma, wave=wave, amplitude=amplitude, wave_mode=1, seed=seed, **kw)


def _positions(w: Workload, rng: np.random.Generator, n: int) -> np.ndarray:
    u = rng.random(n)
    if w.density_ripple == 0.0:
        x = w.L * u
    else:
        # inverse CDF of (1 + eps cos(k x)) / L on [0, L): solve x + (eps/k) sin(k x) = u L
        k = 2.0 * math.pi * w.ripple_mode / w.L
        eps = w.density_ripple
        target = u * w.L
        x = target.copy()
        for _ in range(60):   # Newton; quadratic, so a few steps reach round-off
            f = x + (eps / k) * np.sin(k * x) - target
            x = x - f / (1.0 + eps * np.cos(k * x))
            if np.abs(f).max(initial=0.0) <= 1e-15 * w.L:
                break
        x = np.mod(x, w.L)
    x[x >= w.L] = 0.0
    return x


def _fields(w: Workload, rng: np.random.Generator):
    M, p, dx = w.M, w.degree, w.dx
    greville = (np.arange(M) + 0.5 * (p + 1)) * dx     # V0 (degree p) abscissae
    k = 2.0 * math.pi * w.wave_mode / w.L
    ay = np.zeros(M); az = np.zeros(M); ey = np.zeros(M); ez = np.zeros(M)
    if w.wave == "linear_y":
        # +x travelling linear wave A_y = a cos(kx - wt), E_y = -dA_y/dt, w^2 = k^2 + 1
        om = math.sqrt(k * k + 1.0)
        ay = w.amplitude * np.cos(k * greville)
        ey = -w.amplitude * om * np.sin(k * greville)
    elif w.wave == "cp":
        # circularly polarised pump A = a0 (cos(kx - wt), sin(kx - wt)), E = -dA/dt,
        # relativistic dispersion w^2 = k^2 + 1/gamma0, gamma0 = sqrt(1 + a0^2)
        g0 = math.sqrt(1.0 + w.amplitude ** 2)
        om = math.sqrt(k * k + 1.0 / g0)
        ay = w.amplitude * np.cos(k * greville)
        az = w.amplitude * np.sin(k * greville)
        ey = -w.amplitude * om * np.sin(k * greville)
        ez = w.amplitude * om * np.cos(k * greville)
    elif w.wave == "paper":
        # Section 5.1 initial fields: E_y = E0 cos kx, E_z = E0 sin kx, A_y = -E0 sin kx, A_z = E0 cos kx
        E0 = w.amplitude
        ey = E0 * np.cos(k * greville)
        ez = E0 * np.sin(k * greville)
        ay = -E0 * np.sin(k * greville)
        az = E0 * np.cos(k * greville)
    if w.coef_noise > 0.0:
        ay = ay + rng.normal(0.0, w.coef_noise, M)
        az = az + rng.normal(0.0, w.coef_noise, M)
    return ey, ez, ay, az


def generate(w: Workload, n: Optional[int] = None, seed: Optional[int] = None) -> dict:
    """Initial state arrays for workload ``w`` (float64, host).

    Returns a dict with x, p (length n) and ey, ez, ay, az (length M), and with
    spin sx, sy, sz (length n); e_x is left to the discrete Poisson solve of each
    implementation.
    """
    n = w.n_particles if n is None else int(n)
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    x = _positions(w, rng, n)
    p = rng.normal(0.0, w.sigma, n)
    ey, ez, ay, az = _fields(w, rng)
    out = {"x": x.astype(np.float64), "p": p.astype(np.float64), "ey": ey, "ez": ez, "ay": ay, "az": az}
    if w.spin == "z":
        out.update(sx=np.zeros(n), sy=np.zeros(n), sz=np.ones(n))
    elif w.spin == "sphere":
        # uniform on the unit sphere: cos(theta) uniform in [-1, 1], azimuth uniform
        u = rng.uniform(-1.0, 1.0, n)
        phi = rng.uniform(0.0, 2.0 * math.pi, n)
        r = np.sqrt(1.0 - u * u)
        out.update(sx=r * np.cos(phi), sy=r * np.sin(phi), sz=u)
    return out
