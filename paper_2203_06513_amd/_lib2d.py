"""ctypes binding of the 2D entry points of libecpic.so (include/ecpic2d.h):
argument marshalling only.

Every computation happens in the HIP library on the GPU.  If the library is not
built, or no gfx950 device is usable, the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from ._lib import EcpicError, load as _load1

# Every symbol include/ecpic2d.h declares.
EXPORTS_2D = (
    "ecpic2d_create", "ecpic2d_destroy", "ecpic2d_set_particles", "ecpic2d_get_particles",
    "ecpic2d_set_spins", "ecpic2d_get_spins", "ecpic2d_set_fields", "ecpic2d_get_fields", "ecpic2d_solve_gauss", "ecpic2d_substep_I",
    "ecpic2d_substep_II", "ecpic2d_substep_III", "ecpic2d_substep_IV", "ecpic2d_step", "ecpic2d_energy",
    "ecpic2d_gauss_residual", "ecpic2d_deposit_charge", "ecpic2d_profile_enable", "ecpic2d_kernel_time",
)


class Config2D(C.Structure):
    _fields_ = [("L1", C.c_double), ("L2", C.c_double), ("M1", C.c_int32), ("M2", C.c_int32),
                ("degree", C.c_int32), ("picard_max_iter", C.c_int32), ("n_particles", C.c_int64),
                ("weight", C.c_double), ("dt", C.c_double), ("picard_tol", C.c_double), ("device", C.c_int32),
                ("spin", C.c_int32), ("hbar", C.c_double)]


class IterStats2D(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("reserved", C.c_int32), ("residual", C.c_double)]


class EnergyParts2D(C.Structure):
    _fields_ = [("kinetic", C.c_double), ("e_xy", C.c_double), ("b_z", C.c_double), ("e_z", C.c_double),
                ("a_z", C.c_double), ("total", C.c_double), ("zeeman", C.c_double)]


_bound = False


def load() -> C.CDLL:
    global _bound
    L = _load1()
    if not _bound:
        V = C.c_void_p
        D = C.POINTER(C.c_double)
        I32P = C.POINTER(C.c_int32)
        sig = {
            "ecpic2d_create": [C.POINTER(Config2D), C.POINTER(V)],
            "ecpic2d_destroy": [V],
            "ecpic2d_set_particles": [V, V, V, V, V, C.c_int64],
            "ecpic2d_get_particles": [V, V, V, V, V, C.c_int64],
            "ecpic2d_set_spins": [V, V, V, V, C.c_int64],
            "ecpic2d_get_spins": [V, V, V, V, C.c_int64],
            "ecpic2d_set_fields": [V, V, V, V, V, V],
            "ecpic2d_get_fields": [V, V, V, V, V, V],
            "ecpic2d_solve_gauss": [V],
            "ecpic2d_substep_I": [V, C.c_double, C.POINTER(IterStats2D)],
            "ecpic2d_substep_II": [V, C.c_double],
            "ecpic2d_substep_III": [V, C.c_double, C.POINTER(IterStats2D)],
            "ecpic2d_substep_IV": [V, C.c_double],
            "ecpic2d_step": [V, C.c_int32, I32P, I32P],
            "ecpic2d_energy": [V, C.POINTER(EnergyParts2D)],
            "ecpic2d_gauss_residual": [V, D, V],
            "ecpic2d_deposit_charge": [V, V],
            "ecpic2d_profile_enable": [V, C.c_int32],
            "ecpic2d_kernel_time": [V, C.c_char_p, D, C.POINTER(C.c_int64)],
        }
        for f, args in sig.items():
            fn = getattr(L, f)
            fn.argtypes = args
            fn.restype = C.c_int
        _bound = True
    return L


def _check(status: int, what: str):
    if status != 0:
        raise EcpicError(status, what)


def _vec(a, n: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context2D:
    """One 2D simulation context on one GPU (ecpic2d_create ... ecpic2d_destroy)."""

    def __init__(self, L1, L2, M1, M2, degree, n_particles, dt, tol, weight=0.0, kmax=0, device=0, spin=0,
                 hbar=0.0):
        self.cfg = Config2D(float(L1), float(L2), int(M1), int(M2), int(degree), int(kmax), int(n_particles),
                            float(weight), float(dt), float(tol), int(device), int(spin), float(hbar))
        self.spin = bool(spin)
        self.M1, self.M2, self.N = int(M1), int(M2), int(n_particles)
        self.Nc = self.M1 * self.M2
        self._h = C.c_void_p()
        _check(load().ecpic2d_create(C.byref(self.cfg), C.byref(self._h)), "ecpic2d_create")

    @classmethod
    def from_workload(cls, w, n=None, **kw):
        n = w.n_particles if n is None else int(n)
        spin = getattr(w, "spin", "none") != "none"
        args = dict(L1=w.L1, L2=w.L2, M1=w.M1, M2=w.M2, degree=w.degree, n_particles=n, dt=w.dt, tol=w.tol,
                    weight=w.L1 * w.L2 / n if n else 0.0, kmax=w.kmax, spin=int(spin),
                    hbar=getattr(w, "hbar", 0.0) if spin else 0.0)
        args.update(kw)
        return cls(**args)

    def close(self):
        if self._h:
            load().ecpic2d_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state ------------------------------------------------------------
    def set_particles(self, x1, x2, p1, p2):
        a = [_vec(v, self.N) for v in (x1, x2, p1, p2)]
        _check(load().ecpic2d_set_particles(self._h, *[_p(v) for v in a], self.N), "ecpic2d_set_particles")

    def get_particles(self):
        out = [np.empty(self.N) for _ in range(4)]
        _check(load().ecpic2d_get_particles(self._h, *[_p(v) for v in out], self.N), "ecpic2d_get_particles")
        return dict(zip(("x1", "x2", "p1", "p2"), out))

    def set_spins(self, sx, sy, sz):
        a = [_vec(v, self.N) for v in (sx, sy, sz)]
        _check(load().ecpic2d_set_spins(self._h, *[_p(v) for v in a], self.N), "ecpic2d_set_spins")

    def get_spins(self):
        out = [np.empty(self.N) for _ in range(3)]
        _check(load().ecpic2d_get_spins(self._h, *[_p(v) for v in out], self.N), "ecpic2d_get_spins")
        return dict(zip(("sx", "sy", "sz"), out))

    def set_fields(self, e=None, bz=None, ez=None, az=None):
        """e: V1 coefficients e1 then e2 (2 M1 M2); bz, ez, az: M1 M2 each; None sets zero."""
        N = self.Nc
        e1 = e2 = None
        if e is not None:
            e = _vec(e, 2 * N)
            e1, e2 = e[:N].copy(), e[N:].copy()
        arrs = [e1, e2] + [None if v is None else _vec(v, N) for v in (bz, ez, az)]
        _check(load().ecpic2d_set_fields(self._h, *[_p(v) for v in arrs]), "ecpic2d_set_fields")

    def get_fields(self):
        out = [np.empty(self.Nc) for _ in range(5)]
        _check(load().ecpic2d_get_fields(self._h, *[_p(v) for v in out]), "ecpic2d_get_fields")
        return {"e": np.concatenate(out[:2]), "bz": out[2], "ez": out[3], "az": out[4]}

    def load(self, arrays: dict, solve_gauss: bool = True):
        """Particles and fields from a generator dict (x1, x2, p1, p2, e, bz, ez, az; sx,
        sy, sz with spin)."""
        self.set_particles(arrays["x1"], arrays["x2"], arrays["p1"], arrays["p2"])
        if self.spin:
            self.set_spins(arrays["sx"], arrays["sy"], arrays["sz"])
        self.set_fields(arrays["e"], arrays["bz"], arrays["ez"], arrays["az"])
        if solve_gauss:
            self.solve_gauss()

    def state(self) -> dict:
        s = self.get_particles()
        if self.spin:
            s.update(self.get_spins())
        s.update(self.get_fields())
        return s

    def solve_gauss(self):
        _check(load().ecpic2d_solve_gauss(self._h), "ecpic2d_solve_gauss")

    # -- substeps -----------------------------------------------------------
    def substep_I(self, dt=None):
        st = IterStats2D()
        dt = self.cfg.dt if dt is None else float(dt)
        _check(load().ecpic2d_substep_I(self._h, dt, C.byref(st)), "ecpic2d_substep_I")
        return st.sweeps, st.residual

    def substep_II(self, dt=None):
        dt = self.cfg.dt if dt is None else float(dt)
        _check(load().ecpic2d_substep_II(self._h, dt), "ecpic2d_substep_II")

    def substep_III(self, dt=None):
        st = IterStats2D()
        dt = self.cfg.dt if dt is None else float(dt)
        _check(load().ecpic2d_substep_III(self._h, dt, C.byref(st)), "ecpic2d_substep_III")
        return st.sweeps, st.residual

    def substep_IV(self, dt=None):
        dt = self.cfg.dt if dt is None else float(dt)
        _check(load().ecpic2d_substep_IV(self._h, dt), "ecpic2d_substep_IV")

    def step(self, nsteps=1):
        """nsteps Lie-Trotter steps: (sweeps_I, iters_III) per step."""
        kI = np.zeros(nsteps, dtype=np.int32)
        kIII = np.zeros(nsteps, dtype=np.int32)
        I32P = C.POINTER(C.c_int32)
        _check(load().ecpic2d_step(self._h, int(nsteps), kI.ctypes.data_as(I32P), kIII.ctypes.data_as(I32P)),
               "ecpic2d_step")
        return kI, kIII

    # -- diagnostics -----------------------------------------------------------
    def energy(self):
        """[kinetic, 1/2 e^T M1 e, 1/2 b^T M2 b, 1/2 e_z^T M0 e_z, 1/2 a^T K a, H, Zeeman]
        (H includes the Zeeman term; 0 without spin)."""
        e = EnergyParts2D()
        _check(load().ecpic2d_energy(self._h, C.byref(e)), "ecpic2d_energy")
        return np.array([e.kinetic, e.e_xy, e.b_z, e.e_z, e.a_z, e.total, e.zeeman])

    def gauss_residual(self, vec=False):
        m = C.c_double()
        v = np.empty(self.Nc) if vec else None
        _check(load().ecpic2d_gauss_residual(self._h, C.byref(m), _p(v)), "ecpic2d_gauss_residual")
        return (m.value, v) if vec else m.value

    def deposit_charge(self):
        rho = np.empty(self.Nc)
        _check(load().ecpic2d_deposit_charge(self._h, _p(rho)), "ecpic2d_deposit_charge")
        return rho

    def profile(self, on: bool = True):
        _check(load().ecpic2d_profile_enable(self._h, int(bool(on))), "ecpic2d_profile_enable")

    def kernel_time(self, name: str):
        ms = C.c_double()
        n = C.c_int64()
        _check(load().ecpic2d_kernel_time(self._h, name.encode(), C.byref(ms), C.byref(n)), "ecpic2d_kernel_time")
        return ms.value, n.value
