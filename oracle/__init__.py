"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The HIP library never imports, links or
calls anything here, and this module never imports the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")
SRC2D_PATH = os.path.join(_HERE, "oracle2d.c")

OK, ENOTCONV = 0, -3


def build(force: bool = True) -> str:
    """Compile the oracle (1D and 2D) with gcc (strict IEEE: no contraction, no fast-math)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", LIB_PATH, SRC_PATH, SRC2D_PATH, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB_PATH


class Cfg(C.Structure):
    _fields_ = [("L", C.c_double), ("M", C.c_int32), ("p", C.c_int32), ("n", C.c_int64),
                ("w", C.c_double), ("dt", C.c_double), ("tol", C.c_double),
                ("kmax", C.c_int32), ("commit_unconverged", C.c_int32), ("seidel", C.c_int32),
                ("splitting", C.c_int32), ("warm_previous", C.c_int32), ("hbar", C.c_double)]


_lib: Optional[C.CDLL] = None
_D = C.POINTER(C.c_double)


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(Cfg)
        L.orc_bspline.restype = C.c_double
        L.orc_bspline.argtypes = [C.c_int, C.c_double]
        for f in ("orc_lambda0", "orc_lambda1"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [P, C.c_long, C.c_double]
        for f in ("orc_field0", "orc_field1"):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [P, _D, C.c_double]
        L.orc_mass_row.restype = None
        L.orc_mass_row.argtypes = [C.c_int, _D]
        for f in ("orc_apply_M0", "orc_apply_M1", "orc_apply_G", "orc_apply_GT", "orc_apply_K",
                  "orc_apply_cn_plus", "orc_apply_cn_minus", "orc_solve_M1", "orc_solve_M0",
                  "orc_solve_cn"):
            getattr(L, f).restype = None
            getattr(L, f).argtypes = [P, _D, _D]
        for f in ("orc_line_mean", "orc_line_mean2"):
            getattr(L, f).restype = C.c_int
            getattr(L, f).argtypes = [P, C.c_double, C.c_double, C.POINTER(C.c_long), _D]
        L.orc_deposit_current.restype = None
        L.orc_deposit_current.argtypes = [P, _D, _D, C.c_int64, _D]
        L.orc_deposit_charge.restype = None
        L.orc_deposit_charge.argtypes = [P, _D, _D]
        L.orc_energy.restype = None
        L.orc_energy.argtypes = [P, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_gauss_residual.restype = C.c_double
        L.orc_gauss_residual.argtypes = [P, _D, _D, _D]
        L.orc_solve_gauss.restype = None
        L.orc_solve_gauss.argtypes = [P, _D, _D]
        L.orc_particle_map.restype = None
        L.orc_particle_map.argtypes = [P, C.c_double, C.c_double, C.c_double, _D, _D, _D, _D, _D,
                                       _D, _D, C.POINTER(C.c_long), C.POINTER(C.c_int), _D]
        I32 = C.POINTER(C.c_int32)
        L.orc_substep_I.restype = C.c_int
        L.orc_substep_I.argtypes = [P, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_I_h.restype = C.c_int
        L.orc_substep_I_h.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_I_adjoint.restype = C.c_int
        L.orc_substep_I_adjoint.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_particle_map_adjoint.restype = None
        L.orc_particle_map_adjoint.argtypes = [P, C.c_double, C.c_double, C.c_double, _D, _D, _D, _D, _D,
                                               _D, _D, _D]
        L.orc_substep_II.restype = C.c_int
        L.orc_substep_II.argtypes = [P, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_II_h.restype = C.c_int
        L.orc_substep_II_h.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [P, C.c_int32, _D, _D, _D, _D, _D, _D, _D, I32, I32, I32, _D]
        # spin
        L.orc_particle_map_spin.restype = None
        L.orc_particle_map_spin.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                            _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_substep_I_hs.restype = C.c_int
        L.orc_substep_I_hs.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_I_adjoint_s.restype = C.c_int
        L.orc_substep_I_adjoint_s.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_II_hs.restype = C.c_int
        L.orc_substep_II_hs.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D, _D, _D, I32, _D]
        L.orc_substep_III_h.restype = None
        L.orc_substep_III_h.argtypes = [P, C.c_double, _D, _D, _D, _D, _D, _D]
        L.orc_energy_s.restype = None
        L.orc_energy_s.argtypes = [P, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D]
        L.orc_step_s.restype = C.c_int
        L.orc_step_s.argtypes = [P, C.c_int32, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D, I32, I32, I32, _D]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """The oracle bound to one configuration (L, M, p, n, w, dt, tol, kmax)."""

    def __init__(self, L, M, p, n, w=None, dt=0.05, tol=1e-13, kmax=50, commit_unconverged=False,
                 seidel=False, splitting=0, warm_previous=False, hbar=0.0):
        if w is None:
            w = L / n if n > 0 else 0.0
        self.cfg = Cfg(float(L), int(M), int(p), int(n), float(w),
                       float(dt), float(tol), int(kmax), int(bool(commit_unconverged)),
                       int(bool(seidel)), int(splitting), int(bool(warm_previous)), float(hbar))
        self._c = C.byref(self.cfg)

    @classmethod
    def from_workload(cls, w, n=None, **kw):
        n = w.n_particles if n is None else n
        args = dict(L=w.L, M=w.M, p=w.degree, n=n, w=w.L / n, dt=w.dt, tol=w.tol, kmax=w.kmax,
                    hbar=getattr(w, "hbar", 0.0))
        args.update(kw)
        return cls(**args)

    # -- bases and matrices --------------------------------------------------
    @staticmethod
    def bspline(d, u):
        return lib().orc_bspline(int(d), float(u))

    @staticmethod
    def mass_row(d):
        row = np.zeros(2 * d + 1)
        lib().orc_mass_row(int(d), _ptr(row))
        return row

    def lambda0(self, j, x):
        return lib().orc_lambda0(self._c, int(j), float(x))

    def lambda1(self, j, x):
        return lib().orc_lambda1(self._c, int(j), float(x))

    def field0(self, coef, x):
        coef = _f64(coef)
        return lib().orc_field0(self._c, _ptr(coef), float(x))

    def field1(self, coef, x):
        coef = _f64(coef)
        return lib().orc_field1(self._c, _ptr(coef), float(x))

    def _op(self, name, v):
        v = _f64(v)
        out = np.zeros(self.cfg.M)
        getattr(lib(), name)(self._c, _ptr(v), _ptr(out))
        return out

    def M0(self, v): return self._op("orc_apply_M0", v)
    def M1(self, v): return self._op("orc_apply_M1", v)
    def G(self, v): return self._op("orc_apply_G", v)
    def GT(self, v): return self._op("orc_apply_GT", v)
    def K(self, v): return self._op("orc_apply_K", v)
    def cn_plus(self, v): return self._op("orc_apply_cn_plus", v)
    def cn_minus(self, v): return self._op("orc_apply_cn_minus", v)
    def solve_M1(self, v): return self._op("orc_solve_M1", v)
    def solve_M0(self, v): return self._op("orc_solve_M0", v)
    def solve_cn(self, v): return self._op("orc_solve_cn", v)

    def line_mean(self, x0, x1):
        jlo = C.c_long(0)
        vals = np.zeros(16)
        nj = lib().orc_line_mean(self._c, float(x0), float(x1), C.byref(jlo), _ptr(vals))
        return jlo.value, vals[:nj].copy()

    def line_mean2(self, x0, x1):
        """Means of the degree p-2 splines over the segment (the spin force's divided
        differences)."""
        jlo = C.c_long(0)
        vals = np.zeros(16)
        nj = lib().orc_line_mean2(self._c, float(x0), float(x1), C.byref(jlo), _ptr(vals))
        return jlo.value, vals[:nj].copy()

    def deposit_current(self, x0, x1):
        x0 = _f64(x0); x1 = _f64(x1)
        J = np.zeros(self.cfg.M)
        lib().orc_deposit_current(self._c, _ptr(x0), _ptr(x1), len(x0), _ptr(J))
        return J

    def deposit_charge(self, x):
        x = _f64(x)
        assert len(x) == self.cfg.n
        rho = np.zeros(self.cfg.M)
        lib().orc_deposit_charge(self._c, _ptr(x), _ptr(rho))
        return rho

    def particle_map(self, x0, p0, delta, ay, az, gy, gz, ebar):
        arrs = [_f64(a) for a in (ay, az, gy, gz, ebar)]
        p1 = C.c_double(0); dn = C.c_double(0); jlo = C.c_long(0); nj = C.c_int(0)
        lbar = np.zeros(16)
        lib().orc_particle_map(self._c, float(x0), float(p0), float(delta), *[_ptr(a) for a in arrs],
                               C.byref(p1), C.byref(dn), C.byref(jlo), C.byref(nj), _ptr(lbar))
        return p1.value, dn.value, jlo.value, lbar[:nj.value].copy()

    def particle_map_spin(self, x0, p0, delta, sy, sz, ay, az, gy, gz, hy, hz, ebar):
        """One evaluation of the Subsystem I map with the spin force (hy = G G a_y)."""
        arrs = [_f64(a) for a in (ay, az, gy, gz, hy, hz, ebar)]
        p1 = C.c_double(0); dn = C.c_double(0)
        lib().orc_particle_map_spin(self._c, float(x0), float(p0), float(delta), float(sy), float(sz),
                                    *[_ptr(a) for a in arrs], C.byref(p1), C.byref(dn))
        return p1.value, dn.value

    # -- state-level operations ---------------------------------------------
    def _spins(self, s):
        """The state's spin arrays (s_x, s_y, s_z), or None if it carries none."""
        return (s["sx"], s["sy"], s["sz"]) if "sx" in s else None

    def energy(self, s):
        """[kinetic, e_x part, e_perp part, a_perp part, H]; with spins H includes the
        Zeeman term, kept in self.last_zeeman."""
        sp = self._spins(s)
        if sp is None:
            parts = np.zeros(5)
            lib().orc_energy(self._c, *[_ptr(s[k]) for k in ("x", "p", "ex", "ey", "ez", "ay", "az")],
                             _ptr(parts))
            return parts
        six = np.zeros(6)
        lib().orc_energy_s(self._c, _ptr(s["x"]), _ptr(s["p"]), _ptr(sp[1]), _ptr(sp[2]),
                           *[_ptr(s[k]) for k in ("ex", "ey", "ez", "ay", "az")], _ptr(six))
        self.last_zeeman = six[4]
        return six[[0, 1, 2, 3, 5]]

    def gauss_residual(self, x, ex, vec=False):
        x = _f64(x); ex = _f64(ex)
        r = np.zeros(self.cfg.M)
        m = lib().orc_gauss_residual(self._c, _ptr(x), _ptr(ex), _ptr(r))
        return (m, r) if vec else m

    def solve_gauss(self, x):
        x = _f64(x)
        ex = np.zeros(self.cfg.M)
        lib().orc_solve_gauss(self._c, _ptr(x), _ptr(ex))
        return ex

    def substep_I(self, s, h=None, dstart=None, dcommit=None):
        """In place on state dict s (x, p, ex, ay, az), over time step h (the configured dt
        if None), from the increments dstart if given (else the explicit start); dcommit
        (array of n) receives the committed increments.  Returns (status, sweeps, residual)."""
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        ds = None if dstart is None else _f64(dstart)
        sp = self._spins(s)
        sy, sz = (sp[1], sp[2]) if sp is not None and self.cfg.hbar != 0.0 else (None, None)
        st = lib().orc_substep_I_hs(self._c, h, _ptr(s["x"]), _ptr(s["p"]), _ptr(s["ex"]), _ptr(s["ay"]),
                                    _ptr(s["az"]), _ptr(sy), _ptr(sz), _ptr(ds), _ptr(dcommit),
                                    C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_I_adjoint(self, s, h=None, dcommit=None):
        """The adjoint Subsystem I scheme over h, in place.  Returns (status, sweeps, residual)."""
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        sp = self._spins(s)
        sy, sz = (sp[1], sp[2]) if sp is not None and self.cfg.hbar != 0.0 else (None, None)
        st = lib().orc_substep_I_adjoint_s(self._c, h, _ptr(s["x"]), _ptr(s["p"]), _ptr(s["ex"]),
                                           _ptr(s["ay"]), _ptr(s["az"]), _ptr(sy), _ptr(sz), _ptr(dcommit),
                                           C.byref(k), C.byref(r))
        return st, k.value, r.value

    def particle_map_adjoint(self, x0, p0, P, ay, az, gy, gz, ebar):
        """One evaluation of the adjoint map: (delta of P, new momentum, its delta)."""
        arrs = [_f64(a) for a in (ay, az, gy, gz, ebar)]
        d = C.c_double(0); Pn = C.c_double(0); dn = C.c_double(0)
        lib().orc_particle_map_adjoint(self._c, float(x0), float(p0), float(P), *[_ptr(a) for a in arrs],
                                       C.byref(d), C.byref(Pn), C.byref(dn))
        return d.value, Pn.value, dn.value

    def substep_II(self, s, h=None):
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        sp = self._spins(s)
        sy, sz = (sp[1], sp[2]) if sp is not None and self.cfg.hbar != 0.0 else (None, None)
        st = lib().orc_substep_II_hs(self._c, h, _ptr(s["x"]), _ptr(s["p"]), _ptr(sy), _ptr(sz),
                                     _ptr(s["ey"]), _ptr(s["ez"]), _ptr(s["ay"]), _ptr(s["az"]),
                                     C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_III(self, s, h=None):
        """Subsystem III (the spins rotate about (0, dA_z/dx, -dA_y/dx)) over h, in place."""
        h = self.cfg.dt if h is None else float(h)
        lib().orc_substep_III_h(self._c, h, _ptr(s["x"]), _ptr(s["ay"]), _ptr(s["az"]), _ptr(s["sx"]),
                                _ptr(s["sy"]), _ptr(s["sz"]))

    def step(self, s, nsteps=1, energies=False):
        """Steps in place (Lie-Trotter, or the symmetric composition with splitting=1).
        Returns (status, sweeps_I, iters_II, energy[nsteps+1,5]); with splitting=1 the
        sweeps of the adjoint substeps are kept in self.last_sweeps_I2."""
        I32 = C.POINTER(C.c_int32)
        kI = np.zeros(nsteps, dtype=np.int32); kII = np.zeros(nsteps, dtype=np.int32)
        kI2 = np.zeros(nsteps, dtype=np.int32)
        if self._spins(s) is not None:   # I, II, III (or the symmetric composition with III)
            E6 = np.zeros((nsteps + 1, 6)) if energies else None
            st = lib().orc_step_s(self._c, int(nsteps),
                                  *[_ptr(s[k]) for k in ("x", "p", "sx", "sy", "sz", "ex", "ey", "ez", "ay", "az")],
                                  kI.ctypes.data_as(I32), kII.ctypes.data_as(I32), kI2.ctypes.data_as(I32),
                                  _ptr(E6))
            self.last_sweeps_I2 = kI2
            E = None
            if energies:
                E = E6[:, [0, 1, 2, 3, 5]].copy()
                self.last_zeeman = E6[:, 4].copy()
            return st, kI, kII, E
        E = np.zeros((nsteps + 1, 5)) if energies else None
        st = lib().orc_step(self._c, int(nsteps), *[_ptr(s[k]) for k in ("x", "p", "ex", "ey", "ez", "ay", "az")],
                            kI.ctypes.data_as(I32), kII.ctypes.data_as(I32), kI2.ctypes.data_as(I32), _ptr(E))
        self.last_sweeps_I2 = kI2
        return st, kI, kII, E


def initial_state(orc: Oracle, arrays: dict) -> dict:
    """Copy the generator's arrays into an oracle state and solve for e_x."""
    keys = ("x", "p", "ey", "ez", "ay", "az") + (("sx", "sy", "sz") if "sx" in arrays else ())
    s = {k: _f64(arrays[k]).copy() for k in keys}
    s["ex"] = orc.solve_gauss(s["x"])
    return s
