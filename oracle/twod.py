"""ctypes wrapper of the plain FP64 CPU oracle of the reduced 2D model (``oracle2d.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of ``bench.py``.  The HIP library never imports, links or calls
anything here, and this module never imports the HIP library.

State dict keys: x1, x2, p1, p2 (length n); e (V1: e1 then e2, 2 M1 M2), bz (V2),
ez, az (V0), every grid row-major with index i1 M2 + i2.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import lib as _lib1

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


class Cfg2(C.Structure):
    _fields_ = [("L1", C.c_double), ("L2", C.c_double), ("M1", C.c_int32), ("M2", C.c_int32),
                ("p", C.c_int32), ("kmax", C.c_int32), ("n", C.c_int64), ("w", C.c_double),
                ("dt", C.c_double), ("tol", C.c_double)]


_bound = False


def lib() -> C.CDLL:
    global _bound
    L = _lib1()
    if not _bound:
        P = C.POINTER(Cfg2)
        for f, res, args in [
            ("orc2_eval", C.c_double, [P, _D, C.c_int, C.c_int, C.c_double, C.c_double]),
            ("orc2_line_mean", C.c_double, [P, _D, C.c_int, C.c_int] + [C.c_double] * 4),
            ("orc2_line_deposit", None, [P, _D, C.c_int, C.c_int] + [C.c_double] * 5),
            ("orc2_apply_M0", None, [P, _D, _D]), ("orc2_apply_M1", None, [P, _D, _D]),
            ("orc2_apply_M2", None, [P, _D, _D]), ("orc2_apply_G", None, [P, _D, _D]),
            ("orc2_apply_GT", None, [P, _D, _D]), ("orc2_apply_C", None, [P, _D, _D]),
            ("orc2_apply_CT", None, [P, _D, _D]), ("orc2_apply_K", None, [P, _D, _D]),
            ("orc2_solve_M1", None, [P, _D, _D]),
            ("orc2_deposit_charge", None, [P, _D, _D, _D]),
            ("orc2_gauss_residual", C.c_double, [P, _D, _D, _D, _D]),
            ("orc2_solve_gauss", None, [P, _D, _D, _D]),
            ("orc2_energy", None, [P] + [_D] * 9),
            ("orc2_particle_map", None, [P] + [C.c_double] * 6 + [_D] * 5),
            ("orc2_substep_I", C.c_int, [P, C.c_double] + [_D] * 6 + [_I32, _D]),
            ("orc2_substep_II", None, [P, C.c_double] + [_D] * 6),
            ("orc2_substep_III", C.c_int, [P, C.c_double] + [_D] * 6 + [_I32, _D]),
            ("orc2_substep_IV", None, [P, C.c_double, _D, _D]),
            ("orc2_step", C.c_int, [P, C.c_int32] + [_D] * 8 + [_I32, _I32]),
            ("orc2_bfield", None, [P, _D, _D, C.c_double, C.c_double, _D]),
            ("orc2_energy_s", None, [P, C.c_double] + [_D] * 12),
            ("orc2_particle_map_s", None, [P, C.c_double, _D, _D, _D, C.c_int64] + [C.c_double] * 6 + [_D] * 5),
            ("orc2_substep_I_s", C.c_int, [P, C.c_double, C.c_double] + [_D] * 10 + [_I32, _D]),
            ("orc2_substep_II_s", None, [P, C.c_double] + [_D] * 9),
            ("orc2_spin_sources", None, [P] + [_D] * 7),
            ("orc2_substep_III_s", C.c_int, [P, C.c_double, C.c_double] + [_D] * 8 + [_I32, _D]),
            ("orc2_substep_IV_s", None, [P, C.c_double, C.c_double] + [_D] * 5),
            ("orc2_step_s", C.c_int, [P, C.c_double, C.c_int32] + [_D] * 11 + [_I32, _I32]),
        ]:
            fn = getattr(L, f)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


STATE_KEYS = ("x1", "x2", "p1", "p2", "e", "bz", "ez", "az")
SPIN_KEYS = ("sx", "sy", "sz")


class Oracle2D:
    """The 2D oracle bound to one configuration."""

    def __init__(self, L1, L2, M1, M2, p, n, w=None, dt=0.05, tol=1e-13, kmax=50, hbar=0.0):
        if w is None:
            w = L1 * L2 / n if n > 0 else 0.0
        self.cfg = Cfg2(float(L1), float(L2), int(M1), int(M2), int(p), int(kmax), int(n), float(w),
                        float(dt), float(tol))
        self._c = C.byref(self.cfg)
        self.N = int(M1) * int(M2)
        self.hbar = float(hbar)   # the _s methods (spin terms)

    @classmethod
    def from_workload(cls, w, n=None, **kw):
        n = w.n_particles if n is None else n
        args = dict(L1=w.L1, L2=w.L2, M1=w.M1, M2=w.M2, p=w.degree, n=n, w=w.L1 * w.L2 / n, dt=w.dt,
                    tol=w.tol, kmax=w.kmax, hbar=getattr(w, "hbar", 0.0))
        args.update(kw)
        return cls(**args)

    # -- fields, means, operators ------------------------------------------
    def eval(self, coef, d1, d2, x1, x2):
        coef = _f64(coef)
        return lib().orc2_eval(self._c, _ptr(coef), int(d1), int(d2), float(x1), float(x2))

    def line_mean(self, coef, d1, d2, a, b):
        coef = _f64(coef)
        return lib().orc2_line_mean(self._c, _ptr(coef), int(d1), int(d2), float(a[0]), float(a[1]),
                                    float(b[0]), float(b[1]))

    def line_deposit(self, d1, d2, a, b, q=1.0, grid=None):
        grid = np.zeros(self.N) if grid is None else grid
        lib().orc2_line_deposit(self._c, _ptr(grid), int(d1), int(d2), float(a[0]), float(a[1]), float(b[0]),
                                float(b[1]), float(q))
        return grid

    def _op(self, name, v, nout):
        v = _f64(v)
        out = np.zeros(nout)
        getattr(lib(), name)(self._c, _ptr(v), _ptr(out))
        return out

    def M0(self, v): return self._op("orc2_apply_M0", v, self.N)
    def M1(self, v): return self._op("orc2_apply_M1", v, 2 * self.N)
    def M2(self, v): return self._op("orc2_apply_M2", v, self.N)
    def G(self, v): return self._op("orc2_apply_G", v, 2 * self.N)
    def GT(self, v): return self._op("orc2_apply_GT", v, self.N)
    def C(self, v): return self._op("orc2_apply_C", v, self.N)
    def CT(self, v): return self._op("orc2_apply_CT", v, 2 * self.N)
    def K(self, v): return self._op("orc2_apply_K", v, self.N)
    def solve_M1(self, v): return self._op("orc2_solve_M1", v, 2 * self.N)

    def particle_map(self, x, p, d, ebar, az, ga):
        """One evaluation of the Subsystem I map for one particle: (p^{k+1}, d^{k+1})."""
        arrs = [_f64(a) for a in (ebar, az, ga)]
        pn = np.zeros(2); dn = np.zeros(2)
        lib().orc2_particle_map(self._c, float(x[0]), float(x[1]), float(p[0]), float(p[1]), float(d[0]),
                                float(d[1]), *[_ptr(a) for a in arrs], _ptr(pn), _ptr(dn))
        return pn, dn

    # -- state-level --------------------------------------------------------
    def deposit_charge(self, s):
        rho = np.zeros(self.N)
        lib().orc2_deposit_charge(self._c, _ptr(s["x1"]), _ptr(s["x2"]), _ptr(rho))
        return rho

    def gauss_residual(self, s, vec=False):
        r = np.zeros(self.N)
        m = lib().orc2_gauss_residual(self._c, _ptr(s["x1"]), _ptr(s["x2"]), _ptr(s["e"]), _ptr(r))
        return (m, r) if vec else m

    def solve_gauss(self, s):
        lib().orc2_solve_gauss(self._c, _ptr(s["x1"]), _ptr(s["x2"]), _ptr(s["e"]))

    def energy(self, s):
        """[kinetic, 1/2 e^T M1 e, 1/2 b^T M2 b, 1/2 e_z^T M0 e_z, 1/2 a^T K a, H]."""
        out = np.zeros(6)
        lib().orc2_energy(self._c, *[_ptr(s[k]) for k in STATE_KEYS], _ptr(out))
        return out

    def substep_I(self, s, h=None):
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        st = lib().orc2_substep_I(self._c, h, *[_ptr(s[k_]) for k_ in ("x1", "x2", "p1", "p2", "e", "az")],
                                  C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_II(self, s, h=None):
        h = self.cfg.dt if h is None else float(h)
        lib().orc2_substep_II(self._c, h, *[_ptr(s[k]) for k in ("x1", "x2", "p1", "p2", "bz", "az")])

    def substep_III(self, s, h=None):
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        st = lib().orc2_substep_III(self._c, h, *[_ptr(s[k_]) for k_ in ("x1", "x2", "p1", "p2", "ez", "az")],
                                    C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_IV(self, s, h=None):
        h = self.cfg.dt if h is None else float(h)
        lib().orc2_substep_IV(self._c, h, _ptr(s["e"]), _ptr(s["bz"]))

    def step(self, s, nsteps=1):
        """Lie-Trotter steps I, II, III, IV in place: (status, sweeps_I, iters_III)."""
        kI = np.zeros(nsteps, dtype=np.int32); kIII = np.zeros(nsteps, dtype=np.int32)
        st = lib().orc2_step(self._c, int(nsteps), *[_ptr(s[k]) for k in STATE_KEYS],
                             kI.ctypes.data_as(_I32), kIII.ctypes.data_as(_I32))
        return st, kI, kIII


    # -- with spin (Zeeman term hbar sum_a w s_a . B_h(x_a)) -----------------
    def bfield(self, az, bz, x1, x2):
        """B_h = (dA_z/dx2, -dA_z/dx1, B_z) at a point."""
        ga = self.G(az)
        B = np.zeros(3)
        lib().orc2_bfield(self._c, _ptr(ga), _ptr(_f64(bz)), float(x1), float(x2), _ptr(B))
        return B

    def energy_s(self, s):
        """[kinetic, 1/2 e^T M1 e, 1/2 b^T M2 b, 1/2 e_z^T M0 e_z, 1/2 a^T K a, Zeeman, H]."""
        out = np.zeros(7)
        lib().orc2_energy_s(self._c, self.hbar, *[_ptr(s[k]) for k in ("x1", "x2", "p1", "p2", "sx", "sy", "sz",
                                                                         "e", "bz", "ez", "az")], _ptr(out))
        return out

    def particle_map_s(self, s, a, x, p, d, ebar):
        """One evaluation of the Subsystem I map with spin for particle a of state s
        (its spins, a_z and b_z): (p^{k+1}, d^{k+1})."""
        pn = np.zeros(2); dn = np.zeros(2)
        lib().orc2_particle_map_s(self._c, self.hbar, _ptr(s["sx"]), _ptr(s["sy"]), _ptr(s["sz"]), int(a),
                                  float(x[0]), float(x[1]), float(p[0]), float(p[1]), float(d[0]), float(d[1]),
                                  _ptr(_f64(ebar)), _ptr(s["az"]), _ptr(s["bz"]), _ptr(pn), _ptr(dn))
        return pn, dn

    def spin_sources(self, s):
        """(G*^T Lambda1*(X)^T W S_xy, Lambda2(X)^T W S_z) at the state's particles."""
        sxy = np.zeros(self.N); dz = np.zeros(self.N)
        lib().orc2_spin_sources(self._c, *[_ptr(s[k]) for k in ("x1", "x2", "sx", "sy", "sz")], _ptr(sxy),
                                _ptr(dz))
        return sxy, dz

    def substep_I_s(self, s, h=None):
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        st = lib().orc2_substep_I_s(self._c, h, self.hbar, *[_ptr(s[k_]) for k_ in (
            "x1", "x2", "p1", "p2", "sx", "sy", "sz", "e", "az", "bz")], C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_II_s(self, s, h=None):
        h = self.cfg.dt if h is None else float(h)
        lib().orc2_substep_II_s(self._c, h, *[_ptr(s[k]) for k in ("x1", "x2", "p1", "p2", "sx", "sy", "sz",
                                                                     "bz", "az")])

    def substep_III_s(self, s, h=None):
        k = C.c_int32(0); r = C.c_double(0)
        h = self.cfg.dt if h is None else float(h)
        st = lib().orc2_substep_III_s(self._c, h, self.hbar, *[_ptr(s[k_]) for k_ in (
            "x1", "x2", "p1", "p2", "sx", "sy", "ez", "az")], C.byref(k), C.byref(r))
        return st, k.value, r.value

    def substep_IV_s(self, s, h=None):
        h = self.cfg.dt if h is None else float(h)
        lib().orc2_substep_IV_s(self._c, h, self.hbar, _ptr(s["x1"]), _ptr(s["x2"]), _ptr(s["sz"]), _ptr(s["e"]),
                                _ptr(s["bz"]))

    def step_s(self, s, nsteps=1):
        """Lie-Trotter steps with spin in place: (status, sweeps_I, iters_III)."""
        kI = np.zeros(nsteps, dtype=np.int32); kIII = np.zeros(nsteps, dtype=np.int32)
        st = lib().orc2_step_s(self._c, self.hbar, int(nsteps), *[_ptr(s[k]) for k in (
            "x1", "x2", "p1", "p2", "sx", "sy", "sz", "e", "bz", "ez", "az")],
            kI.ctypes.data_as(_I32), kIII.ctypes.data_as(_I32))
        return st, kI, kIII


def initial_state2d(orc: Oracle2D, arrays: dict) -> dict:
    """Copy the generator's arrays (and spins, if any) into an oracle state and correct
    e_xy so that the discrete Gauss law holds."""
    s = {k: _f64(arrays[k]).copy() for k in STATE_KEYS + SPIN_KEYS if k in arrays}
    orc.solve_gauss(s)
    return s
