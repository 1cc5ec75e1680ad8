"""ctypes binding of libecpic.so (include/ecpic.h): argument marshalling only.

Every computation happens in the HIP library on the GPU.  If the library is not
built, or no gfx950 device is usable, the calls raise; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ECPIC_LIB") or os.path.join(_HERE, "libecpic.so")

OK, EINVAL, ENOMEM, ENOTCONV, EDEVICE, ENONFINITE, ECFL, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32_MIXED = 0, 1
WS_EXPLICIT, WS_PREVIOUS, WS_MLP = 0, 1, 2
MAP_JACOBI, MAP_SEIDEL = 0, 1
LIE_TROTTER, SYMMETRIC = 0, 1

# Every symbol include/ecpic.h declares.
EXPORTS = (
    "ecpic_create", "ecpic_destroy", "ecpic_set_particles", "ecpic_get_particles",
    "ecpic_set_particles_dev", "ecpic_get_particles_dev", "ecpic_set_fields", "ecpic_get_fields",
    "ecpic_solve_gauss", "ecpic_substep_particles", "ecpic_substep_particles_adjoint", "ecpic_substep_fields",
    "ecpic_step", "ecpic_set_spins", "ecpic_get_spins", "ecpic_substep_spin",
    "ecpic_deposit_current", "ecpic_deposit_current_noalloc", "ecpic_deposit_charge", "ecpic_energy",
    "ecpic_gauss_residual",
    "ecpic_profile_enable", "ecpic_kernel_time", "ecpic_bandwidth_probe", "ecpic_strerror",
    "ecpic_ws_record", "ecpic_ws_records", "ecpic_ws_get_records", "ecpic_ws_train", "ecpic_ws_n_params",
    "ecpic_ws_get_weights", "ecpic_ws_set_weights", "ecpic_ws_enable", "ecpic_ws_grad", "ecpic_ws_table",
)


class EcpicError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_strerror(status)} ({status})")


class Config(C.Structure):
    _fields_ = [("L", C.c_double), ("M", C.c_int32), ("degree", C.c_int32), ("n_particles", C.c_int64),
                ("weight", C.c_double), ("dt", C.c_double), ("picard_tol", C.c_double),
                ("picard_max_iter", C.c_int32), ("precision", C.c_int32), ("warmstart", C.c_int32),
                ("map", C.c_int32), ("device", C.c_int32), ("stream", C.c_void_p), ("fp32_sweeps", C.c_int32),
                ("sweep_guess", C.c_int32), ("waves_per_item", C.c_int32), ("splitting", C.c_int32),
                ("item_particles", C.c_int32), ("spin", C.c_int32), ("hbar", C.c_double)]


class IterStats(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("fp32_sweeps", C.c_int32), ("residual", C.c_double),
                ("crossing_queue", C.c_int32), ("sweeps_adjoint", C.c_int32), ("residual_hist", C.c_double * 4)]


class WsTrainConfig(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("seed", C.c_uint64)]


class EnergyParts(C.Structure):
    _fields_ = [("kinetic", C.c_double), ("e_long", C.c_double), ("e_trans", C.c_double),
                ("b_trans", C.c_double), ("total", C.c_double), ("zeeman", C.c_double)]


_lib: Optional[C.CDLL] = None
_D = C.POINTER(C.c_double)


def _one_hip_runtime():
    """PyTorch for ROCm ships its own HIP runtime library under a name that does not match
    the one the library links; loaded after the library, it would be a second runtime in
    the process, whose streams and allocations the library's runtime does not know.  When
    torch is installed it is therefore imported first, so the library binds to the
    runtime torch already holds and a torch stream or tensor can be handed over."""
    try:
        import torch  # noqa: F401
    except ImportError:
        pass


def load() -> C.CDLL:
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2203_06513_amd/build.py "
                               "(or __graft_entry__.build())")
        _one_hip_runtime()
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        L.ecpic_create.argtypes = [C.POINTER(Config), C.POINTER(V)]
        L.ecpic_destroy.argtypes = [V]
        for f in ("ecpic_set_particles", "ecpic_get_particles", "ecpic_set_particles_dev",
                  "ecpic_get_particles_dev"):
            getattr(L, f).argtypes = [V, V, V, C.c_int64]
        L.ecpic_set_fields.argtypes = [V, V, V, V, V, V]
        L.ecpic_get_fields.argtypes = [V, V, V, V, V, V]
        L.ecpic_solve_gauss.argtypes = [V]
        L.ecpic_substep_particles.argtypes = [V, C.c_double, C.POINTER(IterStats)]
        L.ecpic_substep_particles_adjoint.argtypes = [V, C.c_double, C.POINTER(IterStats)]
        L.ecpic_substep_fields.argtypes = [V, C.c_double, C.POINTER(IterStats)]
        L.ecpic_step.argtypes = [V, C.c_int32, C.POINTER(IterStats), C.POINTER(IterStats), C.POINTER(C.c_int32)]
        L.ecpic_set_spins.argtypes = [V, V, V, V, C.c_int64]
        L.ecpic_get_spins.argtypes = [V, V, V, V, C.c_int64]
        L.ecpic_substep_spin.argtypes = [V, C.c_double]
        L.ecpic_deposit_current.argtypes = [V, V, V, C.c_int64, V]
        L.ecpic_deposit_current_noalloc.argtypes = [V, V, V, C.c_int64, V, V]
        L.ecpic_deposit_charge.argtypes = [V, V]
        L.ecpic_energy.argtypes = [V, C.POINTER(EnergyParts)]
        L.ecpic_gauss_residual.argtypes = [V, C.POINTER(C.c_double), V]
        L.ecpic_profile_enable.argtypes = [V, C.c_int32]
        L.ecpic_kernel_time.argtypes = [V, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.ecpic_bandwidth_probe.argtypes = [V, C.c_int64, C.c_int32, C.POINTER(C.c_double)]
        I64P = C.POINTER(C.c_int64)
        FP = C.POINTER(C.c_float)
        L.ecpic_ws_record.argtypes = [V, C.c_int32, C.c_int64]
        L.ecpic_ws_records.argtypes = [V, I64P]
        L.ecpic_ws_get_records.argtypes = [V, V, V, C.c_int64]
        L.ecpic_ws_train.argtypes = [V, C.POINTER(WsTrainConfig), FP]
        L.ecpic_ws_n_params.argtypes = [V, I64P]
        L.ecpic_ws_get_weights.argtypes = [V, V, C.c_int64]
        L.ecpic_ws_set_weights.argtypes = [V, V, C.c_int64]
        L.ecpic_ws_enable.argtypes = [V, C.c_int32]
        L.ecpic_ws_grad.argtypes = [V, V, V, C.c_int64, V, FP]
        L.ecpic_ws_table.argtypes = [V, V]
        L.ecpic_strerror.argtypes = [C.c_int]
        L.ecpic_strerror.restype = C.c_char_p
        for f in EXPORTS:
            if f != "ecpic_strerror":
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _strerror(status: int) -> str:
    try:
        return load().ecpic_strerror(int(status)).decode()
    except Exception:  # the library itself may be what is missing
        return "error"


def _arr(a: Optional[np.ndarray], n: int):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def _ck(rc: int, what: str):
    if rc != OK:
        raise EcpicError(rc, what)


class Context:
    """One simulation state on one GPU (see include/ecpic.h)."""

    def __init__(self, L: float, M: int, degree: int, n_particles: int, dt: float, tol: float,
                 weight: float = 0.0, max_iter: int = 0, precision: int = FP64,
                 warmstart: int = WS_EXPLICIT, map: int = MAP_JACOBI, device: int = 0,
                 stream: Optional[int] = None, fp32_sweeps: int = 0, sweep_guess: int = 0,
                 waves_per_item: int = 0, splitting: int = LIE_TROTTER, item_particles: int = 0,
                 spin: bool = False, hbar: float = 0.0):
        self._lib = load()
        self.cfg = Config(float(L), int(M), int(degree), int(n_particles), float(weight), float(dt),
                          float(tol), int(max_iter), int(precision), int(warmstart), int(map), int(device),
                          C.c_void_p(stream) if stream else None, int(fp32_sweeps), int(sweep_guess),
                          int(waves_per_item), int(splitting), int(item_particles), int(bool(spin)),
                          float(hbar))
        self.spin = bool(spin)
        self.dt = float(dt)
        self.M = int(M)
        self.N = int(n_particles)
        h = C.c_void_p()
        _ck(self._lib.ecpic_create(C.byref(self.cfg), C.byref(h)), "ecpic_create")
        self._h = h

    @classmethod
    def from_workload(cls, w, n: Optional[int] = None, **kw):
        n = w.n_particles if n is None else n
        args = dict(L=w.L, M=w.M, degree=w.degree, n_particles=n, dt=w.dt, tol=w.tol, max_iter=w.kmax)
        if getattr(w, "spin", "none") != "none":
            args.update(spin=True, hbar=w.hbar)
        args.update(kw)
        return cls(**args)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ecpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- state ----------------------------------------------------------------
    def set_particles(self, x, p):
        x = _arr(x, self.N); p = _arr(p, self.N)
        _ck(self._lib.ecpic_set_particles(self._h, x.ctypes.data, p.ctypes.data, self.N), "set_particles")

    def get_particles(self):
        x = np.empty(self.N); p = np.empty(self.N)
        _ck(self._lib.ecpic_get_particles(self._h, x.ctypes.data, p.ctypes.data, self.N), "get_particles")
        return x, p

    def set_particles_dev(self, x_ptr: int, p_ptr: int):
        _ck(self._lib.ecpic_set_particles_dev(self._h, x_ptr, p_ptr, self.N), "set_particles_dev")

    def get_particles_dev(self, x_ptr: int, p_ptr: int):
        _ck(self._lib.ecpic_get_particles_dev(self._h, x_ptr, p_ptr, self.N), "get_particles_dev")

    def set_fields(self, ex=None, ey=None, ez=None, ay=None, az=None):
        arrs = [_arr(a, self.M) for a in (ex, ey, ez, ay, az)]
        ptrs = [a.ctypes.data if a is not None else None for a in arrs]
        _ck(self._lib.ecpic_set_fields(self._h, *ptrs), "set_fields")

    def get_fields(self) -> dict:
        out = {k: np.empty(self.M) for k in ("ex", "ey", "ez", "ay", "az")}
        _ck(self._lib.ecpic_get_fields(self._h, *[out[k].ctypes.data for k in ("ex", "ey", "ez", "ay", "az")]),
            "get_fields")
        return out

    def set_spins(self, sx, sy, sz):
        a = [_arr(v, self.N) for v in (sx, sy, sz)]
        _ck(self._lib.ecpic_set_spins(self._h, *[v.ctypes.data for v in a], self.N), "set_spins")

    def get_spins(self):
        out = [np.empty(self.N) for _ in range(3)]
        _ck(self._lib.ecpic_get_spins(self._h, *[v.ctypes.data for v in out], self.N), "get_spins")
        return tuple(out)

    def substep_spin(self, dt: Optional[float] = None):
        """Subsystem III (the spins' exact rotation) over dt (the configured step if None)."""
        _ck(self._lib.ecpic_substep_spin(self._h, self.dt if dt is None else float(dt)), "substep_spin")

    def load(self, arrays: dict, solve_gauss: bool = True):
        """Particles, spins (if the dict has them) and transverse fields from a workload
        dict; e_x from the Poisson solve."""
        self.set_particles(arrays["x"], arrays["p"])
        if self.spin and "sx" in arrays:
            self.set_spins(arrays["sx"], arrays["sy"], arrays["sz"])
        self.set_fields(arrays.get("ex"), arrays["ey"], arrays["ez"], arrays["ay"], arrays["az"])
        if solve_gauss:
            self.solve_gauss()

    def state(self) -> dict:
        x, p = self.get_particles()
        s = self.get_fields()
        s["x"] = x
        s["p"] = p
        if self.spin:
            s["sx"], s["sy"], s["sz"] = self.get_spins()
        return s

    # -- the method -------------------------------------------------------------
    def solve_gauss(self):
        _ck(self._lib.ecpic_solve_gauss(self._h), "solve_gauss")

    def substep_particles(self, dt: Optional[float] = None, check: bool = True):
        """Subsystem I over dt (the configured step if None).  Returns (sweeps, residual);
        last_stats_I keeps (sweeps, fp32_sweeps, residual, crossing_queue, status)."""
        st = IterStats()
        rc = self._lib.ecpic_substep_particles(self._h, self.dt if dt is None else float(dt), C.byref(st))
        self.last_stats_I = (st.sweeps, st.fp32_sweeps, st.residual, st.crossing_queue, rc)
        self.last_res_hist_I = np.array(st.residual_hist[:])
        if check:
            _ck(rc, "substep_particles")
        return st.sweeps, st.residual

    def substep_particles_adjoint(self, dt: Optional[float] = None, check: bool = True):
        """The adjoint Subsystem I scheme over dt.  Returns (sweeps, residual)."""
        st = IterStats()
        rc = self._lib.ecpic_substep_particles_adjoint(self._h, self.dt if dt is None else float(dt),
                                                       C.byref(st))
        self.last_stats_I = (st.sweeps, st.fp32_sweeps, st.residual, st.crossing_queue, rc)
        if check:
            _ck(rc, "substep_particles_adjoint")
        return st.sweeps, st.residual

    def substep_fields(self, dt: Optional[float] = None):
        st = IterStats()
        rc = self._lib.ecpic_substep_fields(self._h, self.dt if dt is None else float(dt), C.byref(st))
        _ck(rc, "substep_fields")
        return st.sweeps, st.residual

    def step(self, nsteps: int = 1, check: bool = True):
        """Returns (status, steps_done, sweeps_I[n], sweeps_II[n], fp32_sweeps_I[n])."""
        sI = (IterStats * max(nsteps, 1))()
        sII = (IterStats * max(nsteps, 1))()
        done = C.c_int32(0)
        rc = self._lib.ecpic_step(self._h, int(nsteps), sI, sII, C.byref(done))
        if check:
            _ck(rc, "step")
        kI = np.array([sI[i].sweeps for i in range(nsteps)], dtype=np.int32)
        kII = np.array([sII[i].sweeps for i in range(nsteps)], dtype=np.int32)
        k32 = np.array([sI[i].fp32_sweeps for i in range(nsteps)], dtype=np.int32)
        self.last_queue_I = np.array([sI[i].crossing_queue for i in range(nsteps)], dtype=np.int32)
        self.last_sweeps_I2 = np.array([sI[i].sweeps_adjoint for i in range(nsteps)], dtype=np.int32)
        self.last_res_hist_I = np.array([sI[i].residual_hist[:] for i in range(nsteps)]).reshape(nsteps, 4)
        return rc, done.value, kI, kII, k32

    # -- diagnostics ------------------------------------------------------------
    def energy(self) -> np.ndarray:
        e = EnergyParts()
        _ck(self._lib.ecpic_energy(self._h, C.byref(e)), "energy")
        self.last_zeeman = e.zeeman
        return np.array([e.kinetic, e.e_long, e.e_trans, e.b_trans, e.total])

    def gauss_residual(self, vec: bool = False):
        m = C.c_double(0.0)
        r = np.empty(self.M)
        _ck(self._lib.ecpic_gauss_residual(self._h, C.byref(m), r.ctypes.data), "gauss_residual")
        return (m.value, r) if vec else m.value

    def deposit_charge(self) -> np.ndarray:
        rho = np.empty(self.M)
        _ck(self._lib.ecpic_deposit_charge(self._h, rho.ctypes.data), "deposit_charge")
        return rho

    def deposit_current(self, x0, x1) -> np.ndarray:
        x0 = np.ascontiguousarray(x0, dtype=np.float64); x1 = np.ascontiguousarray(x1, dtype=np.float64)
        J = np.empty(self.M)
        _ck(self._lib.ecpic_deposit_current(self._h, x0.ctypes.data, x1.ctypes.data, len(x0), J.ctypes.data),
            "deposit_current")
        return J

    def deposit_current_noalloc(self, x0_ptr: int, x1_ptr: int, n: int, J_ptr: int, flags_ptr: int = 0) -> int:
        """Device pointers in and out; enqueued on the context's stream, nothing allocated,
        not waited for.  Returns the status (not raised: the caller may be capturing)."""
        return self._lib.ecpic_deposit_current_noalloc(self._h, x0_ptr, x1_ptr, int(n), J_ptr, flags_ptr or None)

    # -- learned warm start -----------------------------------------------------
    def ws_record(self, stride: int, capacity: int = 0):
        _ck(self._lib.ecpic_ws_record(self._h, int(stride), int(capacity)), "ws_record")

    def ws_records(self) -> int:
        n = C.c_int64(0)
        _ck(self._lib.ecpic_ws_records(self._h, C.byref(n)), "ws_records")
        return n.value

    def ws_n_features(self) -> int:
        return 3 + 6 * (self.cfg.degree + 1)

    def ws_get_records(self, n: Optional[int] = None):
        n = self.ws_records() if n is None else int(n)
        f = np.empty((n, self.ws_n_features()), np.float32)
        t = np.empty((n, 2), np.float32)
        _ck(self._lib.ecpic_ws_get_records(self._h, f.ctypes.data, t.ctypes.data, n), "ws_get_records")
        return f, t

    def ws_train(self, steps: int = 0, batch: int = 0, lr: float = 0.0, seed: int = 0) -> float:
        cfg = WsTrainConfig(int(steps), int(batch), float(lr), int(seed))
        loss = C.c_float(0.0)
        _ck(self._lib.ecpic_ws_train(self._h, C.byref(cfg), C.byref(loss)), "ws_train")
        return loss.value

    def ws_n_params(self) -> int:
        n = C.c_int64(0)
        _ck(self._lib.ecpic_ws_n_params(self._h, C.byref(n)), "ws_n_params")
        return n.value

    def ws_get_weights(self) -> np.ndarray:
        w = np.empty(self.ws_n_params(), np.float32)
        _ck(self._lib.ecpic_ws_get_weights(self._h, w.ctypes.data, len(w)), "ws_get_weights")
        return w

    def ws_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _ck(self._lib.ecpic_ws_set_weights(self._h, w.ctypes.data, len(w)), "ws_set_weights")

    def ws_enable(self, on: bool = True):
        _ck(self._lib.ecpic_ws_enable(self._h, int(bool(on))), "ws_enable")

    def ws_grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32); y = np.ascontiguousarray(y, dtype=np.float32)
        n = x.shape[0]
        D = self.ws_n_features()
        g = np.empty(self.ws_n_params() - 2 * (D + 2) - 2, np.float32)
        loss = C.c_float(0.0)
        _ck(self._lib.ecpic_ws_grad(self._h, x.ctypes.data, y.ctypes.data, n, g.ctypes.data, C.byref(loss)),
            "ws_grad")
        return g, loss.value

    def ws_table(self) -> np.ndarray:
        t = np.empty((self.M, 8, 8), np.float32)
        _ck(self._lib.ecpic_ws_table(self._h, t.ctypes.data), "ws_table")
        return t

    # -- timing -----------------------------------------------------------------
    def profile(self, enable: bool = True):
        _ck(self._lib.ecpic_profile_enable(self._h, int(enable)), "profile_enable")

    def bandwidth_probe(self, nbytes: int, reps: int = 20) -> float:
        """Mean ms of a plain copy kernel that reads and writes nbytes each."""
        ms = C.c_double(0.0)
        _ck(self._lib.ecpic_bandwidth_probe(self._h, int(nbytes), int(reps), C.byref(ms)), "bandwidth_probe")
        return ms.value

    def kernel_time(self, name: str):
        ms = C.c_double(0.0); n = C.c_int64(0)
        _ck(self._lib.ecpic_kernel_time(self._h, name.encode(), C.byref(ms), C.byref(n)), "kernel_time")
        return ms.value, n.value
