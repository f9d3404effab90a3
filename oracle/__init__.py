"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the plain FP64 CPU oracle.

The oracle (``lbm_oracle.c``) is an independent, slow, obviously-correct CPU
implementation of the EOS-based multiphase MRT lattice Boltzmann step of
arXiv 2103.08301, Sec. 2.  Only ``tests/``, the package's ``smoke()`` check and
the CPU-baseline leg of ``bench.py`` may use it.  It imports nothing from the
GPU package and the GPU package imports nothing from it.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

EOS_CS = 0
EOS_PR = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no FMA contraction, OpenMP over rows."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
               _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("eos", C.c_int), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double),
        ("omega", C.c_double), ("T_over_Tc", C.c_double), ("k", C.c_double),
        ("kappa", C.c_double), ("tau", C.c_double), ("s_e", C.c_double),
        ("s_eps", C.c_double), ("s_q", C.c_double), ("s_j", C.c_double),
        ("rho_wall", C.c_double), ("dp", C.c_double), ("x_periodic", C.c_int),
        ("y_periodic", C.c_int), ("check_every", C.c_int), ("v_limit", C.c_double),
        ("forcing", C.c_int),
    ]


class Summary(C.Structure):
    _fields_ = [
        ("step", C.c_int64),
        ("tau_max", C.c_double * 2), ("tau_min", C.c_double * 2),
        ("p_max", C.c_double * 2), ("p_min", C.c_double * 2),
        ("x_tau_max", C.c_int32 * 2), ("x_tau_min", C.c_int32 * 2),
        ("x_p_max", C.c_int32 * 2), ("x_p_min", C.c_int32 * 2),
        ("sum_tau2", C.c_double), ("int_peak_tau2", C.c_double), ("int_tau2", C.c_double),
        ("run_tau_max", C.c_double * 2), ("run_tau_min", C.c_double * 2),
        ("run_p_max", C.c_double * 2), ("run_p_min", C.c_double * 2),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


class Component(C.Structure):
    _fields_ = [
        ("first_cell", C.c_int64), ("cells", C.c_int32), ("wall", C.c_int32),
        ("mass", C.c_double), ("excess_mass", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        P = C.POINTER(Params)
        sig = {
            "orc_params_default": (None, [P]),
            "orc_critical": (C.c_int, [P, _D, _D]),
            "orc_alpha": (C.c_double, [P, C.c_double, C.c_double]),
            "orc_p0": (C.c_double, [P, C.c_double, C.c_double]),
            "orc_dp0": (C.c_double, [P, C.c_double, C.c_double, C.c_int]),
            "orc_coexistence": (C.c_int, [P, C.c_double, _D, _D, _D]),
            "orc_velocities": (None, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _D]),
            "orc_moment_matrix": (None, [_D]),
            "orc_equilibrium": (None, [C.c_double, C.c_double, C.c_double, _D]),
            "orc_collide_node": (None, [P, _D, C.c_double, C.c_double, _D, _D, _D, _D]),
            "orc_grad_field": (None, [_D, C.c_int, C.c_int, _D, _D]),
            "orc_lap_field": (None, [_D, C.c_int, C.c_int, _D]),
            "orc_splitmix64": (C.c_uint64, [C.c_uint64, C.c_uint64]),
            "orc_threads": (C.c_int, []),
            "orc_create": (C.c_int, [C.c_int, C.c_int, P, C.POINTER(C.c_void_p)]),
            "orc_destroy": (None, [C.c_void_p]),
            "orc_state": (C.c_int, [C.c_void_p, _D, _D, _D, _D, _D]),
            "orc_init_plug": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double,
                                        C.c_double, C.c_uint64]),
            "orc_init_density": (C.c_int, [C.c_void_p, _D]),
            "orc_set_f": (None, [C.c_void_p, _D]),
            "orc_get_f": (None, [C.c_void_p, _D]),
            "orc_step": (C.c_int, [C.c_void_p, C.c_int64]),
            "orc_step_count": (C.c_int64, [C.c_void_p]),
            "orc_unstable_step": (C.c_int64, [C.c_void_p]),
            "orc_fields": (None, [C.c_void_p, _D, _D, _D]),
            "orc_force": (None, [C.c_void_p, _D, _D]),
            "orc_wall": (None, [C.c_void_p, _D, _D, _D, _D]),
            "orc_eval_force": (None, [C.c_void_p, _D, _D, _D, _D, _D]),
            "orc_history": (C.c_int64, [C.c_void_p, C.POINTER(Summary), C.c_int64]),
            "orc_totals": (None, [C.c_void_p, _D, _D, _D]),
            "orc_interface": (C.c_int, [C.c_void_p, _D, _D, C.POINTER(C.c_int)]),
            "orc_components_field": (C.c_int64, [_D, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                                 C.c_int, C.POINTER(Component), C.c_int64]),
            "orc_components": (C.c_int64, [C.c_void_p, C.c_double, C.c_int, C.POINTER(Component), C.c_int64]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def components_field(rho: np.ndarray, threshold: float, rho_g: float = 0.0, connectivity: int = 4,
                     x_periodic: int = 0, y_periodic: int = 0) -> list:
    """Liquid components (rho > threshold) of an arbitrary field rho[ny][nx]."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    n = lib().orc_components_field(_ptr(rho), nx, ny, x_periodic, y_periodic, threshold, rho_g, connectivity, None, 0)
    if n < 0:
        raise ValueError(f"orc_components_field failed: {n}")
    buf = (Component * max(n, 1))()
    lib().orc_components_field(_ptr(rho), nx, ny, x_periodic, y_periodic, threshold, rho_g, connectivity, buf, n)
    return [buf[i].as_dict() for i in range(n)]


def params(**kw) -> Params:
    """Oracle parameters: defaults are config C1's CS model, overridden by keywords."""
    p = Params()
    lib().orc_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def critical(p: Params):
    rc, tc = C.c_double(), C.c_double()
    st = lib().orc_critical(C.byref(p), C.byref(rc), C.byref(tc))
    if st:
        raise ValueError(f"orc_critical failed: {st}")
    return rc.value, tc.value


def coexistence(p: Params, T: float):
    g, l, ps = C.c_double(), C.c_double(), C.c_double()
    st = lib().orc_coexistence(C.byref(p), T, C.byref(g), C.byref(l), C.byref(ps))
    if st:
        raise ValueError(f"orc_coexistence failed: {st}")
    return g.value, l.value, ps.value


def p0(p: Params, T: float, rho: float) -> float:
    return lib().orc_p0(C.byref(p), T, rho)


def dp0(p: Params, T: float, rho: float, order: int) -> float:
    return lib().orc_dp0(C.byref(p), T, rho, order)


def alpha(p: Params, T: float, Tc: float) -> float:
    return lib().orc_alpha(C.byref(p), T, Tc)


def velocities():
    ex, ey, w = C.c_int(), C.c_int(), C.c_double()
    out = []
    for i in range(9):
        lib().orc_velocities(i, C.byref(ex), C.byref(ey), C.byref(w))
        out.append((ex.value, ey.value, w.value))
    return out


def moment_matrix() -> np.ndarray:
    m = np.zeros(81)
    lib().orc_moment_matrix(_ptr(m))
    return m.reshape(9, 9)


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    f = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, _ptr(f))
    return f


def collide_node(p: Params, f9, Fx: float, Fy: float):
    f = np.ascontiguousarray(f9, dtype=np.float64)
    out = np.zeros(9)
    r, vx, vy = C.c_double(), C.c_double(), C.c_double()
    lib().orc_collide_node(C.byref(p), _ptr(f), Fx, Fy, _ptr(out), C.byref(r), C.byref(vx), C.byref(vy))
    return out, r.value, vx.value, vy.value


def grad_field(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    h, w = a.shape
    gx = np.zeros((h - 2, w - 2))
    gy = np.zeros((h - 2, w - 2))
    lib().orc_grad_field(_ptr(a), w, h, _ptr(gx), _ptr(gy))
    return gx, gy


def lap_field(a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    h, w = a.shape
    out = np.zeros((h - 2, w - 2))
    lib().orc_lap_field(_ptr(a), w, h, _ptr(out))
    return out


def threads() -> int:
    return lib().orc_threads()


def splitmix64(seed: int, counter: int) -> int:
    return lib().orc_splitmix64(seed, counter)


class Sim:
    """One oracle simulation on an nx x ny grid (FP64, CPU)."""

    def __init__(self, nx: int, ny: int, p: Params):
        self.nx, self.ny, self.p = nx, ny, p
        h = C.c_void_p()
        st = lib().orc_create(nx, ny, C.byref(p), C.byref(h))
        if st:
            raise ValueError(f"orc_create failed: {st}")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    def state(self) -> dict:
        v = [C.c_double() for _ in range(5)]
        lib().orc_state(self._h, *[C.byref(x) for x in v])
        return dict(zip(["T", "Tc", "rho_g", "rho_l", "rho_w"], [x.value for x in v]))

    def init_plug(self, plug_len, film, x_center=math.nan, noise_amp=1e-3, seed=1):
        st = lib().orc_init_plug(self._h, plug_len, film, x_center, noise_amp, seed)
        if st:
            raise ValueError(f"orc_init_plug failed: {st}")

    def init_density(self, rho: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        assert rho.shape == (self.ny, self.nx)
        lib().orc_init_density(self._h, _ptr(rho))

    def set_f(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        assert f.shape == (9, self.ny, self.nx)
        lib().orc_set_f(self._h, _ptr(f))

    def get_f(self) -> np.ndarray:
        f = np.zeros((9, self.ny, self.nx))
        lib().orc_get_f(self._h, _ptr(f))
        return f

    def step(self, n: int) -> int:
        return lib().orc_step(self._h, n)

    @property
    def steps(self) -> int:
        return lib().orc_step_count(self._h)

    @property
    def unstable_step(self) -> int:
        return lib().orc_unstable_step(self._h)

    def fields(self):
        r = np.zeros((self.ny, self.nx))
        vx = np.zeros_like(r)
        vy = np.zeros_like(r)
        lib().orc_fields(self._h, _ptr(r), _ptr(vx), _ptr(vy))
        return r, vx, vy

    def force(self):
        fx = np.zeros((self.ny, self.nx))
        fy = np.zeros_like(fx)
        lib().orc_force(self._h, _ptr(fx), _ptr(fy))
        return fx, fy

    def eval_force(self, rho: np.ndarray):
        """(Fx, Fy, p_bot, p_top) of a given density field [ny][nx] by the step's own force and
        wall-pressure stages (eqs. 2.17 and 2.8); replaces this simulation's density and force."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        assert rho.shape == (self.ny, self.nx)
        fx = np.zeros((self.ny, self.nx))
        fy = np.zeros_like(fx)
        pb = np.zeros(self.nx)
        pt = np.zeros(self.nx)
        lib().orc_eval_force(self._h, _ptr(rho), _ptr(fx), _ptr(fy), _ptr(pb), _ptr(pt))
        return fx, fy, pb, pt

    def wall(self):
        a = [np.zeros(self.nx) for _ in range(4)]
        lib().orc_wall(self._h, *[_ptr(x) for x in a])
        return dict(zip(["tau_bot", "tau_top", "p_bot", "p_top"], a))

    def history(self, cap: int = 1 << 20):
        buf = (Summary * cap)()
        n = lib().orc_history(self._h, buf, cap)
        return [buf[i].as_dict() for i in range(n)]

    def totals(self):
        m, px, py = C.c_double(), C.c_double(), C.c_double()
        lib().orc_totals(self._h, C.byref(m), C.byref(px), C.byref(py))
        return m.value, px.value, py.value

    def interface(self):
        xr, xf, cols = C.c_double(), C.c_double(), C.c_int()
        lib().orc_interface(self._h, C.byref(xr), C.byref(xf), C.byref(cols))
        return xr.value, xf.value, cols.value

    def components(self, threshold: float = math.nan, connectivity: int = 4) -> list:
        """Liquid components of the current density (threshold NaN = (rho_g + rho_l) / 2)."""
        n = lib().orc_components(self._h, threshold, connectivity, None, 0)
        if n < 0:
            raise RuntimeError(f"orc_components failed: {n}")
        buf = (Component * max(n, 1))()
        lib().orc_components(self._h, threshold, connectivity, buf, n)
        return [buf[i].as_dict() for i in range(n)]
