"""Thin ctypes binding of the C ABI in include/lbm.h (argument marshalling only).

The functions below carry the C names (lbm_create, lbm_bind, lbm_step, ...).
`Lattice` strings them together: torch supplies the device workspace and the
HIP stream, the library does every step of the method in its own kernels.  The
binding raises if liblbm.so is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_ESTATE = 0, -1, -2, -3, -4, -5
LBM_EOS_CS, LBM_EOS_PR = 0, 1
LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S, LBM_F32D, LBM_F32S, LBM_F64T, LBM_F16R = 0, 1, 2, 3, 4, 5, 6, 7
OBJECTIVES = {"sum": 0, "peak": 1}  # lbm_adjoint_objective_kind
STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S, "f32d": LBM_F32D,
           "f32s": LBM_F32S, "f64t": LBM_F64T, "f16r": LBM_F16R}

EXPORTED = [
    "lbm_params_default", "lbm_create", "lbm_workspace", "lbm_bind", "lbm_state", "lbm_init_plug",
    "lbm_init_density", "lbm_step", "lbm_step_count", "lbm_fields", "lbm_wall_stress", "lbm_stress_history",
    "lbm_check_state", "lbm_components", "lbm_components_field", "lbm_get_f", "lbm_set_f", "lbm_destroy",
    "lbm_last_error", "lbm_batch_create", "lbm_batch_workspace", "lbm_batch_bind", "lbm_batch_case",
    "lbm_batch_step", "lbm_batch_destroy", "lbm_batch_last_error", "lbm_set_tangent", "lbm_get_f_tangent",
    "lbm_reset_stress_extremes", "lbm_adjoint_workspace", "lbm_adjoint_bind", "lbm_adjoint_forward",
    "lbm_adjoint_backward", "lbm_adjoint_state_gradient", "lbm_autotune", "lbm_batch_autotune",
    "lbm_fields_device", "lbm_save", "lbm_load", "lbm_launch_config", "lbm_adjoint_objective",
    "lbm_capture", "lbm_batch_capture", "lbm_check_state_noalloc",
]


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class lbm_params(C.Structure):
    _fields_ = [
        ("eos", C.c_int), ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("omega", C.c_double),
        ("T_over_Tc", C.c_double), ("k", C.c_double), ("kappa", C.c_double), ("s_e", C.c_double),
        ("s_eps", C.c_double), ("s_q", C.c_double), ("s_j", C.c_double), ("rho_wall", C.c_double),
        ("dp", C.c_double), ("x_periodic", C.c_int), ("y_periodic", C.c_int), ("storage", C.c_int),
        ("rho0_shift", C.c_double), ("check_every", C.c_int), ("v_limit", C.c_double),
        ("history_cap", C.c_int), ("tile_rows", C.c_int), ("schedule", C.c_int),
        ("tile_waves", C.c_int), ("pipe_blocks", C.c_int), ("graph_steps", C.c_int),
        ("fused_steps", C.c_int),
    ]


class lbm_stress_summary(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("tau_max", C.c_double * 2), ("tau_min", C.c_double * 2),
        ("p_max", C.c_double * 2), ("p_min", C.c_double * 2), ("x_tau_max", C.c_int32 * 2),
        ("x_tau_min", C.c_int32 * 2), ("x_p_max", C.c_int32 * 2), ("x_p_min", C.c_int32 * 2),
        ("sum_tau2", C.c_double), ("int_peak_tau2", C.c_double), ("int_tau2", C.c_double),
        ("run_tau_max", C.c_double * 2), ("run_tau_min", C.c_double * 2),
        ("run_p_max", C.c_double * 2), ("run_p_min", C.c_double * 2),
        ("d_sum_tau2", C.c_double), ("d_int_tau2", C.c_double),
    ]


class lbm_check_result(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass", C.c_double), ("momx", C.c_double), ("momy", C.c_double),
        ("vmax", C.c_double), ("nan_count", C.c_int64), ("x_rear", C.c_double), ("x_front", C.c_double),
        ("liquid_columns", C.c_int32), ("rupture_step", C.c_int64), ("unstable_step", C.c_int64),
    ]


class lbm_component(C.Structure):
    _fields_ = [
        ("first_cell", C.c_int64), ("cells", C.c_int32), ("wall", C.c_int32),
        ("mass", C.c_double), ("excess_mass", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
    ]


class lbm_aerosol_summary(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("components", C.c_int64), ("aerosols", C.c_int64), ("aerosol_cells", C.c_int64),
        ("threshold", C.c_double), ("liquid_mass", C.c_double), ("aerosol_mass", C.c_double),
        ("aerosol_excess_mass", C.c_double),
    ]


def struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


_lib = None
_D = C.POINTER(C.c_double)
_P = C.c_void_p


def library():
    """Loads liblbm.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        PP = C.POINTER(lbm_params)
        sig = {
            "lbm_params_default": (None, [PP]),
            "lbm_create": (C.c_int, [C.c_int, C.c_int, C.c_double, PP, C.POINTER(_P)]),
            "lbm_workspace": (C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
            "lbm_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "lbm_state": (C.c_int, [_P, _D, _D, _D, _D, _D]),
            "lbm_init_plug": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_uint64]),
            "lbm_init_density": (C.c_int, [_P, _D]),
            "lbm_step": (C.c_int, [_P, C.c_int64]),
            "lbm_capture": (C.c_int, [_P, C.c_int64]),
            "lbm_batch_capture": (C.c_int, [_P, C.c_int64]),
            "lbm_step_count": (C.c_int, [_P, C.POINTER(C.c_int64)]),
            "lbm_fields": (C.c_int, [_P, _D, _D, _D]),
            "lbm_fields_device": (C.c_int, [_P, _P, _P, _P, C.c_int]),
            "lbm_save": (C.c_int, [_P, C.c_char_p]),
            "lbm_launch_config": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                            C.POINTER(C.c_int)]),
            "lbm_load": (C.c_int, [_P, C.c_char_p]),
            "lbm_wall_stress": (C.c_int, [_P, _D, _D, _D, _D, C.POINTER(lbm_stress_summary)]),
            "lbm_stress_history": (C.c_int, [_P, C.POINTER(lbm_stress_summary), C.c_int64,
                                             C.POINTER(C.c_int64)]),
            "lbm_check_state": (C.c_int, [_P, C.POINTER(lbm_check_result)]),
            "lbm_check_state_noalloc": (C.c_int, [_P, C.POINTER(lbm_check_result)]),
            "lbm_components": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(lbm_component), C.c_int64,
                                         C.POINTER(C.c_int64), C.POINTER(lbm_aerosol_summary)]),
            "lbm_components_field": (C.c_int, [_D, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                               C.c_int, C.POINTER(lbm_component), C.c_int64, C.POINTER(C.c_int64),
                                               C.POINTER(lbm_aerosol_summary)]),
            "lbm_reset_stress_extremes": (C.c_int, [_P]),
            "lbm_autotune": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _D]),
            "lbm_batch_autotune": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _D]),
            "lbm_adjoint_workspace": (C.c_int, [_P, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
            "lbm_adjoint_bind": (C.c_int, [_P, _P, C.c_size_t, C.c_int64, C.c_int64]),
            "lbm_adjoint_forward": (C.c_int, [_P, _D]),
            "lbm_adjoint_objective": (C.c_int, [_P, C.c_int]),
            "lbm_adjoint_backward": (C.c_int, [_P, C.c_double, _D]),
            "lbm_adjoint_state_gradient": (C.c_int, [_P, _D]),
            "lbm_set_tangent": (C.c_int, [_P, _D]),
            "lbm_get_f_tangent": (C.c_int, [_P, _D]),
            "lbm_get_f": (C.c_int, [_P, _D]),
            "lbm_set_f": (C.c_int, [_P, _D]),
            "lbm_destroy": (None, [_P]),
            "lbm_last_error": (C.c_char_p, [_P]),
            "lbm_batch_create": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _D, PP,
                                           C.POINTER(_P)]),
            "lbm_batch_workspace": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
            "lbm_batch_bind": (C.c_int, [_P, _P, C.c_size_t, _P]),
            "lbm_batch_case": (C.c_int, [_P, C.c_int, C.POINTER(_P)]),
            "lbm_batch_step": (C.c_int, [_P, C.c_int64, C.POINTER(C.c_int)]),
            "lbm_batch_destroy": (None, [_P]),
            "lbm_batch_last_error": (C.c_char_p, [_P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _check(ctx, st: int):
    if st != LBM_OK:
        msg = library().lbm_last_error(ctx)
        raise LbmError(st, msg.decode() if msg else "")


# ---- C-named wrappers -------------------------------------------------------

def lbm_params_default(**overrides) -> lbm_params:
    p = lbm_params()
    library().lbm_params_default(C.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(f"unknown lbm_params field {k!r}")
        setattr(p, k, STORAGE[v] if k == "storage" and isinstance(v, str) else v)
    return p


def lbm_create(nx: int, ny: int, tau: float, p: lbm_params):
    h = C.c_void_p()
    st = library().lbm_create(nx, ny, tau, C.byref(p), C.byref(h))
    if st != LBM_OK:
        raise LbmError(st, f"lbm_create({nx}, {ny}, {tau}) rejected the parameters")
    return h


def lbm_workspace(ctx, with_align: bool = False):
    """Device bytes to allocate and bind (and, with_align, their required alignment)."""
    n, a = C.c_size_t(), C.c_size_t()
    _check(ctx, library().lbm_workspace(ctx, C.byref(n), C.byref(a)))
    return (n.value, a.value) if with_align else n.value


def lbm_bind(ctx, device_ptr: int, nbytes: int, stream: int):
    _check(ctx, library().lbm_bind(ctx, C.c_void_p(device_ptr), nbytes, C.c_void_p(stream)))


def lbm_state(ctx) -> dict:
    v = [C.c_double() for _ in range(5)]
    _check(ctx, library().lbm_state(ctx, *[C.byref(x) for x in v]))
    return dict(zip(["T", "Tc", "rho_g", "rho_l", "rho_w"], [x.value for x in v]))


def lbm_init_plug(ctx, plug_len, film, x_center=math.nan, noise_amp=1e-3, seed=1):
    _check(ctx, library().lbm_init_plug(ctx, plug_len, film, x_center, noise_amp, seed))


def lbm_init_density(ctx, rho: np.ndarray):
    _check(ctx, library().lbm_init_density(ctx, _ptr(np.ascontiguousarray(rho, dtype=np.float64))))


def lbm_step(ctx, n: int) -> int:
    """Returns the status (LBM_OK or LBM_EUNSTABLE); other failures raise."""
    st = library().lbm_step(ctx, n)
    if st not in (LBM_OK, LBM_EUNSTABLE):
        _check(ctx, st)
    return st


def lbm_capture(ctx, n: int):
    _check(ctx, library().lbm_capture(ctx, n))


def lbm_step_count(ctx) -> int:
    n = C.c_int64()
    _check(ctx, library().lbm_step_count(ctx, C.byref(n)))
    return n.value


def lbm_fields(ctx, rho, vx, vy):
    _check(ctx, library().lbm_fields(ctx, _ptr(rho), _ptr(vx), _ptr(vy)))


def lbm_fields_device(ctx, rho_ptr: int, vx_ptr: int, vy_ptr: int, fp64: bool):
    """Device pointers (ints, 0 for none) of caller-owned [ny][nx] arrays."""
    _check(ctx, library().lbm_fields_device(ctx, rho_ptr or None, vx_ptr or None, vy_ptr or None, int(fp64)))


def lbm_save(ctx, path: str):
    _check(ctx, library().lbm_save(ctx, os.fsencode(path)))


def lbm_load(ctx, path: str):
    _check(ctx, library().lbm_load(ctx, os.fsencode(path)))


def lbm_wall_stress(ctx, tau_bot, tau_top, p_bot, p_top) -> dict:
    s = lbm_stress_summary()
    _check(ctx, library().lbm_wall_stress(ctx, _ptr(tau_bot), _ptr(tau_top), _ptr(p_bot), _ptr(p_top),
                                          C.byref(s)))
    return struct_dict(s)


def lbm_stress_history(ctx, cap: int) -> list:
    buf = (lbm_stress_summary * max(cap, 1))()
    n = C.c_int64()
    _check(ctx, library().lbm_stress_history(ctx, buf, cap, C.byref(n)))
    return [struct_dict(buf[i]) for i in range(n.value)]


def lbm_check_state(ctx) -> dict:
    r = lbm_check_result()
    _check(ctx, library().lbm_check_state(ctx, C.byref(r)))
    return struct_dict(r)


def lbm_check_state_noalloc(ctx) -> dict:
    r = lbm_check_result()
    _check(ctx, library().lbm_check_state_noalloc(ctx, C.byref(r)))
    return struct_dict(r)


def lbm_components(ctx, threshold: float = math.nan, connectivity: int = 4):
    """(components as dicts, summary dict) of the last step's density."""
    n, summ = C.c_int64(), lbm_aerosol_summary()
    _check(ctx, library().lbm_components(ctx, threshold, connectivity, None, 0, C.byref(n), None))
    buf = (lbm_component * max(n.value, 1))()
    _check(ctx, library().lbm_components(ctx, threshold, connectivity, buf, n.value, C.byref(n), C.byref(summ)))
    return [struct_dict(buf[i]) for i in range(n.value)], struct_dict(summ)


def lbm_components_field(rho: np.ndarray, threshold: float, rho_g: float = 0.0, connectivity: int = 4,
                         x_periodic: int = 0, y_periodic: int = 0):
    """(components, summary) of a host field rho[ny][nx]; host code only, no device."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    ny, nx = rho.shape
    n, summ = C.c_int64(), lbm_aerosol_summary()
    st = library().lbm_components_field(_ptr(rho), nx, ny, x_periodic, y_periodic, threshold, rho_g, connectivity,
                                        None, 0, C.byref(n), None)
    if st != LBM_OK:
        raise LbmError(st, "lbm_components_field: invalid arguments")
    buf = (lbm_component * max(n.value, 1))()
    library().lbm_components_field(_ptr(rho), nx, ny, x_periodic, y_periodic, threshold, rho_g, connectivity, buf,
                                   n.value, C.byref(n), C.byref(summ))
    return [struct_dict(buf[i]) for i in range(n.value)], struct_dict(summ)


def lbm_set_tangent(ctx, dtheta):
    d = np.ascontiguousarray(dtheta, dtype=np.float64)
    assert d.shape == (4,)
    _check(ctx, library().lbm_set_tangent(ctx, _ptr(d)))


def lbm_get_f_tangent(ctx, df: np.ndarray):
    _check(ctx, library().lbm_get_f_tangent(ctx, _ptr(df)))


def lbm_autotune(ctx, trial_steps: int = 50) -> dict:
    r, w, us = C.c_int(), C.c_int(), C.c_double()
    _check(ctx, library().lbm_autotune(ctx, trial_steps, C.byref(r), C.byref(w), C.byref(us)))
    return dict(tile_rows=r.value, tile_waves=w.value, us_per_step=us.value,
                fused_steps=lbm_launch_config(ctx)["fused_steps"])


def lbm_launch_config(ctx) -> dict:
    v = [C.c_int() for _ in range(4)]
    _check(ctx, library().lbm_launch_config(ctx, *(C.byref(x) for x in v)))
    return dict(zip(["tile_rows", "tile_waves", "fused_steps", "graph_steps"], (x.value for x in v)))


def lbm_adjoint_workspace(ctx, nsteps: int, segment: int = 0) -> int:
    n = C.c_size_t()
    st = library().lbm_adjoint_workspace(ctx, nsteps, segment, C.byref(n))
    if st != LBM_OK:
        raise LbmError(st, f"lbm_adjoint_workspace({nsteps}, {segment}) rejected the request")
    return n.value


def lbm_adjoint_bind(ctx, device_ptr: int, nbytes: int, nsteps: int, segment: int = 0):
    _check(ctx, library().lbm_adjoint_bind(ctx, C.c_void_p(device_ptr), nbytes, nsteps, segment))


def lbm_adjoint_forward(ctx) -> tuple:
    """Returns (status, J): status LBM_OK or LBM_EUNSTABLE; other failures raise."""
    J = C.c_double(math.nan)
    st = library().lbm_adjoint_forward(ctx, C.byref(J))
    if st not in (LBM_OK, LBM_EUNSTABLE):
        _check(ctx, st)
    return st, J.value


def lbm_adjoint_backward(ctx, seed: float = 1.0) -> np.ndarray:
    g = np.empty(4)
    _check(ctx, library().lbm_adjoint_backward(ctx, seed, _ptr(g)))
    return g


def lbm_adjoint_state_gradient(ctx, out: np.ndarray):
    _check(ctx, library().lbm_adjoint_state_gradient(ctx, _ptr(out)))


def lbm_get_f(ctx, f: np.ndarray):
    _check(ctx, library().lbm_get_f(ctx, _ptr(f)))


def lbm_set_f(ctx, f: np.ndarray):
    _check(ctx, library().lbm_set_f(ctx, _ptr(np.ascontiguousarray(f, dtype=np.float64))))


def lbm_destroy(ctx):
    library().lbm_destroy(ctx)


def lbm_last_error(ctx) -> str:
    m = library().lbm_last_error(ctx)
    return m.decode() if m else ""


# ---- convenience object -----------------------------------------------------

def _batch_check(b, st: int):
    if st != LBM_OK:
        msg = library().lbm_batch_last_error(b)
        raise LbmError(st, msg.decode() if msg else "")


class Lattice:
    """One D2Q9 channel on one GPU.  torch provides the device workspace and the stream."""

    def __init__(self, nx: int, ny: int, tau: float, device: str = "cuda:0", stream=None, **params):
        import torch

        self.nx, self.ny, self.tau = nx, ny, tau
        self.params = lbm_params_default(**params)
        self._ctx = lbm_create(nx, ny, tau, self.params)
        self._owner = None
        nbytes, align = lbm_workspace(self._ctx, with_align=True)
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        if self.workspace.data_ptr() % align:
            raise RuntimeError(f"torch returned a workspace not aligned to {align} bytes")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            lbm_bind(self._ctx, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)

    @classmethod
    def _case_of(cls, batch, k: int, nx: int, ny: int, tau: float, params):
        """View of case k of a batch (stepped by the batch; keeps the batch alive)."""
        self = cls.__new__(cls)
        self.nx, self.ny, self.tau, self.params = nx, ny, tau, params
        ctx = _P()
        _batch_check(batch._b, library().lbm_batch_case(batch._b, k, C.byref(ctx)))
        self._ctx = ctx
        self._owner = batch
        self.device, self.stream, self.workspace = batch.device, batch.stream, None
        return self

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and getattr(self, "_owner", None) is None:
            lbm_destroy(ctx)
        self._ctx = None

    @property
    def ctx(self):
        return self._ctx

    def state(self) -> dict:
        return lbm_state(self._ctx)

    def init_plug(self, plug_len, film, x_center=math.nan, noise_amp=1e-3, seed=1):
        lbm_init_plug(self._ctx, plug_len, film, x_center, noise_amp, seed)

    def init_density(self, rho: np.ndarray):
        assert rho.shape == (self.ny, self.nx)
        lbm_init_density(self._ctx, rho)

    def step(self, n: int) -> int:
        """Enqueues n steps on the lattice's stream; waits only for the checks at multiples of check_every."""
        return lbm_step(self._ctx, n)

    def capture(self, n: int):
        """Captures the HIP graphs a call step(n) made now would replay (nothing runs)."""
        lbm_capture(self._ctx, n)

    @property
    def steps(self) -> int:
        return lbm_step_count(self._ctx)

    def fields(self):
        r = np.empty((self.ny, self.nx))
        vx = np.empty_like(r)
        vy = np.empty_like(r)
        lbm_fields(self._ctx, r, vx, vy)
        return r, vx, vy

    def fields_device(self, dtype=None):
        """rho, vx, vy of the last step as device tensors [ny][nx] (float64, or float32), written on the
        lattice's stream."""
        import torch

        dtype = torch.float64 if dtype is None else dtype
        if dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be torch.float64 or torch.float32")
        with torch.cuda.stream(self.stream):
            out = [torch.empty((self.ny, self.nx), dtype=dtype, device=self.device) for _ in range(3)]
        lbm_fields_device(self._ctx, *(t.data_ptr() for t in out), dtype == torch.float64)
        return tuple(out)

    def save(self, path: str):
        """Checkpoint of the run (lbm_save)."""
        lbm_save(self._ctx, path)

    def load(self, path: str):
        """Continue a run saved by a lattice with the same sizes, tau and parameters (lbm_load)."""
        lbm_load(self._ctx, path)

    def wall(self):
        a = [np.empty(self.nx) for _ in range(4)]
        s = lbm_wall_stress(self._ctx, *a)
        return dict(zip(["tau_bot", "tau_top", "p_bot", "p_top"], a)), s

    def history(self, cap: int = 1 << 16) -> list:
        return lbm_stress_history(self._ctx, cap)

    def check(self) -> dict:
        return lbm_check_state(self._ctx)

    def reset_stress_extremes(self):
        """Restart the running wall-stress extremes from the next step on."""
        _check(self._ctx, library().lbm_reset_stress_extremes(self._ctx))

    def components(self, threshold: float = math.nan, connectivity: int = 4):
        """Liquid components of the last step's density and the aerosol totals."""
        return lbm_components(self._ctx, threshold, connectivity)

    def get_f(self) -> np.ndarray:
        f = np.empty((9, self.ny, self.nx))
        lbm_get_f(self._ctx, f)
        return f

    def set_tangent(self, dp: float = 0.0, a: float = 0.0, b: float = 0.0, T: float = 0.0):
        """F64T storage: tangent direction in (dp, a, b, absolute T); the state's tangent restarts at zero
        with each initialisation."""
        lbm_set_tangent(self._ctx, [dp, a, b, T])

    def get_f_tangent(self) -> np.ndarray:
        df = np.empty((9, self.ny, self.nx))
        lbm_get_f_tangent(self._ctx, df)
        return df

    def set_f(self, f: np.ndarray):
        assert f.shape == (9, self.ny, self.nx)
        lbm_set_f(self._ctx, f)

    def autotune(self, trial_steps: int = 50) -> dict:
        """Times every tile shape of the tile schedule, and two steps per launch, on the current state and keeps
        the fastest."""
        return lbm_autotune(self._ctx, trial_steps)

    def launch_config(self) -> dict:
        return lbm_launch_config(self._ctx)

    def adjoint_bind(self, nsteps: int, segment: int = 0, objective: str = "sum"):
        """Device workspace for recording nsteps steps with a checkpoint every `segment` steps; objective "sum"
        (J = sum over steps, walls, columns of tau_w^2) or "peak" (J = sum over steps of the peak tau_w^2)."""
        import torch

        nbytes = lbm_adjoint_workspace(self._ctx, nsteps, segment)
        self.adjoint_workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            lbm_adjoint_bind(self._ctx, self.adjoint_workspace.data_ptr(), nbytes, nsteps, segment)
        _check(self._ctx, library().lbm_adjoint_objective(self._ctx, OBJECTIVES[objective]))

    def adjoint_forward(self) -> tuple:
        """Runs and records the bound number of steps; returns (status, J = int of sum tau_w^2)."""
        return lbm_adjoint_forward(self._ctx)

    def adjoint_backward(self, seed: float = 1.0) -> np.ndarray:
        """seed * dJ/d(dp, a, b, T) by one reverse sweep over the recorded steps."""
        return lbm_adjoint_backward(self._ctx, seed)

    def adjoint_state_gradient(self) -> np.ndarray:
        g = np.empty((9, self.ny, self.nx))
        lbm_adjoint_state_gradient(self._ctx, g)
        return g


class Batch:
    """Many independent channels advanced by one kernel launch per step.

    cases: a list of dicts with nx, ny, tau and any lbm_params fields; keywords
    given to the constructor apply to every case (storage, eos, tile_rows,
    tile_waves and check_every must agree).  batch[k] is case k as a Lattice
    (initialise and read it there); batch.step(n) advances all cases."""

    def __init__(self, cases: list, device: str = "cuda:0", stream=None, **common):
        import torch

        n = len(cases)
        specs = [dict(common, **c) for c in cases]
        nx = (C.c_int * n)(*[int(c.pop("nx")) for c in specs])
        ny = (C.c_int * n)(*[int(c.pop("ny")) for c in specs])
        tau = (C.c_double * n)(*[float(c.pop("tau")) for c in specs])
        params = (lbm_params * n)(*[lbm_params_default(**c) for c in specs])
        b = _P()
        st = library().lbm_batch_create(n, nx, ny, tau, params, C.byref(b))
        if st != LBM_OK:
            raise LbmError(st, "lbm_batch_create: the cases disagree on storage/eos/tile shape/check cadence, "
                               "or a case is invalid")
        self._b = b
        size = C.c_size_t()
        _batch_check(b, library().lbm_batch_workspace(b, C.byref(size)))
        self.device = torch.device(device)
        self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            _batch_check(b, library().lbm_batch_bind(b, self.workspace.data_ptr(), size.value,
                                                     self.stream.cuda_stream))
        self.cases = [Lattice._case_of(self, k, nx[k], ny[k], tau[k], params[k]) for k in range(n)]

    def __len__(self):
        return len(self.cases)

    def __getitem__(self, k: int) -> Lattice:
        return self.cases[k]

    def step(self, n: int) -> int:
        failed = C.c_int(-1)
        st = library().lbm_batch_step(self._b, n, C.byref(failed))
        if st != LBM_OK:
            msg = library().lbm_batch_last_error(self._b)
            err = LbmError(st, msg.decode() if msg else "")
            err.case = failed.value
            raise err
        return LBM_OK

    def capture(self, n: int):
        """Captures the HIP graphs a call step(n) made now would replay (nothing runs)."""
        _batch_check(self._b, library().lbm_batch_capture(self._b, n))

    def autotune(self, trial_steps: int = 20) -> dict:
        """Times every tile shape on all cases at once and keeps the fastest for the batch."""
        r, w, us = C.c_int(), C.c_int(), C.c_double()
        _batch_check(self._b, library().lbm_batch_autotune(self._b, trial_steps, C.byref(r), C.byref(w),
                                                           C.byref(us)))
        return dict(tile_rows=r.value, tile_waves=w.value, us_per_step=us.value)

    def __del__(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            self.cases = []
            library().lbm_batch_destroy(b)
            self._b = None


# ---- autograd ------------------------------------------------------------------

def _check_wall_shear_spec(spec: dict):
    """The adjoint holds the wall ghost density fixed.  Without an explicit rho_wall the library
    sets it to rho_l(T) of each theta, so the forward J would depend on theta through the wall
    density and the returned gradient would not be the gradient of J: such a spec is refused."""
    rw = spec.get("params", {}).get("rho_wall")
    if rw is None or not math.isfinite(float(rw)):
        raise ValueError("WallShearObjective needs spec['params']['rho_wall'] (a finite wall density): the "
                         "gradient holds the wall density fixed, and by default it would follow rho_l(theta)")


def _wall_shear_lattice(theta, spec: dict):
    """A lattice at theta = (dp, a, b, T) with T absolute, initialised with spec['rho_init']."""
    dp, a, b, T = (float(v) for v in theta)
    kw = dict(spec.get("params", {}))
    kw.update(a=a, b=b, dp=dp)
    probe = Lattice(spec["nx"], spec["ny"], spec["tau"], device=spec.get("device", "cuda:0"),
                    T_over_Tc=spec.get("T_over_Tc_probe", 0.9), **kw)
    tc = probe.state()["Tc"]  # the library's critical temperature of (a, b, R)
    del probe
    lat = Lattice(spec["nx"], spec["ny"], spec["tau"], device=spec.get("device", "cuda:0"), T_over_Tc=T / tc, **kw)
    lat.init_density(spec["rho_init"])
    return lat


class WallShearObjective:
    """J(theta) = time integral over `nsteps` steps of the squared wall shear summed over both walls, as a
    differentiable function of theta = (dp, a, b, T) (a float64 tensor of 4; T absolute).  Forward runs the
    lattice on the GPU and records checkpoints; backward is one reverse (adjoint) sweep of the hand-written
    adjoint kernels.

    spec: nx, ny, tau, nsteps, rho_init (ny x nx initial density, held fixed), params (other lbm_params
    fields; rho_wall is required: the gradient holds the wall density fixed, so it must not follow theta),
    optional segment, device and objective ("sum", the default, or "peak": the time integral of the squared
    peak wall shear).

        J = WallShearObjective.apply(theta, spec); J.backward()  ->  theta.grad
    """

    _fn = None

    @staticmethod
    def _function():
        if WallShearObjective._fn is not None:
            return WallShearObjective._fn
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, theta, spec):
                _check_wall_shear_spec(spec)
                lat = _wall_shear_lattice(theta.detach().cpu().tolist(), spec)
                lat.adjoint_bind(spec["nsteps"], spec.get("segment", 0), spec.get("objective", "sum"))
                st, J = lat.adjoint_forward()
                if st != LBM_OK:
                    raise LbmError(st, "the forward run went unstable")
                ctx.lattice = lat
                ctx.theta_dtype, ctx.theta_device = theta.dtype, theta.device
                return torch.tensor(J, dtype=theta.dtype, device=theta.device)

            @staticmethod
            def backward(ctx, grad_out):
                g = ctx.lattice.adjoint_backward(float(grad_out))
                ctx.lattice = None
                return torch.tensor(g, dtype=ctx.theta_dtype, device=ctx.theta_device), None

        WallShearObjective._fn = _Fn
        return _Fn

    @classmethod
    def apply(cls, theta, spec: dict):
        return cls._function().apply(theta, spec)
