"""Python binding of ``liblbm.so`` (declared in ``include/lbm.h``).

Argument marshalling only: every step of the scheme runs in the HIP
kernels.  The functions carry the C names; a non-OK status raises
:class:`LbmError`.  :class:`Channel` wraps a context whose device memory is
a torch tensor and whose stream is torch's current stream.

There is no CPU fallback: if the library is not built, loading raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LATTICES = {"D2Q16": 0, "D2Q17": 1, "D3Q121": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "fp16": 3, "fp32s": 4}
FIELDS = ("rho", "ux", "uy", "uz", "T", "sxy", "qx", "qy", "qz")

LBM_OK = 0
LBM_EINVAL = -1
LBM_ENOMEM = -2
LBM_EDEVICE = -3
LBM_ENONFINITE = -4
LBM_ENEGATIVE = -5
LBM_EUNSUPPORTED = -6


class LbmError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lbm_strerror(status) if _lib is not None else str(status)
        if _lib is not None and status in (LBM_EDEVICE, LBM_ENOMEM):
            msg += " [%s]" % _lib.lbm_last_device_error().decode()
        super().__init__("%s: %s (status %d)" % (what, msg, status))


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class _Wall(ctypes.Structure):
    _fields_ = [("ux", ctypes.c_double), ("uz", ctypes.c_double), ("T", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("liblbm.so is not built (%s); run `python -m "
                           "paper_1209_5201_amd.build`" % LIB_PATH)
    # torch ships its own HIP runtime under the same soname
    # (libamdhip64.so.7).  Loading torch first makes the library bind to that
    # runtime, so the process has one HIP runtime, torch's memory and streams
    # are native handles, and devices are visible to both.  (Loading the
    # library first would pull in a second runtime that sees no device.)
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "lbm_lattice_info": (ctypes.c_int, [ctypes.c_int, _ip, _ip, _ip, _ip, _dp, _ip, _dp]),
        "lbm_tau_from_kn": (ctypes.c_double, [ctypes.c_int, ctypes.c_int32, ctypes.c_double]),
        "lbm_required_bytes": (ctypes.c_size_t, [ctypes.c_int, _Grid, ctypes.c_int]),
        "lbm_create": (ctypes.c_int, [ctypes.c_int, _Grid, ctypes.c_double,
                                      ctypes.POINTER(_Wall), ctypes.POINTER(_Wall),
                                      ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
        "lbm_create_in": (ctypes.c_int, [ctypes.c_int, _Grid, ctypes.c_double,
                                         ctypes.POINTER(_Wall), ctypes.POINTER(_Wall),
                                         ctypes.c_int, _vp, _vp, ctypes.c_size_t,
                                         ctypes.POINTER(_vp)]),
        "lbm_init": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
        "lbm_step": (ctypes.c_int, [_vp, ctypes.c_int64]),
        "lbm_field": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
        "lbm_moments": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
        "lbm_residual": (ctypes.c_int, [_vp, _dp]),
        "lbm_mass": (ctypes.c_int, [_vp, _dp]),
        "lbm_steps_done": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
        "lbm_state_bytes": (ctypes.c_size_t, [_vp]),
        "lbm_save": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "lbm_load": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
        "lbm_batch_step": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int64,
                                          _dp]),
        "lbm_batch_run": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                         ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_int64),
                                         _ip]),
        "lbm_set_accommodation": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
        "lbm_set_viscosity_law": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double]),
        "lbm_set_body_force": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double]),
        "lbm_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
        "lbm_kernel_time": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int64), _dp,
                                           ctypes.POINTER(ctypes.c_int64)]),
        "lbm_destroy": (None, [_vp]),
        "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "lbm_last_device_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C ABI entry points this binding expects."""
    return ["lbm_lattice_info", "lbm_tau_from_kn", "lbm_required_bytes", "lbm_create",
            "lbm_create_in", "lbm_init", "lbm_step", "lbm_field", "lbm_moments",
            "lbm_residual", "lbm_mass", "lbm_steps_done", "lbm_state_bytes", "lbm_save",
            "lbm_load", "lbm_batch_step", "lbm_batch_run", "lbm_set_accommodation",
            "lbm_set_viscosity_law", "lbm_set_body_force", "lbm_set_timing", "lbm_kernel_time", "lbm_destroy", "lbm_strerror",
            "lbm_last_device_error"]


def _check(st: int, what: str):
    if st != LBM_OK:
        raise LbmError(st, what)


def _lat(lattice) -> int:
    return LATTICES[lattice.upper()] if isinstance(lattice, str) else int(lattice)


def _prec(prec) -> int:
    return PRECISIONS[prec.lower()] if isinstance(prec, str) else int(prec)


def _dptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_dp)


# ------------------------------------------------------------- C names ---

def lbm_strerror(status: int) -> str:
    return _load().lbm_strerror(int(status)).decode()


def lbm_lattice_info(lattice) -> dict:
    lib = _load()
    Q, D, N, EQ = (ctypes.c_int() for _ in range(4))
    r = ctypes.c_double()
    _check(lib.lbm_lattice_info(_lat(lattice), ctypes.byref(Q), ctypes.byref(D),
                                ctypes.byref(N), ctypes.byref(EQ), ctypes.byref(r),
                                None, None), "lbm_lattice_info")
    e = np.zeros((Q.value, 3), dtype=np.int32)
    w = np.zeros(Q.value, dtype=np.float64)
    _check(lib.lbm_lattice_info(_lat(lattice), None, None, None, None, None,
                                e.ctypes.data_as(_ip), _dptr(w)), "lbm_lattice_info")
    return {"Q": Q.value, "D": D.value, "N": N.value, "eq_order": EQ.value, "r": r.value,
            "e": e, "w": w}


def lbm_tau_from_kn(lattice, ny: int, kn: float) -> float:
    return float(_load().lbm_tau_from_kn(_lat(lattice), int(ny), float(kn)))


def lbm_required_bytes(lattice, nx: int, ny: int, prec) -> int:
    return int(_load().lbm_required_bytes(_lat(lattice), _Grid(nx, ny), _prec(prec)))


def lbm_create(lattice, nx, ny, tau, bottom=(0.0, 0.0, 1.0), top=(0.0, 0.0, 1.0),
               prec="fp64", stream=None):
    ctx = _vp()
    _check(_load().lbm_create(_lat(lattice), _Grid(nx, ny), float(tau),
                              ctypes.byref(_Wall(*bottom)), ctypes.byref(_Wall(*top)),
                              _prec(prec), stream, ctypes.byref(ctx)), "lbm_create")
    return ctx


def lbm_create_in(lattice, nx, ny, tau, bottom, top, prec, stream, dev_ptr, nbytes):
    ctx = _vp()
    _check(_load().lbm_create_in(_lat(lattice), _Grid(nx, ny), float(tau),
                                 ctypes.byref(_Wall(*bottom)), ctypes.byref(_Wall(*top)),
                                 _prec(prec), stream, _vp(dev_ptr), int(nbytes),
                                 ctypes.byref(ctx)), "lbm_create_in")
    return ctx


def lbm_init(ctx, rho=None, ux=None, uy=None, T=None):
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).ravel()
            for a in (rho, ux, uy, T)]
    _check(_load().lbm_init(ctx, *[_dptr(a) for a in arrs]), "lbm_init")


def lbm_step(ctx, n: int):
    _check(_load().lbm_step(ctx, int(n)), "lbm_step")


def lbm_field(ctx, field, nx: int, ny: int) -> np.ndarray:
    fid = FIELDS.index(field) if isinstance(field, str) else int(field)
    out = np.empty((ny, nx), dtype=np.float64)
    _check(_load().lbm_field(ctx, fid, _dptr(out)), "lbm_field")
    return out


def lbm_moments(ctx, nx: int, ny: int) -> dict:
    return {k: lbm_field(ctx, k, nx, ny) for k in FIELDS}


def lbm_residual(ctx) -> float:
    r = ctypes.c_double()
    _check(_load().lbm_residual(ctx, ctypes.byref(r)), "lbm_residual")
    return r.value


def lbm_mass(ctx) -> float:
    m = ctypes.c_double()
    _check(_load().lbm_mass(ctx, ctypes.byref(m)), "lbm_mass")
    return m.value


def lbm_steps_done(ctx) -> int:
    s = ctypes.c_int64()
    _check(_load().lbm_steps_done(ctx, ctypes.byref(s)), "lbm_steps_done")
    return s.value


def lbm_state_bytes(ctx) -> int:
    return int(_load().lbm_state_bytes(ctx))


def lbm_save(ctx) -> bytearray:
    n = lbm_state_bytes(ctx)
    buf = bytearray(n)
    cbuf = (ctypes.c_char * n).from_buffer(buf)
    _check(_load().lbm_save(ctx, ctypes.cast(cbuf, _vp), n), "lbm_save")
    return buf


def lbm_load(ctx, state: bytearray):
    cbuf = (ctypes.c_char * len(state)).from_buffer(state)
    _check(_load().lbm_load(ctx, ctypes.cast(cbuf, _vp), len(state)), "lbm_load")


def lbm_batch_step(ctxs, k_steps: int) -> np.ndarray:
    """Advance several contexts k_steps in one persistent launch per storage
    format; returns their residuals (NaN where a case went non-finite)."""
    n = len(ctxs)
    arr = (_vp * n)(*[c.value if isinstance(c, _vp) else c for c in ctxs])
    out = np.empty(n, dtype=np.float64)
    _check(_load().lbm_batch_step(arr, n, int(k_steps), _dptr(out)), "lbm_batch_step")
    return out


def lbm_batch_run(ctxs, budgets, window: int, tol: float):
    """Advance contexts in residual windows until converged (residual < tol)
    or out of budget; returns (residuals, steps advanced, states)."""
    n = len(ctxs)
    arr = (_vp * n)(*[c.value if isinstance(c, _vp) else c for c in ctxs])
    b = np.ascontiguousarray(budgets, dtype=np.int64)
    res = np.empty(n, dtype=np.float64)
    steps = np.empty(n, dtype=np.int64)
    state = np.empty(n, dtype=np.int32)
    _check(_load().lbm_batch_run(arr, n, b.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 int(window), float(tol), _dptr(res),
                                 steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 state.ctypes.data_as(_ip)), "lbm_batch_run")
    return res, steps, state


def lbm_set_accommodation(ctx, alpha_bottom: float, alpha_top: float):
    _check(_load().lbm_set_accommodation(ctx, float(alpha_bottom), float(alpha_top)),
           "lbm_set_accommodation")


def lbm_set_viscosity_law(ctx, exponent):
    """exponent w of mu = T^w for the local relaxation time; None: constant tau."""
    _check(_load().lbm_set_viscosity_law(ctx, int(exponent is not None),
                                         0.0 if exponent is None else float(exponent)),
           "lbm_set_viscosity_law")


def lbm_set_body_force(ctx, ax: float, ay: float = 0.0, az: float = 0.0):
    _check(_load().lbm_set_body_force(ctx, float(ax), float(ay), float(az)),
           "lbm_set_body_force")


def lbm_set_timing(ctx, enable: bool):
    _check(_load().lbm_set_timing(ctx, int(bool(enable))), "lbm_set_timing")


def lbm_kernel_time(ctx) -> dict:
    um, wm = ctypes.c_double(), ctypes.c_double()
    un, wn = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().lbm_kernel_time(ctx, ctypes.byref(um), ctypes.byref(un), ctypes.byref(wm),
                                   ctypes.byref(wn)), "lbm_kernel_time")
    return {"update_ms": um.value, "update_launches": un.value, "wall_ms": wm.value,
            "wall_launches": wn.value}


def lbm_destroy(ctx):
    if ctx:
        _load().lbm_destroy(ctx)


# ------------------------------------------------------------ convenience ---

class Channel:
    """One channel problem on the GPU.  Device memory comes from torch (one
    uint8 tensor of lbm_required_bytes), work runs on torch's current
    stream of `device`."""

    def __init__(self, lattice, nx, ny, tau, bottom=(0.0, 0.0, 1.0), top=(0.0, 0.0, 1.0),
                 prec="fp64", device="cuda:0", kn=None, accommodation=(1.0, 1.0),
                 viscosity_exp=None, force=None):
        import torch
        self.lattice = lattice if isinstance(lattice, str) else \
            {v: k for k, v in LATTICES.items()}[lattice]
        self.nx, self.ny, self.prec = int(nx), int(ny), prec
        if kn is not None:
            tau = lbm_tau_from_kn(lattice, ny, kn)
        self.tau = float(tau)
        nbytes = lbm_required_bytes(lattice, nx, ny, prec)
        if nbytes == 0:
            raise LbmError(LBM_EINVAL, "lbm_required_bytes")
        self._buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.device = self._buf.device
        self._stream = torch.cuda.current_stream(self.device)
        self.ctx = lbm_create_in(lattice, nx, ny, tau, bottom, top, prec,
                                 self._stream.cuda_stream, self._buf.data_ptr(), nbytes)
        if tuple(accommodation) != (1.0, 1.0):
            self.set_accommodation(*accommodation)
        if viscosity_exp is not None:
            self.set_viscosity_law(viscosity_exp)
        if force is not None:
            self.set_body_force(*force)

    def set_body_force(self, ax, ay=0.0, az=0.0):
        lbm_set_body_force(self.ctx, ax, ay, az)

    def set_viscosity_law(self, exponent):
        lbm_set_viscosity_law(self.ctx, exponent)

    def set_accommodation(self, alpha_bottom: float, alpha_top: float):
        lbm_set_accommodation(self.ctx, alpha_bottom, alpha_top)

    def init(self, rho=None, ux=None, uy=None, T=None):
        lbm_init(self.ctx, rho, ux, uy, T)

    def step(self, n: int):
        lbm_step(self.ctx, n)

    def field(self, name: str) -> np.ndarray:
        return lbm_field(self.ctx, name, self.nx, self.ny)

    def moments(self) -> dict:
        return lbm_moments(self.ctx, self.nx, self.ny)

    def residual(self) -> float:
        return lbm_residual(self.ctx)

    def mass(self) -> float:
        return lbm_mass(self.ctx)

    def steps_done(self) -> int:
        return lbm_steps_done(self.ctx)

    def save(self) -> bytearray:
        return lbm_save(self.ctx)

    def load(self, state):
        lbm_load(self.ctx, state)

    def run_to_residual(self, tol: float, window: int = 100, max_steps: int = 10 ** 7) -> int:
        """Step in windows until the residual rate drops below tol."""
        while self.steps_done() < max_steps:
            self.step(window)
            r = self.residual()
            if not math.isfinite(r):
                raise LbmError(LBM_ENONFINITE, "run_to_residual")
            if r < tol:
                break
        return self.steps_done()

    def close(self):
        if getattr(self, "ctx", None):
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
