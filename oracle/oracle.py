"""Python driver of the FP64 oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the oracle checks the product path and is never
part of it.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.

The C core is built on first use with the system C compiler (no HIP, no
shared headers with the product).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

from . import lattices as _lat

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = False) -> str:
    """Compile the oracle core with gcc (strict IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", _SRC, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lat = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   _ip, _dp, ctypes.c_double]
            lib.orc_geq.argtypes = lat + [_dp, ctypes.c_double, _dp]
            lib.orc_geq.restype = None
            lib.orc_init.argtypes = lat + [ctypes.c_int, ctypes.c_int, _dp, _dp,
                                           _dp, _dp]
            lib.orc_init.restype = None
            lib.orc_run.argtypes = lat + [ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, _dp, _dp, ctypes.c_double,
                                          ctypes.c_double, _dp, ctypes.c_long, _dp, _dp, _dp]
            lib.orc_run.restype = ctypes.c_int
            lib.orc_moments.argtypes = lat + [ctypes.c_int, ctypes.c_int,
                                              ctypes.c_double, _dp, _dp, _dp, _dp]
            lib.orc_moments.restype = None
            _lib = lib
    return _lib


def _p(a: np.ndarray, t=_dp):
    return a.ctypes.data_as(t)


class _LatArgs:
    """Keeps the contiguous int32/float64 copies of a lattice alive."""

    def __init__(self, lat: _lat.OracleLattice):
        self.lat = lat
        self.e = np.ascontiguousarray(lat.e, dtype=np.int32)
        self.w = np.ascontiguousarray(lat.w, dtype=np.float64)

    def args(self):
        L = self.lat
        return (L.Q, L.D, L.eq_order, int(L.thermal), _p(self.e, _ip),
                _p(self.w), L.r)


FIELDS = ("rho", "ux", "uy", "uz", "T", "sxy", "qx", "qy", "qz")


def geq(lattice, u, T=1.0) -> np.ndarray:
    """g^eq_a(u, T) of Eq. (eq:feq) for every velocity (unit density)."""
    lat = _lat.by_name(lattice) if isinstance(lattice, str) else lattice
    la = _LatArgs(lat)
    uu = np.zeros(3)
    uu[:len(u)] = u
    out = np.empty(lat.Q)
    _load().orc_geq(*la.args(), _p(uu), float(T), _p(out))
    return out


def tau_from_kn(lattice, ny: int, kn: float) -> float:
    """Relaxation time in time steps for a channel of ny rows.

    Non-dimensional tau = mu/p * sqrt(2/pi) Kn (Sec. II and the Kn definition
    of Sec. IV, with mu = p = 1); lengths are scaled by the channel height,
    so dx = 1/ny and, with c = r e, dt = dx / r.
    """
    lat = _lat.by_name(lattice) if isinstance(lattice, str) else lattice
    return math.sqrt(2.0 / math.pi) * kn * lat.r * ny


class OracleCase:
    """One channel: nx periodic columns, ny rows between two diffuse walls.

    walls are (ux, uz, T) per wall; bottom wall below row 0, top above row
    ny-1; accommodation = (alpha_b, alpha_t) of the Maxwell-type scattering
    kernel (1: fully diffuse, the paper's wall).  Initial fields default to
    rho = 1, u = 0, T = 1.  viscosity_exp = omega_v switches to the local
    relaxation time tau T^(omega_v - 1) / rho (mu = T^omega_v, p = rho T);
    None keeps tau constant.  force = (a_x, a_y, a_z): a body force, the
    acceleration of every node per time step (None: no force).
    """

    def __init__(self, lattice, nx, ny, tau, wall_b=(0.0, 0.0, 1.0),
                 wall_t=(0.0, 0.0, 1.0), rho0=None, u0=None, T0=None,
                 accommodation=(1.0, 1.0), viscosity_exp=None, force=None):
        self.alpha = (float(accommodation[0]), float(accommodation[1]))
        self.law = None if viscosity_exp is None else np.array([float(viscosity_exp)])
        self.force = None if force is None else np.array([float(v) for v in force])
        self.lat = _lat.by_name(lattice) if isinstance(lattice, str) else lattice
        self._la = _LatArgs(self.lat)
        self.nx, self.ny, self.tau = int(nx), int(ny), float(tau)
        self.wall_b = np.array(wall_b, dtype=np.float64)
        self.wall_t = np.array(wall_t, dtype=np.float64)
        nodes = self.nx * self.ny
        rho = np.ones(nodes) if rho0 is None else \
            np.ascontiguousarray(rho0, dtype=np.float64).reshape(nodes)
        u = np.zeros((3, nodes))
        if u0 is not None:
            u0 = np.asarray(u0, dtype=np.float64)
            for i in range(u0.shape[0]):
                u[i] = u0[i].reshape(nodes)
        T = np.ones(nodes) if T0 is None else \
            np.ascontiguousarray(T0, dtype=np.float64).reshape(nodes)
        self.f = np.empty((self.ny, self.nx, self.lat.Q))
        u = np.ascontiguousarray(u)
        _load().orc_init(*self._la.args(), self.nx, self.ny, _p(rho), _p(u),
                         _p(T), _p(self.f))
        self.t = 0

    def run(self, nsteps: int, record_flux: bool = False):
        flux = np.zeros((max(int(nsteps), 1), 4)) if record_flux else None
        rc = _load().orc_run(*self._la.args(), self.nx, self.ny, self.tau,
                             _p(self.wall_b), _p(self.wall_t), self.alpha[0], self.alpha[1],
                             _p(self.f), int(nsteps), _p(flux) if record_flux else None,
                             None if self.law is None else _p(self.law),
                             None if self.force is None else _p(self.force))
        if rc != 0:
            raise RuntimeError("oracle run failed (%d)" % rc)
        self.t += int(nsteps)
        return flux[:nsteps] if record_flux else None

    def moments(self) -> dict:
        out = np.empty((len(FIELDS), self.ny, self.nx))
        _load().orc_moments(*self._la.args(), self.nx, self.ny, self.tau,
                            _p(self.f), _p(out), None if self.law is None else _p(self.law),
                            None if self.force is None else _p(self.force))
        return {k: out[i] for i, k in enumerate(FIELDS)}

    def mass(self) -> float:
        return float(np.sum(self.f))


def residual_rate(prev: dict, cur: dict, k_steps: int, u_ref: float) -> float:
    """Convergence measure used to stop a steady solve.

    The paper states no criterion; the reading used here is a per-step rate
    of change over a window of k_steps steps, so that single precision can
    reach small tolerances:
      R = max(|u(t) - u(t-K)|_2 / (K U_ref sqrt(n)), |T(t) - T(t-K)|_2 / (K sqrt(n)))
    with n the number of nodes and U_ref the largest wall speed (1 if 0).
    """
    n = cur["ux"].size
    du = np.sqrt(sum(np.sum((cur[c] - prev[c]) ** 2) for c in ("ux", "uy", "uz")))
    dT = np.sqrt(np.sum((cur["T"] - prev["T"]) ** 2))
    uref = u_ref if u_ref > 0 else 1.0
    return max(du / (k_steps * uref * math.sqrt(n)), dT / (k_steps * math.sqrt(n)))
