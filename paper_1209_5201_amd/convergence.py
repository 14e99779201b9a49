"""Grid-convergence study of the thermal Couette flow (Sec. IV).

Solves the Couette problem at several resolutions N_G (rows across the
channel) to a steady state on the GPU, takes the finest as the reference
U_Delta, T_Delta, and forms the global relative errors of Sec. IV:

    E_U = sqrt( sum_j (U_j - U_Delta(Y_j))^2 / sum_j U_Delta(Y_j)^2 )
    E_T = sqrt( sum_j (T_j - T_Delta(Y_j))^2 / sum_j (T_Delta(Y_j) - T_w)^2 )

with the reference interpolated (cubic) onto the coarse nodes
Y_j = (j + 1/2) / N_G.  The observed order is the least-squares slope of
log E against log N_G.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm as _l


def steady_profile(lattice: str, ny: int, kn: float, U: float, Tw: float, prec: str = "fp64",
                   tol: float = 1e-11, window: int = 1000, max_steps: int = 5_000_000):
    ch = _l.Channel(lattice, 1, ny, 0.0, (-U, 0.0, Tw), (U, 0.0, Tw), prec=prec, kn=kn)
    steps = ch.run_to_residual(tol, window=window, max_steps=max_steps)
    m = ch.moments()
    r = ch.residual()
    ch.close()
    return {"ux": m["ux"][:, 0], "T": m["T"][:, 0], "steps": steps, "residual": r}


def cubic_interp(xs, ys, x):
    """Piecewise cubic (Catmull-Rom style, four nearest nodes) interpolation
    of a smooth profile sampled at ascending xs."""
    xs = np.asarray(xs)
    ys = np.asarray(ys)
    out = np.empty_like(np.asarray(x, dtype=np.float64))
    for k, xv in enumerate(np.atleast_1d(x)):
        i = int(np.clip(np.searchsorted(xs, xv) - 2, 0, len(xs) - 4))
        xx, yy = xs[i:i + 4], ys[i:i + 4]
        v = 0.0
        for a in range(4):           # Lagrange form on the four nodes
            term = yy[a]
            for b in range(4):
                if b != a:
                    term *= (xv - xx[b]) / (xx[a] - xx[b])
            v += term
        out[k] = v
    return out


def convergence_study(grids=(20, 50, 100, 200), reference=500, lattice="D3Q121", kn=0.01,
                      U=0.2, Tw=1.0, prec="fp64", tol=1e-11):
    ref = steady_profile(lattice, reference, kn, U, Tw, prec, tol)
    Yr = (np.arange(reference) + 0.5) / reference
    rows = []
    for n in grids:
        p = steady_profile(lattice, n, kn, U, Tw, prec, tol)
        Y = (np.arange(n) + 0.5) / n
        Ur = cubic_interp(Yr, ref["ux"], Y)
        Tr = cubic_interp(Yr, ref["T"], Y)
        EU = math.sqrt(np.sum((p["ux"] - Ur) ** 2) / np.sum(Ur ** 2))
        ET = math.sqrt(np.sum((p["T"] - Tr) ** 2) / np.sum((Tr - Tw) ** 2))
        rows.append({"N_G": n, "E_U": EU, "E_T": ET, "steps": p["steps"]})
    lg = np.log([r["N_G"] for r in rows])
    order_u = -np.polyfit(lg, np.log([r["E_U"] for r in rows]), 1)[0]
    order_t = -np.polyfit(lg, np.log([r["E_T"] for r in rows]), 1)[0]
    return {"rows": rows, "reference": reference, "reference_steps": ref["steps"],
            "order_U": float(order_u), "order_T": float(order_t)}
