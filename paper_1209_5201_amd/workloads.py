"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
runs.  Only random draws and problem parameters live here: no arithmetic of
the scheme (relaxation times are derived from Kn by each side itself).

The workloads follow the paper's own synthetic Couette set-up (Sec. IV:
plates at Y = 0 and Y = 1 moving in opposite directions at the same speed);
the paper uses no external dataset.
"""
from __future__ import annotations

import numpy as np


def random_fields(nx: int, ny: int, seed: int, thermal: bool, amp: float = 0.02):
    """Smooth-ish random start fields: rho, ux, uy (and T) perturbations."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + amp * rng.standard_normal((ny, nx))
    ux = 0.5 * amp * rng.standard_normal((ny, nx))
    uy = 0.5 * amp * rng.standard_normal((ny, nx))
    T = 1.0 + amp * rng.random((ny, nx)) if thermal else None
    return rho, ux, uy, T


# Isothermal Couette, the lowest-order lattice, FP64.
C1 = dict(name="isothermal Couette", lattices=("D2Q16", "D2Q17"), nx=1, ny=32,
          bottom=(-0.1, 0.0, 1.0), top=(0.1, 0.0, 1.0), kn=0.1, steps=2000)

# Thermal Couette, the highest-order lattice, FP32 vs FP64, run to 1e-8.
C2 = dict(name="thermal Couette", lattice="D3Q121", nx=4, ny=256,
          bottom=(-0.2, 0.0, 1.0), top=(0.2, 0.0, 1.1), kns=(0.01, 0.1, 0.5),
          tol=1e-8, window=100)

# 2-D bulk bandwidth case: D2Q17 (the mid-order lattice), FP32, 2048 x 2048,
# walls at rest at T = 1, Kn = 0.05, rho = 1 + 1e-3 N(0,1), u = 0, 1000 steps.
C3 = dict(name="2D bulk bandwidth", lattice="D2Q17", nx=2048, ny=2048,
          bottom=(0.0, 0.0, 1.0), top=(0.0, 0.0, 1.0), kn=0.05, steps=1000,
          prec="fp32", seed=0, amp=1e-3)

# Reduced-precision storage: D3Q121, 1024 x 1024, walls -+0.1, T = 1,
# Kn = 0.05, rest start, 5000 steps, BF16 / FP16 deviations.
C5 = dict(name="reduced-precision storage", lattice="D3Q121", nx=1024, ny=1024,
          bottom=(-0.1, 0.0, 1.0), top=(0.1, 0.0, 1.0), kn=0.05, steps=5000)


def c3_density(nx: int = 2048, ny: int = 2048, seed: int = 0, amp: float = 1e-3,
               period_x: int | None = None) -> np.ndarray:
    """rho = 1 + amp N(0,1), drawn row-major (y outer).  With period_x the
    draw covers period_x columns and is tiled along x."""
    rng = np.random.default_rng(seed)
    if period_x is None:
        return 1.0 + amp * rng.standard_normal((ny, nx))
    tile = 1.0 + amp * rng.standard_normal((ny, period_x))
    return np.tile(tile, (1, nx // period_x))


def serving_requests(n: int = 1024, seed: int = 1, rate: float = 100.0,
                     ny_range=(16, 512), channel_fraction: float = 0.0):
    """Couette requests: lattice uniform over the three, Ny uniform, Kn
    log-uniform in [0.01, 0.5], U uniform in [0.01, 0.2] (walls -U / +U),
    top-wall T uniform in [1, 1.2] for the thermal lattice (1 otherwise),
    Poisson arrivals at `rate` per second.  With channel_fraction > 0 that
    share of the requests (drawn from a second stream, so the Couette draws
    are unchanged) are force-driven channels instead: walls at rest at
    T = 1, driven by the body force whose no-slip Navier-Stokes peak
    velocity is U (key "umax"; each side derives the force itself)."""
    rng = np.random.default_rng(seed)
    kind = np.random.default_rng([seed, 7])
    names = ("D2Q16", "D2Q17", "D3Q121")
    out = []
    t = 0.0
    for i in range(n):
        lat = names[int(rng.integers(0, 3))]
        ny = int(rng.integers(ny_range[0], ny_range[1] + 1))
        kn = float(np.exp(rng.uniform(np.log(0.01), np.log(0.5))))
        U = float(rng.uniform(0.01, 0.2))
        Tt = float(rng.uniform(1.0, 1.2)) if lat == "D3Q121" else 1.0
        t += float(rng.exponential(1.0 / rate))
        if channel_fraction > 0 and kind.random() < channel_fraction:
            out.append(dict(id=i, lattice=lat, nx=1, ny=ny, kn=kn, bottom=(0.0, 0.0, 1.0),
                            top=(0.0, 0.0, 1.0), umax=U, arrival=t))
        else:
            out.append(dict(id=i, lattice=lat, nx=1, ny=ny, kn=kn, bottom=(-U, 0.0, 1.0),
                            top=(U, 0.0, Tt), arrival=t))
    return out
