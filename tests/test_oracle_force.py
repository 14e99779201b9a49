"""Pins of the oracle's body force (not in the paper; the force-driven
channel).  Reading: the force term of the Boltzmann equation, -a . grad_c f,
projected on the Hermite polynomials up to the equilibrium's order, is
a . d f^eq / du at fixed rho and T; the trapezoidal change of variable of
Sec. II applied to collision + force then shifts the velocity of the stored
f~ by a/2, its temperature by a^2/(4D), and adds tau/(tau + 1/2) F to the
collision."""
import math

import numpy as np
import pytest

from oracle import lattices as L
from oracle import oracle as O
from paper_1209_5201_amd import workloads as W

LATS = ["D2Q16", "D2Q17", "D3Q121"]


@pytest.mark.parametrize("name", LATS)
def test_uniform_acceleration_between_specular_walls(name):
    """A uniform state between specular walls (no wall friction) under a
    uniform force stays uniform and accelerates exactly:
    u(t) = u0 + a (t + 1/2) (f~(0) = f^eq(u0) carries half a step of force),
    with rho and T unchanged and no shear stress."""
    lat = L.by_name(name)
    a = (2e-3, 0.0, 1e-3 if lat.D == 3 else 0.0)
    ny, nx, t = 8, 2, 40
    u0 = np.stack([np.full((ny, nx), 0.01), np.zeros((ny, nx)), np.zeros((ny, nx))])
    T0 = np.full((ny, nx), 1.05) if lat.thermal else None
    c = O.OracleCase(name, nx, ny, 0.7, (0, 0, 1.0), (0, 0, 1.0), u0=u0, T0=T0,
                     accommodation=(0, 0), force=a)
    m0 = c.moments()
    c.run(t)
    m = c.moments()
    assert np.abs(m["ux"] - (0.01 + a[0] * (t + 0.5))).max() < 1e-14
    assert np.abs(m["uz"] - a[2] * (t + 0.5)).max() < 1e-14
    assert np.abs(m["uy"]).max() < 1e-15
    assert np.abs(m["rho"] - 1).max() < 1e-14
    assert np.abs(m["T"] - m0["T"]).max() < 1e-13
    assert np.abs(m["sxy"]).max() < 1e-15


@pytest.mark.parametrize("name", ["D2Q17", "D3Q121"])
def test_momentum_budget(name):
    """From a random start between specular walls the total momentum of the
    physical f grows by M a every step, exactly (the force term's first
    moment is rho a, its zeroth zero)."""
    lat = L.by_name(name)
    rho, ux, uy, T = W.random_fields(5, 12, seed=4, thermal=lat.thermal)
    a = 1e-3
    c = O.OracleCase(name, 5, 12, 0.8, (0, 0, 1.0), (0, 0, 1.0), rho0=rho,
                     u0=np.stack([ux, uy, 0 * ux]), T0=T, accommodation=(0, 0),
                     force=(a, 0, 0))

    def momentum():
        m = c.moments()
        return (m["rho"] * m["ux"]).sum(), m["rho"].sum()
    p0, M = momentum()
    c.run(25)
    p1, M1 = momentum()
    assert abs(M1 / M - 1) < 1e-14
    assert abs((p1 - p0) / (25 * a * M) - 1) < 1e-12


@pytest.mark.parametrize("name,tol", [("D3Q121", 1e-2), ("D2Q17", 2e-2)])
def test_poiseuille_near_continuum(name, tol):
    """Force-driven channel between diffuse walls at rest, Kn = 0.01: the NS
    solution with the first-order slip length Kn of the Couette pin,
    u(Y) = a/(2 nu) (Y (1 - Y) + Kn); in channel units a/nu =
    a_lat r ny / (sqrt(2/pi) Kn) (a_lat the velocity gained per step).
    Measured deviations: 0.5 % (D3Q121), 1.3 % (D2Q17) of the peak."""
    lat = L.by_name(name)
    ny, kn, a_over_nu = 32, 0.01, 0.4
    a_lat = a_over_nu * math.sqrt(2 / math.pi) * kn / (lat.r * ny)
    c = O.OracleCase(name, 1, ny, O.tau_from_kn(name, ny, kn), (0, 0, 1.0), (0, 0, 1.0),
                     force=(a_lat, 0, 0))
    prev = c.moments()
    while c.t < 400000:
        c.run(1000)
        cur = c.moments()
        if O.residual_rate(prev, cur, 1000, 0.05) < 1e-12:
            break
        prev = cur
    Y = (np.arange(ny) + 0.5) / ny
    ns = a_over_nu / 2 * (Y * (1 - Y) + kn)
    assert np.abs(cur["ux"][:, 0] - ns).max() < tol * ns.max()
