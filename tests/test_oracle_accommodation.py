"""Pins of the oracle's generic scattering wall (Sec. III: f^O = sum R f^I
with the normalised, non-negative kernel R), used with the Maxwell-type
kernel R = alpha R_D + (1 - alpha) R_S: alpha = 1 is the paper's diffuse
wall of Eq. (eq:dkboundary), alpha = 0 specular reflection."""
import math

import numpy as np
import pytest

from oracle import lattices as L
from oracle import oracle as O

LATS = ["D2Q16", "D2Q17", "D3Q121"]


def mirror_index(lat):
    idx = {tuple(v): i for i, v in enumerate(lat.e)}
    return np.array([idx[(v[0], -v[1], v[2])] for v in lat.e])


def periodic_reference(lat, f0, tau, steps):
    """Wall-free reference: nx = 1, rows periodic in y, written directly
    from Eq. (eq:scheme) with the (separately pinned) equilibrium."""
    f = f0.copy()
    om = 1.0 / (tau + 0.5)
    c = lat.r * lat.e.astype(float)
    for _ in range(steps):
        fs = np.empty_like(f)
        for j in range(f.shape[0]):
            rho = f[j].sum()
            u = f[j] @ c / rho
            T = (f[j] @ np.sum((c - u) ** 2, axis=1)) / (rho * lat.D) if lat.thermal else 1.0
            fs[j] = f[j] - om * (f[j] - rho * O.geq(lat, u, T))
        for q in range(lat.Q):
            f[:, q] = np.roll(fs[:, q], lat.e[q, 1])
    return f


@pytest.mark.parametrize("name", LATS)
def test_specular_walls_are_mirrors(name):
    """With alpha = 0 both walls reflect specularly: the channel evolves
    exactly like the lower half of a wall-free periodic channel of twice the
    height started from the field and its mirror image."""
    lat = L.by_name(name)
    ny, tau, steps = 8, 0.7, 12
    rng = np.random.default_rng(21)
    rho0 = 1 + 0.03 * rng.standard_normal((ny, 1))
    u0 = 0.04 * rng.standard_normal((3, ny, 1))
    if lat.D == 2:
        u0[2] = 0
    T0 = 1 + 0.03 * rng.random((ny, 1)) if lat.thermal else None
    wall = (0.13, 0.0, 1.1 if lat.thermal else 1.0)   # ignored by specular walls
    c = O.OracleCase(name, 1, ny, tau, wall, wall, rho0=rho0, u0=u0, T0=T0,
                     accommodation=(0.0, 0.0))
    m = mirror_index(lat)
    full = np.concatenate([c.f[:, 0, :], c.f[::-1, 0, :][:, m]], axis=0)
    ref = periodic_reference(lat, full, tau, steps)
    c.run(steps)
    assert np.abs(c.f[:, 0, :] - ref[:ny]).max() < 1e-14


@pytest.mark.parametrize("name", LATS)
def test_mass_and_zero_net_flux_for_any_accommodation(name):
    rng = np.random.default_rng(2)
    rho0 = 1 + 0.02 * rng.standard_normal((10, 3))
    c = O.OracleCase(name, 3, 10, 0.6, (-0.1, 0, 1.0), (0.1, 0, 1.0), rho0=rho0,
                     accommodation=(0.3, 0.8))
    m0 = c.mass()
    for _ in range(20):
        fl = c.run(1, record_flux=True)[0]
        assert abs(c.mass() - m0) < 1e-13 * m0
        assert abs(fl[0] - fl[1]) < 1e-14 * fl[0] and abs(fl[2] - fl[3]) < 1e-14 * fl[2]
        m0 = c.mass()


@pytest.mark.parametrize("name", ["D2Q16", "D3Q121"])
def test_collisionless_closed_form_with_accommodation(name):
    """No collisions, x-invariant, rest start, both walls alpha: velocities
    leaving the bottom wall carry [A_b g^b + (1 - alpha) A_t P g^t] / (2 - alpha)
    (P: normal reversal), the amplitudes A_b, A_t being those of the fully
    diffuse case (zero net flux, total mass)."""
    lat = L.by_name(name)
    alpha, U = 0.6, 0.1
    c = O.OracleCase(name, 1, 12, math.inf, (-U, 0, 1.0), (U, 0, 1.0),
                     accommodation=(alpha, alpha))
    c.run(20000)
    gb, gt = O.geq(lat, (-U, 0, 0), 1.0), O.geq(lat, (U, 0, 0), 1.0)
    ey = lat.e[:, 1]
    P = mirror_index(lat)
    Db, Dt = np.sum(ey[ey > 0] * gb[ey > 0]), np.sum(-ey[ey < 0] * gt[ey < 0])
    A = np.array([[Db, -Dt], [gb[ey > 0].sum(), gt[ey < 0].sum()]])
    Ab, At = np.linalg.solve(A, [0.0, 1.0 - lat.w[ey == 0].sum()])
    up = (Ab * gb + (1 - alpha) * At * gt[P]) / (2 - alpha)
    down = (At * gt + (1 - alpha) * Ab * gb[P]) / (2 - alpha)
    want = np.where(ey > 0, up, np.where(ey < 0, down, lat.w))
    assert np.abs(c.f[:, 0, :] - want).max() < 3e-13


def test_maxwell_slip_near_continuum():
    """Sec. IV's NS slip solution with Maxwell's slip coefficient
    (2 - alpha)/alpha: U = (2Y - 1) U_w / (1 + 2 Kn (2 - alpha)/alpha)."""
    name, ny, kn, U, alpha = "D3Q121", 32, 0.01, 0.05, 0.5
    c = O.OracleCase(name, 1, ny, O.tau_from_kn(name, ny, kn), (-U, 0, 1.0), (U, 0, 1.0),
                     accommodation=(alpha, alpha))
    prev = c.moments()
    while c.t < 100000:
        c.run(200)
        cur = c.moments()
        if O.residual_rate(prev, cur, 200, U) < 1e-11:
            break
        prev = cur
    Y = (np.arange(ny) + 0.5) / ny
    s = (2 - alpha) / alpha
    ns = (2 * Y - 1) * U / (1 + 2 * kn * s)
    assert np.abs(cur["ux"][:, 0] - ns).max() < 1.2e-2 * U
    mid = slice(ny // 4, 3 * ny // 4)
    fit = np.polyfit(Y[mid], cur["ux"][mid, 0], 1)
    slip = U - np.polyval(fit, 1.0)
    assert abs(slip / (U * 2 * kn * s / (1 + 2 * kn * s)) - 1) < 0.1
