"""Pins of the oracle's stream-collide step and diffuse wall (Eq. (eq:scheme),
Sec. III, Eq. (eq:dkboundary)) by invariants and closed forms the paper's
equations imply.
"""
import math

import numpy as np
import pytest

from oracle import lattices as L
from oracle import oracle as O

LATS = ["D2Q16", "D2Q17", "D3Q121"]


@pytest.mark.parametrize("name", LATS)
def test_rest_state_is_invariant(name):
    """Walls at rest, T_w = 1, f~ = w: the diffuse wall gives back exactly
    what arrives, the collision leaves an equilibrium alone."""
    c = O.OracleCase(name, 3, 8, 0.7)
    w = c.lat.w
    c.run(25)
    assert np.abs(c.f - w).max() < 1e-14


@pytest.mark.parametrize("name,T", [("D2Q16", 1.0), ("D2Q17", 1.0), ("D3Q121", 1.15)])
def test_uniform_translation_is_invariant(name, T):
    """Both walls move tangentially at U with T_w = T and the gas starts at
    f^eq(1, U, T): zero normal momentum makes the pooled mass equal the
    re-emitted one, so nothing changes."""
    U = (0.08, 0.0, -0.05) if name == "D3Q121" else (0.08, 0.0, 0.0)
    wall = (U[0], U[2], T)
    u0 = np.zeros((3, 6, 2))
    for i in range(3):
        u0[i] = U[i]
    c = O.OracleCase(name, 2, 6, 0.9, wall_b=wall, wall_t=wall, u0=u0,
                     T0=np.full((6, 2), T))
    f0 = c.f.copy()
    c.run(20)
    assert np.abs(c.f - f0).max() < 2e-15


@pytest.mark.parametrize("name", LATS)
def test_mass_conservation_and_zero_wall_flux_each_step(name):
    rng = np.random.default_rng(5)
    nx, ny = 4, 10
    rho0 = 1.0 + 0.05 * rng.standard_normal((ny, nx))
    u0 = 0.05 * rng.standard_normal((3, ny, nx))
    if name != "D3Q121":
        u0[2] = 0
    T0 = 1.0 + 0.05 * rng.random((ny, nx)) if name == "D3Q121" else None
    wt = 1.1 if name == "D3Q121" else 1.0
    c = O.OracleCase(name, nx, ny, 0.6, wall_b=(-0.1, 0.0, 1.0),
                     wall_t=(0.1, 0.0, wt), rho0=rho0, u0=u0, T0=T0)
    m_prev = c.mass()
    for _ in range(30):
        flux = c.run(1, record_flux=True)[0]
        m = c.mass()
        assert abs(m - m_prev) <= 1e-13 * m_prev
        m_prev = m
        assert flux[0] > 0 and flux[2] > 0
        assert abs(flux[0] - flux[1]) <= 1e-14 * flux[0]
        assert abs(flux[2] - flux[3]) <= 1e-14 * flux[2]


def collisionless_closed_form(lat, ub, ut):
    """Steady state with no collisions, x-invariant, rest start: each
    population with e_y > 0 is A_b g^b, each with e_y < 0 is A_t g^t, e_y = 0
    keeps its start value; zero net flux and total mass fix A_b, A_t."""
    gb = O.geq(lat, (ub, 0, 0), 1.0)
    gt = O.geq(lat, (ut, 0, 0), 1.0)
    ey = lat.e[:, 1]
    Db = np.sum(ey[ey > 0] * gb[ey > 0])
    Dt = np.sum(-ey[ey < 0] * gt[ey < 0])
    A = np.array([[Db, -Dt], [gb[ey > 0].sum(), gt[ey < 0].sum()]])
    Ab, At = np.linalg.solve(A, [0.0, 1.0 - lat.w[ey == 0].sum()])
    return np.where(ey > 0, Ab * gb, np.where(ey < 0, At * gt, lat.w))


@pytest.mark.parametrize("name,steps,tol", [("D2Q16", 400, 1e-15),
                                            ("D2Q17", 60000, 1e-12),
                                            ("D3Q121", 12000, 3e-13)])
def test_collisionless_limit_matches_closed_form(name, steps, tol):
    # tol: the transient's rounding drift of the total mass (~1e-12 relative
    # for D3Q121) sets the floor
    lat = L.by_name(name)
    c = O.OracleCase(name, 1, 12, math.inf, wall_b=(-0.1, 0, 1.0),
                     wall_t=(0.1, 0, 1.0))
    c.run(steps)
    want = collisionless_closed_form(lat, -0.1, 0.1)
    assert np.abs(c.f[:, 0, :] - want).max() < tol


def test_collisionless_shear_stress_values():
    """Same closed form, as a free-molecular shear stress (U = 0.1):
    sigma_xy = sum_a f_a c_x c_y at the steady state."""
    want = {"D2Q16": -0.0894427191, "D2Q17": -0.0597147711, "D3Q121": -0.0694789146}
    for name, val in want.items():
        lat = L.by_name(name)
        f = collisionless_closed_form(lat, -0.1, 0.1)
        c = lat.r * lat.e.astype(float)
        rho = f.sum()
        ux = (f @ c[:, 0]) / rho
        s = np.sum(f * (c[:, 0] - ux) * c[:, 1])
        assert abs(s - val) < 1e-10
        # and the oracle's own moment output agrees on that state
        case = O.OracleCase(name, 1, 8, math.inf)
        case.f[:] = f
        assert abs(case.moments()["sxy"].mean() - val) < 1e-10


@pytest.mark.parametrize("name", LATS)
def test_mirror_symmetry(name):
    """Walls -U / +U at equal T: the problem is invariant under a half-turn
    about the channel axis (x -> -x, y -> -y), so u_x and u_y are odd and rho,
    T, sigma_xy even about mid-channel; u_z vanishes (z mirror)."""
    ny = 14
    tau = O.tau_from_kn(name, ny, 0.05)
    c = O.OracleCase(name, 1, ny, tau, wall_b=(-0.1, 0, 1.0), wall_t=(0.1, 0, 1.0))
    c.run(300)
    m = c.moments()
    assert np.abs(m["ux"][:, 0] + m["ux"][::-1, 0]).max() < 1e-14
    assert np.abs(m["rho"][:, 0] - m["rho"][::-1, 0]).max() < 1e-14
    assert np.abs(m["T"][:, 0] - m["T"][::-1, 0]).max() < 1e-14
    assert np.abs(m["sxy"][:, 0] - m["sxy"][::-1, 0]).max() < 1e-14
    assert np.abs(m["uy"][:, 0] + m["uy"][::-1, 0]).max() < 1e-15
    assert np.abs(m["uz"]).max() < 1e-16


@pytest.mark.parametrize("name", LATS)
def test_x_translation_equivariance(name):
    """Periodic x: shifting the start field by s columns shifts the result."""
    rng = np.random.default_rng(9)
    nx, ny, s = 5, 8, 2
    rho0 = 1.0 + 0.02 * rng.standard_normal((ny, nx))
    a = O.OracleCase(name, nx, ny, 0.8, wall_b=(-0.05, 0, 1.0), wall_t=(0.1, 0, 1.0),
                     rho0=rho0)
    b = O.OracleCase(name, nx, ny, 0.8, wall_b=(-0.05, 0, 1.0), wall_t=(0.1, 0, 1.0),
                     rho0=np.roll(rho0, s, axis=1))
    a.run(12)
    b.run(12)
    assert np.abs(np.roll(a.f, s, axis=1) - b.f).max() < 1e-15


@pytest.mark.parametrize("name", LATS)
def test_x_invariant_field_matches_single_column(name):
    """nx columns of an x-invariant problem reproduce the nx = 1 run."""
    tau = 1.3
    a = O.OracleCase(name, 1, 9, tau, wall_b=(-0.1, 0, 1.0), wall_t=(0.1, 0, 1.0))
    b = O.OracleCase(name, 4, 9, tau, wall_b=(-0.1, 0, 1.0), wall_t=(0.1, 0, 1.0))
    a.run(20)
    b.run(20)
    for x in range(4):
        assert np.abs(b.f[:, x, :] - a.f[:, 0, :]).max() < 1e-15


def post_collision(case):
    m = case.moments()
    om = 1.0 / (case.tau + 0.5)
    fs = np.empty_like(case.f)
    for j in range(case.ny):
        u = (m["ux"][j, 0], m["uy"][j, 0], m["uz"][j, 0])
        g = m["rho"][j, 0] * O.geq(case.lat, u, m["T"][j, 0])
        fs[j, 0] = case.f[j, 0] - om * (case.f[j, 0] - g)
    return fs, m


def interface_momentum_flux(case):
    """x-momentum carried across each interior interface between rows j and
    j+1 in one step, by the post-collision populations."""
    lat = case.lat
    fs, m = post_collision(case)
    cx = lat.r * lat.e[:, 0]
    ey = lat.e[:, 1]
    P = []
    for j in range(lat.N - 1, case.ny - lat.N):
        s = 0.0
        for a in range(lat.Q):
            if ey[a] > 0:
                s += cx[a] * sum(fs[j - k, 0, a] for k in range(ey[a]))
            elif ey[a] < 0:
                s -= cx[a] * sum(fs[j + 1 + k, 0, a] for k in range(-ey[a]))
        P.append(s)
    return np.array(P), m


@pytest.mark.parametrize("name,kn,ny", [("D2Q17", 0.1, 16), ("D2Q16", 0.1, 16),
                                        ("D3Q121", 0.05, 16)])
def test_steady_couette_momentum_flux_is_uniform(name, kn, ny):
    """At steady state the x-momentum flux across every row interface is the
    same (momentum balance of each row); the mid-channel shear stress output
    equals that flux times dx/dt = r up to the curvature of f across rows."""
    tau = O.tau_from_kn(name, ny, kn)
    c = O.OracleCase(name, 1, ny, tau, wall_b=(-0.1, 0, 1.0), wall_t=(0.1, 0, 1.0))
    c.run(12000)
    P, m = interface_momentum_flux(c)
    assert (P.max() - P.min()) < 1e-12 * abs(P).max()
    smid = m["sxy"][ny // 2, 0]
    assert abs(smid - c.lat.r * P.mean()) < 2e-3 * abs(smid)


@pytest.mark.parametrize("name", LATS)
def test_positivity_is_kept(name):
    ny = 12
    tau = O.tau_from_kn(name, ny, 0.05)
    wt = 1.2 if name == "D3Q121" else 1.0
    c = O.OracleCase(name, 2, ny, tau, wall_b=(-0.2, 0, 1.0), wall_t=(0.2, 0, wt))
    assert np.all(O.geq(name, (0.2, 0, 0), wt) > 0)
    for _ in range(10):
        c.run(40)
        assert c.f.min() > 0
