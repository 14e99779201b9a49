"""Pins of the oracle's local relaxation time (end of Sec. II: for thermal
problems tau may follow the local temperature).  Reading: the
non-dimensional tau = mu / p of Sec. II with p = rho T and a power-law
viscosity mu = T^w, i.e. tau_node = tau T^(w - 1) / rho; the stress and heat
flux conversion of Sec. II then uses each node's own tau."""
import numpy as np
import pytest

from oracle import oracle as O

LAT = "D3Q121"


def steady(case, uref, window=500, tol=1e-12, max_steps=200000):
    prev = case.moments()
    while case.t < max_steps:
        case.run(window)
        cur = case.moments()
        if O.residual_rate(prev, cur, window, uref) < tol:
            return cur
        prev = cur
    raise AssertionError("no steady state")


@pytest.mark.parametrize("w", [None, 0.5, 1.0])
def test_conduction_follows_the_viscosity_law(w):
    """Walls at rest at T = 1 and 1.5, near continuum (Kn = 0.01): the
    energy equation reduces to d/dy (k dT/dy) = 0 with BGK's conductivity
    k proportional to p tau = T^w, so T^(w + 1) is linear across the channel
    and the mid-channel temperature is ((1 + 1.5^(w+1)) / 2)^(1/(w+1)).
    Constant tau gives k proportional to p, uniform: the w = 0 profile."""
    ny, Tt = 32, 1.5
    c = O.OracleCase(LAT, 1, ny, O.tau_from_kn(LAT, ny, 0.01), (0, 0, 1.0), (0, 0, Tt),
                     viscosity_exp=w)
    T = steady(c, 0.0)["T"][:, 0]
    Y = (np.arange(ny) + 0.5) / ny
    we = 0.0 if w is None else w

    def nonlinearity(e):
        z = T ** (e + 1.0)
        return np.abs(z - np.polyval(np.polyfit(Y, z, 1), Y)).max() / np.ptp(z)

    # the closed forms for w = 0, 0.5, 1 are 1.2500, 1.2626, 1.2748; the
    # O(Kn) temperature jumps at the walls shift the profile by ~2e-3
    mid = ((1 + Tt ** (we + 1)) / 2) ** (1 / (we + 1))
    assert abs(np.interp(0.5, Y, T) - mid) < 3e-3
    assert nonlinearity(we) < 6e-3
    for other in (0.0, 0.5, 1.0):
        if other != we:
            assert nonlinearity(other) > 1.5e-2


@pytest.mark.parametrize("w", [0.5, 1.0])
def test_shear_stress_uses_each_nodes_relaxation_time(w):
    """Couette flow across a temperature difference (walls -+0.1, T 1 and
    1.5): momentum conservation makes the shear stress uniform across the
    bulk.  The conversion f - f^eq = tau/(tau + 1/2) (f~ - f^eq) of Sec. II
    must take each node's tau: with the reference tau everywhere the bulk
    stress would vary by 6-19 %."""
    ny = 32
    c = O.OracleCase(LAT, 1, ny, O.tau_from_kn(LAT, ny, 0.01), (-0.1, 0, 1.0), (0.1, 0, 1.5),
                     viscosity_exp=w)
    s = steady(c, 0.1)["sxy"][3:-3, 0]
    assert np.ptp(s) / abs(s.mean()) < 1.5e-2
