"""Near-continuum Couette against the Navier-Stokes slip / jump solutions of
Sec. IV (the paper's validation), as tolerance pins of the whole oracle.

NS references (Sec. IV), walls at Y = 0 and Y = 1 moving at -U_w and +U_w:
  U_NS = (2Y - 1) U_w / (1 + 2 Kn)
  T_NS = T_w + zeta Kn K + K Y (1 - Y),  K = 2 Pr a^2 / Cp,  a = U_w/(1+2Kn),
         zeta = 2 gamma / ((gamma + 1) Pr)
which is the printed T_NS with the square restored on U_w in its last term
(Cp = 5/2, Pr = 1 give zeta = 5/4 and reproduce every other printed term).
Shear stress and heat flux of the same solution: sigma_xy = -mu dU/dY,
q_y = -(Cp/Pr) mu dT/dY with mu = sqrt(2/pi) Kn (Kn definition, Sec. IV).
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
FACTS = json.load(open(os.path.join(GOLD, "paper_facts.json")))


def steady(name, kn, ny, U, Tb=1.0, Tt=1.0, tol=1e-11, K=200, max_steps=200000):
    tau = O.tau_from_kn(name, ny, kn)
    c = O.OracleCase(name, 1, ny, tau, wall_b=(-U, 0, Tb), wall_t=(U, 0, Tt))
    prev = c.moments()
    while c.t < max_steps:
        c.run(K)
        cur = c.moments()
        r = O.residual_rate(prev, cur, K, U)
        prev = cur
        if r < tol:
            return c, cur
    raise AssertionError("no steady state")


def ns(Y, kn, U, Tw, Cp, Pr):
    a = U / (1 + 2 * kn)
    K = 2 * Pr * a * a / Cp
    gamma = Cp / (Cp - 1)
    zeta = 2 * gamma / ((gamma + 1) * Pr)
    mu = math.sqrt(2 / math.pi) * kn
    T = Tw + zeta * kn * K + K * Y * (1 - Y)
    return {"u": (2 * Y - 1) * a, "T": T, "sxy": -mu * 2 * a,
            "qy": -(Cp / Pr) * mu * K * (1 - 2 * Y)}


def test_printed_temperature_formula_with_restored_square():
    """The printed T_NS (square restored) equals the closed form above."""
    Cp, Pr, Tw = 2.5, 1.0, 1.0
    for kn in (0.01, 0.1):
        for U in (0.05, 0.2):
            Y = np.linspace(0, 1, 11)
            printed = (kn * (8 * Cp * Tw + 5 * U ** 2) + 8 * Cp * Tw * kn ** 2
                       + 2 * Cp * Tw - 4 * Pr * U ** 2 * (Y - 1) * Y) \
                / (2 * Cp * (2 * kn + 1) ** 2)
            assert np.allclose(printed, ns(Y, kn, U, Tw, Cp, Pr)["T"], rtol=0, atol=1e-15)


@pytest.mark.parametrize("name,ny", [("D2Q17", 32), ("D2Q16", 64)])
def test_isothermal_couette_near_continuum(name, ny):
    U = FACTS["isothermal_couette"]["U_w"]
    kn = 0.01
    c, m = steady(name, kn, ny, U)
    Y = (np.arange(ny) + 0.5) / ny
    ref = ns(Y, kn, U, 1.0, 2.5, 1.0)
    assert np.abs(m["ux"][:, 0] - ref["u"]).max() < 1e-2 * U
    assert abs(m["sxy"][ny // 2, 0] / ref["sxy"] - 1) < 1e-2
    assert np.all(m["T"] == 1.0)


def test_thermal_couette_near_continuum():
    th = FACTS["thermal_couette"]
    U, Tw, Cp, Pr = th["U_w"], th["T_w"], th["Cp"], th["Pr"]
    kn, ny = 0.01, 32
    c, m = steady("D3Q121", kn, ny, U, Tw, Tw)
    Y = (np.arange(ny) + 0.5) / ny
    ref = ns(Y, kn, U, Tw, Cp, Pr)
    rise = ref["T"].max() - Tw
    assert np.abs(m["ux"][:, 0] - ref["u"]).max() < 1e-2 * U
    assert np.abs(m["T"][:, 0] - ref["T"]).max() < 3e-2 * rise
    assert abs(m["sxy"][ny // 2, 0] / ref["sxy"] - 1) < 1e-2
    mid = slice(ny // 4, 3 * ny // 4)
    assert np.abs(m["qy"][mid, 0] - ref["qy"][mid]).max() < 1e-2 * np.abs(ref["qy"]).max()
    # the first node sits in the Knudsen layer: above T_w, near the NS value
    assert abs((m["T"][0, 0] - Tw) / (ref["T"][0] - Tw) - 1) < 0.15


def fitted_slip(m, ny, U):
    Y = (np.arange(ny) + 0.5) / ny
    mid = slice(ny // 4, 3 * ny // 4)
    p = np.polyfit(Y[mid], m["ux"][mid, 0], 1)
    return U - np.polyval(p, 1.0)


def test_slip_follows_ns_at_small_kn_and_grows_with_kn():
    U, ny = 0.05, 32
    _, m = steady("D3Q121", 0.01, ny, U, tol=1e-10)
    assert abs(fitted_slip(m, ny, U) / (U * 2 * 0.01 / 1.02) - 1) < 3e-2
    for name in ("D2Q16", "D2Q17"):
        slips = []
        for kn in (0.02, 0.05, 0.1):
            _, m = steady(name, kn, ny, U, tol=1e-10)
            slips.append(fitted_slip(m, ny, U))
        assert slips[0] < slips[1] < slips[2] < U
    # D2Q16 stays close to the NS slip into the early transition regime
    for kn in (0.05, 0.1):
        _, m = steady("D2Q16", kn, ny, U, tol=1e-10)
        assert abs(fitted_slip(m, ny, U) / (U * 2 * kn / (1 + 2 * kn)) - 1) < 5e-2
