"""Pins of the oracle's velocity sets (the tables the paper omits, Sec. IV).

The pins are independent of how the oracle solves for the tables:
  * every monomial (all of them, odd ones included, not only the symmetry
    classes the solver uses) is checked against the unit-Gaussian moment;
  * arbitrary polynomials are integrated against numpy's Gauss-Hermite rule;
  * D2Q17 is compared with a hand-derived closed form;
  * N = 3 ghost layers for D2Q17 is the number the paper prints (Sec. III).
"""
import itertools
import json
import math
import os

import mpmath
import numpy as np
import pytest

from oracle import lattices as L

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gauss_moment(m):
    v = 1.0
    for k in m:
        if k % 2:
            return 0.0
        v *= float(mpmath.fac2(k - 1)) if k > 0 else 1.0
    return v


def lattice_moment(lat, m):
    c = lat.r * lat.e[:, :lat.D].astype(np.float64)
    return float(np.sum(lat.w * np.prod(c ** np.array(m), axis=1)))


@pytest.mark.parametrize("name,Q,D,N", [("D2Q16", 16, 2, 3), ("D2Q17", 17, 2, 3),
                                        ("D3Q121", 121, 3, 3)])
def test_shape_positivity_symmetry(name, Q, D, N):
    lat = L.by_name(name)
    assert lat.Q == Q and lat.D == D and lat.N == N
    assert np.all(lat.w > 0)
    assert abs(np.sum(lat.w) - 1.0) < 1e-15
    rows = {tuple(v) for v in lat.e}
    assert len(rows) == Q
    # closed under reflection of each axis (the wall mirror e_y -> -e_y in particular)
    for v in lat.e:
        for ax in range(D):
            m = list(v)
            m[ax] = -m[ax]
            assert tuple(m) in rows


def test_d2q17_ghost_layers_match_paper():
    facts = json.load(open(os.path.join(GOLD, "paper_facts.json")))
    assert L.d2q17().N == facts["ghost_layers_d2q17"]["value"]


@pytest.mark.parametrize("name", ["D2Q17", "D3Q121"])
def test_all_monomials_to_degree(name):
    lat = L.by_name(name)
    worst = 0.0
    for m in itertools.product(range(lat.degree + 1), repeat=lat.D):
        if sum(m) > lat.degree:
            continue
        got, want = lattice_moment(lat, m), gauss_moment(m)
        worst = max(worst, abs(got - want) / max(1.0, abs(want)))
    assert worst < 2e-14, worst


@pytest.mark.parametrize("name", ["D2Q17", "D3Q121"])
def test_degree_is_sharp(name):
    """The next even degree is not integrated exactly (the degree is the
    lattice's, not an accident of the check)."""
    lat = L.by_name(name)
    d = lat.degree + 1
    worst = 0.0
    for m in itertools.product(range(d + 1), repeat=lat.D):
        if sum(m) == d:
            worst = max(worst, abs(lattice_moment(lat, m) - gauss_moment(m)))
    assert worst > 1e-3


def test_d2q16_tensor_rule():
    """Builder's D2Q16: exact for every monomial with exponents <= 3 per axis."""
    lat = L.d2q16()
    for m in itertools.product(range(4), repeat=2):
        assert abs(lattice_moment(lat, m) - gauss_moment(m)) < 1e-15
    # largest attainable 4th moment of a {+-1,+-3} rule with exact M0, M2
    assert abs(lattice_moment(lat, (4, 0)) - 25.0 / 9.0) < 1e-14


@pytest.mark.parametrize("name", ["D2Q17", "D3Q121"])
def test_random_polynomials_against_gauss_hermite(name):
    """Integrate random polynomials of total degree <= lattice degree with
    numpy's probabilists' Gauss-Hermite rule (a library routine)."""
    lat = L.by_name(name)
    x, wx = np.polynomial.hermite_e.hermegauss(12)
    wx = wx / np.sqrt(2 * np.pi)
    rng = np.random.default_rng(7)
    c = lat.r * lat.e[:, :lat.D].astype(np.float64)
    exps = [m for m in itertools.product(range(lat.degree + 1), repeat=lat.D)
            if sum(m) <= lat.degree]
    for _ in range(5):
        coef = rng.standard_normal(len(exps))
        lat_val = sum(k * np.sum(lat.w * np.prod(c ** np.array(m), axis=1))
                      for k, m in zip(coef, exps))
        gh = 0.0
        for k, m in zip(coef, exps):
            term = k
            for i in range(lat.D):
                term *= np.sum(wx * x ** m[i])
            gh += term
        assert abs(lat_val - gh) < 1e-11 * max(1.0, abs(gh))


def test_d2q17_closed_form():
    gold = json.load(open(os.path.join(GOLD, "d2q17_closed_form.json")))
    mpmath.mp.dps = 30
    env = {"sqrt": mpmath.sqrt}
    lat = L.d2q17()
    r2 = float(eval(gold["r2"], env))
    assert abs(lat.r ** 2 - r2) < 4e-16 * r2
    for key, expr in gold["w"].items():
        a, b = (int(t) for t in key.split(","))
        want = float(eval(expr, env))
        sel = [i for i, v in enumerate(lat.e)
               if sorted(map(abs, v[:2])) == sorted((a, b))]
        assert len(sel) == (1 if (a, b) == (0, 0) else 4)
        for i in sel:
            assert abs(lat.w[i] - want) <= 2e-16 * want + 1e-20


def test_d3q121_y_marginal_is_1d_degree9_rule():
    """Summing D3Q121 over x and z leaves a 7-point 1-D rule on
    r*{0,+-1,+-2,+-3}; degree 9 in 3-D forces it to be degree 9 in 1-D."""
    lat = L.d3q121()
    marg = {k: float(np.sum(lat.w[lat.e[:, 1] == k])) for k in range(-3, 4)}
    for p in range(10):
        s = sum(wk * (lat.r * k) ** p for k, wk in marg.items())
        assert abs(s - gauss_moment((p,))) < 1e-13 * max(1, gauss_moment((p,)))
