"""Pins of the oracle's truncated Maxwellian, Eq. (eq:feq).

Independent references:
  * pointwise: the printed polynomial must equal the Hermite series of the
    Maxwellian truncated at the same order, sum_k a^(k) : H^(k)(c) / k!,
    with the tensor Hermite polynomials written from their textbook
    definition and the coefficients a^(k) = E[H^(k)(c)] over the Maxwellian
    obtained by numpy's Gauss-Hermite rule;
  * moments: on each lattice, sum_a f^eq_a c_a^m must equal the Maxwellian's
    moment (Gauss-Hermite again) for every monomial up to the order the
    lattice and the truncation can both carry (Sec. II).
"""
import itertools

import numpy as np
import pytest

from oracle import lattices as L
from oracle import oracle as O


def hermite_tensors(c, kmax):
    """H^(0..kmax)(c) for one point c (length D), probabilists' convention."""
    D = c.shape[0]
    d = np.eye(D)
    H = [np.array(1.0), c.copy()]
    H.append(np.einsum("i,j->ij", c, c) - d)
    H.append(np.einsum("i,j,k->ijk", c, c, c)
             - (np.einsum("i,jk->ijk", c, d) + np.einsum("j,ik->ijk", c, d)
                + np.einsum("k,ij->ijk", c, d)))
    cc = np.einsum("i,j->ij", c, c)
    H.append(np.einsum("i,j,k,l->ijkl", c, c, c, c)
             - (np.einsum("ij,kl->ijkl", cc, d) + np.einsum("ik,jl->ijkl", cc, d)
                + np.einsum("il,jk->ijkl", cc, d) + np.einsum("jk,il->ijkl", cc, d)
                + np.einsum("jl,ik->ijkl", cc, d) + np.einsum("kl,ij->ijkl", cc, d))
             + (np.einsum("ij,kl->ijkl", d, d) + np.einsum("ik,jl->ijkl", d, d)
                + np.einsum("il,jk->ijkl", d, d)))
    return H[:kmax + 1]


def gh_points(D, n=10):
    x, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / np.sqrt(2 * np.pi)
    pts, wts = [], []
    for idx in itertools.product(range(n), repeat=D):
        pts.append([x[i] for i in idx])
        wts.append(np.prod([w[i] for i in idx]))
    return np.array(pts), np.array(wts)


def maxwellian_hermite_coeffs(u, T, kmax):
    D = u.shape[0]
    z, wz = gh_points(D)
    a = None
    for zi, wi in zip(z, wz):
        H = hermite_tensors(u + np.sqrt(T) * zi, kmax)
        a = [wi * h for h in H] if a is None else [ak + wi * h for ak, h in zip(a, H)]
    return a


def series(c, a, kmax):
    H = hermite_tensors(c, kmax)
    s, fact = 0.0, 1.0
    for k in range(kmax + 1):
        fact *= max(k, 1)
        s += np.sum(a[k] * H[k]) / fact
    return s


@pytest.mark.parametrize("name", ["D2Q17", "D3Q121", "D2Q16"])
def test_feq_equals_truncated_hermite_series(name):
    lat = L.by_name(name)
    rng = np.random.default_rng(11)
    for _ in range(4):
        u = np.zeros(3)
        u[:lat.D] = rng.uniform(-0.3, 0.3, lat.D)
        T = rng.uniform(0.8, 1.25) if lat.thermal else 1.0
        a = maxwellian_hermite_coeffs(u[:lat.D], T, lat.eq_order)
        g = O.geq(lat, u, T)
        for i in range(lat.Q):
            c = lat.r * lat.e[i, :lat.D].astype(float)
            want = lat.w[i] * series(c, a, lat.eq_order)
            assert abs(g[i] - want) < 1e-14 * max(lat.w[i], 1e-3), (i, g[i], want)


def maxwellian_moment(u, T, m):
    z, wz = gh_points(len(u))
    c = u + np.sqrt(T) * z
    return float(np.sum(wz * np.prod(c ** np.array(m), axis=1)))


@pytest.mark.parametrize("name,order", [("D2Q17", 3), ("D3Q121", 4)])
def test_feq_moments_match_maxwellian(name, order):
    lat = L.by_name(name)
    rng = np.random.default_rng(3)
    cvec = lat.r * lat.e[:, :lat.D].astype(float)
    for _ in range(3):
        u = np.zeros(3)
        u[:lat.D] = rng.uniform(-0.25, 0.25, lat.D)
        T = rng.uniform(0.85, 1.2) if lat.thermal else 1.0
        rho = rng.uniform(0.9, 1.1)
        feq = rho * O.geq(lat, u, T)
        for m in itertools.product(range(order + 1), repeat=lat.D):
            if sum(m) > order:
                continue
            got = float(np.sum(feq * np.prod(cvec ** np.array(m), axis=1)))
            want = rho * maxwellian_moment(u[:lat.D], T, m)
            assert abs(got - want) < 1e-13, (m, got, want)


def test_d2q16_second_order_conserves_mass_momentum_and_shear():
    lat = L.d2q16()
    cvec = lat.r * lat.e[:, :2].astype(float)
    for u in ([0.1, -0.05], [-0.2, 0.15]):
        uu = np.array(u + [0.0])
        feq = O.geq(lat, uu)
        assert abs(feq.sum() - 1.0) < 1e-15
        assert np.allclose(feq @ cvec, u, atol=1e-15, rtol=0)
        assert abs(np.sum(feq * cvec[:, 0] * cvec[:, 1]) - u[0] * u[1]) < 1e-15


def test_rest_equilibrium_is_the_weights():
    for name in ("D2Q16", "D2Q17", "D3Q121"):
        lat = L.by_name(name)
        assert np.allclose(O.geq(lat, (0, 0, 0), 1.0), lat.w, rtol=0, atol=1e-17)
