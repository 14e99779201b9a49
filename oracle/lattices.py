"""Discrete velocity sets for the oracle.

TEST INFRASTRUCTURE ONLY.  Nothing under ``oracle/`` is part of the product
path; only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it.

The paper names three lattices (D2Q17, D2Q16, D3Q121; Sec. IV) but omits
their tables (Sec. IV: "details ... omitted"), so the oracle derives them
from the defining property of a lattice ``xi = {c_a, w_a}`` (Sec. II, the
notation introduced before Eq. (eq:feq)): with ``c_a = r * e_a`` on integer
vectors ``e_a``, the weighted sums ``sum_a w_a c_a^m`` must equal the moments
of the unit Gaussian for every monomial ``m`` up to the quadrature degree.

Readings (each recorded in the design notes):

* D2Q17 - shells (0,0),(1,0),(1,1),(2,2),(3,0), degree 7.  The only positive
  solution; its largest wall-normal component 3 matches N = 3 given for this
  lattice in Sec. III.
* D3Q121 - degree 9 on the shells (000),(100),(111),(210),(220),(222),(300),
  (311),(320),(333): one of several positive degree-9 121-velocity rules.
* D2Q16 - tensor product of the 1-D set {+-1, +-3} with weights 9/20, 1/20
  and r = sqrt(5)/3 (the choice that reproduces the 0th and 2nd moments and
  maximises the 4th).  Used with the 2nd-order equilibrium (Sec. II: the
  second-order truncation).  This table is a labelled construction: the
  paper's own D2Q16 cannot be recovered from the text.

The derivation works in 40-digit arithmetic (mpmath) and rounds to float64
once at the end.
"""
from __future__ import annotations

import functools
import itertools
from dataclasses import dataclass

import mpmath
import numpy as np


@dataclass(frozen=True)
class OracleLattice:
    name: str
    D: int                 # velocity-space dimension (enters T and f^eq)
    e: np.ndarray          # (Q, 3) int64 integer velocities
    w: np.ndarray          # (Q,) float64 weights
    r: float               # scale: c_a = r * e_a
    eq_order: int          # truncation order of Eq. (eq:feq)
    thermal: bool          # False: T is fixed to 1 (Sec. II, after eq:feq)
    degree: int            # exact quadrature degree

    @property
    def Q(self) -> int:
        return int(self.e.shape[0])

    @property
    def N(self) -> int:
        """Ghost layers = largest wall-normal integer speed (Sec. III)."""
        return int(np.max(np.abs(self.e[:, 1])))


def _orbit(shell, D):
    """All sign changes and coordinate permutations of one shell vector."""
    s = list(shell) + [0] * (D - len(shell))
    pts = set()
    for perm in itertools.permutations(range(D)):
        for signs in itertools.product((1, -1), repeat=D):
            pts.add(tuple(signs[i] * s[perm[i]] for i in range(D)))
    return sorted(pts)


def _gauss_moment(m):
    """E[prod z_i^{m_i}] for independent standard normal z_i."""
    v = mpmath.mpf(1)
    for k in m:
        if k % 2:
            return mpmath.mpf(0)
        v *= mpmath.fac2(k - 1) if k > 0 else 1
    return v


def _even_monomials(D, degree):
    """One representative (non-increasing exponents) per symmetry class."""
    out = []
    for tot in range(0, degree + 1, 2):
        for m in itertools.product(range(0, tot + 1, 2), repeat=D):
            if sum(m) == tot and list(m) == sorted(m, reverse=True):
                out.append(m)
    return out


def _solve_rule(shells, D, degree, r_guess):
    """Solve the moment equations for (r, per-shell weights).

    With S shells there are S+1 symmetry classes of even monomials up to the
    degree, i.e. S+1 equations, linear in the S weights for fixed r.  r is
    the root of the determinant of the augmented (S+1)x(S+1) system.
    """
    mpmath.mp.dps = 40
    monos = _even_monomials(D, degree)
    orbits = [_orbit(s, D) for s in shells]
    if len(monos) != len(shells) + 1:
        raise ValueError("moment system is not square in (weights, r)")

    def augmented(r):
        rows = []
        for m in monos:
            row = []
            for orb in orbits:
                acc = mpmath.mpf(0)
                for v in orb:
                    t = mpmath.mpf(1)
                    for i in range(D):
                        t *= (r * v[i]) ** m[i]
                    acc += t
                row.append(acc)
            row.append(_gauss_moment(m))
            rows.append(row)
        return mpmath.matrix(rows)

    r = mpmath.findroot(lambda x: mpmath.det(augmented(x)), mpmath.mpf(r_guess))
    A = augmented(r)
    S = len(shells)
    lhs = mpmath.matrix([[A[i, j] for j in range(S)] for i in range(S)])
    rhs = mpmath.matrix([A[i, S] for i in range(S)])
    wts = mpmath.lu_solve(lhs, rhs)
    return r, [wts[i] for i in range(S)], orbits


def _assemble(name, D, orbits, shell_w, r, eq_order, thermal, degree):
    e, w = [], []
    for orb, ws in zip(orbits, shell_w):
        for v in orb:
            e.append(tuple(v) + (0,) * (3 - D))
            w.append(float(ws))
    return OracleLattice(name=name, D=D, e=np.array(e, dtype=np.int64),
                         w=np.array(w, dtype=np.float64), r=float(r),
                         eq_order=eq_order, thermal=thermal, degree=degree)


@functools.lru_cache(maxsize=None)
def d2q17() -> OracleLattice:
    shells = [(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)]
    r, ws, orbs = _solve_rule(shells, 2, 7, 1.6)
    if min(ws) <= 0:
        raise RuntimeError("D2Q17 solve landed on a non-positive root")
    return _assemble("D2Q17", 2, orbs, ws, r, 4, False, 7)


@functools.lru_cache(maxsize=None)
def d3q121() -> OracleLattice:
    shells = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0), (2, 2, 0), (2, 2, 2),
              (3, 0, 0), (3, 1, 1), (3, 2, 0), (3, 3, 3)]
    r, ws, orbs = _solve_rule(shells, 3, 9, 1.2)
    if min(ws) <= 0:
        raise RuntimeError("D3Q121 solve landed on a non-positive root")
    return _assemble("D3Q121", 3, orbs, ws, r, 4, True, 9)


@functools.lru_cache(maxsize=None)
def d2q16() -> OracleLattice:
    """Tensor product of the 1-D rule {+-1: 9/20, +-3: 1/20}, r = sqrt(5)/3."""
    mpmath.mp.dps = 40
    one_d = {1: mpmath.mpf(9) / 20, -1: mpmath.mpf(9) / 20,
             3: mpmath.mpf(1) / 20, -3: mpmath.mpf(1) / 20}
    e, w = [], []
    for a in (-3, -1, 1, 3):
        for b in (-3, -1, 1, 3):
            e.append((a, b, 0))
            w.append(float(one_d[a] * one_d[b]))
    return OracleLattice(name="D2Q16", D=2, e=np.array(e, dtype=np.int64),
                         w=np.array(w, dtype=np.float64),
                         r=float(mpmath.sqrt(5) / 3), eq_order=2,
                         thermal=False, degree=3)


def by_name(name: str) -> OracleLattice:
    return {"D2Q16": d2q16, "D2Q17": d2q17, "D3Q121": d3q121}[name.upper()]()
