"""Writes ``lattice_tables.h``: the velocity sets the HIP library is compiled
against.

The paper leaves the three lattice tables out (Sec. IV), so they are
recovered from what defines a lattice (Sec. II): integer velocities e_a with
c_a = r e_a and weights w_a such that sum_a w_a c_a^m equals the unit
Gaussian's moment for every monomial m up to the quadrature degree.

  D2Q17  shells (0,0),(1,0),(1,1),(2,2),(3,0); degree 7; 4th-order f^eq
  D3Q121 shells (000),(100),(111),(210),(220),(222),(300),(311),(320),(333);
         degree 9; 4th-order f^eq; thermal
  D2Q16  tensor product of {+-1: 9/20, +-3: 1/20}, r = sqrt(5)/3;
         2nd-order f^eq (a labelled construction, see the design notes)

Method: Newton iteration on the full square system (shell weights and r
together), started from the least-squares weights at a rough r.
40-digit arithmetic, printed with 21 significant digits.

Run:  python paper_1209_5201_amd/csrc/gen_lattice_tables.py
"""
import itertools
import os

import mpmath as mp

mp.mp.dps = 40


def shell_members(shell, dim):
    s = list(shell) + [0] * (dim - len(shell))
    out = set()
    for perm in itertools.permutations(s):
        for flips in itertools.product((1, -1), repeat=dim):
            out.add(tuple(f * p for f, p in zip(flips, perm)))
    return sorted(out)


def gaussian(expo):
    v = mp.mpf(1)
    for k in expo:
        if k % 2:
            return mp.mpf(0)
        for j in range(k - 1, 0, -2):
            v *= j
    return v


def classes(dim, degree):
    res = []
    for d in range(0, degree + 1, 2):
        for combo in itertools.combinations_with_replacement(range(d, -1, -2), dim):
            if sum(combo) == d and all(c % 2 == 0 for c in combo):
                key = tuple(sorted(combo, reverse=True))
                if key not in res:
                    res.append(key)
    return res


def shell_sum(members, expo, r):
    tot = mp.mpf(0)
    for v in members:
        t = mp.mpf(1)
        for comp, k in zip(v, expo):
            t *= (r * comp) ** k
        tot += t
    return tot


def newton_rule(shells, dim, degree, r0):
    mem = [shell_members(s, dim) for s in shells]
    eqs = classes(dim, degree)
    S = len(shells)
    assert len(eqs) == S + 1

    def F(*z):
        ws, r = z[:S], z[S]
        return [sum(ws[s] * shell_sum(mem[s], m, r) for s in range(S)) - gaussian(m)
                for m in eqs]

    def J(*z):
        ws, r = z[:S], z[S]
        rows = []
        for m in eqs:
            sums = [shell_sum(mem[s], m, r) for s in range(S)]
            # every term of a class-m sum is homogeneous of degree |m| in r
            rows.append(sums + [sum(ws[s] * sums[s] for s in range(S)) * sum(m) / r])
        return mp.matrix(rows)

    # start: least-squares weights of all S+1 equations at r0
    A = mp.matrix([[shell_sum(mem[s], m, r0) for s in range(S)] for m in eqs])
    b = mp.matrix([gaussian(m) for m in eqs])
    w0 = mp.lu_solve(A.T * A, A.T * b)
    sol = mp.findroot(F, [w0[i] for i in range(S)] + [mp.mpf(r0)], J=J, maxsteps=200)
    ws = [sol[i] for i in range(S)]
    r = sol[S]
    if min(ws) <= 0:
        raise RuntimeError("non-positive weight")
    return ws, r, mem


def emit(name, dim, eq_order, thermal, vel, wts, r):
    order = sorted(range(len(vel)), key=lambda i: (vel[i][1], vel[i][2], vel[i][0]))
    Q = len(vel)
    N = max(abs(v[1]) for v in vel)
    lines = ["struct %s {" % name,
             "  static constexpr int Q = %d;" % Q,
             "  static constexpr int D = %d;" % dim,
             "  static constexpr int N = %d;      // ghost layers per wall" % N,
             "  static constexpr int EQ = %d;     // truncation order of f^eq" % eq_order,
             "  static constexpr bool THERMAL = %s;" % ("true" if thermal else "false"),
             "  static constexpr double R = %s;" % mp.nstr(r, 21),
             "  static constexpr signed char E[%d][3] = {" % Q]
    row = []
    for i in order:
        row.append("{%d,%d,%d}" % vel[i])
    for k in range(0, Q, 8):
        lines.append("    " + ", ".join(row[k:k + 8]) + ",")
    lines.append("  };")
    lines.append("  static constexpr double W[%d] = {" % Q)
    for k in range(0, Q, 3):
        lines.append("    " + ", ".join(mp.nstr(wts[i], 21, min_fixed=0, max_fixed=0)
                                         for i in order[k:k + 3]) + ",")
    lines.append("  };")
    lines.append("};")
    return "\n".join(lines)


def build():
    blocks = []
    # D2Q16 (tensor product rule)
    one = {1: mp.mpf(9) / 20, 3: mp.mpf(1) / 20}
    vel, wts = [], []
    for a in (-3, -1, 1, 3):
        for b in (-3, -1, 1, 3):
            vel.append((a, b, 0))
            wts.append(one[abs(a)] * one[abs(b)])
    blocks.append(emit("D2Q16", 2, 2, False, vel, wts, mp.sqrt(5) / 3))
    # D2Q17
    ws, r, mem = newton_rule([(0, 0), (1, 0), (1, 1), (2, 2), (3, 0)], 2, 7, 1.6)
    vel = [m + (0,) for s in mem for m in s]
    wts = [ws[i] for i, s in enumerate(mem) for _ in s]
    blocks.append(emit("D2Q17", 2, 4, False, vel, wts, r))
    # D3Q121
    shells = [(0, 0, 0), (1, 0, 0), (1, 1, 1), (2, 1, 0), (2, 2, 0), (2, 2, 2),
              (3, 0, 0), (3, 1, 1), (3, 2, 0), (3, 3, 3)]
    ws, r, mem = newton_rule(shells, 3, 9, 1.2)
    vel = [m for s in mem for m in s]
    wts = [ws[i] for i, s in enumerate(mem) for _ in s]
    blocks.append(emit("D3Q121", 3, 4, True, vel, wts, r))
    head = ("// Generated by gen_lattice_tables.py - do not edit.\n"
            "// Velocity sets c_a = R * E_a with weights W_a integrating the unit\n"
            "// Gaussian exactly up to the lattice's degree (D2Q17: 7, D3Q121: 9,\n"
            "// D2Q16: tensor product of a 1-D degree-3 rule).  Velocities are\n"
            "// sorted by (e_y, e_z, e_x).\n"
            "#pragma once\n\nnamespace lbm {\n\n")
    return head + "\n\n".join(blocks) + "\n\n}  // namespace lbm\n"


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_tables.h")
    with open(out, "w") as fh:
        fh.write(build())
    print("wrote", out)
