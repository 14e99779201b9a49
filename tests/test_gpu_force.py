"""GPU parity of the body force (force-driven channel; the Hermite-projected
force term a . d f^eq / du with the half-step shift of Sec. II's change of
variable) against the FP64 oracle, through the C ABI (lbm_set_body_force),
on the linear, row-tiled and batched kernels."""
import math
import sys

import numpy as np
import pytest

import paper_1209_5201_amd as lbm
from paper_1209_5201_amd import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "uz", "T", "sxy", "qx", "qy", "qz")
GROUPS = {"ux": ("ux", "uy", "uz"), "uy": ("ux", "uy", "uz"), "uz": ("ux", "uy", "uz"),
          "qx": ("qx", "qy", "qz"), "qy": ("qx", "qy", "qz"), "qz": ("qx", "qy", "qz")}
LATS = ["D2Q16", "D2Q17", "D3Q121"]
WALLS = {"D2Q16": ((-0.05, 0.0, 1.0), (0.02, 0.0, 1.0)),
         "D2Q17": ((-0.05, 0.0, 1.0), (0.02, 0.0, 1.0)),
         "D3Q121": ((-0.05, 0.02, 1.0), (0.02, 0.0, 1.1))}
FORCE = {"D2Q16": (3e-4, -1e-4, 0.0), "D2Q17": (3e-4, -1e-4, 0.0), "D3Q121": (3e-4, -1e-4, 2e-4)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_err(got, want, atol, fields=FIELDS):
    errs = {}
    for k in fields:
        scale = max(np.abs(want[j]).max() for j in GROUPS.get(k, (k,)))
        d = max(np.abs(got[k] - want[k]).max() - atol, 0.0)
        errs[k] = d / scale if scale > 0 else d
    say("   errors", {k: "%.1e" % v for k, v in errs.items()})
    return max(errs.values())


def pair(lat, nx, ny, tau, prec="fp64", seed=3, accommodation=(1.0, 1.0), force=None):
    force = FORCE[lat] if force is None else force
    rho, ux, uy, T = W.random_fields(nx, ny, seed=seed, thermal=(lat == "D3Q121"))
    g = lbm.Channel(lat, nx, ny, tau, *WALLS[lat], prec=prec, accommodation=accommodation,
                    force=force)
    g.init(rho=rho, ux=ux, uy=uy, T=T)
    o = O.OracleCase(lat, nx, ny, tau, *WALLS[lat], rho0=rho,
                     u0=np.stack([ux, uy, np.zeros_like(ux)]), T0=T,
                     accommodation=accommodation, force=force)
    return g, o


@pytest.mark.parametrize("lat", LATS)
@pytest.mark.parametrize("nx,ny", [(13, 24), (256, 12)])
def test_fp64_force(lat, nx, ny):
    say("case force fp64", lat, nx, ny)
    g, o = pair(lat, nx, ny, 0.7)
    assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12
    for t in (1, 20):
        g.step(t)
        o.run(t)
        assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12, o.t
    g.close()


# Heat flux of an isothermal set from a random start: a near-zero
# non-equilibrium quantity (see the accommodation tests); FP32 arithmetic
# meets 1e-4 of its largest value there, 1e-5 on every other result.
ISO_Q_TOL = 1e-4


@pytest.mark.parametrize("lat", ["D2Q17", "D3Q121"])
@pytest.mark.parametrize("prec", ["fp32", "fp32s"])
def test_single_precision_force(lat, prec):
    say("case force", lat, prec)
    g, o = pair(lat, 256, 16, 0.8, prec=prec, seed=5, accommodation=(0.6, 0.9))
    g.step(40)
    o.run(40)
    got, want = g.moments(), o.moments()
    if lat == "D3Q121" or prec == "fp32s":
        assert max_err(got, want, 1e-9) <= 1e-5
    else:
        assert max_err(got, want, 1e-9, FIELDS[:6]) <= 1e-5
        assert max_err(got, want, 1e-9, FIELDS[6:]) <= ISO_Q_TOL
    g.close()


def test_batched_mix_of_forced_and_free_cases():
    """Forced and force-free cases of two formats in one lbm_batch_step call
    (one launch per format and force variant) against the oracle."""
    specs = [("D2Q17", "fp64", True), ("D3Q121", "fp64", False), ("D2Q16", "fp64", True),
             ("D3Q121", "fp64", True), ("D2Q17", "fp64", False)]
    chans, orcs = [], []
    for i, (lat, prec, forced) in enumerate(specs):
        g, o = pair(lat, 1, 18, 0.9, prec=prec, seed=30 + i,
                    force=None if forced else (0.0, 0.0, 0.0))
        if not forced:
            o.force = None
        chans.append(g)
        orcs.append(o)
    say("case force batch")
    lbm.lbm_batch_step([c.ctx for c in chans], 60)
    for o in orcs:
        o.run(60)
    for g, o in zip(chans, orcs):
        assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12, g.lattice
    for c in chans:
        c.close()


def test_poiseuille_steady_state_fp32():
    """The force-driven channel (walls at rest, Kn = 0.05) run to a steady
    state in FP32 through the serving path, against the FP64 oracle run to
    the same step count."""
    lat, ny, kn = "D2Q17", 48, 0.05
    tau = lbm.lbm_tau_from_kn(lat, ny, kn)
    a = 0.4 * math.sqrt(2 / math.pi) * kn / (lbm.lbm_lattice_info(lat)["r"] * ny)
    say("case poiseuille fp32")
    g = lbm.Channel(lat, 1, ny, tau, prec="fp32", force=(a, 0.0, 0.0))
    res, steps, state = lbm.lbm_batch_run([g.ctx], [200000], 100, 1e-8)
    assert state[0] == 1, (res, steps)
    o = O.OracleCase(lat, 1, ny, O.tau_from_kn(lat, ny, kn), force=(a, 0.0, 0.0))
    o.run(int(steps[0]))
    got, want = g.moments(), o.moments()
    assert max_err(got, want, 1e-9, ("rho", "ux", "uy", "sxy")) <= 1e-5
    g.close()


def test_force_is_refused_where_it_does_not_apply():
    ch = lbm.Channel("D2Q17", 4, 16, 0.8)
    for bad in ((0.0, 0.0, 1e-3), (float("nan"), 0.0, 0.0), (2.0, 0.0, 0.0)):
        with pytest.raises(lbm.LbmError):
            ch.set_body_force(*bad)
    ch.close()


# 16-bit storage with every wall / collision option at once: the force
# variant of the 16-bit kernels, partial accommodation and (D3Q121) the
# viscosity law, against the FP64 oracle, node by node (no averaging).  Bars
# from the storage rounding of a random start (2^-8 relative per value in
# BF16, 2^-11 in FP16, accumulated over 40 steps): rho, u, T to 1e-2 / 1e-3
# of their scale; sigma_xy, the small non-equilibrium part, to 2e-2 / 2e-3
# (measured: BF16 7-9e-3, FP16 1.0e-3).
REDUCED16 = {"bf16": (1e-2, 2e-2), "fp16": (1e-3, 2e-3)}


@pytest.mark.parametrize("lat", ["D2Q17", "D3Q121"])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_16bit_with_force_accommodation_and_law(lat, prec):
    say("case 16-bit options", lat, prec)
    w = 0.7 if lat == "D3Q121" else None
    rho, ux, uy, T = W.random_fields(256, 16, seed=17, thermal=(lat == "D3Q121"))
    g = lbm.Channel(lat, 256, 16, 0.8, *WALLS[lat], prec=prec, accommodation=(0.6, 0.9),
                    force=FORCE[lat], viscosity_exp=w)
    g.init(rho=rho, ux=ux, uy=uy, T=T)
    o = O.OracleCase(lat, 256, 16, 0.8, *WALLS[lat], rho0=rho,
                     u0=np.stack([ux, uy, np.zeros_like(ux)]), T0=T,
                     accommodation=(0.6, 0.9), force=FORCE[lat], viscosity_exp=w)
    g.step(40)
    o.run(40)
    got, want = g.moments(), o.moments()
    bar, bar_s = REDUCED16[prec]
    assert max_err(got, want, 0.0, FIELDS[:5]) <= bar
    assert max_err(got, want, 0.0, ("sxy",)) <= bar_s
    g.close()
