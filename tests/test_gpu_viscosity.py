"""GPU parity of the local relaxation time (tau = mu/p with mu = T^w,
p = rho T, end of Sec. II) against the FP64 oracle, through the C ABI
(lbm_set_viscosity_law), on the linear, row-tiled and batched kernels."""
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
LAT = "D3Q121"
WALLS = ((-0.1, 0.03, 1.0), (0.1, 0.0, 1.3))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def max_err(got, want, atol):
    errs = {}
    for k in FIELDS:
        scale = max(np.abs(want[j]).max() for j in GROUPS.get(k, (k,)))
        d = max(np.abs(got[k] - want[k]).max() - atol, 0.0)
        errs[k] = d / scale if scale > 0 else d
    say("   errors", {k: "%.1e" % v for k, v in errs.items()})
    return max(errs.values())


def pair(nx, ny, tau, w, prec="fp64", seed=3):
    rho, ux, uy, T = W.random_fields(nx, ny, seed=seed, thermal=True, amp=0.05)
    g = lbm.Channel(LAT, nx, ny, tau, *WALLS, prec=prec, viscosity_exp=w)
    g.init(rho=rho, ux=ux, uy=uy, T=T)
    o = O.OracleCase(LAT, nx, ny, tau, *WALLS, rho0=rho,
                     u0=np.stack([ux, uy, np.zeros_like(ux)]), T0=T, viscosity_exp=w)
    return g, o


@pytest.mark.parametrize("w", [0.5, 0.81])
@pytest.mark.parametrize("nx,ny", [(13, 24), (256, 12)])
def test_fp64_local_tau(nx, ny, w):
    """13 columns: linear update with a separate wall launch; 256 columns:
    row-tiled update with fused wall sums."""
    say("case viscosity law fp64", nx, ny, w)
    g, o = pair(nx, ny, 0.6, w)
    for t in (1, 20):
        g.step(t)
        o.run(t)
        assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12, o.t
    g.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("fp32s", 1e-5)])
def test_single_precision_local_tau(prec, tol):
    say("case viscosity law", prec)
    g, o = pair(256, 16, 0.7, 0.5, prec=prec, seed=9)
    g.step(40)
    o.run(40)
    assert max_err(g.moments(), o.moments(), 1e-9) <= tol
    g.close()


def test_batched_path_and_switching():
    """The batched kernel with the law on some cases, then switched off on
    one and on for another between launches, against the oracle."""
    chans, orcs = [], []
    for i, w in enumerate((0.5, None, 1.0)):
        g, o = pair(1, 20, 0.8, w, seed=20 + i)
        chans.append(g)
        orcs.append(o)
    say("case viscosity law batch")
    lbm.lbm_batch_step([c.ctx for c in chans], 50)
    for o in orcs:
        o.run(50)
    for g, o in zip(chans, orcs):
        assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12
    # the library's state after a call is post-collision: a new law acts
    # from the collision of the next step on, which is the oracle's second
    # collision from here (its state is pre-collision)
    chans[0].set_viscosity_law(None)
    chans[1].set_viscosity_law(0.7)
    lbm.lbm_batch_step([c.ctx for c in chans], 30)
    for o in orcs:
        o.run(1)
    orcs[0].law = None
    orcs[1].law = np.array([0.7])
    for o in orcs:
        o.run(29)
    for g, o in zip(chans, orcs):
        assert max_err(g.moments(), o.moments(), 1e-15) <= 1e-12
    for c in chans:
        c.close()


def test_law_is_refused_where_it_does_not_apply():
    iso = lbm.Channel("D2Q17", 4, 16, 0.8)
    with pytest.raises(lbm.LbmError):
        iso.set_viscosity_law(0.5)
    iso.close()
    free = lbm.Channel(LAT, 1, 16, float("inf"))
    with pytest.raises(lbm.LbmError):
        free.set_viscosity_law(0.5)
    free.close()


def test_fp32_split_node_batched_with_law_and_accommodation():
    """The FP32 batched kernel splits each D3Q121 node over four groups of
    waves (velocity subsets with partial moment sums combined in LDS); 300
    rows take two passes of 256 nodes.  With the viscosity law and partial
    accommodation on both walls: against the FP64 oracle at the FP32 bar,
    and against the same case on the per-node kernel, which sums each node's
    moments in one lane (the two differ only in rounding order)."""
    say("case split node batched fp32 D3Q121 ny 300 law + accommodation")
    g, o = pair(1, 300, 0.7, 0.5, prec="fp32", seed=31)
    h, _ = pair(1, 300, 0.7, 0.5, prec="fp32", seed=31)
    for c in (g, h):
        c.set_accommodation(0.6, 0.85)
    o.alpha = (0.6, 0.85)
    lbm.lbm_batch_step([g.ctx], 40)
    h.step(40)
    o.run(40)
    assert max_err(g.moments(), o.moments(), 1e-9) <= 1e-5
    assert max_err(g.moments(), h.moments(), 1e-9) <= 1e-5
    g.close()
    h.close()
