"""GPU tests of the batched small-case path (lbm_batch_step) and the
continuous-batching server."""
import math
import sys

import numpy as np
import pytest

import paper_1209_5201_amd as lbm
from paper_1209_5201_amd import serve
from paper_1209_5201_amd import workloads as W
from oracle import lattices as OL
from oracle import oracle as O

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "uz", "T", "sxy", "qx", "qy", "qz")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [("D2Q16", 1, 32, 0.1, (-0.1, 0.0, 1.0), (0.1, 0.0, 1.0)),
         ("D2Q17", 3, 40, 0.05, (-0.05, 0.0, 1.0), (0.1, 0.0, 1.0)),
         ("D3Q121", 2, 24, 0.2, (-0.2, 0.0, 1.0), (0.2, 0.0, 1.1)),
         ("D2Q17", 1, 300, 0.02, (-0.1, 0.0, 1.0), (0.1, 0.0, 1.0))]


def open_case(lat, nx, ny, kn, b, t, prec):
    return lbm.Channel(lat, nx, ny, lbm.lbm_tau_from_kn(lat, ny, kn), b, t, prec=prec)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5), ("fp32s", 1e-7)])
def test_batch_matches_single_context_path(prec, tol):
    """The batched persistent kernel against lbm_step's per-step kernels:
    the same scheme, compiled in another kernel (the compiler may contract
    differently), so fields agree to rounding."""
    say("case batch == step", prec)
    a = [open_case(*c, prec) for c in CASES]
    b = [open_case(*c, prec) for c in CASES]
    for _ in range(3):
        res = lbm.lbm_batch_step([c.ctx for c in a], 50)
        for c in b:
            c.step(50)
        for ca, cb, r in zip(a, b, res):
            ma, mb = ca.moments(), cb.moments()
            for k in FIELDS:
                grp = ("ux", "uy", "uz") if k[0] == "u" else ("qx", "qy", "qz") \
                    if k[0] == "q" else (k,)
                scale = max(np.abs(mb[j]).max() for j in grp)
                assert np.abs(ma[k] - mb[k]).max() <= tol * scale + 1e-15, (prec, k)
            assert ca.steps_done() == cb.steps_done()
            assert abs(r - cb.residual()) <= 1e-3 * abs(cb.residual())
    for c in a + b:
        c.close()


def test_batch_run_stops_each_case_at_its_own_window():
    """lbm_batch_run: a case stops at the first window whose residual meets
    the tolerance, independently of its budget and of the other cases."""
    say("case batch_run stop")
    a = [open_case(*c, "fp32") for c in CASES[:3]]
    res, steps, state = lbm.lbm_batch_run([c.ctx for c in a], [100000, 3000, 100000], 100, 1e-6)
    assert state[1] in (0, 1) and steps[1] <= 3000
    # the same cases one at a time with other budgets stop at the same step
    for i, c in enumerate(CASES[:3]):
        if state[i] != 1:
            continue
        b = open_case(*c, "fp32")
        r2, s2, st2 = lbm.lbm_batch_run([b.ctx], [steps[i] + 5000], 100, 1e-6)
        assert st2[0] == 1 and s2[0] == steps[i] and r2[0] == res[i]
        for k in ("ux", "sxy"):
            assert np.array_equal(b.field(k), a[i].field(k))
        b.close()
    for c in a:
        c.close()


def test_batch_matches_oracle_fp64():
    say("case batch vs oracle")
    chans = [open_case(*c, "fp64") for c in CASES]
    lbm.lbm_batch_step([c.ctx for c in chans], 120)
    for (lat, nx, ny, kn, bw, tw), ch in zip(CASES, chans):
        o = O.OracleCase(lat, nx, ny, O.tau_from_kn(lat, ny, kn), bw, tw)
        o.run(120)
        want, got = o.moments(), ch.moments()
        for k in ("rho", "ux", "uy", "T", "sxy", "qy"):
            scale = max(np.abs(want[j]).max() for j in (("ux", "uy") if k[0] == "u" else (k,)))
            assert np.abs(got[k] - want[k]).max() <= 1e-12 * scale + 1e-15, (lat, k)
        ch.close()


def test_each_result_is_the_same_alone_and_in_the_mix():
    """A request served inside a mix of others returns bit-identical profiles
    and step counts to the same request served alone."""
    reqs = W.serving_requests(n=12, seed=11, rate=1e9, ny_range=(16, 64), channel_fraction=0.4)
    for r in reqs:
        r["kn"] = max(r["kn"], 0.1)   # keep the test short
    say("case alone == mix", len(reqs))
    mix = serve.Server(prec="fp32", window=100, tol=1e-7, max_active=8).run(reqs,
                                                                           realtime=False)
    assert mix["solves"] == len(reqs)
    by_id = {r.id: r for r in mix["results"]}
    for req in reqs[:4]:
        alone = serve.Server(prec="fp32", window=100, tol=1e-7, max_active=1).run(
            [req], realtime=False)["results"][0]
        inmix = by_id[req["id"]]
        assert alone.steps == inmix.steps and alone.converged and inmix.converged
        for k in ("ux", "T", "sxy", "qy"):
            assert np.array_equal(alone.profiles[k], inmix.profiles[k]), (req["id"], k)


def test_served_fp32_results_match_fp64_oracle():
    """Served FP32 Couette solves (run to the residual tolerance) against the
    FP64 oracle run the same number of steps."""
    reqs = [dict(id=0, lattice="D2Q17", ny=32, kn=0.1, bottom=(-0.1, 0, 1.0),
                 top=(0.1, 0, 1.0), arrival=0.0),
            dict(id=1, lattice="D3Q121", ny=24, kn=0.3, bottom=(-0.15, 0, 1.0),
                 top=(0.15, 0, 1.1), arrival=0.0),
            dict(id=2, lattice="D2Q16", ny=40, kn=0.2, bottom=(-0.05, 0, 1.0),
                 top=(0.05, 0, 1.0), arrival=0.0)]
    say("case served vs oracle")
    out = serve.Server(prec="fp32", window=100, tol=1e-8).run(reqs, realtime=False)
    for res, req in zip(out["results"], reqs):
        assert res.converged
        o = O.OracleCase(req["lattice"], 1, req["ny"],
                         O.tau_from_kn(req["lattice"], req["ny"], req["kn"]),
                         req["bottom"], req["top"])
        o.run(res.steps)
        want = o.moments()
        for k in ("ux", "sxy") + (("T", "qy") if req["lattice"] == "D3Q121" else ()):
            w = want[k][:, 0]
            scale = np.abs(w - (1.0 if k == "T" else 0.0)).max()
            assert np.abs(res.profiles[k] - w).max() <= 1e-5 * scale + 1e-9, (req["lattice"], k)


def test_served_channel_requests_match_fp64_oracle():
    """Force-driven channel requests served in FP32 beside a Couette request,
    each against the FP64 oracle run the same number of steps with the force
    derived from the oracle's own lattice tables."""
    reqs = [dict(id=0, lattice="D2Q17", ny=32, kn=0.1, bottom=(0, 0, 1.0), top=(0, 0, 1.0),
                 umax=0.08, arrival=0.0),
            dict(id=1, lattice="D3Q121", ny=24, kn=0.2, bottom=(0, 0, 1.0), top=(0, 0, 1.0),
                 umax=0.1, arrival=0.0),
            dict(id=2, lattice="D2Q16", ny=40, kn=0.05, bottom=(0, 0, 1.0), top=(0, 0, 1.0),
                 umax=0.05, arrival=0.0),
            dict(id=3, lattice="D2Q17", ny=20, kn=0.3, bottom=(-0.1, 0, 1.0), top=(0.1, 0, 1.0),
                 arrival=0.0)]
    say("case served channels vs oracle")
    out = serve.Server(prec="fp32", window=100, tol=1e-8).run(reqs, realtime=False)
    for res, req in zip(out["results"], reqs):
        assert res.converged
        lat = OL.by_name(req["lattice"])
        force = None
        if "umax" in req:
            a = 8 * req["umax"] * math.sqrt(2 / math.pi) * req["kn"] / (lat.r * req["ny"])
            force = (a, 0.0, 0.0)
        o = O.OracleCase(lat, 1, req["ny"], O.tau_from_kn(lat, req["ny"], req["kn"]),
                         req["bottom"], req["top"], force=force)
        o.run(res.steps)
        want = o.moments()
        for k in ("ux", "sxy") + (("T", "qy") if req["lattice"] == "D3Q121" else ()):
            w = want[k][:, 0]
            scale = np.abs(w - (1.0 if k == "T" else 0.0)).max()
            assert np.abs(res.profiles[k] - w).max() <= 1e-5 * scale + 1e-9, (req["lattice"], k)


def poison(ch):
    """Overwrite node 0's first population with NaN through a checkpoint:
    the failure is forced from the host; the GPU only computes with it."""
    state = ch.save()
    nan = np.array([np.nan], dtype=np.float32 if ch.prec == "fp32" else np.float64)
    state[16:16 + nan.nbytes] = nan.tobytes()
    ch.load(state)


def test_nonfinite_state_is_reported_not_crashed():
    say("case nonfinite")
    ch = open_case("D2Q17", 1, 32, 0.1, (-0.1, 0, 1.0), (0.1, 0, 1.0), "fp32")
    ch.step(20)
    poison(ch)
    ch.step(20)
    with pytest.raises(lbm.LbmError) as ei:
        ch.residual()
    assert ei.value.status == lbm.lbm.LBM_ENONFINITE
    ch.close()


def test_poisoned_case_retires_without_touching_the_others():
    say("case poisoned batch")
    good = [open_case(*c, "fp32") for c in CASES[:3]]
    ref = [open_case(*c, "fp32") for c in CASES[:3]]
    bad = open_case(*CASES[1], "fp32")
    poison(bad)
    r1, s1, st1 = lbm.lbm_batch_run([c.ctx for c in good] + [bad.ctx], [4000] * 4, 100, 1e-7)
    r2, s2, st2 = lbm.lbm_batch_run([c.ctx for c in ref], [4000] * 3, 100, 1e-7)
    assert st1[3] == -1 and np.isnan(r1[3]) and s1[3] == 100
    assert np.array_equal(s1[:3], s2) and np.array_equal(st1[:3], st2)
    for a, b in zip(good, ref):
        for k in ("ux", "T", "sxy"):
            assert np.array_equal(a.field(k), b.field(k))
    for c in good + ref + [bad]:
        c.close()


def test_grid_convergence_is_second_order():
    """Sec. IV: thermal Couette (D3Q121, Kn = 0.01, U_w = 0.2, T_w = 1); the
    global errors E_U, E_T against a fine reference fall at second order."""
    from paper_1209_5201_amd import convergence
    say("case grid convergence")
    out = convergence.convergence_study(grids=(20, 40, 80), reference=320)
    say("   ", out)
    assert 1.7 < out["order_U"] < 2.5, out
    assert 1.7 < out["order_T"] < 2.5, out
