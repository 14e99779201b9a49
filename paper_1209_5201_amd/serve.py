"""Continuous batching of Couette / channel solves on one GPU.

Requests (a channel: velocity set, ny, Kn, walls, and optionally a body
force for a force-driven channel) arrive over time.  The
server admits arrived requests while it has free slots and free HBM (each
case's footprint is lbm_required_bytes), advances every admitted case by one
step budget in a single lbm_batch_run call (one persistent launch per
storage format; the cases' work overlaps on the device, and each case checks
its residual after every window inside the launch and stops once converged),
retires the converged cases (copying out their profiles and freeing their
memory), and admits waiting requests into the freed slots.

A case's step budget per launch is inversely proportional to its cost per
step, so that cheap cases do not idle while an expensive one finishes its
windows; the budget depends only on the case itself, and a case stops at
the first window that meets the tolerance whatever its budget, so the
result of a request is the same whether it runs alone or in any mix.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import lbm as _l


@dataclass
class Result:
    id: int
    lattice: str
    ny: int
    kn: float
    steps: int
    residual: float
    arrival: float          # seconds from the start of the run
    admitted: float
    retired: float
    converged: bool
    profiles: dict = field(default_factory=dict)   # x-averaged u_x, T, sigma_xy, q_y


def channel_force(lattice: str, ny: int, kn: float, umax: float) -> float:
    """Acceleration per time step that gives a force-driven channel of ny
    rows at Knudsen number kn the no-slip Navier-Stokes peak velocity umax:
    u_max = (a/nu)/8 in channel units, where a/nu = a_lat r ny / (sqrt(2/pi) Kn)
    (nu = tau T with tau = sqrt(2/pi) Kn, one step dt = 1/(r ny))."""
    r = _l.lbm_lattice_info(lattice)["r"]
    return 8.0 * umax * math.sqrt(2.0 / math.pi) * kn / (r * ny)


def percentile(vals, p):
    return float(np.percentile(np.asarray(vals, dtype=np.float64), p)) if len(vals) else math.nan


class Server:
    # launch length: REF_WINDOWS windows of the most expensive case (D3Q121,
    # 512 nodes; see _step_cost)
    REF_WINDOWS = 4

    def __init__(self, prec: str = "fp32", window: int = 100, tol: float = 1e-8,
                 max_active: int = 256, hbm_budget: Optional[int] = None,
                 max_steps: int = 2_000_000, device: str = "cuda:0", keep_profiles=True,
                 ref_windows: int = REF_WINDOWS):
        import torch
        self.torch = torch
        self.ref_windows = int(ref_windows)
        self.prec, self.window, self.tol = prec, int(window), float(tol)
        self.max_active, self.max_steps = int(max_active), int(max_steps)
        self.device = device
        self.keep_profiles = keep_profiles
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info(torch.device(device))
            hbm_budget = int(0.5 * free)
        self.hbm_budget = int(hbm_budget)

    def _footprint(self, req) -> int:
        return _l.lbm_required_bytes(req["lattice"], req.get("nx", 1), req["ny"], self.prec)

    def _step_cost(self, lattice: str, nodes: int, force: bool) -> float:
        """Time of one step of a case in the batched kernel, in microseconds
        (measured on MI355X; only the per-launch budgets use it, and they do
        not change results).  The FP32 instance without a force gives a
        case 1024 threads and splits D3Q121 nodes over four groups (256
        nodes per pass; 2-D sets 1024 per pass): about 16 us plus 7 us per
        further pass for D3Q121, 3.6 us plus 1.5 us per pass for the 2-D
        sets.  The other instances run 256 threads and whole nodes."""
        big = lattice == "D3Q121"
        if self.prec == "fp32" and not force:
            per_pass = 256 if big else 1024
        else:
            per_pass = 256
        passes = -(-nodes // per_pass)
        base, extra = (16.0, 7.0) if big else (3.6, 1.5)
        if not (self.prec == "fp32" and not force):
            base, extra = (2.0 * base, 2.0 * extra) if big else (base, 2.0 * extra)
        return base + extra * (passes - 1)

    def _budget(self, req) -> int:
        """Steps per launch for a case: REF_WINDOWS windows for the most
        expensive case, proportionally more for cheaper ones, so that the
        cases of a launch take about the same time."""
        force = bool(req.get("force") or req.get("umax"))
        ref = self._step_cost("D3Q121", 512, force)
        cost = self._step_cost(req["lattice"], req.get("nx", 1) * req["ny"], force)
        windows = max(1, int(round(self.ref_windows * ref / cost)))
        return self.window * windows

    def _open(self, req):
        force = req.get("force")
        if force is None and req.get("umax"):
            force = (channel_force(req["lattice"], req["ny"], req["kn"], req["umax"]), 0.0, 0.0)
        return _l.Channel(req["lattice"], req.get("nx", 1), req["ny"], 0.0,
                          req["bottom"], req["top"], prec=self.prec, device=self.device,
                          kn=req["kn"], force=force)

    def _finish(self, slot, now, converged, residual):
        ch, req, t_admit, fp = slot
        prof = {}
        if self.keep_profiles:
            m = ch.moments()
            prof = {k: m[k].mean(axis=1) for k in ("ux", "T", "sxy", "qy")}
        res = Result(id=req["id"], lattice=req["lattice"], ny=req["ny"], kn=req["kn"],
                     steps=ch.steps_done(), residual=residual, arrival=req["arrival"],
                     admitted=t_admit, retired=now, converged=converged, profiles=prof)
        ch.close()
        return res, fp

    def run(self, requests: List[dict], realtime: bool = True) -> dict:
        """Serve `requests` (dicts with id, lattice, ny, kn, bottom, top,
        arrival [s]).  realtime=False admits every request at t = 0."""
        pending = sorted(requests, key=lambda r: (r["arrival"] if realtime else 0.0, r["id"]))
        active = []          # (channel, request, t_admit, footprint)
        used = 0
        results: List[Result] = []
        launches = 0
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            # admit arrived requests while slots and memory allow (FIFO)
            while pending and len(active) < self.max_active:
                req = pending[0]
                if realtime and req["arrival"] > now:
                    break
                fp = self._footprint(req)
                if used + fp > self.hbm_budget and active:
                    break
                pending.pop(0)
                active.append((self._open(req), req, time.perf_counter() - t0, fp))
                used += fp
            if not active:
                wait = pending[0]["arrival"] - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
                continue
            budgets = [min(self._budget(sl[1]),
                           max(self.window, self.max_steps - sl[0].steps_done()))
                       for sl in active]
            res, _adv, state = _l.lbm_batch_run([sl[0].ctx for sl in active], budgets,
                                                self.window, self.tol)
            launches += 1
            now = time.perf_counter() - t0
            keep = []
            for slot, r, st in zip(active, res, state):
                if st != 0 or slot[0].steps_done() >= self.max_steps:
                    out, fp = self._finish(slot, now, bool(st == 1), float(r))
                    results.append(out)
                    used -= fp
                else:
                    keep.append(slot)
            active = keep
        wall = time.perf_counter() - t0
        tts = [r.retired - r.arrival for r in results]
        svc = [r.retired - r.admitted for r in results]
        first = min(r.arrival for r in results) if results else 0.0
        last = max(r.retired for r in results) if results else 0.0
        return {"results": sorted(results, key=lambda r: r.id),
                "solves": len(results),
                "converged": sum(r.converged for r in results),
                "wall_s": wall,
                "solves_per_s": len(results) / (last - first) if last > first else math.nan,
                "p50_s": percentile(tts, 50), "p99_s": percentile(tts, 99),
                "p50_service_s": percentile(svc, 50), "p99_service_s": percentile(svc, 99),
                "launches": launches,
                "node_updates": float(sum(r.steps * r.ny for r in results))}


def one_at_a_time(requests: List[dict], prec: str = "fp64", window: int = 100,
                  tol: float = 1e-8, max_steps: int = 2_000_000, device: str = "cuda:0") -> dict:
    """Baseline: each request solved alone, one after the other, with the
    same residual windows (the persistent kernel on a single case, with a
    long budget so a solve takes few launches)."""
    srv = Server(prec=prec, window=window, tol=tol, max_active=1, max_steps=max_steps,
                 device=device, keep_profiles=True, ref_windows=64)
    return srv.run(requests, realtime=False)
