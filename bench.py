#!/usr/bin/env python3
"""Throughput of the fused stream-collide update on one MI355X.

Workload: the 2-D bulk bandwidth case - D2Q17, 2048 x 2048 nodes, periodic
in x, diffuse walls (at rest, T = 1) top and bottom, Kn = 0.05,
rho = 1 + 1e-3 N(0,1) (seed 0), u = 0, FP32 populations.  One benchmark step
is one time step of the whole grid (one fused launch: wall sums in the wall
rows, pull, collide, store; the output fields, mass and residual are
refreshed after the last step of the timed call).  Inputs are resident in
HBM before timing starts.

Also measured (the "serving" object): the Couette serving stream - 1024
seeded requests over the three velocity sets, Ny in [16, 512], Kn log-uniform
in [0.01, 0.5], each run to a residual rate of 1e-8 in FP32 - as saturated
solves/s and, at 100 Poisson arrivals per second, p50/p99 time-to-solution,
beside the same requests solved one at a time in FP64.

Prints one JSON line: MLUPS (million lattice-node updates per second), the
HBM roofline of the fused update kernel (algorithmic bytes 2*Q*4 per node;
kernel time from a HIP event pair on the library's stream around the timed
K steps, less a one-step call that holds the field-writing launch and the
reductions, over K - 1), and the FP64 oracle timed on the host on a bounded
sample of the same workload.  Beside it, a practical ceiling measured in the
same run (libceiling.so): the update's own pull-and-store pattern with no
collision arithmetic, and a copy, both alternating between two buffers.

    python bench.py --traffic-from FETCH.csv WRITE.csv
rewrites profiles/traffic.json from two rocprofv3 --pmc counter files
(FETCH_SIZE, WRITE_SIZE) of a bench run, each calibrated by the same counter
on the 1 GiB device copy the bench performs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published
KERNEL = "step_rows_kernel<D2Q17, CF32, false, false>"
WORKLOAD = "D2Q17 2048x2048 FP32"


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SOURCES = ("lbm_device.hpp", "lattice_tables.h", "lbm_internal.hpp")


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1209_5201_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated by the copy kernel), if it
    was taken on the current kernel sources; else None."""
    try:
        with open(TRAFFIC_JSON) as fh:
            ent = json.load(fh)[kernel]
        if ent.get("workload") != workload or ent.get("source_sha") != kernel_source_digest():
            return None
        return float(ent["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def write_traffic(fetch_csv: str, write_csv: str, kernel_match: str, kernel: str,
                  workload: str):
    """Per-dispatch KiB of FETCH_SIZE / WRITE_SIZE for the kernel, each scaled
    by (bytes the 1 GiB copy moves) / (what the counter reads for it)."""
    import csv

    def per_kernel(path, counter):
        copy, kern = [], []
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            val = float(row["Counter_Value"]) * 1024.0
            if "copyBuffer" in row["Kernel_Name"] and int(row["Grid_Size"]) >= 131072:
                copy.append(val)
            elif kernel_match in row["Kernel_Name"]:
                kern.append(val)
        return sum(copy) / len(copy), sum(kern) / len(kern), len(kern)

    gib = float(1 << 30)
    c_f, k_f, n_f = per_kernel(fetch_csv, "FETCH_SIZE")
    c_w, k_w, n_w = per_kernel(write_csv, "WRITE_SIZE")
    fetch = k_f * gib / c_f
    write = k_w * gib / c_w
    try:
        data = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        data = {}
    data[kernel] = {"workload": workload, "source_sha": kernel_source_digest(),
                    "bytes_per_launch": fetch + write, "fetch_bytes": fetch,
                    "write_bytes": write, "fetch_scale": gib / c_f, "write_scale": gib / c_w,
                    "dispatches": [n_f, n_w]}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(data, fh, indent=1)
    print(json.dumps(data[kernel]))


def cpu_baseline(cfg, nsteps: int):
    """The FP64 oracle on the host: same grid and start field, nsteps steps."""
    import numpy as np  # noqa: F401
    from oracle import oracle as O
    from paper_1209_5201_amd import workloads as W
    rho = W.c3_density(cfg["nx"], cfg["ny"], seed=cfg["seed"], amp=cfg["amp"])
    case = O.OracleCase(cfg["lattice"], cfg["nx"], cfg["ny"],
                        O.tau_from_kn(cfg["lattice"], cfg["ny"], cfg["kn"]),
                        cfg["bottom"], cfg["top"], rho0=rho)
    t0 = time.perf_counter()
    case.run(nsteps)
    dt = time.perf_counter() - t0
    return {"value": cfg["nx"] * cfg["ny"] * nsteps / dt / 1e6, "unit": "MLUPS",
            "cores": 1, "kind": "oracle",
            "sample": "%s %dx%d FP64, %d steps (%.1f s), single-threaded C"
                      % (cfg["lattice"], cfg["nx"], cfg["ny"], nsteps, dt)}


def serving(n_requests: int, rate: float, baseline_cases: int):
    """Couette serving stream (FP32, residual 1e-8): saturated throughput
    with every request queued at t = 0, then latency at a fixed Poisson
    arrival rate; the same stream with a quarter of the requests replaced by
    force-driven channels; the same first `baseline_cases` requests solved
    one at a time in FP64 as the baseline."""
    from paper_1209_5201_amd import serve
    from paper_1209_5201_amd import workloads as W
    reqs = W.serving_requests(n=n_requests, seed=1, rate=rate)
    sat = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
        reqs, realtime=False)
    live = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
        reqs, realtime=True)
    mixed_reqs = W.serving_requests(n=n_requests, seed=1, rate=rate, channel_fraction=0.25)
    mixed_sat = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
        mixed_reqs, realtime=False)
    mixed_live = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
        mixed_reqs, realtime=True)
    base = serve.one_at_a_time(reqs[:baseline_cases], prec="fp64")
    same = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
        reqs[:baseline_cases], realtime=False)

    def r(x):
        return round(x, 4)
    return {"requests": n_requests, "precision": "fp32", "tolerance": 1e-8,
            "saturated_solves_per_s": r(sat["solves_per_s"]),
            "saturated_converged": sat["converged"],
            "arrival_rate_per_s": rate,
            "solves_per_s": r(live["solves_per_s"]),
            "p50_time_to_solution_s": r(live["p50_s"]), "p99_time_to_solution_s": r(live["p99_s"]),
            "p50_service_s": r(live["p50_service_s"]), "p99_service_s": r(live["p99_service_s"]),
            "with_channels": {
                "requests": n_requests, "force_driven_channels": sum("umax" in q for q in mixed_reqs),
                "saturated_solves_per_s": r(mixed_sat["solves_per_s"]),
                "saturated_converged": mixed_sat["converged"],
                "solves_per_s": r(mixed_live["solves_per_s"]),
                "p50_time_to_solution_s": r(mixed_live["p50_s"]),
                "p99_time_to_solution_s": r(mixed_live["p99_s"])},
            "baseline": {"kind": "one at a time, FP64, same library", "requests": baseline_cases,
                         "solves_per_s": r(base["solves_per_s"]),
                         "batched_fp32_same_requests_solves_per_s": r(same["solves_per_s"])}}


def precision_table(torch, steps_2d: int = 200, steps_3d: int = 60):
    """MLUPS and algorithmic HBM rate of the fused update per velocity set and
    storage format: the bulk 2048^2 case on D2Q16 and D2Q17, and the D3Q121
    1024^2 case (walls -0.1 / +0.1, Kn 0.05).  Wall clock over back-to-back steps (one
    launch per step); fields refreshed once at the end.  Each row also gives
    the same-run pull ceiling for its element size and the fraction of it the
    update reaches."""
    import paper_1209_5201_amd as lbm
    from paper_1209_5201_amd import workloads as W
    rows = []
    for lat, nx, ny, steps, walls in (
            ("D2Q16", 2048, 2048, steps_2d, (W.C3["bottom"], W.C3["top"])),
            ("D2Q17", 2048, 2048, steps_2d, (W.C3["bottom"], W.C3["top"])),
            ("D3Q121", W.C5["nx"], W.C5["ny"], steps_3d, (W.C5["bottom"], W.C5["top"]))):
        Q = lbm.lbm_lattice_info(lat)["Q"]
        ceilings = {}   # pull ceiling per element size, for this set and grid
        for prec, b in (("fp64", 8), ("fp32", 4), ("fp32s", 4), ("bf16", 2), ("fp16", 2)):
            ch = lbm.Channel(lat, nx, ny, lbm.lbm_tau_from_kn(lat, ny, 0.05), *walls, prec=prec)
            ch.step(10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch.step(steps)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ch.close()
            gbps = 2.0 * Q * b * nx * ny / dt / 1e9
            row = {"lattice": lat, "grid": "%dx%d" % (nx, ny), "precision": prec,
                   "MLUPS": round(nx * ny / dt / 1e6, 1), "us_per_step": round(dt * 1e6, 1),
                   "alg_GBps": round(gbps, 1), "frac_hbm": round(gbps / HBM_PEAK_GBPS, 3)}
            if b not in ceilings:
                ceilings[b] = practical_ceiling(lat, nx, ny, elem_bytes=b)["pull_GBps"]
            row["pull_ceiling_GBps"] = round(ceilings[b], 1)
            row["frac_of_pull_ceiling"] = round(gbps / ceilings[b], 3)
            rows.append(row)
    return rows


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy rate (read + write bytes / time) as a practical
    HBM ceiling, measured in the same run."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    e.synchronize()
    return 2.0 * nbytes * reps / (s.elapsed_time(e) * 1e-3) / 1e9


def practical_ceiling(lattice: str, nx: int, ny: int, elem_bytes: int = 4,
                      reps: int = 50) -> dict:
    """Bandwidth references from libceiling.so, measured in the same run: the
    update's own pull-and-store pattern with no collision arithmetic, on
    elements of the storage format's size, and a 16-byte-per-lane copy of the
    same state.  Both alternate between
    two buffers, as the update does; with a fixed source buffer, part of
    every read would come from the memory-side cache."""
    import ctypes
    from paper_1209_5201_amd.lbm import LATTICES
    path = os.path.join(ROOT, "paper_1209_5201_amd", "libceiling.so")
    if not os.path.exists(path):
        raise RuntimeError("libceiling.so is not built (python -m paper_1209_5201_amd.build)")
    fn = ctypes.CDLL(path).lbm_ceiling
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)] * 4
    out = [ctypes.c_double() for _ in range(4)]
    rc = fn(LATTICES[lattice], elem_bytes, nx, ny, reps, *[ctypes.byref(v) for v in out])
    if rc != 0:
        raise RuntimeError("lbm_ceiling failed (%d)" % rc)
    pull_us, copy_us, pull_bytes, copy_bytes = (v.value for v in out)
    return {"pull_GBps": pull_bytes / pull_us / 1e3, "pull_us": pull_us,
            "copy_GBps": copy_bytes / copy_us / 1e3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--serving-requests", type=int, default=1024)
    ap.add_argument("--serving-rate", type=float, default=100.0)
    ap.add_argument("--serving-baseline", type=int, default=16)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-precisions", action="store_true")
    ap.add_argument("--profile-formats", type=int, metavar="STEPS",
                    help="only run the D3Q121 1024^2 channel STEPS steps in every storage "
                         "format (a short run to trace under rocprofv3) and exit")
    ap.add_argument("--profile-serving", type=int, metavar="REQUESTS",
                    help="only serve the first REQUESTS requests of the serving stream "
                         "(FP32, all queued at t = 0; a run to trace) and exit")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args.traffic_from[0], args.traffic_from[1],
                      "step_rows_kernel<lbm::D2Q17, lbm::dev::CF32, false, false>", KERNEL,
                      WORKLOAD)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the single-GPU share is the "
              "workload (a multi-GPU run would split x into slabs with a "
              "3-column halo exchange, which this library does not implement)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch
    import paper_1209_5201_amd as lbm
    from paper_1209_5201_amd import workloads as W

    if args.profile_formats:
        c = W.C5
        out = {}
        for prec in ("fp64", "fp32", "fp32s", "bf16", "fp16"):
            ch = lbm.Channel("D3Q121", c["nx"], c["ny"],
                             lbm.lbm_tau_from_kn("D3Q121", c["ny"], c["kn"]), c["bottom"],
                             c["top"], prec=prec)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ch.step(args.profile_formats)
            torch.cuda.synchronize()
            out[prec] = round((time.perf_counter() - t0) / args.profile_formats * 1e6, 1)
            ch.close()
        print(json.dumps({"workload": "D3Q121 1024x1024 Couette, every format",
                          "us_per_step": out}), flush=True)
        return
    if args.profile_serving:
        from paper_1209_5201_amd import serve
        reqs = W.serving_requests(n=args.profile_serving, seed=1, rate=args.serving_rate)
        res = serve.Server(prec="fp32", window=100, tol=1e-8, keep_profiles=False).run(
            reqs, realtime=False)
        print(json.dumps({"workload": "serving stream, first %d requests" % args.profile_serving,
                          "solves": res["solves"], "solves_per_s": round(res["solves_per_s"], 1),
                          "launches": res["launches"]}), flush=True)
        return

    torch.cuda.set_device(0)
    cfg = W.C3
    nx, ny, lat = cfg["nx"], cfg["ny"], cfg["lattice"]
    Q = lbm.lbm_lattice_info(lat)["Q"]
    tau = lbm.lbm_tau_from_kn(lat, ny, cfg["kn"])
    ch = lbm.Channel(lat, nx, ny, tau, cfg["bottom"], cfg["top"], prec=cfg["prec"])
    ch.init(rho=W.c3_density(nx, ny, seed=cfg["seed"], amp=cfg["amp"]))
    if args.warmup:
        ch.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, nothing else on the stream; a HIP event pair on
    # the library's stream brackets it
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    ch.step(args.steps)
    ev[1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mass = ch.mass()
    # a one-step call: the launch that also writes the output fields and the
    # two reduction launches, which close every call; the other K - 1
    # launches of the timed region are the plain fused update
    ev[2].record(stream)
    ch.step(1)
    ev[3].record(stream)
    torch.cuda.synchronize()
    region_ms = ev[0].elapsed_time(ev[1])
    tail_ms = ev[2].elapsed_time(ev[3])
    elapsed = t1 - t0
    nodes = nx * ny
    mlups = nodes * args.steps / elapsed / 1e6
    upd_s = (region_ms - tail_ms) / max(args.steps - 1, 1) * 1e-3
    alg_bytes = 2.0 * Q * 4 * nodes          # read Q + write Q FP32 populations
    achieved = alg_bytes / upd_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic_from_profile(KERNEL, WORKLOAD),
            "kernel": KERNEL, "kernel_us": round(upd_s * 1e6, 2),
            "bytes_per_launch": alg_bytes,
            "kernel_timing": "HIP events on the library stream around the timed K steps, "
                             "less a one-step call (field-writing launch + reductions), "
                             "over K - 1"}
    line = {
        "metric": "MLUPS (FP32 fused stream-collide, HBM roofline)",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D bulk bandwidth: D2Q17 2048x2048, diffuse walls at rest, "
                               "Kn=0.05, rho=1+1e-3 N(0,1) seed 0, FP32 populations",
                   "nx": nx, "ny": ny, "lattice": lat, "precision": "fp32",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "copy_ref_GBps": round(copy_bandwidth(torch), 1),
        "mass_after": mass,
    }
    ceil = practical_ceiling(lat, nx, ny)
    line["practical_ceiling"] = {
        "kind": "same run, FP32, two buffers alternating: the update's pull-and-store pattern "
                "with no collision arithmetic (rows N..ny-N-1), and a 16-byte copy of the state",
        "pull_no_arithmetic_GBps": round(ceil["pull_GBps"], 1),
        "copy_GBps": round(ceil["copy_GBps"], 1),
        "kernel_frac_of_pull": round(achieved / ceil["pull_GBps"], 4)}
    ch.close()
    if not args.no_precisions:
        line["precisions"] = precision_table(torch)
    if not args.no_serving:
        line["serving"] = serving(args.serving_requests, args.serving_rate,
                                  args.serving_baseline)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, args.cpu_steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
