"""Builds ``liblbm.so`` (the HIP library for gfx950) in-tree with hipcc,
and ``libceiling.so``, the bandwidth references that ``bench.py`` reports
beside the update (``csrc/ceiling_probe.hip``; not used by ``liblbm.so``).

    python -m paper_1209_5201_amd.build [--verbose]

Always recompiles.  --verbose prints the per-kernel register / LDS / spill
report of the compiler.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblbm.so")
CEILING_LIB = os.path.join(PKG, "libceiling.so")
CEILING_SOURCES = [os.path.join(CSRC, "ceiling_probe.hip")]
BUILD = os.path.join(PKG, "_build")
SOURCES = [os.path.join(CSRC, "lbm_set_%s_%s%s.hip" % (s, p, f))
           for s in ("d3q121", "d2q17", "d2q16") for p in ("fp64", "fp32", "bf16", "fp16", "fp32s")
           for f in ("", "_force")] + \
    [os.path.join(CSRC, "lbm_batch_%s%s.hip" % (p, f))
     for p in ("fp64", "fp32", "bf16", "fp16", "fp32s") for f in ("", "_force")] + \
    [os.path.join(CSRC, "lbm_batch_%s_3d%s.hip" % (p, f))
     for p in ("fp64", "fp32s") for f in ("", "_force")] + \
    [os.path.join(CSRC, "lbm_dispatch.hip"), os.path.join(CSRC, "lbm_api.cpp")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 VALU forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if verbose:
        cmd += ["-Rpass-analysis=kernel-resource-usage"]
    cmd += ["-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return obj, res


def _link(objs, out: str):
    tmp = out + ".tmp%d" % os.getpid()
    link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link of %s failed (exit %d)" % (os.path.basename(out), res.returncode))
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one process each) and link both
    libraries; returns the path of liblbm.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    sources = SOURCES + CEILING_SOURCES
    workers = max(1, min(len(sources), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), sources))
    for obj, res in results:
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed on %s (exit %d)" % (obj, res.returncode))
        if verbose:
            sys.stderr.write(res.stderr)
    objs = [obj for obj, _ in results]
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], CEILING_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
