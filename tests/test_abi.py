"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/lbm.h declares, reports velocity sets that satisfy
their defining moment conditions, and rejects invalid arguments before any
device work."""
import ctypes
import itertools
import math
import os
import re

import mpmath
import numpy as np
import pytest

import paper_1209_5201_amd as lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(lbm.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 17
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers every declaration
    assert set(names) <= set(lbm.lbm.exported_symbols())


def gauss(m):
    v = 1.0
    for k in m:
        if k % 2:
            return 0.0
        v *= float(mpmath.fac2(k - 1)) if k > 0 else 1.0
    return v


@pytest.mark.parametrize("name,degree,Q,N", [("D2Q17", 7, 17, 3), ("D3Q121", 9, 121, 3)])
def test_library_lattice_tables_satisfy_moment_conditions(name, degree, Q, N):
    info = lbm.lbm_lattice_info(name)
    assert info["Q"] == Q and info["N"] == N and info["eq_order"] == 4
    D = info["D"]
    c = info["r"] * info["e"][:, :D].astype(float)
    w = info["w"]
    assert np.all(w > 0)
    for m in itertools.product(range(degree + 1), repeat=D):
        if sum(m) <= degree:
            got = float(np.sum(w * np.prod(c ** np.array(m), axis=1)))
            assert abs(got - gauss(m)) < 2e-14 * max(1.0, gauss(m)), m


def test_library_d2q16_is_the_tensor_rule():
    info = lbm.lbm_lattice_info("D2Q16")
    assert info["Q"] == 16 and info["eq_order"] == 2
    assert abs(info["r"] - math.sqrt(5) / 3) < 1e-16
    one = {1: 0.45, 3: 0.05}
    for e, w in zip(info["e"], info["w"]):
        assert abs(w - one[abs(e[0])] * one[abs(e[1])]) < 1e-17


def test_tau_from_kn():
    r = lbm.lbm_lattice_info("D3Q121")["r"]
    assert abs(lbm.lbm_tau_from_kn("D3Q121", 256, 0.1) - math.sqrt(2 / math.pi) * 0.1 * r * 256) \
        < 1e-12
    assert math.isnan(lbm.lbm_tau_from_kn("D2Q17", 32, -1.0))


def test_required_bytes_and_limits():
    b = lbm.lbm_required_bytes("D2Q17", 2048, 2048, "fp32")
    pops = 2 * 17 * 2048 * 2048 * 4
    assert pops < b <= pops + 13 * 8 * 2048 * 2048 + (1 << 20) * 2
    assert lbm.lbm_required_bytes("D2Q17", 1, 5, "fp64") == 0     # ny < 2N
    assert lbm.lbm_required_bytes("D2Q17", 0, 32, "fp64") == 0
    assert lbm.lbm_required_bytes("D3Q121", 1024, 1024, "bf16") < \
        lbm.lbm_required_bytes("D3Q121", 1024, 1024, "fp32") == \
        lbm.lbm_required_bytes("D3Q121", 1024, 1024, "fp32s")
    assert lbm.lbm_required_bytes("D2Q17", 64, 64, 5) == 0    # no such format


@pytest.mark.parametrize("kwargs", [
    dict(lattice="D2Q17", nx=1, ny=32, tau=0.0),                       # tau <= 0
    dict(lattice="D2Q17", nx=1, ny=4, tau=1.0),                        # ny < 2N
    dict(lattice="D2Q17", nx=1, ny=32, tau=1.0, top=(0.1, 0.0, 1.1)),  # T != 1 isothermal
    dict(lattice="D2Q16", nx=1, ny=32, tau=1.0, top=(0.1, 0.2, 1.0)),  # uz on a 2-D set
    dict(lattice="D3Q121", nx=1, ny=32, tau=1.0, top=(float("nan"), 0.0, 1.0)),
    dict(lattice="D3Q121", nx=1, ny=32, tau=1.0, top=(0.0, 0.0, -1.0)),
])
def test_create_rejects_invalid_arguments_without_device_work(kwargs):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.lbm_create(**kwargs)
    assert ei.value.status == lbm.lbm.LBM_EINVAL


def test_null_context_is_rejected():
    lib = ctypes.CDLL(lbm.LIB_PATH)
    lib.lbm_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
    assert lib.lbm_step(None, 1) == lbm.lbm.LBM_EINVAL
    assert lbm.lbm_strerror(lbm.lbm.LBM_ENEGATIVE).startswith("wall Maxwellian")
    lib.lbm_set_accommodation.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double]
    assert lib.lbm_set_accommodation(None, 0.5, 0.5) == lbm.lbm.LBM_EINVAL


def test_ceiling_library_rejects_invalid_arguments_before_device_work():
    """libceiling.so (the bandwidth references bench.py reports) exports its
    one entry point and refuses unusable shapes without touching a device."""
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1209_5201_amd", "libceiling.so"))
    fn = lib.lbm_ceiling
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)] * 4
    out = [ctypes.c_double(-1.0) for _ in range(4)]
    refs = [ctypes.byref(v) for v in out]
    assert fn(1, 4, 2048, 2048, 10, None, *refs[1:]) == -1   # null output
    assert fn(3, 4, 2048, 2048, 10, *refs) == -1             # no such set
    assert fn(1, 3, 2048, 2048, 10, *refs) == -1             # no such element size
    assert fn(1, 4, 2000, 2048, 10, *refs) == -1             # nx not a multiple of 256
    assert fn(1, 2, 2048, 6, 10, *refs) == -1                # ny <= 2N
    assert fn(2, 8, 1024, 1024, 0, *refs) == -1              # no repetitions
    assert all(v.value == -1.0 for v in out)
