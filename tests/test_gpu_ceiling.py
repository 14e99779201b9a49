"""GPU check of libceiling.so, the bandwidth references bench.py reports
beside the fused update: on a small grid every element size runs, the byte
counts are the pattern's (2 Q b per node over the rows N..ny-N-1; twice the
padded state for the copy) and the rates are positive and below the HBM
peak by a margin no real run exceeds."""
import ctypes
import os
import sys

import pytest

import paper_1209_5201_amd as lbm

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ceiling(lattice, elem_bytes, nx, ny, reps):
    fn = ctypes.CDLL(os.path.join(ROOT, "paper_1209_5201_amd", "libceiling.so")).lbm_ceiling
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_double)] * 4
    out = [ctypes.c_double(-1.0) for _ in range(4)]
    rc = fn(lbm.lbm.LATTICES[lattice], elem_bytes, nx, ny, reps, *[ctypes.byref(v) for v in out])
    return rc, [v.value for v in out]


@pytest.mark.parametrize("lattice,nx,ny", [("D2Q17", 512, 64), ("D3Q121", 256, 16)])
@pytest.mark.parametrize("elem_bytes", [8, 4, 2])
def test_ceiling_kernels_run_and_count_bytes(lattice, nx, ny, elem_bytes):
    print("case ceiling", lattice, nx, ny, elem_bytes, flush=True)
    sys.stdout.flush()
    info = lbm.lbm_lattice_info(lattice)
    Q, N = info["Q"], info["N"]
    rc, (pull_us, copy_us, pull_bytes, copy_bytes) = ceiling(lattice, elem_bytes, nx, ny, 3)
    assert rc == 0
    assert pull_bytes == 2.0 * elem_bytes * Q * nx * (ny - 2 * N)
    plane = (nx * ny + 63) // 64 * 64 + 128
    assert copy_bytes == 2.0 * elem_bytes * Q * plane
    for us, nbytes in ((pull_us, pull_bytes), (copy_us, copy_bytes)):
        assert us > 0.0
        assert nbytes / (us * 1e-6) < 1.5 * 8e12   # bytes per second, peak 8 TB/s
