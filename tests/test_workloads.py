"""Host-side request generation and the force-driven channel recipe (no
GPU): the serving stream is seeded and its Couette draws do not depend on
the share of channel requests; the server's body force, derived from the
library's tables, gives the no-slip Navier-Stokes peak velocity by the
oracle's own tables."""
import math

import numpy as np

from oracle import lattices as OL
from paper_1209_5201_amd import serve
from paper_1209_5201_amd import workloads as W


def test_serving_stream_is_seeded_and_kind_draws_are_separate():
    a = W.serving_requests(64, seed=3)
    b = W.serving_requests(64, seed=3)
    c = W.serving_requests(64, seed=3, channel_fraction=0.5)
    assert a == b
    for x, y in zip(a, c):
        assert (x["lattice"], x["ny"], x["kn"], x["arrival"]) == \
            (y["lattice"], y["ny"], y["kn"], y["arrival"])
        if "umax" in y:
            assert y["bottom"][0] == 0.0 and y["top"][0] == 0.0
            assert abs(y["umax"] - x["top"][0]) < 1e-15
    n = sum("umax" in r for r in W.serving_requests(2000, seed=1, channel_fraction=0.25))
    assert 400 < n < 600
    t = [r["arrival"] for r in a]
    assert all(np.diff(t) > 0)


def test_channel_force_gives_the_navier_stokes_peak():
    """u_max = (a/nu)/8 in channel units with nu = sqrt(2/pi) Kn (tau of
    Sec. II with mu = p = 1) and one step = 1/(r ny) of time."""
    for name in ("D2Q16", "D2Q17", "D3Q121"):
        r = OL.by_name(name).r
        for ny, kn, U in ((32, 0.01, 0.1), (200, 0.3, 0.02)):
            a_lat = serve.channel_force(name, ny, kn, U)
            dt = 1.0 / (r * ny)
            nu = math.sqrt(2 / math.pi) * kn
            assert abs((a_lat / dt) / nu / 8 - U) < 1e-12 * U
