"""Host-side grouping of batched cases by storage format (one launch per
format present): every case gets one slot, the groups tile 0..n exactly
and keep input order.  Compiled with the system C++ compiler; no GPU."""
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1209_5201_amd", "csrc")

DRIVER = r"""
#include "batch_plan.hpp"
#include <cstdio>
int main() {
  int nfmt, n;
  while (std::scanf("%d %d", &nfmt, &n) == 2) {
    int fmt[256], start[16], pos[256];
    for (int i = 0; i < n; ++i) std::scanf("%d", &fmt[i]);
    const bool ok = lbm::plan_groups(fmt, n, nfmt, start, pos);
    std::printf("%d", ok ? 1 : 0);
    if (ok) {
      for (int p = 0; p <= nfmt; ++p) std::printf(" %d", start[p]);
      for (int i = 0; i < n; ++i) std::printf(" %d", pos[i]);
    }
    std::printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def planner(tmp_path_factory):
    d = tmp_path_factory.mktemp("plan")
    src, exe = d / "drv.cpp", d / "drv"
    src.write_text(DRIVER)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)])

    def run(nfmt, fmts):
        out = subprocess.run([str(exe)], input="%d %d %s\n" % (nfmt, len(fmts),
                                                              " ".join(map(str, fmts))),
                             capture_output=True, text=True, check=True).stdout.split()
        vals = list(map(int, out))
        if vals[0] == 0:
            return None
        return vals[1:nfmt + 2], vals[nfmt + 2:]
    return run


@pytest.mark.parametrize("nfmt", [4, 5])
def test_groups_tile_the_cases_in_order(planner, nfmt):
    rng = np.random.default_rng(nfmt)
    cases = [[0] * 4, [nfmt - 1] * 3, [1, 0, 1, 0]] + \
        [list(rng.integers(0, nfmt, size=int(rng.integers(1, 60)))) for _ in range(20)]
    for fmts in cases:
        start, pos = planner(nfmt, fmts)
        n = len(fmts)
        assert start[0] == 0 and start[nfmt] == n
        assert all(start[p + 1] - start[p] >= 0 for p in range(nfmt))
        assert sorted(pos) == list(range(n))
        for i, f in enumerate(fmts):
            assert start[f] <= pos[i] < start[f + 1]
            for j in range(i):
                if fmts[j] == f:
                    assert pos[j] < pos[i]


def test_out_of_range_format_is_rejected(planner):
    assert planner(5, [0, 5, 1]) is None
    assert planner(5, [-1]) is None
