"""Compile-time checks of the velocity bookkeeping the kernels rely on, by
hipcc on the host (syntax only, no GPU): the opposite of a velocity is an
involution with -c, the f^eq pairing and the node split keep each pair
{c, -c} together, every velocity belongs to exactly one part, the parts are
balanced, and the rest velocity goes to part 0.  A failed static_assert is
a compile error."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1209_5201_amd", "csrc")
INCLUDE = os.path.join(HERE, "..", "include")

CHECKS = r"""
#include "lbm_device.hpp"

namespace chk {
using namespace lbm;
using namespace lbm::dev;

template <class L>
constexpr bool opposite_is_minus_c() {
  for (int q = 0; q < L::Q; ++q) {
    const int o = opposite<L>(q);
    if (o < 0 || opposite<L>(o) != q) return false;
    for (int k = 0; k < 3; ++k)
      if (L::E[o][k] != -L::E[q][k]) return false;
    const bool rest = L::E[q][0] == 0 && L::E[q][1] == 0 && L::E[q][2] == 0;
    if ((o == q) != rest) return false;
  }
  return true;
}

template <class L, int P, int PART>
constexpr int part_size() {
  int n = 0;
  for (int q = 0; q < L::Q; ++q) n += in_part<L, PART, P>(q) ? 1 : 0;
  return n;
}

template <class L, int P>
constexpr bool partition_ok() {
  static_assert(P >= 1 && P <= 4, "checked for up to four parts");
  int lo = L::Q, hi = 0, total = 0;
  for (int q = 0; q < L::Q; ++q) {
    int owners = 0;
    for (int p = 0; p < P; ++p) {
      const bool in = p == 0 ? in_part<L, 0, P>(q) : p == 1 ? in_part<L, 1, P>(q)
                    : p == 2 ? in_part<L, 2, P>(q) : in_part<L, 3, P>(q);
      if (in) {
        ++owners;
        // the pair stays in one part
        const int o = opposite<L>(q);
        const bool oin = p == 0 ? in_part<L, 0, P>(o) : p == 1 ? in_part<L, 1, P>(o)
                       : p == 2 ? in_part<L, 2, P>(o) : in_part<L, 3, P>(o);
        if (!oin) return false;
        // the rest velocity belongs to part 0
        if (o == q && p != 0) return false;
      }
    }
    if (owners != 1) return false;
  }
  const int sizes[4] = {part_size<L, P, 0>(), P > 1 ? part_size<L, P, 1>() : 0,
                        P > 2 ? part_size<L, P, 2>() : 0, P > 3 ? part_size<L, P, 3>() : 0};
  for (int p = 0; p < P; ++p) {
    total += sizes[p];
    lo = sizes[p] < lo ? sizes[p] : lo;
    hi = sizes[p] > hi ? sizes[p] : hi;
  }
  // one pair (two velocities) plus the rest velocity at most between parts
  return total == L::Q && hi - lo <= 3;
}

template <class L>
constexpr bool whole_set_is_part_minus_one() {
  for (int q = 0; q < L::Q; ++q)
    if (!in_part<L, -1, 1>(q)) return false;
  return true;
}

static_assert(opposite_is_minus_c<D2Q16>(), "D2Q16 opposite");
static_assert(opposite_is_minus_c<D2Q17>(), "D2Q17 opposite");
static_assert(opposite_is_minus_c<D3Q121>(), "D3Q121 opposite");
static_assert(whole_set_is_part_minus_one<D3Q121>(), "PART = -1 is the whole set");
static_assert(partition_ok<D2Q16, 2>() && partition_ok<D2Q16, 4>(), "D2Q16 parts");
static_assert(partition_ok<D2Q17, 2>() && partition_ok<D2Q17, 4>(), "D2Q17 parts");
static_assert(partition_ok<D3Q121, 2>() && partition_ok<D3Q121, 4>(), "D3Q121 parts");
// the split the batched FP32 kernel uses: 31 / 30 / 30 / 30 velocities
static_assert(part_size<D3Q121, 4, 0>() == 31 && part_size<D3Q121, 4, 3>() == 30, "sizes");
// the batched kernel's launch shape and split
static_assert(batch_threads<CF32, false>() == 1024 && batch_parts<D3Q121, CF32, false>() == 4,
              "FP32 split");
static_assert(batch_parts<D3Q121, CF32, true>() == 1 && batch_parts<D2Q17, CF32, false>() == 1,
              "whole nodes elsewhere");
}  // namespace chk
"""


def test_velocity_pairs_and_parts_compile(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "checks.hip"
    src.write_text(CHECKS)
    # the checks evaluate every (velocity, part) pair at compile time: more
    # constant-evaluation steps than clang's default allows on D3Q121; the
    # host pass alone evaluates them
    res = subprocess.run([hipcc, "-std=c++17", "--offload-arch=gfx950", "--cuda-host-only",
                          "-fsyntax-only", "-fconstexpr-steps=100000000", "-I", INCLUDE, "-I",
                          CSRC, str(src)],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-4000:]
