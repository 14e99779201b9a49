// Device code for gfx950 (MI355X): the fused pull-stream + diffuse-wall +
// BGK-collide update of the multi-speed lattice Boltzmann scheme of
// Meng & Zhang (arXiv:1209.5201), plus its initialisation and the FP64
// reductions.
//
// Data layout: structure-of-arrays population planes, plane q holds f*_q of
// every node at element q*plane + y*nx + x.  A step reads plane set A and
// writes plane set B (no in-place hazards).
//
// Per step, two launches:
//  1. wall_kernel: one wavefront per (wall, ghost column) gathers the mass
//     that the post-collision populations send into the N ghost layers of
//     that column (the numerator of Eq. (eq:dkboundary)), summing the terms
//     in FP64 in a fixed order, and stores ratio = M / D.
//  2. step_kernel: one thread per node pulls f~_q(x, y) = f*_q(x - e_x,
//     y - e_y); when the source lies in a ghost layer the value is the
//     re-emitted g^eq_q(u_w, T_w) * ratio of that ghost column (same-step
//     re-emission).  Then moments, f^eq (Eq. (eq:feq)) and the relaxation of
//     Eq. (eq:scheme), and a coalesced store of f*.
// The velocity set is a compile-time table: every per-velocity constant
// (integer e, weight w, |c|^2) is an immediate and the loop over velocities
// is fully unrolled.  The stencil is HBM-bound (2 Q element transfers per
// node update), so no matrix cores are involved.
#pragma once

#include "lbm_internal.hpp"
#include "lattice_tables.h"

#include <hip/hip_fp16.h>

#include <cstdint>
#include <type_traits>

namespace lbm {
namespace dev {

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// acc + k * v for a small compile-time integer k, without multiplies for
// k = +-1.
template <int K, class R>
__device__ __forceinline__ R add_scaled(R acc, R v) {
  if constexpr (K == 0) return acc;
  else if constexpr (K == 1) return acc + v;
  else if constexpr (K == -1) return acc - v;
  else return acc + R(K) * v;
}

// k * v for a small compile-time integer k (the first term of a sum: no
// addition to a zero, which IEEE arithmetic cannot drop because of -0).
template <int K, class R>
__device__ __forceinline__ R scaled(R v) {
  if constexpr (K == 1) return v;
  else if constexpr (K == -1) return -v;
  else return R(K) * v;
}

// acc + k * v, or k * v alone when FIRST (acc not yet assigned).
template <int K, bool FIRST, class R>
__device__ __forceinline__ R accum(R acc, R v) {
  if constexpr (K == 0) return acc;
  else if constexpr (FIRST) return scaled<K>(v);
  else return add_scaled<K>(acc, v);
}

// e_x a + e_y b + e_z c for a compile-time integer vector e.
template <int EX, int EY, int EZ, class R>
__device__ __forceinline__ R dot_e(R a, R b, R c) {
  if constexpr (EX != 0) return add_scaled<EZ>(add_scaled<EY>(scaled<EX>(a), b), c);
  else if constexpr (EY != 0) return add_scaled<EZ>(scaled<EY>(b), c);
  else if constexpr (EZ != 0) return scaled<EZ>(c);
  else return R(0);
}

// Index of the velocity -c_q, and the first velocity with a nonzero
// component k (k = 3: nonzero |c|^2).
template <class L>
constexpr int opposite(int q) {
  for (int p = 0; p < L::Q; ++p)
    if (L::E[p][0] == -L::E[q][0] && L::E[p][1] == -L::E[q][1] && L::E[p][2] == -L::E[q][2])
      return p;
  return -1;
}
// Velocity subsets for a node split over P groups of lanes: the pairs
// {c, -c} in the order of their lower index are dealt round-robin to the
// parts, the rest velocity to part 0.  PART = -1 is the whole set.
template <class L>
constexpr int pair_rank(int q) {
  const int o = opposite<L>(q);
  if (o == q) return -1;
  const int lo = q < o ? q : o;
  int r = 0;
  for (int p = 0; p < lo; ++p)
    if (opposite<L>(p) > p) ++r;
  return r;
}
template <class L, int PART, int P>
constexpr bool in_part(int q) {
  if constexpr (PART < 0) {
    return true;
  } else {
    const int r = pair_rank<L>(q);
    return (r < 0 ? 0 : r % P) == PART;
  }
}

template <class L>
constexpr int first_nonzero(int k) {
  for (int p = 0; p < L::Q; ++p) {
    const int v = k < 3 ? L::E[p][k]
                        : L::E[p][0] * L::E[p][0] + L::E[p][1] * L::E[p][1] + L::E[p][2] * L::E[p][2];
    if (v != 0) return p;
  }
  return -1;
}

// ---------------------------------------------------------------- codecs --
// Population planes are accessed through buffer resources (one descriptor
// per plane set): the per-velocity plane offset q * plane * bytes is a
// scalar (SGPR) operand and the in-plane node offset a 32-bit vector
// operand shared by every velocity with the same shift, so the unrolled
// Q-velocity pulls need no 64-bit address arithmetic.  Accesses beyond the
// descriptor's size return 0 instead of faulting.
using Rsrc = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  // word 3 = 0x00020000: raw (untyped) dword access on the gfx9 family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, int(bytes), 0x00020000);
}

// Storage <-> arithmetic.  Every format holds the deviation g = f - w_q from
// the rest state, so rounding acts on the (small) deviation, not on f.
// 16-bit formats hold h = g * S for a per-format power of two S (a
// compile-time constant: 2^12 for FP16, 1 for BF16) and decode to float.  They round
// stochastically: a slowly varying population rounded to nearest is rounded
// the same way every step, and that bias accumulates in the conserved
// moments over the flow's momentum-diffusion time; unbiased rounding leaves a
// random walk instead (about 20x smaller errors for FP16 and BF16 in channel
// flows).  The random bits come from a counter-based hash of (node,
// velocity, step), so runs are reproducible.
// Stores of the grid-wide update are nontemporal (cache policy 2 = nt): a
// step's output is read only by the next step, after the whole grid has been
// written, so keeping it in L2 buys nothing and streaming stores sustain a
// higher HBM write rate.  The persistent small-case kernel stores with the
// default policy (0): its next step reads the data back from cache.
constexpr int kStoreNT = 2;
constexpr int kStoreCached = 0;

// 32 well-mixed bits from a 32-bit counter ("lowbias32" integer finaliser,
// C. Wellons).
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

struct CF64 {
  using S = double;
  using R = double;
  static constexpr uint32_t B = 8;
  static constexpr bool kRandom = false;
  static constexpr int kRandBits = 0;
  static constexpr bool kWallRowsFirst = false;  // row order of the row-tiled update
  static constexpr int kScale = 1;  // registers hold (f - w) * kScale
  __device__ static R ld(Rsrc r, uint32_t vo, uint32_t so, const Tables*) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
  }
  template <int POL>
  __device__ static void st(Rsrc r, uint32_t vo, uint32_t so, R g, const Tables*, uint32_t) {
    using U2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, g), r, vo, so, POL);
  }
};

struct CF32 {
  using S = float;
  using R = float;
  static constexpr uint32_t B = 4;
  static constexpr bool kRandom = false;
  static constexpr int kRandBits = 0;
  static constexpr bool kWallRowsFirst = false;  // row order of the row-tiled update
  static constexpr int kScale = 1;  // registers hold (f - w) * kScale
  __device__ static R ld(Rsrc r, uint32_t vo, uint32_t so, const Tables*) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
  }
  template <int POL>
  __device__ static void st(Rsrc r, uint32_t vo, uint32_t so, R g, const Tables*, uint32_t) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(g), r, vo, so, POL);
  }
};

// FP32 storage of the deviations, all arithmetic in double: the storage
// rounding is the only single-precision error, at the traffic of FP32.  The
// rounding is stochastic (to one of the two neighbouring floats, with
// probability by distance): near a steady state a deterministic rounding
// makes the same error at every step, a bias that the slow diffusive modes
// accumulate over their relaxation time; unbiased rounding leaves noise.
struct CF32S {
  using S = float;
  using R = double;
  static constexpr uint32_t B = 4;
  static constexpr bool kRandom = true;
  static constexpr int kRandBits = 29;
  static constexpr bool kWallRowsFirst = true;  // row order of the row-tiled update
  static constexpr int kScale = 1;  // registers hold (f - w) * kScale
  __device__ static R ld(Rsrc r, uint32_t vo, uint32_t so, const Tables*) {
    return double(__uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0)));
  }
  // Add 29 random bits below the float's last significand bit to the
  // double's sign-magnitude word (a carry rounds the magnitude up, for
  // either sign) and clear them.  In the float normal range the result is a
  // float and the conversion exact; below 2^-126 the conversion rounds the
  // result once more to the nearest subnormal (no deviation is that small);
  // zero stays zero, infinity infinity, a quiet NaN a NaN (its top
  // significand bit survives).
  template <int POL>
  __device__ static void st(Rsrc r, uint32_t vo, uint32_t so, R g, const Tables*,
                            uint32_t rnd) {
    const uint64_t u = (uint64_t(__double_as_longlong(g)) + uint64_t(rnd & 0x1fffffffu)) &
                       ~uint64_t(0x1fffffffu);
    const float f = float(__longlong_as_double((long long)u));
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(f), r, vo, so, POL);
  }
};

// BF16 has FP32's exponent range: the deviations are stored unscaled.
struct CBF16 {
  using S = uint16_t;
  using R = float;
  static constexpr uint32_t B = 2;
  static constexpr bool kRandom = true;
  static constexpr int kRandBits = 16;
  static constexpr bool kWallRowsFirst = true;  // row order of the row-tiled update
  static constexpr int kScale = 1;  // registers hold (f - w) * kScale
  __device__ static R ld(Rsrc r, uint32_t vo, uint32_t so, const Tables*) {
    const uint32_t h = __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    return __uint_as_float(h << 16);
  }
  // Stochastic rounding to the 8-bit significand: add 16 random bits below
  // the kept ones to the sign-magnitude word (a carry rounds the magnitude
  // up, for either sign) and keep the top half.  Infinity stays infinity;
  // a NaN is stored as the quiet NaN.
  template <int POL>
  __device__ static void st(Rsrc r, uint32_t vo, uint32_t so, R g, const Tables*,
                            uint32_t rnd) {
    uint32_t u = __float_as_uint(g) + (rnd & 0xffffu);
    u = g != g ? 0x7fc00000u : u;
    __builtin_amdgcn_raw_buffer_store_b16(uint16_t(u >> 16), r, vo, so, POL);
  }
};

// FP16 keeps (f - w) * 2^12: deviations |f - w| < 1 fit its range (65504)
// and small ones stay above its normal limit 2^-14.  The update works on the
// scaled values themselves (kScale: every step is linear in the deviations
// and a power-of-two scale commutes with rounding, so the results match
// unscaled arithmetic to rounding), and loads and stores carry no multiply.  The
// scale is a compile-time constant: one read from memory would have to be
// re-read after every population store (the stores may alias it), each
// re-read waiting for all stores in flight.
struct CFP16 {
  using S = _Float16;
  using R = float;
  static constexpr uint32_t B = 2;
  static constexpr bool kRandom = true;
  static constexpr int kRandBits = 13;
  static constexpr bool kWallRowsFirst = true;  // row order of the row-tiled update
  static constexpr int kScale = 4096;  // registers hold (f - w) * kScale
  __device__ static R ld(Rsrc r, uint32_t vo, uint32_t so, const Tables*) {
    const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    return float(__builtin_bit_cast(_Float16, h));
  }
  // Stochastic rounding to FP16's 10-bit significand: add 13 random bits
  // below the kept ones to the (scaled) float's sign-magnitude word (a carry
  // rounds the magnitude up, for either sign) and clear them.  In FP16's
  // normal range [2^-14, 65504] the result is an FP16 value and the
  // conversion exact; below it (deviations under 2^-26 with the scale) the
  // conversion rounds once more to the nearest subnormal; above it the
  // conversion overflows to infinity as round-to-nearest would.  A quiet
  // NaN stays a NaN.
  template <int POL>
  __device__ static void st(Rsrc r, uint32_t vo, uint32_t so, R g, const Tables*,
                            uint32_t rnd) {
    const uint32_t u = (__float_as_uint(g) + (rnd & 0x1fffu)) & 0xffffe000u;
    const _Float16 h = _Float16(__uint_as_float(u));
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, h), r, vo, so, POL);
  }
};

// Descriptor over one plane set of the current step.
template <class L, class C>
__device__ __forceinline__ Rsrc plane_set(const void* p, long long plane) {
  return make_rsrc(p, uint32_t(uint64_t(L::Q) * uint64_t(plane) * C::B));
}

// ------------------------------------------------------------ equilibrium --
// Eq. (eq:feq) regrouped as a polynomial in x = c.u whose coefficients
// depend on the node (rho, u.u, theta = T-1) and on the velocity only through
// cc = |c|^2, written for the deviation from the rest weight:
//   f^eq_q - w_q = w_q (A0 + x (A1 + x (A2 + x (A3 + x A4)))),
//   A0 = (rho - 1) + rho (k0 - 1),  Ai = rho ki  (i >= 1),
//   k0 - 1 = k0a + cc (k0b + cc k0c), k1 = k1a + cc k1b, k2 = k2a + cc k2b.
// An exact rearrangement of the printed terms (the constant 1 is taken out
// analytically, so no O(1) term enters the rounding).
template <class L, class R>
struct EqCoef {
  R k0a, k0b, k0c, k1a, k1b, k2a, k2b, k3, k4;
  // d (f^eq_q / w_q) / d(u.u) at fixed x = c.u, theta: d0a + cc d0b + x (d1 + x d2)
  R d0a, d0b, d1, d2;

  __host__ __device__ static EqCoef make(R rho, R drho, R uu, R th) {
    constexpr R D = R(L::D);
    EqCoef c{};
    if constexpr (L::EQ >= 4) {
      c.k0a = drho + rho * (-R(0.5) * uu - R(0.5) * D * th + R(0.125) * uu * uu +
                            R(0.25) * (D + 2) * th * uu + R(0.125) * D * (D + 2) * th * th);
      c.k0b = rho * (R(0.5) * th - R(0.25) * th * uu - R(0.25) * (D + 2) * th * th);
      c.k0c = rho * (R(0.125) * th * th);
      c.k1a = rho * (R(1) - R(0.5) * uu - R(0.5) * (D + 2) * th);
      c.k1b = rho * (R(0.5) * th);
      c.k2a = rho * (R(0.5) - R(0.25) * uu - R(0.25) * (D + 4) * th);
      c.k2b = rho * (R(0.25) * th);
      c.k3 = rho * R(1.0 / 6.0);
      c.k4 = rho * R(1.0 / 24.0);
      c.d0a = rho * (-R(0.5) + R(0.25) * uu + R(0.25) * (D + 2) * th);
      c.d0b = rho * (-R(0.25) * th);
      c.d1 = rho * -R(0.5);
      c.d2 = rho * -R(0.25);
    } else if constexpr (L::EQ == 3) {
      c.k0a = drho + rho * (-R(0.5) * uu - R(0.5) * D * th);
      c.k0b = rho * (R(0.5) * th);
      c.k1a = rho * (R(1) - R(0.5) * uu - R(0.5) * (D + 2) * th);
      c.k1b = rho * (R(0.5) * th);
      c.k2a = rho * R(0.5);
      c.k3 = rho * R(1.0 / 6.0);
      c.d0a = rho * -R(0.5);
      c.d1 = rho * -R(0.5);
    } else {
      c.k0a = drho + rho * (-R(0.5) * uu - R(0.5) * D * th);
      c.k0b = rho * (R(0.5) * th);
      c.k1a = rho;
      c.k2a = rho * R(0.5);
      c.d0a = rho * -R(0.5);
    }
    return c;
  }

  // (f^eq_q - w_q) / w_q at x = c_q.u, for |e_q|^2 = EE.
  template <int EE>
  __host__ __device__ R poly(R x) const {
    constexpr R cc = R(L::R * L::R * EE);
    R K0, K1, K2;
    if constexpr (L::THERMAL) {
      K0 = k0a + cc * (k0b + cc * k0c);
      K1 = k1a + cc * k1b;
      K2 = k2a + cc * k2b;
    } else {
      K0 = k0a;
      K1 = k1a;
      K2 = k2a;
    }
    if constexpr (L::EQ >= 4) return K0 + x * (K1 + x * (K2 + x * (k3 + x * k4)));
    else if constexpr (L::EQ == 3) return K0 + x * (K1 + x * (K2 + x * k3));
    else return K0 + x * (K1 + x * K2);
  }

  // poly<EE> at x and at -x (velocities c and -c): the parts even and odd in
  // x are shared.
  template <int EE>
  __host__ __device__ void poly_pair(R x, R& plus, R& minus) const {
    constexpr R cc = R(L::R * L::R * EE);
    R K0, K1, K2;
    if constexpr (L::THERMAL) {
      K0 = k0a + cc * (k0b + cc * k0c);
      K1 = k1a + cc * k1b;
      K2 = k2a + cc * k2b;
    } else {
      K0 = k0a;
      K1 = k1a;
      K2 = k2a;
    }
    const R x2 = x * x;
    R even, odd;
    if constexpr (L::EQ >= 4) {
      even = K0 + x2 * (K2 + x2 * k4);
      odd = K1 + x2 * k3;
    } else if constexpr (L::EQ == 3) {
      even = K0 + x2 * K2;
      odd = K1 + x2 * k3;
    } else {
      even = K0 + x2 * K2;
      odd = K1;
    }
    plus = even + x * odd;
    minus = even - x * odd;
  }

  // poly at the rest velocity (c = 0, x = 0)
  __host__ __device__ R poly0() const { return k0a; }

  // Body-force term (f^eq's directional derivative in u at fixed rho, T)
  // over w_q: F_q / w_q = (a.c) dP/dx + 2 (a.u) dP/d(u.u), P = f^eq_q / w_q,
  // for the pair c, -c at once: x and a.c change sign together, so with
  // dP/dx = Pe + Po and dP/d(u.u) = Ue + Uo split into parts even and odd
  // in x, F(c) / w = Se + So and F(-c) / w = Se - So, where
  // Se = (a.c) Po + 2 (a.u) Ue and So = (a.c) Pe + 2 (a.u) Uo.
  template <int EE>
  __host__ __device__ void force_pair(R x, R ac, R au, R& plus, R& minus) const {
    constexpr R cc = R(L::R * L::R * EE);
    R K1, K2;
    if constexpr (L::THERMAL) {
      K1 = k1a + cc * k1b;
      K2 = k2a + cc * k2b;
    } else {
      K1 = k1a;
      K2 = k2a;
    }
    const R x2 = x * x;
    R pe, po, ue, uo;
    if constexpr (L::EQ >= 4) {
      pe = K1 + R(3) * k3 * x2;
      po = x * (R(2) * K2 + R(4) * k4 * x2);
      ue = d0a + cc * d0b + d2 * x2;
      uo = d1 * x;
    } else if constexpr (L::EQ == 3) {
      pe = K1 + R(3) * k3 * x2;
      po = R(2) * K2 * x;
      ue = d0a;
      uo = d1 * x;
    } else {
      pe = K1;
      po = R(2) * K2 * x;
      ue = d0a;
      uo = R(0);
    }
    const R se = ac * po + R(2) * au * ue, so = ac * pe + R(2) * au * uo;
    plus = se + so;
    minus = se - so;
  }

  // force at the rest velocity (c = 0): 2 (a.u) dP/d(u.u) at x = 0
  __host__ __device__ R force0(R au) const { return R(2) * au * d0a; }
};

template <class R>
struct Macro {
  R rho, drho, ux, uy, uz, th;
};

// Eq. (eq:summac) from the deviations: rho = 1 + sum g, rho u = sum g c
// (sum w c = 0), and for the thermal set rho D T = D + sum g |c|^2 - rho u^2
// (sum w |c|^2 = D); theta = T - 1.  Isothermal sets use T = 1.
// A is the arithmetic type, G the type the deviations are held in.
template <class R>
struct Sums {
  R drho, mx, my, mz, e2;  // sum g, sum g e, sum g |e|^2
};

// The sums of Eq. (eq:summac) over the deviations of velocity subset PART
// (of P); the whole set for PART = -1.
template <class L, class R, class G = R, int PART = -1, int P = 1>
__device__ __forceinline__ Sums<R> sums(const G (&g)[L::Q]) {
  R drho = 0, mx = 0, my = 0, mz = 0, e2 = 0;
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    if constexpr (in_part<L, PART, P>(q)) {
      const R v = R(g[q]);
      if constexpr (PART < 0) {
        drho = q == 0 ? v : drho + v;
        mx = accum<ex, q == first_nonzero<L>(0)>(mx, v);
        my = accum<ey, q == first_nonzero<L>(1)>(my, v);
        mz = accum<ez, q == first_nonzero<L>(2)>(mz, v);
        if constexpr (L::THERMAL)
          e2 = accum<ex * ex + ey * ey + ez * ez, q == first_nonzero<L>(3)>(e2, v);
      } else {
        drho += v;
        mx = add_scaled<ex>(mx, v);
        my = add_scaled<ey>(my, v);
        mz = add_scaled<ez>(mz, v);
        if constexpr (L::THERMAL) e2 = add_scaled<ex * ex + ey * ey + ez * ez>(e2, v);
      }
    }
  };
  static_for<0, L::Q>(body);
  return Sums<R>{drho, mx, my, mz, e2};
}

template <class L, class R>
__device__ __forceinline__ Macro<R> macro_from(const Sums<R>& t) {
  const R drho = t.drho, mx = t.mx, my = t.my, mz = t.mz, e2 = t.e2;
  Macro<R> m;
  m.drho = drho;
  m.rho = R(1) + drho;
  const R inv = R(1) / m.rho;
  constexpr R r = R(L::R);
  m.ux = r * mx * inv;
  m.uy = r * my * inv;
  m.uz = L::D == 3 ? r * mz * inv : R(0);
  if constexpr (L::THERMAL) {
    const R uu = L::D == 3 ? m.ux * m.ux + m.uy * m.uy + m.uz * m.uz : m.ux * m.ux + m.uy * m.uy;
    m.th = (R(L::R * L::R) * e2 - m.rho * uu - R(L::D) * drho) * (inv * R(1.0 / L::D));
  } else {
    m.th = R(0);
  }
  return m;
}


// g* = g - omega (g - (f^eq - w)), in place.  With MOM, also writes the
// output fields of the pre-collision state f~ at node n (Eq. (eq:summac)):
// rho, u, T, and the stress and heat flux of the original f, obtained from
// f~ by the conversion of Sec. II, f - f^eq = tau/(tau+1/2) (f~ - f^eq).
// With C = c - u, sigma_xy = sum f C_x C_y and q_i = 1/2 sum f |C|^2 C_i.
// The equilibrium parts are exact closed forms of the lattice's moments, so
// only the small non-equilibrium part f~ - f^eq is summed (no cancellation
// of O(u) terms in single precision):
//   sum_q f^eq_q C_x C_y = 0 (second moments of f^eq are exact on every set);
//   sum_q f^eq_q |C|^2 C_i = 0 on sets whose f^eq reproduces the third
//   moments (fourth-order f^eq on D2Q17 and D3Q121).
// D2Q16's second-order f^eq does not: its heat flux sums f - w and adds
//   sum_q w_q |C|^2 C_i = -u_i (D + 2 + |u|^2).
// FORCE: a body force a (not in the paper).  Its Hermite-projected term is
// F = a . d f^eq / du; the trapezoidal change of variable of Sec. II applied
// to collision + force gives g* = g + omega (f^eq - w - g) + tau/(tau+1/2) F
// with f^eq and F at the moments of f: u = u[f~] + a/2, T = T[f~] + a^2/(4D).
// relax() = sums() + macro_from() + relax_part() over the whole set +
// write_fields(); the batched kernel's split nodes call the parts itself
// (case_nodes_part).
template <class R>
struct NeqSums {
  R sxy, qx, qy, qz;  // non-equilibrium sums of the stress and heat flux
};

// The collision of velocity subset PART (of P; all for PART = -1) given the
// node's moments m of f~ (turned into those of f under a force, in place).
// With MOM, also returns the subset's stress and heat-flux sums in ns.
// Returns tau/(tau+1/2) of the node.
template <class L, class R, bool MOM, bool FORCE, int PART = -1, int P = 1, int SC = 1>
__device__ __forceinline__ R relax_part(R (&g)[L::Q], const StepArgs& a, Macro<R>& m,
                                        NeqSums<R>& ns) {
  R fax = 0, fay = 0, faz = 0;
  if constexpr (FORCE) {
    // moments of f from those of f~: u + a/2, T + a^2/(4D)
    fax = R(a.ax);
    fay = R(a.ay);
    faz = R(a.az);
    m.ux += R(0.5) * fax;
    m.uy += R(0.5) * fay;
    m.uz += R(0.5) * faz;
    if constexpr (L::THERMAL) m.th += (fax * fax + fay * fay + faz * faz) * R(0.25 / L::D);
  }
  const R uu = L::D == 3 ? m.ux * m.ux + m.uy * m.uy + m.uz * m.uz : m.ux * m.ux + m.uy * m.uy;
  const auto k = EqCoef<L, R>::make(m.rho, m.drho, uu, m.th);
  constexpr R r = R(L::R);
  const R sx = r * m.ux, sy = r * m.uy, sz = r * m.uz;
  R omega = R(a.omega), kf = R(a.kfac);
  if constexpr (L::THERMAL) {
    if (a.law) {
      // local relaxation time tau = mu / p (Sec. II) with mu = T^w, p = rho T
      const R tn = R(a.tau) * pow(R(1) + m.th, R(a.vexp) - R(1)) / m.rho;
      omega = R(1) / (tn + R(0.5));
      kf = tn * omega;
    }
  }
  const R au = fax * m.ux + fay * m.uy + faz * m.uz;
  R sxy = 0, qx = 0, qy = 0, qz = 0;
  // velocity q at x = c_q.u, with geq = f^eq_q - w_q
  // F: the force term of velocity q (zero without a force)
  auto finish = [&](auto qc, R geq, R F) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    if constexpr (MOM) {
      // f~ - f^eq (+ F/2 under a force: f - f^eq = tau/(tau+1/2) (f~ + F/2 - f^eq))
      const R neq = FORCE ? g[q] - geq + R(0.5) * F : g[q] - geq;
      const R Cx = R(L::R * ex) - m.ux, Cy = R(L::R * ey) - m.uy, Cz = R(L::R * ez) - m.uz;
      const R C2 = Cx * Cx + Cy * Cy + Cz * Cz;
      sxy += neq * Cx * Cy;
      const R fq = L::EQ >= 3 ? neq : geq + kf * neq;  // D2Q16: deviation of f from w
      qx += fq * C2 * Cx;
      qy += fq * C2 * Cy;
      qz += fq * C2 * Cz;
    }
    if constexpr (FORCE)
      g[q] = g[q] + omega * (geq - g[q]) + kf * F;
    else
      g[q] = g[q] + omega * (geq - g[q]);
  };
  // The velocities come in pairs c, -c (and the rest velocity): x changes
  // sign within a pair, and f^eq's even and odd parts in x are shared.
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int o = opposite<L>(q);
    static_assert(o >= 0, "velocity set not closed under c -> -c");
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    constexpr int EE = ex * ex + ey * ey + ez * ez;
    if constexpr (!in_part<L, PART, P>(q)) {
      // another part's velocity
    } else if constexpr (o == q) {
      finish(qc, R(L::W[q] * SC) * k.poly0(), FORCE ? R(L::W[q] * SC) * k.force0(au) : R(0));
    } else if constexpr (q < o) {
      const R x = dot_e<ex, ey, ez>(sx, sy, sz);
      R plus, minus, fplus = R(0), fminus = R(0);
      k.template poly_pair<EE>(x, plus, minus);
      if constexpr (FORCE)
        k.template force_pair<EE>(x, r * dot_e<ex, ey, ez>(fax, fay, faz), au, fplus, fminus);
      finish(qc, R(L::W[q] * SC) * plus, R(L::W[q] * SC) * fplus);
      finish(std::integral_constant<int, o>{}, R(L::W[o] * SC) * minus, R(L::W[o] * SC) * fminus);
    }
  };
  static_for<0, L::Q>(body);
  constexpr R inv = R(1.0 / SC);
  ns = NeqSums<R>{sxy * inv, qx * inv, qy * inv, qz * inv};
  return kf;
}

// The output fields of node n from its moments, tau/(tau+1/2) and the
// non-equilibrium sums.
template <class L, class R>
__device__ __forceinline__ void write_fields(double* mom, long long nodes, long long n,
                                             const Macro<R>& m, R kf, const NeqSums<R>& ns) {
  const R sxy = ns.sxy, qx = ns.qx, qy = ns.qy, qz = ns.qz;
  {
    mom[0 * nodes + n] = 1.0 + double(m.drho);
    mom[1 * nodes + n] = double(m.ux);
    mom[2 * nodes + n] = double(m.uy);
    mom[3 * nodes + n] = double(m.uz);
    mom[4 * nodes + n] = 1.0 + double(m.th);
    mom[5 * nodes + n] = double(kf * sxy);
    if constexpr (L::EQ >= 3) {
      mom[6 * nodes + n] = 0.5 * double(kf * qx);
      mom[7 * nodes + n] = 0.5 * double(kf * qy);
      mom[8 * nodes + n] = 0.5 * double(kf * qz);
    } else {
      const R uu =
          L::D == 3 ? m.ux * m.ux + m.uy * m.uy + m.uz * m.uz : m.ux * m.ux + m.uy * m.uy;
      const R rest = -(R(L::D + 2) + uu);
      mom[6 * nodes + n] = 0.5 * double(m.ux * rest + qx);
      mom[7 * nodes + n] = 0.5 * double(m.uy * rest + qy);
      mom[8 * nodes + n] = 0.5 * double(m.uz * rest + qz);
    }
  }
}

// SC: the deviations in g are scaled by SC (a power of two; the codec's
// kScale); the moments, fields and f^eq are those of the unscaled values.
template <class L, class R, bool MOM = false, bool FORCE = false, int SC = 1>
__device__ __forceinline__ void relax(R (&g)[L::Q], const StepArgs& a, double* mom = nullptr,
                                      long long nodes = 0, long long n = 0) {
  Sums<R> t = sums<L, R>(g);
  if constexpr (SC != 1) {
    constexpr R inv = R(1.0 / SC);
    t = Sums<R>{t.drho * inv, t.mx * inv, t.my * inv, t.mz * inv, t.e2 * inv};
  }
  Macro<R> m = macro_from<L, R>(t);
  NeqSums<R> ns;
  const R kf = relax_part<L, R, MOM, FORCE, -1, 1, SC>(g, a, m, ns);
  if constexpr (MOM) write_fields<L, R>(mom, nodes, n, m, kf, ns);
}

// Blocks are dealt round-robin to the 8 XCDs (block b runs on XCD b % 8,
// each with its own L2).  Remap so that each XCD gets a contiguous run of
// logical tiles: neighbouring rows and x-segments, whose shifted reads share
// cache lines, then meet in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int per = nb / X, rem = nb % X, xcd = b % X, idx = b / X;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Columns x - s (periodic) for s = -NS..NS.  FAST requires nx >= NS, where
// one conditional add either way is enough; otherwise any nx >= 1.
template <int NS, bool FAST>
__device__ __forceinline__ void wrapped_columns(int x, int nx, int (&xw)[2 * NS + 1]) {
  for (int s = -NS; s <= NS; ++s) {
    int c = x - s;
    if constexpr (FAST) {
      c += c < 0 ? nx : 0;
      c -= c >= nx ? nx : 0;
    } else {
      while (c < 0) c += nx;
      while (c >= nx) c -= nx;
    }
    xw[s + NS] = c;
  }
}

// Index of the velocity with the normal (y) component reversed.
template <class L>
constexpr int mirror_y(int q) {
  for (int m = 0; m < L::Q; ++m)
    if (L::E[m][0] == L::E[q][0] && L::E[m][1] == -L::E[q][1] && L::E[m][2] == L::E[q][2])
      return m;
  return -1;
}

template <class L>
constexpr int max_ex() {
  int m = 0;
  for (int q = 0; q < L::Q; ++q) {
    const int a = L::E[q][0] < 0 ? -L::E[q][0] : L::E[q][0];
    m = a > m ? a : m;
  }
  return m;
}

// ------------------------------------------------------------ wall sums --
template <class L>
struct WallTerms {
  struct Term {
    int q, j, ex;
  };
  static constexpr int count() {
    int n = 0;
    for (int q = 0; q < L::Q; ++q)
      if (L::E[q][1] < 0) n += -L::E[q][1];
    return n;
  }
  static constexpr int NT = count();
  struct Arr {
    Term t[NT];
  };
  // Bottom wall: a population with e_y < 0 leaving fluid row j lands in a
  // ghost layer iff j + e_y < 0, i.e. j = 0 .. -e_y - 1.
  static constexpr Arr bottom() {
    Arr a{};
    int n = 0;
    for (int q = 0; q < L::Q; ++q)
      for (int j = 0; j < -L::E[q][1]; ++j) a.t[n++] = Term{q, j, L::E[q][0]};
    return a;
  }
  // Top wall (mirror): e_y > 0 from rows ny-1-j, j = 0 .. e_y - 1.
  static constexpr Arr top() {
    Arr a{};
    int n = 0;
    for (int q = 0; q < L::Q; ++q)
      for (int j = 0; j < L::E[q][1]; ++j) a.t[n++] = Term{q, j, L::E[q][0]};
    return a;
  }
};

// Pooled incoming mass of ghost column xp (deviations only), the same in
// every lane: the wave issues every term's load at the same (wave-uniform)
// address, with no branch between them, and adds the terms in their fixed
// order.  (A version that gave each lane its own terms behind a per-term
// branch waited for each load in turn: 88 memory latencies per wall and
// step on D3Q121.)
template <class L, class C, bool TOP>
__device__ __forceinline__ double ghost_mass(Rsrc fin, const StepArgs& a, int xp) {
  using W = WallTerms<L>;
  double acc = 0.0;
  auto body = [&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr auto T = TOP ? W::top().t[t] : W::bottom().t[t];
    int xs = xp - T.ex;
    while (xs < 0) xs += a.nx;
    while (xs >= a.nx) xs -= a.nx;
    const int row = TOP ? a.ny - 1 - T.j : T.j;
    acc += double(C::ld(fin, (uint32_t(row) * uint32_t(a.nx) + uint32_t(xs)) * C::B,
                        uint32_t(T.q) * uint32_t(a.plane) * C::B, a.tab));
  };
  static_for<0, W::NT>(body);
  return acc * (1.0 / C::kScale);
}

template <class L, class C>
__global__ __launch_bounds__(kBlock) void wall_kernel(StepArgs a) {
  const int wave = int((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = int(threadIdx.x & 63);
  if (wave >= 2 * a.nx) return;  // wave-uniform
  const Rsrc fin = plane_set<L, C>(a.fin, a.plane);
  const bool top = wave >= a.nx;
  const int xp = top ? wave - a.nx : wave;
  double M;
  if (top)
    M = ghost_mass<L, C, true>(fin, a, xp);
  else
    M = ghost_mass<L, C, false>(fin, a, xp);
  // pooled incoming mass = rest-state part + deviations; ratio of
  // Eq. (eq:dkboundary) numerator to its denominator
  if (lane == 0)
    a.ratio[(top ? a.nx : 0) + xp] =
        top ? (a.tab->Wt + M) / a.tab->Dt : (a.tab->Wb + M) / a.tab->Db;
}

// ------------------------------------------------------------- the step --
// Pull of one node: f~_q(x, y) = f*_q(x - e_x, y - e_y), or, when the source
// row lies in a ghost layer, the value the wall re-emits there:
// g^eq_q(u_w, T_w) * (pooled mass / D) of the source's ghost column (read
// through ratio(wall, q)), Eq. (eq:dkboundary).  Returns deviations from w_q.
// A wall with accommodation below one also reflects part of the incoming
// mass specularly; wall_specular adds that share afterwards.
// Copy of the two wall Maxwellians g^eq(u_w, T_w) (bottom in [0, Q), top in
// [Q, 2Q)) in LDS, for the pulls of the rows next to a wall; by all threads
// of the block, followed by a barrier.
template <class L>
__device__ __forceinline__ void stage_wall_tables(const StepArgs& a, double* wtab, int nthreads) {
  for (int i = int(threadIdx.x); i < 2 * L::Q; i += nthreads)
    wtab[i] = i < L::Q ? a.tab->gb[i] : a.tab->gt[i - L::Q];
  __syncthreads();
}

// wtab: the wall Maxwellians staged by stage_wall_tables (read only in the
// rows next to a wall).  PART / P: only the velocities of that subset.
// UNIFORM_Y: y is the same for the whole workgroup (the row-tiled update).
template <class L, class C, int PART = -1, int P = 1, bool UNIFORM_Y = false, class Ratio>
__device__ __forceinline__ void pull(typename C::R (&f)[L::Q], const StepArgs& a, int y,
                                     const int (&xw)[2 * max_ex<L>() + 1], const double* wtab,
                                     Ratio&& ratio) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  const Rsrc fin = plane_set<L, C>(a.fin, a.plane);
  const uint32_t nx = uint32_t(a.nx);
  const uint32_t pb = uint32_t(a.plane) * C::B;  // bytes per plane
  if (y >= L::N && y < a.ny - L::N) {
    // vector offset: node (x - e_x, y - N), one per e_x; the row shift
    // (N - e_y) rows joins the plane offset in the scalar operand
    uint32_t vo[2 * NS + 1];
    const uint32_t yb = uint32_t(y - L::N) * nx;
    for (int s = 0; s < 2 * NS + 1; ++s) vo[s] = (yb + uint32_t(xw[s])) * C::B;
    const uint32_t rb = nx * C::B;  // bytes per row
    auto body = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      if constexpr (in_part<L, PART, P>(q))
        f[q] = C::ld(fin, vo[ex + NS], uint32_t(q) * pb + uint32_t(L::N - ey) * rb, a.tab);
    };
    static_for<0, L::Q>(body);
  } else if constexpr (UNIFORM_Y) {
    // A row next to a wall, the same for the whole workgroup: which sources
    // lie beyond a wall is uniform, so the per-velocity choice is a scalar
    // branch; a source beyond the wall takes the re-emitted value
    // f = g^eq(u_w, T_w) M / D (wall table and ratios in LDS).
    auto body = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      if constexpr (!in_part<L, PART, P>(q)) return;
      const int ys = y - ey;
      if (ey > 0 && ys < 0)
        f[q] = R((wtab[q] * ratio(0, ex) - L::W[q]) * C::kScale);
      else if (ey < 0 && ys >= a.ny)
        f[q] = R((wtab[L::Q + q] * ratio(1, ex) - L::W[q]) * C::kScale);
      else
        f[q] = C::ld(fin, (uint32_t(ys) * nx + uint32_t(xw[ex + NS])) * C::B, uint32_t(q) * pb,
                     a.tab);
    };
    static_for<0, L::Q>(body);
  } else {
    // Rows next to a wall, y varying across the wave.  Every velocity's
    // load is issued (a source beyond a wall reads this node's column in
    // row y instead, inside the grid), then the sources beyond a wall take
    // the re-emitted value: no divergent branch separates the loads, so
    // they are in flight together rather than one wait per velocity.
    auto load = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      if constexpr (!in_part<L, PART, P>(q)) return;
      const int ys = y - ey;
      const uint32_t row = uint32_t(ys < 0 || ys >= a.ny ? y : ys);
      f[q] = C::ld(fin, (row * nx + uint32_t(xw[ex + NS])) * C::B, uint32_t(q) * pb, a.tab);
    };
    static_for<0, L::Q>(load);
    auto emit = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      if constexpr (!in_part<L, PART, P>(q)) {
        // another part's velocity
      } else if constexpr (ey > 0) {  // bottom wall (y - e_y < 0)
        const R v = R((wtab[q] * ratio(0, ex) - L::W[q]) * C::kScale);
        f[q] = y - ey < 0 ? v : f[q];
      } else if constexpr (ey < 0) {  // top wall (y - e_y >= ny)
        const R v = R((wtab[L::Q + q] * ratio(1, ex) - L::W[q]) * C::kScale);
        f[q] = y - ey >= a.ny ? v : f[q];
      }
    };
    static_for<0, L::Q>(emit);
  }
}

// Maxwell-type scattering at the walls (Sec. III's generic kernel R taken as
// a R_D + (1 - a) R_S, a the wall's accommodation): for the velocities a
// wall re-emits into row y, mix the diffuse value pull() produced with the
// specular image, f~_q = a f_D + (1 - a) f*_{q'}(x - e_x, y'), q' = q with
// e_y reversed and y' the source row reflected at the wall plane (-1 - y_s
// below the bottom wall, 2 ny - 1 - y_s above the top one).  Does nothing
// away from the walls or for a = 1 (the paper's diffuse wall).
template <class L, class C, int PART = -1, int P = 1>
__device__ __forceinline__ void wall_specular(typename C::R (&f)[L::Q], const StepArgs& a, int y,
                                              const int (&xw)[2 * max_ex<L>() + 1]) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  const double ab = a.tab->ab, at = a.tab->at;
  const bool bottom = y < L::N && ab != 1.0, top = y >= a.ny - L::N && at != 1.0;
  if (!bottom && !top) return;
  const Rsrc fin = plane_set<L, C>(a.fin, a.plane);
  const uint32_t nx = uint32_t(a.nx);
  const uint32_t pb = uint32_t(a.plane) * C::B;
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1];
    constexpr int m = mirror_y<L>(q);
    static_assert(m >= 0, "velocity set not symmetric under y reversal");
    if constexpr (!in_part<L, PART, P>(q)) return;
    const int ys = y - ey;
    if (ey > 0 && ys < 0 && bottom) {
      const double gs = double(C::ld(fin, (uint32_t(-1 - ys) * nx + uint32_t(xw[ex + NS])) * C::B,
                                     uint32_t(m) * pb, a.tab));
      f[q] = R(ab * double(f[q]) + (1.0 - ab) * gs);
    } else if (ey < 0 && ys >= a.ny && top) {
      const double gs = double(C::ld(
          fin, (uint32_t(2 * a.ny - 1 - ys) * nx + uint32_t(xw[ex + NS])) * C::B, uint32_t(m) * pb,
          a.tab));
      f[q] = R(at * double(f[q]) + (1.0 - at) * gs);
    }
  };
  static_for<0, L::Q>(body);
}

template <class L, class C, int POL = kStoreNT, int PART = -1, int P = 1>
__device__ __forceinline__ void store(const typename C::R (&f)[L::Q], const StepArgs& a,
                                      uint32_t n) {
  // a subset's stores would not draw the same rounding bits as the whole set's
  static_assert(PART < 0 || !C::kRandom, "velocity subsets only for formats without rounding");
  const Rsrc fout = plane_set<L, C>(a.fout, a.plane);
  const uint32_t pb = uint32_t(a.plane) * C::B;
  // Random bits for the stochastic rounding of the rounded formats: a
  // counter hash of (step, seed, node) seeds Marsaglia's xorshift32 (shift
  // triple 13, 17, 5; never zero), stepped once per velocity, or once per
  // pair of velocities (low half for even q, high half for odd q) where a
  // format needs at most 16 bits.
  uint32_t x = 0u;
  if constexpr (C::kRandom)
    x = mix32(mix32(a.step * 0x9e3779b9u + a.seed) ^ (n * uint32_t(L::Q))) | 1u;
  auto next = [&x]() {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
  };
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    uint32_t rnd = 0u;
    if constexpr (C::kRandom && C::kRandBits <= 16)
      rnd = q % 2 == 0 ? next() : x >> 16;
    else if constexpr (C::kRandom)
      rnd = next();
    if constexpr (in_part<L, PART, P>(q))
      C::template st<POL>(fout, n * C::B, uint32_t(q) * pb, f[q], a.tab, rnd);
  };
  static_for<0, L::Q>(body);
}

// Pooled incoming mass of one ghost column, summed serially in a fixed order
// (deviations only; the rest-state part is added by the caller).
template <class L, class C, bool TOP>
__device__ __forceinline__ double ghost_column_deviation(const StepArgs& a, int xp) {
  using W = WallTerms<L>;
  const Rsrc fin = plane_set<L, C>(a.fin, a.plane);
  double acc = 0.0;
  auto body = [&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr auto T = TOP ? W::top().t[t] : W::bottom().t[t];
    int xs = xp - T.ex;
    xs += xs < 0 ? a.nx : 0;
    xs -= xs >= a.nx ? a.nx : 0;
    const int row = TOP ? a.ny - 1 - T.j : T.j;
    acc += double(C::ld(fin, (uint32_t(row) * uint32_t(a.nx) + uint32_t(xs)) * C::B,
                        uint32_t(T.q) * uint32_t(a.plane) * C::B, a.tab));
  };
  static_for<0, W::NT>(body);
  return acc * (1.0 / C::kScale);
}

// Any grid shape: one thread per node on a linear node index; the ghost
// ratios come from wall_kernel, launched before.
template <class L, class C, bool MOM, bool FORCE>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  __shared__ double wtab_s[2 * L::Q];
  const long long nodes = (long long)a.nx * a.ny;
  const long long base = (long long)xcd_remap(blockIdx.x, gridDim.x) * kBlock;
  // blocks holding a row next to a wall stage the wall Maxwellians
  // (block-uniform test, before any thread leaves)
  const long long last = (base + kBlock < nodes ? base + kBlock : nodes) - 1;
  if (base / a.nx < L::N || last / a.nx >= a.ny - L::N)
    stage_wall_tables<L>(a, wtab_s, kBlock);
  const long long n = base + threadIdx.x;
  if (n >= nodes) return;
  const int y = int(n / a.nx);
  const int x = int(n - (long long)y * a.nx);
  int xw[2 * NS + 1];
  wrapped_columns<NS, false>(x, a.nx, xw);
  R f[L::Q];
  pull<L, C>(f, a, y, xw, wtab_s,
             [&](int wall, int ex) { return a.ratio[wall * a.nx + xw[ex + NS]]; });
  wall_specular<L, C>(f, a, y, xw);
  relax<L, R, MOM, FORCE, C::kScale>(f, a, a.mom, nodes, n);
  store<L, C>(f, a, uint32_t(n));
}

// Rows that are a multiple of kBlock wide: each block owns kBlock
// consecutive nodes of one row (x0 .. x0+kBlock-1), so the row index is
// wave-uniform and no integer division per thread is needed.  Blocks of the
// N rows next to a wall first compute the pooled ghost-column ratios of the
// kBlock + 2 NS columns their pulls can reach into LDS (fusing the wall sums
// into the update: no separate launch, no global round trip).
template <class L, class C, bool MOM, bool FORCE>
__global__ __launch_bounds__(kBlock) void step_rows_kernel(StepArgs a) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  __shared__ double ratio_s[kBlock + 2 * NS];
  __shared__ double wtab_s[2 * L::Q];
  const int bpr = a.nx / kBlock;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int r = b / bpr;
  // Wall-row blocks also sum the ghost columns (a second round of loads
  // before the pull), so they take longest.  The 16-bit and FP32-storage
  // updates schedule the 2N wall rows first, so that they do not form the
  // grid's tail (measured: D3Q121 BF16 159 -> 138 us, D2Q17 BF16 60 -> 57 us,
  // FP32 storage -1 to -2 %; none for FP32 and FP64, which keep the plain
  // order for the cache reuse of neighbouring rows).
  int y = r;
  if constexpr (C::kWallRowsFirst)
    y = r < L::N ? r : r < 2 * L::N ? a.ny - 1 - (r - L::N) : r - L::N;
  const int x0 = (b - r * bpr) * kBlock;
  const int x = x0 + int(threadIdx.x);
  int xw[2 * NS + 1];
  wrapped_columns<NS, true>(x, a.nx, xw);
  const bool bottom = y < L::N, top = y >= a.ny - L::N;  // block-uniform
  if (bottom || top) {
    for (int s = threadIdx.x; s < kBlock + 2 * NS; s += kBlock) {
      int c = x0 - NS + s;
      c += c < 0 ? a.nx : 0;
      c -= c >= a.nx ? a.nx : 0;
      ratio_s[s] = top ? (a.tab->Wt + ghost_column_deviation<L, C, true>(a, c)) / a.tab->Dt
                       : (a.tab->Wb + ghost_column_deviation<L, C, false>(a, c)) / a.tab->Db;
    }
    stage_wall_tables<L>(a, wtab_s, kBlock);  // ends with the barrier
  }
  R f[L::Q];
  // Wall rows: the formats that schedule them first (their wall blocks run
  // beside interior ones) take the branchless pull, which keeps every load
  // in flight (D3Q121 1024^2: FP32 storage 257 -> 233 us, 16-bit 127 -> 123
  // us per step); FP32 and FP64, whose wall blocks end the grid, take the
  // uniform branches, which skip the loads of sources beyond the wall (the
  // branchless pull cost D2Q17 2048^2 FP32 0.65 us per step).
  pull<L, C, -1, 1, !C::kWallRowsFirst>(
      f, a, y, xw, wtab_s, [&](int, int ex) { return ratio_s[int(threadIdx.x) - ex + NS]; });
  if (bottom || top) wall_specular<L, C>(f, a, y, xw);
  const long long nodes = (long long)a.nx * a.ny;
  const uint32_t n = uint32_t(y) * uint32_t(a.nx) + uint32_t(x);
  relax<L, R, MOM, FORCE, C::kScale>(f, a, a.mom, nodes, n);
  store<L, C>(f, a, n);
}

// f~(0) = f^eq(rho0, u0, T0); writes the output fields of f~(0) and stores
// f*(0) = relaxed f~(0), the state every later step pulls from (as
// deviations from the rest weights).
template <class L, class C, bool FORCE>
__global__ __launch_bounds__(kBlock) void init_kernel(StepArgs a, const double* fields) {
  using R = typename C::R;
  const long long nodes = (long long)a.nx * a.ny;
  const long long n = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (n >= nodes) return;
  double rho = 1.0, ux = 0.0, uy = 0.0, uz = 0.0, T = 1.0;
  if (fields) {
    rho = fields[n];
    ux = fields[nodes + n];
    uy = fields[2 * nodes + n];
    uz = fields[3 * nodes + n];
    T = L::THERMAL ? fields[4 * nodes + n] : 1.0;
  }
  const auto k = EqCoef<L, double>::make(rho, rho - 1.0, ux * ux + uy * uy + uz * uz, T - 1.0);
  constexpr double r = L::R;
  R f[L::Q];
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    const double x = r * (ex * ux + ey * uy + ez * uz);
    f[q] = R(L::W[q] * k.template poly<ex * ex + ey * ey + ez * ez>(x) * C::kScale);  // f^eq - w
  };
  static_for<0, L::Q>(body);
  relax<L, R, true, FORCE, C::kScale>(f, a, a.mom, nodes, n);
  store<L, C>(f, a, uint32_t(n));
}

// Fixed-order block reduction of four FP64 partial sums over NT threads;
// every thread gets the totals.
template <int NT = kBlock>
__device__ __forceinline__ void block_sum4(double (&v)[4], double (*sh)[NT]) {
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    __syncthreads();
  }
  for (int k = 0; k < 4; ++k) v[k] = sh[k][0];
  __syncthreads();  // the scratch may be reused right away
}

// Mass, residual sums and nonfinite count of one node's fields; the
// residual snapshot is advanced to the current fields.
__device__ __forceinline__ void residual_terms(const double* mom, double* snap, long long n,
                                               long long i, double (&v)[4]) {
  const double rho = mom[i];
  const double ux = mom[n + i], uy = mom[2 * n + i], uz = mom[3 * n + i];
  const double T = mom[4 * n + i];
  const double dx = ux - snap[i], dy = uy - snap[n + i], dz = uz - snap[2 * n + i];
  const double dT = T - snap[3 * n + i];
  snap[i] = ux;
  snap[n + i] = uy;
  snap[2 * n + i] = uz;
  snap[3 * n + i] = T;
  v[0] += rho;
  v[1] += dx * dx + dy * dy + dz * dz;
  v[2] += dT * dT;
  v[3] += isfinite(rho + ux + uy + uz + T) ? 0.0 : 1.0;
}

// ---------------------------------------------------------- batched cases --
// Persistent update of many small channels: workgroup b owns case b and runs
// its steps itself, so a step costs two workgroup barriers instead of two
// kernel launches.  Per step: each wavefront sums the pooled mass of
// (wall, ghost column) pairs in FP64 into LDS,
// barrier, the threads update the case's nodes (pulls from the ping-pong
// buffers, which stay in cache), barrier.  Steps run in residual windows;
// after each window the case's fields, mass and residual are formed in the
// kernel and the case stops once the residual is below its tolerance.  A
// case's arithmetic and stopping point depend only on its own data, so its
// result is the same alone and in any mix, and whatever its step budget.
// One step of one case's nodes by the workgroup (the ghost-column ratios
// already in LDS).  MOM: the last step of a window, which also writes the
// output fields; its own loop, so that the populations of the two variants
// never share live ranges (one loop with both would hold more registers).
template <class L, class C, bool FORCE, bool MOM, int NT>
__device__ __forceinline__ void case_nodes(const StepArgs& a, int nodes, const double* ratio_s,
                                           const double* wtab_s) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  for (int n = threadIdx.x; n < nodes; n += NT) {
    const int y = n / a.nx;
    const int x = n - y * a.nx;
    int xw[2 * NS + 1];
    wrapped_columns<NS, false>(x, a.nx, xw);
    R f[L::Q];
    pull<L, C>(f, a, y, xw, wtab_s,
               [&](int wall, int ex) { return ratio_s[wall * a.nx + xw[ex + NS]]; });
    wall_specular<L, C>(f, a, y, xw);
    relax<L, R, MOM, FORCE, C::kScale>(f, a, a.mom, nodes, n);
    store<L, C, kStoreCached>(f, a, uint32_t(n));
  }
}

// Threads per case of the batched kernel, and the number of velocity
// subsets a node of set L is split over.  A case runs on one workgroup and
// is latency-bound: the FP32 instance without a body force gives each case
// 1024 threads and splits its D3Q121 nodes over four groups of four waves
// (about 30 velocities per lane instead of 121).  The force variant (whose
// D3Q121 path spills at 128 or 256 registers per lane when split) and the
// other formats keep 256 threads and whole nodes.
template <class C, bool FORCE>
constexpr int batch_threads() {
  return std::is_same<C, CF32>::value && !FORCE ? 1024 : kBatchBlock;
}
template <class L, class C, bool FORCE>
constexpr int batch_parts() {
  return std::is_same<C, CF32>::value && !FORCE && L::Q > 100 ? 4 : 1;
}

// One step of one case's nodes with each node split over P groups of
// NT / P threads (group PART, a compile-time velocity subset; the group
// index is uniform over each wave).  Each group pulls its velocities and
// puts its partial sums of Eq. (eq:summac) in LDS; after a barrier every
// group adds the P partial sums in the same fixed order, forms the moments
// and relaxes and stores its own velocities.  With MOM the stress and heat
// flux sums are combined the same way and group 0 writes the fields.  All
// groups pass the same barriers.  part_s: (5 + 4) x NT values of R.
template <class L, class C, bool FORCE, bool MOM, int NT, int P, int PART>
__device__ __forceinline__ void case_nodes_part(const StepArgs& a, int nodes,
                                                const double* ratio_s, const double* wtab_s,
                                                typename C::R* part_s) {
  using R = typename C::R;
  constexpr int NS = max_ex<L>();
  constexpr int kSlots = NT / P;
  R* psum = part_s;             // [P][5][kSlots]
  R* pneq = part_s + 5 * NT;    // [P][4][kSlots]
  const int slot = int(threadIdx.x) - PART * kSlots;
  for (int base = 0; base < nodes; base += kSlots) {
    const int n = base + slot;
    const bool active = n < nodes;
    R f[L::Q];
    Sums<R> t{R(0), R(0), R(0), R(0), R(0)};
    if (active) {
      const int y = n / a.nx;
      const int x = n - y * a.nx;
      int xw[2 * NS + 1];
      wrapped_columns<NS, false>(x, a.nx, xw);
      pull<L, C, PART, P>(f, a, y, xw, wtab_s, [&](int wall, int ex) {
        return ratio_s[wall * a.nx + xw[ex + NS]];
      });
      wall_specular<L, C, PART, P>(f, a, y, xw);
      t = sums<L, R, R, PART, P>(f);
    }
    psum[(PART * 5 + 0) * kSlots + slot] = t.drho;
    psum[(PART * 5 + 1) * kSlots + slot] = t.mx;
    psum[(PART * 5 + 2) * kSlots + slot] = t.my;
    psum[(PART * 5 + 3) * kSlots + slot] = t.mz;
    psum[(PART * 5 + 4) * kSlots + slot] = t.e2;
    __syncthreads();
    Macro<R> m{};
    R kf = R(0);
    if (active) {
      R v[5];
      for (int k = 0; k < 5; ++k) {
        v[k] = psum[k * kSlots + slot];
        for (int p = 1; p < P; ++p) v[k] += psum[(p * 5 + k) * kSlots + slot];
      }
      constexpr R inv = R(1.0 / C::kScale);
      m = macro_from<L, R>(Sums<R>{v[0] * inv, v[1] * inv, v[2] * inv, v[3] * inv, v[4] * inv});
      NeqSums<R> ns;
      kf = relax_part<L, R, MOM, FORCE, PART, P, C::kScale>(f, a, m, ns);
      store<L, C, kStoreCached, PART, P>(f, a, uint32_t(n));
      if constexpr (MOM) {
        pneq[(PART * 4 + 0) * kSlots + slot] = ns.sxy;
        pneq[(PART * 4 + 1) * kSlots + slot] = ns.qx;
        pneq[(PART * 4 + 2) * kSlots + slot] = ns.qy;
        pneq[(PART * 4 + 3) * kSlots + slot] = ns.qz;
      }
    }
    if constexpr (MOM) {
      __syncthreads();
      if (PART == 0 && active) {
        R w[4];
        for (int k = 0; k < 4; ++k) {
          w[k] = pneq[k * kSlots + slot];
          for (int p = 1; p < P; ++p) w[k] += pneq[(p * 4 + k) * kSlots + slot];
        }
        write_fields<L, R>(a.mom, nodes, n, m, kf, NeqSums<R>{w[0], w[1], w[2], w[3]});
      }
    }
    __syncthreads();  // the partial sums are reused by the next pass
  }
}

// One step of the nodes: whole nodes per thread, or split (see above).
template <class L, class C, bool FORCE, bool MOM, int NT>
__device__ __forceinline__ void case_step(const StepArgs& a, int nodes, const double* ratio_s,
                                          const double* wtab_s, typename C::R* part_s) {
  constexpr int P = batch_parts<L, C, FORCE>();
  if constexpr (P == 1) {
    case_nodes<L, C, FORCE, MOM, NT>(a, nodes, ratio_s, wtab_s);
  } else if constexpr (P == 2) {
    static_assert(NT % (64 * P) == 0, "groups of whole waves");
    const int part = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / (NT / P));
    if (part == 0)
      case_nodes_part<L, C, FORCE, MOM, NT, P, 0>(a, nodes, ratio_s, wtab_s, part_s);
    else
      case_nodes_part<L, C, FORCE, MOM, NT, P, 1>(a, nodes, ratio_s, wtab_s, part_s);
  } else {
    static_assert(P == 4 && NT % (64 * P) == 0, "four groups of whole waves");
    const int part = __builtin_amdgcn_readfirstlane(int(threadIdx.x) / (NT / P));
    switch (part) {
      case 0: case_nodes_part<L, C, FORCE, MOM, NT, P, 0>(a, nodes, ratio_s, wtab_s, part_s); break;
      case 1: case_nodes_part<L, C, FORCE, MOM, NT, P, 1>(a, nodes, ratio_s, wtab_s, part_s); break;
      case 2: case_nodes_part<L, C, FORCE, MOM, NT, P, 2>(a, nodes, ratio_s, wtab_s, part_s); break;
      default: case_nodes_part<L, C, FORCE, MOM, NT, P, 3>(a, nodes, ratio_s, wtab_s, part_s); break;
    }
  }
}

template <class L, class C, bool FORCE, int NT>
__device__ __forceinline__ void run_case(const CaseDesc& cd, CaseOut* out, double* ratio_s,
                                         double (*red)[NT], double* wtab_s,
                                         typename C::R* part_s) {
  StepArgs a = cd.a;
  stage_wall_tables<L>(a, wtab_s, NT);
  const int nodes = a.nx * a.ny;
  const int lane = int(threadIdx.x & 63);
  const int wave = int(threadIdx.x >> 6);
  constexpr int kWaves = NT / 64;
  const int W = cd.window;
  int cur = cd.cur;
  int done = 0;
  double res = __builtin_inf(), mass = 0.0, state = 0.0;
  while (done + W <= cd.budget) {
    for (int s = 0; s < W; ++s) {
      a.fin = cd.f[cur];
      a.fout = cd.f[cur ^ 1];
      a.step = cd.a.step + uint32_t(done + s) + 1u;
      const Rsrc fin = plane_set<L, C>(a.fin, a.plane);
      for (int p = wave; p < 2 * a.nx; p += kWaves) {
        const bool top = p >= a.nx;
        const int xp = top ? p - a.nx : p;
        const double M = top ? ghost_mass<L, C, true>(fin, a, xp)
                             : ghost_mass<L, C, false>(fin, a, xp);
        if (lane == 0)
          ratio_s[p] = top ? (a.tab->Wt + M) / a.tab->Dt : (a.tab->Wb + M) / a.tab->Db;
      }
      __syncthreads();
      if (s == W - 1)
        case_step<L, C, FORCE, true, NT>(a, nodes, ratio_s, wtab_s, part_s);
      else
        case_step<L, C, FORCE, false, NT>(a, nodes, ratio_s, wtab_s, part_s);
      __syncthreads();
      cur ^= 1;
    }
    done += W;
    double v[4] = {0, 0, 0, 0};
    for (int i = threadIdx.x; i < nodes; i += NT) residual_terms(a.mom, cd.snap, nodes, i, v);
    block_sum4<NT>(v, red);
    if (threadIdx.x == 0)
      for (int k = 0; k < 4; ++k) cd.result[k] = v[k];
    const double ru = sqrt(v[1]) / (double(W) * cd.uref * sqrt(double(nodes)));
    const double rt = sqrt(v[2]) / (double(W) * sqrt(double(nodes)));
    mass = v[0];
    if (v[3] != 0.0) {  // the same decision in every thread: v came from LDS
      res = __builtin_nan("");
      state = -1.0;
      break;
    }
    res = fmax(ru, rt);
    if (res < cd.tol) {
      state = 1.0;
      break;
    }
  }
  if (threadIdx.x == 0) {
    out[blockIdx.x].residual = res;
    out[blockIdx.x].mass = mass;
    out[blockIdx.x].steps = double(done);
    out[blockIdx.x].state = state;
  }
}

// SETS: bit mask of the velocity sets the instance carries (1 D2Q16, 2
// D2Q17, 4 D3Q121).  A kernel's registers are those of its largest set, so
// the double-precision formats keep the large set in an instance of its own
// (in one instance with the others its FP64 path spills to scratch and slows
// every case).  A case of a set the instance does not carry reports failure.
template <class C, bool FORCE, int SETS>
__global__ __launch_bounds__((batch_threads<C, FORCE>())) void batch_kernel(
    const CaseDesc* __restrict__ cases, CaseOut* out) {
  constexpr int NT = batch_threads<C, FORCE>();
  // LDS of the split node loop (D3Q121 in the instances that split it)
  constexpr int kPartLds = (SETS & 4) != 0 && batch_parts<D3Q121, C, FORCE>() > 1 ? 9 * NT : 1;
  __shared__ double ratio_s[2 * kBatchMaxNx];
  __shared__ double red[4][NT];
  __shared__ double wtab_s[2 * kQMax];
  __shared__ typename C::R part_s[kPartLds];
  const CaseDesc& cd = cases[blockIdx.x];
  const int lat = cd.lattice;
  if (lat == 0 && (SETS & 1)) {
    if constexpr ((SETS & 1) != 0) run_case<D2Q16, C, FORCE, NT>(cd, out, ratio_s, red, wtab_s, part_s);
  } else if (lat == 1 && (SETS & 2)) {
    if constexpr ((SETS & 2) != 0) run_case<D2Q17, C, FORCE, NT>(cd, out, ratio_s, red, wtab_s, part_s);
  } else if (lat == 2 && (SETS & 4)) {
    if constexpr ((SETS & 4) != 0) run_case<D3Q121, C, FORCE, NT>(cd, out, ratio_s, red, wtab_s, part_s);
  } else if (threadIdx.x == 0) {
    out[blockIdx.x].residual = __builtin_nan("");
    out[blockIdx.x].mass = __builtin_nan("");
    out[blockIdx.x].steps = 0.0;
    out[blockIdx.x].state = -1.0;
  }
}

// hipGetLastError reports the last error of any HIP call on this thread,
// including calls made by other libraries in the process; clear it before a
// launch so the check after the launch sees only the launch itself.
inline void clear_stale_error() { (void)hipGetLastError(); }

inline unsigned grid_for(long long threads) {
  return unsigned((threads + kBlock - 1) / kBlock);
}

// Launchers of one (velocity set, storage format, body force or not)
// triple, instantiated in its own translation unit (lbm_set_*.hip) so that
// they compile in parallel.  The force is a compile-time variant: the
// force-free kernels carry none of its code or registers.
template <class L, class C, bool FORCE>
struct SetOps {
  static hipError_t wall(const StepArgs& a, hipStream_t s);
  static hipError_t step(const StepArgs& a, bool moments, hipStream_t s);
  static hipError_t step_rows(const StepArgs& a, bool moments, hipStream_t s);
  static hipError_t init(const StepArgs& a, const double* fields, hipStream_t s);
};

#ifdef LBM_DEFINE_SET_OPS
template <class L, class C, bool FORCE>
hipError_t SetOps<L, C, FORCE>::wall(const StepArgs& a, hipStream_t s) {
  clear_stale_error();
  hipLaunchKernelGGL((wall_kernel<L, C>), dim3(grid_for(2LL * a.nx * 64)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class L, class C, bool FORCE>
hipError_t SetOps<L, C, FORCE>::step(const StepArgs& a, bool moments, hipStream_t s) {
  const dim3 grid(grid_for((long long)a.nx * a.ny));
  clear_stale_error();
  if (moments)
    hipLaunchKernelGGL((step_kernel<L, C, true, FORCE>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<L, C, false, FORCE>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class L, class C, bool FORCE>
hipError_t SetOps<L, C, FORCE>::step_rows(const StepArgs& a, bool moments, hipStream_t s) {
  const dim3 grid(unsigned(a.nx / kBlock) * unsigned(a.ny));
  clear_stale_error();
  if (moments)
    hipLaunchKernelGGL((step_rows_kernel<L, C, true, FORCE>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((step_rows_kernel<L, C, false, FORCE>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class L, class C, bool FORCE>
hipError_t SetOps<L, C, FORCE>::init(const StepArgs& a, const double* fields, hipStream_t s) {
  clear_stale_error();
  hipLaunchKernelGGL((init_kernel<L, C, FORCE>), dim3(grid_for((long long)a.nx * a.ny)),
                     dim3(kBlock), 0, s, a, fields);
  return hipGetLastError();
}
#endif

// Batched persistent launch of one storage format (lbm_batch_*.hip).
template <class C, bool FORCE, int SETS>
hipError_t batch_launch(const CaseDesc* cases, int ncase, CaseOut* out, hipStream_t s);

#ifdef LBM_DEFINE_BATCH
template <class C, bool FORCE, int SETS>
hipError_t batch_launch(const CaseDesc* cases, int ncase, CaseOut* out, hipStream_t s) {
  clear_stale_error();
  hipLaunchKernelGGL((batch_kernel<C, FORCE, SETS>), dim3(unsigned(ncase)),
                     dim3(batch_threads<C, FORCE>()), 0, s, cases, out);
  return hipGetLastError();
}
#endif


extern template hipError_t batch_launch<CF64, false, 3>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF64, false, 4>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF64, true, 3>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF64, true, 4>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32, false, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32, true, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CBF16, false, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CBF16, true, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CFP16, false, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CFP16, true, 7>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32S, false, 3>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32S, false, 4>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32S, true, 3>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);
extern template hipError_t batch_launch<CF32S, true, 4>(const CaseDesc*, int,
                                                           CaseOut*, hipStream_t);

extern template struct SetOps<D2Q16, CF64, false>;
extern template struct SetOps<D2Q16, CF64, true>;
extern template struct SetOps<D2Q16, CF32, false>;
extern template struct SetOps<D2Q16, CF32, true>;
extern template struct SetOps<D2Q16, CBF16, false>;
extern template struct SetOps<D2Q16, CBF16, true>;
extern template struct SetOps<D2Q16, CFP16, false>;
extern template struct SetOps<D2Q16, CFP16, true>;
extern template struct SetOps<D2Q16, CF32S, false>;
extern template struct SetOps<D2Q16, CF32S, true>;
extern template struct SetOps<D2Q17, CF64, false>;
extern template struct SetOps<D2Q17, CF64, true>;
extern template struct SetOps<D2Q17, CF32, false>;
extern template struct SetOps<D2Q17, CF32, true>;
extern template struct SetOps<D2Q17, CBF16, false>;
extern template struct SetOps<D2Q17, CBF16, true>;
extern template struct SetOps<D2Q17, CFP16, false>;
extern template struct SetOps<D2Q17, CFP16, true>;
extern template struct SetOps<D2Q17, CF32S, false>;
extern template struct SetOps<D2Q17, CF32S, true>;
extern template struct SetOps<D3Q121, CF64, false>;
extern template struct SetOps<D3Q121, CF64, true>;
extern template struct SetOps<D3Q121, CF32, false>;
extern template struct SetOps<D3Q121, CF32, true>;
extern template struct SetOps<D3Q121, CBF16, false>;
extern template struct SetOps<D3Q121, CBF16, true>;
extern template struct SetOps<D3Q121, CFP16, false>;
extern template struct SetOps<D3Q121, CFP16, true>;
extern template struct SetOps<D3Q121, CF32S, false>;
extern template struct SetOps<D3Q121, CF32S, true>;

}  // namespace dev
}  // namespace lbm
