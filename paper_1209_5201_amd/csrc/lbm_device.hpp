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
//     that column (the numerator of Eq. (eq:dkboundary)), reduces it in FP64
//     with a butterfly of lane shuffles, and stores ratio = M / D.
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

// ---------------------------------------------------------------- codecs --
// Storage <-> arithmetic.  Every format holds the deviation g = f - w_q from
// the rest state, so rounding acts on the (small) deviation, not on f.
// 16-bit formats hold h = g * S for a per-format power of two S
// (Tables::dec = 1/S, enc = S) and decode to float.
struct CF64 {
  using S = double;
  using R = double;
  __device__ static R ld(const S* p, const Tables*) { return *p; }
  __device__ static void st(S* p, R g, const Tables*) { *p = g; }
};

struct CF32 {
  using S = float;
  using R = float;
  __device__ static R ld(const S* p, const Tables*) { return *p; }
  __device__ static void st(S* p, R g, const Tables*) { *p = g; }
};

struct CBF16 {
  using S = uint16_t;
  using R = float;
  __device__ static R ld(const S* p, const Tables* t) {
    return __uint_as_float(uint32_t(*p) << 16) * t->dec;
  }
  __device__ static void st(S* p, R g, const Tables* t) {
    uint32_t u = __float_as_uint(g * t->enc);
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      *p = uint16_t(0x7fc0);  // keep NaN a NaN
      return;
    }
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    *p = uint16_t(u >> 16);
  }
};

struct CFP16 {
  using S = _Float16;
  using R = float;
  __device__ static R ld(const S* p, const Tables* t) { return float(*p) * t->dec; }
  __device__ static void st(S* p, R g, const Tables* t) {
    *p = _Float16(g * t->enc);  // v_cvt_f16_f32: round to nearest even
  }
};

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
    } else if constexpr (L::EQ == 3) {
      c.k0a = drho + rho * (-R(0.5) * uu - R(0.5) * D * th);
      c.k0b = rho * (R(0.5) * th);
      c.k1a = rho * (R(1) - R(0.5) * uu - R(0.5) * (D + 2) * th);
      c.k1b = rho * (R(0.5) * th);
      c.k2a = rho * R(0.5);
      c.k3 = rho * R(1.0 / 6.0);
    } else {
      c.k0a = drho + rho * (-R(0.5) * uu - R(0.5) * D * th);
      c.k0b = rho * (R(0.5) * th);
      c.k1a = rho;
      c.k2a = rho * R(0.5);
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
};

template <class R>
struct Macro {
  R rho, drho, ux, uy, uz, th;
};

// Eq. (eq:summac) from the deviations: rho = 1 + sum g, rho u = sum g c
// (sum w c = 0), and for the thermal set rho D T = D + sum g |c|^2 - rho u^2
// (sum w |c|^2 = D); theta = T - 1.  Isothermal sets use T = 1.
template <class L, class R>
__device__ __forceinline__ Macro<R> macro(const R (&g)[L::Q]) {
  R drho = 0, mx = 0, my = 0, mz = 0, e2 = 0;
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    const R v = g[q];
    drho += v;
    mx = add_scaled<ex>(mx, v);
    my = add_scaled<ey>(my, v);
    mz = add_scaled<ez>(mz, v);
    if constexpr (L::THERMAL) e2 = add_scaled<ex * ex + ey * ey + ez * ez>(e2, v);
  };
  static_for<0, L::Q>(body);
  Macro<R> m;
  m.drho = drho;
  m.rho = R(1) + drho;
  const R inv = R(1) / m.rho;
  constexpr R r = R(L::R);
  m.ux = r * mx * inv;
  m.uy = r * my * inv;
  m.uz = r * mz * inv;
  if constexpr (L::THERMAL) {
    const R uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
    m.th = (R(L::R * L::R) * e2 - m.rho * uu - R(L::D) * drho) * (inv * R(1.0 / L::D));
  } else {
    m.th = R(0);
  }
  return m;
}

// g* = g - omega (g - (f^eq - w)), in place.
template <class L, class R>
__device__ __forceinline__ void relax(R (&g)[L::Q], R omega) {
  const Macro<R> m = macro<L, R>(g);
  const R uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const auto k = EqCoef<L, R>::make(m.rho, m.drho, uu, m.th);
  constexpr R r = R(L::R);
  const R sx = r * m.ux, sy = r * m.uy, sz = r * m.uz;
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    R x = R(0);
    x = add_scaled<ex>(x, sx);
    x = add_scaled<ey>(x, sy);
    x = add_scaled<ez>(x, sz);
    const R geq = R(L::W[q]) * k.template poly<ex * ex + ey * ey + ez * ez>(x);
    g[q] = g[q] + omega * (geq - g[q]);
  };
  static_for<0, L::Q>(body);
}

// Output fields of one node from its deviations (always FP64): rho, u, T,
// and the stress / heat flux of f = f^eq + kfac (f~ - f^eq) (conversion of
// Sec. II).
template <class L, class R>
__device__ __forceinline__ void write_fields(const R (&gr)[L::Q], double kfac, double* mom,
                                             long long nodes, long long n) {
  double g[L::Q];
  auto cvt = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    g[q] = double(gr[q]);
  };
  static_for<0, L::Q>(cvt);
  const Macro<double> m = macro<L, double>(g);
  const double uu = m.ux * m.ux + m.uy * m.uy + m.uz * m.uz;
  const auto k = EqCoef<L, double>::make(m.rho, m.drho, uu, m.th);
  constexpr double r = L::R;
  const double sx = r * m.ux, sy = r * m.uy, sz = r * m.uz;
  double sxy = 0, qx = 0, qy = 0, qz = 0;
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
    const double x = ex * sx + ey * sy + ez * sz;
    const double geq = L::W[q] * k.template poly<ex * ex + ey * ey + ez * ez>(x);
    const double fp = L::W[q] + geq + kfac * (g[q] - geq);
    const double Cx = r * ex - m.ux, Cy = r * ey - m.uy, Cz = r * ez - m.uz;
    const double C2 = Cx * Cx + Cy * Cy + Cz * Cz;
    sxy += fp * Cx * Cy;
    qx += fp * C2 * Cx;
    qy += fp * C2 * Cy;
    qz += fp * C2 * Cz;
  };
  static_for<0, L::Q>(body);
  mom[0 * nodes + n] = m.rho;
  mom[1 * nodes + n] = m.ux;
  mom[2 * nodes + n] = m.uy;
  mom[3 * nodes + n] = m.uz;
  mom[4 * nodes + n] = 1.0 + m.th;
  mom[5 * nodes + n] = sxy;
  mom[6 * nodes + n] = 0.5 * qx;
  mom[7 * nodes + n] = 0.5 * qy;
  mom[8 * nodes + n] = 0.5 * qz;
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

// Columns x - s (periodic) for s = -3..3, valid for any nx >= 1.
template <int NS>
__device__ __forceinline__ void wrapped_columns(int x, int nx, int (&xw)[2 * NS + 1]) {
  for (int s = -NS; s <= NS; ++s) {
    int c = x - s;
    while (c < 0) c += nx;
    while (c >= nx) c -= nx;
    xw[s + NS] = c;
  }
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

template <class L, class C, bool TOP>
__device__ __forceinline__ double ghost_mass(const typename C::S* __restrict__ fin,
                                             const StepArgs& a, int xp, int lane) {
  using W = WallTerms<L>;
  double acc = 0.0;
  auto body = [&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr auto T = TOP ? W::top().t[t] : W::bottom().t[t];
    if (lane == (t & 63)) {
      int xs = xp - T.ex;
      while (xs < 0) xs += a.nx;
      while (xs >= a.nx) xs -= a.nx;
      const int row = TOP ? a.ny - 1 - T.j : T.j;
      const uint32_t idx = uint32_t(T.q) * uint32_t(a.plane) + uint32_t(row) * uint32_t(a.nx) +
                           uint32_t(xs);
      acc += double(C::ld(fin + idx, a.tab));
    }
  };
  static_for<0, W::NT>(body);
  // butterfly over the 64 lanes: fixed order, every lane ends with the sum
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  return acc;
}

template <class L, class C>
__global__ __launch_bounds__(kBlock) void wall_kernel(StepArgs a) {
  const int wave = int((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = int(threadIdx.x & 63);
  if (wave >= 2 * a.nx) return;  // wave-uniform
  const auto* fin = static_cast<const typename C::S*>(a.fin);
  const bool top = wave >= a.nx;
  const int xp = top ? wave - a.nx : wave;
  double M;
  if (top)
    M = ghost_mass<L, C, true>(fin, a, xp, lane);
  else
    M = ghost_mass<L, C, false>(fin, a, xp, lane);
  // pooled incoming mass = rest-state part + deviations; ratio of
  // Eq. (eq:dkboundary) numerator to its denominator
  if (lane == 0)
    a.ratio[(top ? a.nx : 0) + xp] =
        top ? (a.tab->Wt + M) / a.tab->Dt : (a.tab->Wb + M) / a.tab->Db;
}

// ------------------------------------------------------------- the step --
template <class L, class C>
__device__ __forceinline__ void pull(typename C::R (&f)[L::Q], const StepArgs& a, int x,
                                     int y) {
  using R = typename C::R;
  using S = typename C::S;
  constexpr int NS = max_ex<L>();
  const auto* __restrict__ fin = static_cast<const S*>(a.fin);
  int xw[2 * NS + 1];
  wrapped_columns<NS>(x, a.nx, xw);
  const uint32_t plane = uint32_t(a.plane);
  const uint32_t nx = uint32_t(a.nx);
  if (y >= L::N && y < a.ny - L::N) {
    auto body = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      const uint32_t idx = uint32_t(q) * plane + uint32_t(y - ey) * nx + uint32_t(xw[ex + NS]);
      f[q] = C::ld(fin + idx, a.tab);
    };
    static_for<0, L::Q>(body);
  } else {
    const double* rb = a.ratio;
    const double* rt = a.ratio + a.nx;
    auto body = [&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int ex = L::E[q][0], ey = L::E[q][1];
      const int ys = y - ey;
      if (ey > 0 && ys < 0) {
        // re-emitted by the bottom wall: f = g^eq(u_b, T_b) M / D
        f[q] = R(a.tab->gb[q] * rb[xw[ex + NS]] - L::W[q]);
      } else if (ey < 0 && ys >= a.ny) {
        f[q] = R(a.tab->gt[q] * rt[xw[ex + NS]] - L::W[q]);  // top wall
      } else {
        const uint32_t idx = uint32_t(q) * plane + uint32_t(ys) * nx + uint32_t(xw[ex + NS]);
        f[q] = C::ld(fin + idx, a.tab);
      }
    };
    static_for<0, L::Q>(body);
  }
}

template <class L, class C>
__device__ __forceinline__ void store(const typename C::R (&f)[L::Q], const StepArgs& a,
                                      uint32_t n) {
  auto* __restrict__ fout = static_cast<typename C::S*>(a.fout);
  const uint32_t plane = uint32_t(a.plane);
  auto body = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    C::st(fout + uint32_t(q) * plane + n, f[q], a.tab);
  };
  static_for<0, L::Q>(body);
}

template <class L, class C, bool MOM>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs a) {
  using R = typename C::R;
  const long long nodes = (long long)a.nx * a.ny;
  const long long n = (long long)xcd_remap(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
  if (n >= nodes) return;
  const int y = int(n / a.nx);
  const int x = int(n - (long long)y * a.nx);
  R f[L::Q];
  pull<L, C>(f, a, x, y);
  if constexpr (MOM) write_fields<L, R>(f, a.kfac, a.mom, nodes, n);
  relax<L, R>(f, R(a.omega));
  store<L, C>(f, a, uint32_t(n));
}

// f~(0) = f^eq(rho0, u0, T0); writes the output fields of f~(0) and stores
// f*(0) = relaxed f~(0), the state every later step pulls from (as
// deviations from the rest weights).
template <class L, class C>
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
    f[q] = R(L::W[q] * k.template poly<ex * ex + ey * ey + ez * ez>(x));  // f^eq - w
  };
  static_for<0, L::Q>(body);
  write_fields<L, R>(f, a.kfac, a.mom, nodes, n);
  relax<L, R>(f, R(a.omega));
  store<L, C>(f, a, uint32_t(n));
}

inline unsigned grid_for(long long threads) {
  return unsigned((threads + kBlock - 1) / kBlock);
}

// Launchers of one (velocity set, storage format) pair, instantiated in its
// own translation unit (lbm_set_*.hip) so that the pairs compile in
// parallel.
template <class L, class C>
struct SetOps {
  static hipError_t wall(const StepArgs& a, hipStream_t s);
  static hipError_t step(const StepArgs& a, bool moments, hipStream_t s);
  static hipError_t init(const StepArgs& a, const double* fields, hipStream_t s);
};

#ifdef LBM_DEFINE_SET_OPS
template <class L, class C>
hipError_t SetOps<L, C>::wall(const StepArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((wall_kernel<L, C>), dim3(grid_for(2LL * a.nx * 64)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class L, class C>
hipError_t SetOps<L, C>::step(const StepArgs& a, bool moments, hipStream_t s) {
  const dim3 grid(grid_for((long long)a.nx * a.ny));
  if (moments)
    hipLaunchKernelGGL((step_kernel<L, C, true>), grid, dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<L, C, false>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class L, class C>
hipError_t SetOps<L, C>::init(const StepArgs& a, const double* fields, hipStream_t s) {
  hipLaunchKernelGGL((init_kernel<L, C>), dim3(grid_for((long long)a.nx * a.ny)), dim3(kBlock),
                     0, s, a, fields);
  return hipGetLastError();
}
#endif

extern template struct SetOps<D2Q16, CF64>;
extern template struct SetOps<D2Q16, CF32>;
extern template struct SetOps<D2Q16, CBF16>;
extern template struct SetOps<D2Q16, CFP16>;
extern template struct SetOps<D2Q17, CF64>;
extern template struct SetOps<D2Q17, CF32>;
extern template struct SetOps<D2Q17, CBF16>;
extern template struct SetOps<D2Q17, CFP16>;
extern template struct SetOps<D3Q121, CF64>;
extern template struct SetOps<D3Q121, CF32>;
extern template struct SetOps<D3Q121, CBF16>;
extern template struct SetOps<D3Q121, CFP16>;

}  // namespace dev
}  // namespace lbm
