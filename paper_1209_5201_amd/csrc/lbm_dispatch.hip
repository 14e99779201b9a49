// Launch dispatch by velocity set, the FP64 reductions, and the host-side
// helpers (wall Maxwellians, set descriptions).
#include "lbm_device.hpp"

namespace lbm {
namespace dev {

// ----------------------------------------------------------- reductions --
// Fixed grid and fixed combination order: the FP64 results are
// deterministic for a given problem size.
__global__ __launch_bounds__(kBlock) void reduce_partial(ReduceArgs r) {
  __shared__ double sh[4][kBlock];
  const long long n = r.nodes;
  double v[4] = {0, 0, 0, 0};
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (long long)gridDim.x * kBlock)
    residual_terms(r.mom, r.snap, n, i, v);
  block_sum4(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) r.partial[blockIdx.x * 4 + k] = v[k];
}

__global__ __launch_bounds__(kBlock) void reduce_final(ReduceArgs r) {
  __shared__ double sh[4][kBlock];
  double v[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < kReduceBlocks; b += kBlock)
    for (int k = 0; k < 4; ++k) v[k] += r.partial[b * 4 + k];
  block_sum4(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) r.result[k] = v[k];
}

}  // namespace dev

namespace {

template <class L, bool FORCE, class F>
hipError_t by_prec_f(int prec, F&& fn) {
  switch (prec) {
    case kFP64: return fn(dev::SetOps<L, dev::CF64, FORCE>{});
    case kFP32: return fn(dev::SetOps<L, dev::CF32, FORCE>{});
    case kBF16: return fn(dev::SetOps<L, dev::CBF16, FORCE>{});
    case kFP16: return fn(dev::SetOps<L, dev::CFP16, FORCE>{});
    case kFP32S: return fn(dev::SetOps<L, dev::CF32S, FORCE>{});
  }
  return hipErrorInvalidValue;
}

// the body-force variant when the step's arguments carry a force
template <class L, class F>
hipError_t by_prec(int prec, const StepArgs& a, F&& fn) {
  return a.force ? by_prec_f<L, true>(prec, fn) : by_prec_f<L, false>(prec, fn);
}

// all sets in one instance (SETS = 7)
template <class C>
hipError_t batch_of(bool force, const CaseDesc* cases, int ncase, CaseOut* out, hipStream_t s) {
  return force ? dev::batch_launch<C, true, 7>(cases, ncase, out, s)
               : dev::batch_launch<C, false, 7>(cases, ncase, out, s);
}

// the 2-D sets (SETS = 3) or the large set (SETS = 4) in separate instances
template <class C>
hipError_t batch_of_split(bool force, bool large, const CaseDesc* cases, int ncase,
                          CaseOut* out, hipStream_t s) {
  if (large)
    return force ? dev::batch_launch<C, true, 4>(cases, ncase, out, s)
                 : dev::batch_launch<C, false, 4>(cases, ncase, out, s);
  return force ? dev::batch_launch<C, true, 3>(cases, ncase, out, s)
               : dev::batch_launch<C, false, 3>(cases, ncase, out, s);
}

template <class F>
hipError_t by_set(int lattice, F&& fn) {
  switch (lattice) {
    case 0: return fn(D2Q16{});
    case 1: return fn(D2Q17{});
    case 2: return fn(D3Q121{});
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_wall(int lattice, int prec, const StepArgs& a, hipStream_t s) {
  return by_set(lattice, [&](auto lat) {
    return by_prec<decltype(lat)>(prec, a, [&](auto ops) { return decltype(ops)::wall(a, s); });
  });
}

hipError_t launch_step(int lattice, int prec, const StepArgs& a, bool moments, hipStream_t s) {
  return by_set(lattice, [&](auto lat) {
    return by_prec<decltype(lat)>(prec, a,
                                  [&](auto ops) { return decltype(ops)::step(a, moments, s); });
  });
}

hipError_t launch_step_rows(int lattice, int prec, const StepArgs& a, bool moments,
                            hipStream_t s) {
  return by_set(lattice, [&](auto lat) {
    return by_prec<decltype(lat)>(
        prec, a, [&](auto ops) { return decltype(ops)::step_rows(a, moments, s); });
  });
}

hipError_t launch_init(int lattice, int prec, const StepArgs& a, const double* fields,
                       hipStream_t s) {
  return by_set(lattice, [&](auto lat) {
    return by_prec<decltype(lat)>(prec, a,
                                  [&](auto ops) { return decltype(ops)::init(a, fields, s); });
  });
}

hipError_t launch_reduce(const ReduceArgs& r, hipStream_t s) {
  dev::clear_stale_error();
  hipLaunchKernelGGL(dev::reduce_partial, dim3(kReduceBlocks), dim3(kBlock), 0, s, r);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dev::reduce_final, dim3(1), dim3(kBlock), 0, s, r);
  return hipGetLastError();
}

bool batch_splits_sets(int prec) { return prec == kFP64 || prec == kFP32S; }

hipError_t launch_batch(int prec, bool force, bool large, const CaseDesc* cases, int ncase,
                        CaseOut* out, hipStream_t s) {
  if (ncase <= 0 || !cases || !out) return hipErrorInvalidValue;  // one workgroup per case
  switch (prec) {
    case kFP64: return batch_of_split<dev::CF64>(force, large, cases, ncase, out, s);
    case kFP32: return batch_of<dev::CF32>(force, cases, ncase, out, s);
    case kBF16: return batch_of<dev::CBF16>(force, cases, ncase, out, s);
    case kFP16: return batch_of<dev::CFP16>(force, cases, ncase, out, s);
    case kFP32S: return batch_of_split<dev::CF32S>(force, large, cases, ncase, out, s);
  }
  return hipErrorInvalidValue;
}

// Host copy of the equilibrium used for the wall Maxwellians (same
// polynomial as the kernels).
void host_geq(int lattice, const double u[3], double T, double* out) {
  by_set(lattice, [&](auto lat) {
    using L = decltype(lat);
    const auto k = dev::EqCoef<L, double>::make(1.0, 0.0, u[0] * u[0] + u[1] * u[1] + u[2] * u[2],
                                           L::THERMAL ? T - 1.0 : 0.0);
    for (int q = 0; q < L::Q; ++q) {
      const double x = L::R * (L::E[q][0] * u[0] + L::E[q][1] * u[1] + L::E[q][2] * u[2]);
      const int ee = L::E[q][0] * L::E[q][0] + L::E[q][1] * L::E[q][1] + L::E[q][2] * L::E[q][2];
      // runtime |e|^2: evaluate the same polynomial with cc = r^2 |e|^2
      const double cc = L::R * L::R * ee;
      double K0 = k.k0a, K1 = k.k1a, K2 = k.k2a;
      if (L::THERMAL) {
        K0 = k.k0a + cc * (k.k0b + cc * k.k0c);
        K1 = k.k1a + cc * k.k1b;
        K2 = k.k2a + cc * k.k2b;
      }
      double p;
      if (L::EQ >= 4) p = K0 + x * (K1 + x * (K2 + x * (k.k3 + x * k.k4)));
      else if (L::EQ == 3) p = K0 + x * (K1 + x * (K2 + x * k.k3));
      else p = K0 + x * (K1 + x * K2);
      out[q] = L::W[q] + L::W[q] * p;
    }
    return hipSuccess;
  });
}

// Lattice description for the host (no device work).
int host_lattice(int lattice, int* Q, int* D, int* N, int* EQ, double* r, int* e, double* w) {
  if (lattice < 0 || lattice > 2) return -1;
  by_set(lattice, [&](auto lat) {
    using L = decltype(lat);
    *Q = L::Q;
    *D = L::D;
    *N = L::N;
    *EQ = L::EQ;
    *r = L::R;
    if (e)
      for (int q = 0; q < L::Q; ++q)
        for (int i = 0; i < 3; ++i) e[3 * q + i] = L::E[q][i];
    if (w)
      for (int q = 0; q < L::Q; ++q) w[q] = L::W[q];
    return hipSuccess;
  });
  return 0;
}

}  // namespace lbm
