// Bandwidth references for the fused update (measurement aids, not part of
// the update path; built into libceiling.so).  Both alternate between two
// buffers, as the update does, so that no launch reads data that a
// memory-side cache kept from the launch before:
//  - pull_only<L, T>: the update's access pattern with no collision
//    arithmetic.  Planes of nx*ny elements of T (8, 4 or 2 bytes, the
//    population formats) with the update's plane stride (the node count
//    rounded up to 64, plus 128), one node per lane, blocks of 256 lanes along a
//    row, the same XCD-aware block order, each velocity pulled from
//    (x - e_x, y - e_y) with x periodic, nontemporal stores; over the rows
//    whose sources all lie inside the grid (N <= y < ny - N).
//  - copy4: a 16-byte-per-lane copy of the same state, nontemporal stores.
//
// extern "C" int lbm_ceiling(int lattice, int elem_bytes, int nx, int ny,
//                            int reps, double* pull_us, double* copy_us,
//                            double* pull_bytes, double* copy_bytes)
//   lattice 0 D2Q16, 1 D2Q17, 2 D3Q121; elem_bytes 8, 4 or 2; nx a multiple
//   of 256, ny > 2N.  Allocates the two state buffers, times reps launches
//   of each kernel (after two untimed ones) with HIP events on a stream of
//   its own, frees everything.  Writes the mean launch time in microseconds
//   and the bytes each launch moves.  Returns 0, -1 for invalid arguments
//   (before any device work), -2 on a HIP error.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice_tables.h"

namespace {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// Blocks are dealt to the XCDs round-robin; give each XCD a contiguous run.
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int per = nb / kXcds, rem = nb % kXcds, xcd = b % kXcds, idx = b / kXcds;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

template <int I, int N, class F>
__device__ __forceinline__ void unroll(F& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll<I + 1, N>(f);
  }
}

template <class L>
constexpr bool shifts_within_n() {
  for (int q = 0; q < L::Q; ++q)
    if (L::E[q][0] > L::N || L::E[q][0] < -L::N || L::E[q][1] > L::N || L::E[q][1] < -L::N)
      return false;
  return true;
}

// Folds a loaded element into a running value and back, so that every
// stored element depends on every load of its lane.
__device__ __forceinline__ double mix(double acc, double v) { return acc + v; }
__device__ __forceinline__ float mix(float acc, float v) { return acc + v; }
__device__ __forceinline__ uint16_t mix(uint16_t acc, uint16_t v) { return uint16_t(acc ^ v); }
__device__ __forceinline__ double fold(double v, double acc) { return v + 1e-15 * acc; }
__device__ __forceinline__ float fold(float v, float acc) { return v + 1e-7f * acc; }
__device__ __forceinline__ uint16_t fold(uint16_t v, uint16_t acc) {
  return uint16_t(v ^ (acc & 1u));
}

template <class L, class T>
__global__ __launch_bounds__(kBlock) void pull_only(const T* __restrict__ src,
                                                    T* __restrict__ dst, int nx,
                                                    unsigned plane) {
  static_assert(shifts_within_n<L>(), "a source row or column beyond N");
  const int bpr = nx / kBlock;
  const int b = xcd_order(int(blockIdx.x), int(gridDim.x));
  const int y = L::N + b / bpr;
  const int x = (b % bpr) * kBlock + int(threadIdx.x);
  T f[L::Q];
  T s = T(0);
  auto load = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    int c = x - L::E[q][0];
    c += c < 0 ? nx : 0;
    c -= c >= nx ? nx : 0;
    f[q] = src[size_t(q) * plane + unsigned(y - L::E[q][1]) * unsigned(nx) + unsigned(c)];
    s = mix(s, f[q]);
  };
  unroll<0, L::Q>(load);
  auto store = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    __builtin_nontemporal_store(fold(f[q], s),
                                dst + size_t(q) * plane + unsigned(y) * unsigned(nx) + unsigned(x));
  };
  unroll<0, L::Q>(store);
}

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void copy4(const f4* __restrict__ src, f4* __restrict__ dst,
                                                size_t n) {
  const size_t i = size_t(blockIdx.x) * kBlock + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

template <class L, class T>
int measure(int nx, int ny, int reps, double* pull_us, double* copy_us, double* pull_bytes,
            double* copy_bytes) {
  if (nx < kBlock || nx % kBlock != 0 || ny <= 2 * L::N || reps < 1) return -1;
  const size_t plane = (size_t(nx) * size_t(ny) + 63) / 64 * 64 + 128;
  const size_t elems = size_t(L::Q) * plane;
  if (plane > 0xffffffffull / 2 || (elems * sizeof(T)) % sizeof(f4) != 0) return -1;
  T* buf[2] = {nullptr, nullptr};
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -2;
  auto ok = [](hipError_t e) { return e == hipSuccess; };
  do {
    if (!ok(hipMalloc(&buf[0], elems * sizeof(T))) || !ok(hipMalloc(&buf[1], elems * sizeof(T))))
      break;
    if (!ok(hipStreamCreate(&s)) || !ok(hipEventCreate(&e0)) || !ok(hipEventCreate(&e1))) break;
    if (!ok(hipMemsetAsync(buf[0], 0, elems * sizeof(T), s)) ||
        !ok(hipMemsetAsync(buf[1], 0, elems * sizeof(T), s)))
      break;
    const dim3 gp(unsigned(nx / kBlock) * unsigned(ny - 2 * L::N));
    const size_t n4 = elems * sizeof(T) / sizeof(f4);
    const dim3 gc(unsigned((n4 + kBlock - 1) / kBlock));
    float ms = 0.0f;
    bool good = true;
    // pull pattern
    for (int r = -2; r < reps && good; ++r) {
      if (r == 0) good = ok(hipEventRecord(e0, s));
      hipLaunchKernelGGL((pull_only<L, T>), gp, dim3(kBlock), 0, s, buf[r & 1], buf[(r + 1) & 1],
                         nx, unsigned(plane));
      good = good && ok(hipGetLastError());
    }
    if (!good || !ok(hipEventRecord(e1, s)) || !ok(hipEventSynchronize(e1)) ||
        !ok(hipEventElapsedTime(&ms, e0, e1)))
      break;
    *pull_us = 1e3 * double(ms) / reps;
    *pull_bytes = 2.0 * sizeof(T) * L::Q * double(nx) * double(ny - 2 * L::N);
    // copy
    for (int r = -2; r < reps && good; ++r) {
      if (r == 0) good = ok(hipEventRecord(e0, s));
      hipLaunchKernelGGL(copy4, gc, dim3(kBlock), 0, s, reinterpret_cast<const f4*>(buf[r & 1]),
                         reinterpret_cast<f4*>(buf[(r + 1) & 1]), n4);
      good = good && ok(hipGetLastError());
    }
    if (!good || !ok(hipEventRecord(e1, s)) || !ok(hipEventSynchronize(e1)) ||
        !ok(hipEventElapsedTime(&ms, e0, e1)))
      break;
    *copy_us = 1e3 * double(ms) / reps;
    *copy_bytes = 2.0 * sizeof(T) * double(elems);
    rc = 0;
  } while (false);
  if (s) (void)hipStreamSynchronize(s);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  for (T* p : buf)
    if (p) (void)hipFree(p);
  return rc;
}

template <class L>
int by_elem(int elem_bytes, int nx, int ny, int reps, double* const (&o)[4]) {
  switch (elem_bytes) {
    case 8: return measure<L, double>(nx, ny, reps, o[0], o[1], o[2], o[3]);
    case 4: return measure<L, float>(nx, ny, reps, o[0], o[1], o[2], o[3]);
    case 2: return measure<L, uint16_t>(nx, ny, reps, o[0], o[1], o[2], o[3]);
  }
  return -1;
}

}  // namespace

extern "C" int lbm_ceiling(int lattice, int elem_bytes, int nx, int ny, int reps,
                           double* pull_us, double* copy_us, double* pull_bytes,
                           double* copy_bytes) {
  if (!pull_us || !copy_us || !pull_bytes || !copy_bytes) return -1;
  double* const out[4] = {pull_us, copy_us, pull_bytes, copy_bytes};
  switch (lattice) {
    case 0: return by_elem<lbm::D2Q16>(elem_bytes, nx, ny, reps, out);
    case 1: return by_elem<lbm::D2Q17>(elem_bytes, nx, ny, reps, out);
    case 2: return by_elem<lbm::D3Q121>(elem_bytes, nx, ny, reps, out);
  }
  return -1;
}
