// Internal types shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbm {

constexpr int kQMax = 121;
constexpr int kFields = 9;          // rho, ux, uy, uz, T, sxy, qx, qy, qz
constexpr int kBlock = 256;         // threads per block of the node kernels
constexpr int kReduceBlocks = 512;  // partial sums of the FP64 reductions

enum Prec : int { kFP64 = 0, kFP32 = 1, kBF16 = 2, kFP16 = 3, kFP32S = 4 };
constexpr int kPrecCount = 5;

// Per-context constants, resident in device memory and read by the kernels
// through a const __restrict__ pointer (wave-uniform, so scalar loads).
// Populations are held as deviations g_q = f_q - w_q from the rest state
// (rho = 1, u = 0, T = 1) in storage and in all arithmetic.
struct Tables {
  double gb[kQMax];   // g^eq(u_b, T_b), unit density: bottom-wall Maxwellian
  double gt[kQMax];   // top-wall Maxwellian
  double Db, Dt;      // sum over layers l and outgoing velocities of g^eq
  double Wb, Wt;      // rest-state part of the pooled mass: sum of w over the
                      // (velocity, row) pairs that cross each wall
  double ab, at;      // accommodation of each wall: the diffuse share of the
                      // scattering kernel R = a R_D + (1 - a) R_specular
};

struct StepArgs {
  const void* fin;      // deviations g* of the previous step (SoA planes)
  void* fout;           // populations written by this step
  const Tables* tab;
  double* ratio;        // [2][nx]: pooled incoming mass / D per ghost column
  double* mom;          // kFields x nodes output fields, or null
  int nx, ny;
  long long plane;      // elements between population planes
  double omega;         // 1 / (tau + 1/2)
  double kfac;          // tau / (tau + 1/2): f~ -> f conversion of sigma, q
  double tau;           // relaxation time at rho = T = 1
  double vexp;          // viscosity exponent w of the local law (law != 0)
  int law;              // 0: constant tau; 1: tau T^(w-1) / rho per node
  int force;            // 1: body force (ax, ay, az) acts
  double ax, ay, az;    // acceleration per time step (velocity units)
  uint32_t step;        // index of the step being produced (rounding counter)
  uint32_t seed;        // per-context rounding seed
};

struct ReduceArgs {
  const double* mom;    // output fields of the current time
  double* snap;         // ux, uy, uz, T at the previous residual point
  double* partial;      // kReduceBlocks x 4
  double* result;       // mass, sum du^2, sum dT^2, nonfinite count
  long long nodes;
};

// One channel of a batched launch (lbm_batch_step): the step arguments of a
// context plus its buffers.  Built on the host, copied to the device.
constexpr int kBatchMaxNx = 64;    // ghost-column ratios of a case live in LDS
constexpr int kBatchBlock = 256;   // threads per case of the batched kernel (FP32: 1024)
struct CaseDesc {
  StepArgs a;           // fin/fout/step are set per step from f, cur, steps
  void* f[2];
  double* snap;         // residual snapshot of the context
  double* result;       // mass, sum du^2, sum dT^2, nonfinite count
  double uref;          // velocity scale of the residual
  double tol;           // stop after a window whose residual is below tol
  int cur;              // f[cur] holds the newest f*
  int lattice;
  int window;           // steps per residual window
  int budget;           // most steps this launch (a multiple of window)
};
// Per-case output of a batched launch.
struct CaseOut {
  double residual;      // residual of the last window (NaN: non-finite)
  double mass;
  double steps;         // steps advanced
  double state;         // 1 converged, 0 budget used up, -1 non-finite
};

// Launchers (lbm_set_*.hip, lbm_dispatch.hip).  lattice: 0 D2Q16, 1 D2Q17, 2 D3Q121.
hipError_t launch_wall(int lattice, int prec, const StepArgs& a, hipStream_t s);
hipError_t launch_step(int lattice, int prec, const StepArgs& a, bool moments,
                       hipStream_t s);
// Same update for nx a multiple of kBlock, with the wall sums fused in: no
// launch_wall needed before it.
hipError_t launch_step_rows(int lattice, int prec, const StepArgs& a, bool moments,
                            hipStream_t s);
// f~ = f^eq(fields) -> collide -> fout; also writes the output fields.
// fields: rho, ux, uy, uz, T (5 x nodes doubles, may alias a.mom).
hipError_t launch_init(int lattice, int prec, const StepArgs& a,
                       const double* fields, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs& r, hipStream_t s);
// One workgroup per case advances every case of one storage precision (and
// one force variant: all cases with or all without a body force) in
// windows of cases[i].window steps, up to cases[i].budget steps, stopping a
// case after the first window whose residual is below cases[i].tol; writes
// each case's fields after its last window, its mass / residual sums into
// its result block, and out[i].
// large: for formats with batch_splits_sets, the launch of the large set's
// cases (else of the 2-D sets' cases); ignored for the other formats, whose
// one launch takes every set.
hipError_t launch_batch(int prec, bool force, bool large, const CaseDesc* cases, int ncase,
                        CaseOut* out, hipStream_t s);
bool batch_splits_sets(int prec);

// Host helpers (no device work).
// g^eq_q(u, T) of every velocity with unit density (wall Maxwellians).
void host_geq(int lattice, const double u[3], double T, double* out);
// Q, D, N (ghost layers), truncation order, r, e (Q x 3) and w (Q) of a set;
// e and w may be null.  Returns -1 for an unknown lattice.
int host_lattice(int lattice, int* Q, int* D, int* N, int* EQ, double* r, int* e, double* w);

}  // namespace lbm
