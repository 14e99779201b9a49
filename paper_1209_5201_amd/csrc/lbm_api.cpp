// C ABI of the library (declared in include/lbm.h): argument checks, device
// memory layout, the per-context wall tables, and the launch sequence of a
// step.  All arithmetic of the scheme runs in the kernels.
#include "batch_plan.hpp"
#include "lbm.h"
#include "lbm_internal.hpp"

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <climits>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

using namespace lbm;

struct lbm_ctx {
  int lattice, prec;
  int nx, ny, Q, N, D;
  double tau, r;
  lbm_wall wb, wt;
  double alpha_b, alpha_t;  // accommodation (1: the paper's diffuse wall)
  int law;                  // 1: local tau from the viscosity law
  double vexp;              // its exponent w
  double acc[3];            // body force (acceleration per step); 0: none
  hipStream_t stream;
  bool owns;
  char* base;
  size_t bytes;
  long long plane;
  int elem;
  void* f[2];
  int cur;  // f[cur] holds the newest f*
  double* ratio;
  Tables* tab;
  double* mom;
  double* snap;
  double* partial;
  double* result;
  int64_t steps;
  int64_t window;  // steps covered by the newest residual
  double uref;
  int status;
  // event timing of the kernels (lbm_set_timing)
  bool timing;
  std::vector<hipEvent_t> ev;
  double t_update_ms, t_wall_ms;
  int64_t n_update, n_wall;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int elem_bytes(int prec) { return prec == kFP64 ? 8 : (prec == kFP32 || prec == kFP32S) ? 4 : 2; }

struct Layout {
  size_t pop, ratio, tab, mom, snap, partial, result, total;
  long long plane;
};

bool layout(int lattice, lbm_grid g, int prec, Layout* L) {
  int Q, D, N, EQ;
  double r;
  if (host_lattice(lattice, &Q, &D, &N, &EQ, &r, nullptr, nullptr) != 0) return false;
  if (prec < 0 || prec >= kPrecCount || g.nx < 1 || g.ny < 2 * N) return false;
  const long long nodes = (long long)g.nx * g.ny;
  // Plane stride: the node count rounded up to 64, plus 128 elements.  With
  // planes a power of two apart (2048^2 nodes) the concurrent plane streams
  // of a pull start at equally aligned addresses; the 128-element skew took
  // the D2Q17 2048^2 update from 103.5 to 101.9 us (FP32) and 56.8 to 54.5 us
  // (BF16), D3Q121 1024^2 BF16 / FP16 by 4-5 %, and left FP64 unchanged
  // (measured pads of 32-65536 elements: some strides, e.g. 256 FP32
  // elements, were slower).
  const long long plane = (nodes + 63) / 64 * 64 + 128;
  // the kernels address a plane set with 32-bit byte offsets
  if ((unsigned long long)Q * plane * elem_bytes(prec) >= (1ULL << 32)) return false;
  L->plane = plane;
  size_t off = 0;
  L->pop = off;
  off += 2 * align256(size_t(Q) * plane * elem_bytes(prec));
  L->ratio = off;
  off += align256(2 * sizeof(double) * g.nx);
  L->tab = off;
  off += align256(sizeof(Tables));
  L->mom = off;
  off += align256(sizeof(double) * kFields * nodes);
  L->snap = off;
  off += align256(sizeof(double) * 4 * nodes);
  L->partial = off;
  off += align256(sizeof(double) * 4 * kReduceBlocks);
  L->result = off;
  off += align256(sizeof(double) * 4);
  L->total = off;
  return true;
}

int fail(lbm_ctx* c, int st) {
  if (c && c->status == LBM_OK) c->status = st;
  return st;
}

// last HIP error seen by the library on this thread (lbm_last_device_error)
thread_local hipError_t g_last_hip = hipSuccess;
thread_local char g_last_msg[256];

// true if e is hipSuccess; otherwise records e for lbm_last_device_error
bool hip_ok(hipError_t e) {
  if (e == hipSuccess) return true;
  g_last_hip = e;
  return false;
}

int device_status(lbm_ctx* c, hipError_t e) {
  if (e == hipSuccess) return LBM_OK;
  g_last_hip = e;
  return fail(c, LBM_EDEVICE);
}

StepArgs make_args(lbm_ctx* c, const void* fin, void* fout, double* mom) {
  StepArgs a{};
  a.fin = fin;
  a.fout = fout;
  a.tab = c->tab;
  a.ratio = c->ratio;
  a.mom = mom;
  a.nx = c->nx;
  a.ny = c->ny;
  a.plane = c->plane;
  a.omega = 1.0 / (c->tau + 0.5);
  a.kfac = std::isinf(c->tau) ? 1.0 : c->tau / (c->tau + 0.5);
  a.tau = c->tau;
  a.vexp = c->vexp;
  a.law = c->law;
  a.ax = c->acc[0];
  a.ay = c->acc[1];
  a.az = c->acc[2];
  a.force = (c->acc[0] != 0.0 || c->acc[1] != 0.0 || c->acc[2] != 0.0) ? 1 : 0;
  a.step = uint32_t(c->steps);
  a.seed = 0x2545f491u;
  return a;
}

ReduceArgs make_reduce(lbm_ctx* c) {
  ReduceArgs r{};
  r.mom = c->mom;
  r.snap = c->snap;
  r.partial = c->partial;
  r.result = c->result;
  r.nodes = (long long)c->nx * c->ny;
  return r;
}

bool wall_ok(const lbm_wall* w) {
  return w && std::isfinite(w->ux) && std::isfinite(w->uz) && std::isfinite(w->T) && w->T > 0;
}

// Wall Maxwellians and the denominators of Eq. (eq:dkboundary):
// D = sum_l sum_{(c - u_w).n > l} g^eq = sum over velocities leaving the
// wall of (normal integer speed) * g^eq.  Returns false if an outgoing
// g^eq is not positive.
bool fill_tables(lbm_ctx* c, Tables* t) {
  std::memset(t, 0, sizeof(*t));
  int Q, D, N, EQ;
  double r;
  std::vector<int> e(3 * kQMax);
  std::vector<double> w(kQMax);
  host_lattice(c->lattice, &Q, &D, &N, &EQ, &r, e.data(), w.data());
  const double ub[3] = {c->wb.ux, 0.0, c->wb.uz};
  const double ut[3] = {c->wt.ux, 0.0, c->wt.uz};
  host_geq(c->lattice, ub, c->wb.T, t->gb);
  host_geq(c->lattice, ut, c->wt.T, t->gt);
  bool positive = true;
  for (int q = 0; q < Q; ++q) {
    const int ey = e[3 * q + 1];
    if (ey > 0) {
      t->Db += ey * t->gb[q];
      t->Wt += ey * w[q];  // rows ny-1 .. ny-e_y send q into the top ghosts
      positive = positive && t->gb[q] > 0;
    }
    if (ey < 0) {
      t->Dt += -ey * t->gt[q];
      t->Wb += -ey * w[q];
      positive = positive && t->gt[q] > 0;
    }
  }
  t->ab = c->alpha_b;
  t->at = c->alpha_t;
  return positive;
}

int finish_step_outputs(lbm_ctx* c) {
  return device_status(c, launch_reduce(make_reduce(c), c->stream));
}

int run_init(lbm_ctx* c, const double* fields_dev) {
  StepArgs a = make_args(c, nullptr, c->f[0], c->mom);
  c->cur = 0;
  int st = device_status(c, launch_init(c->lattice, c->prec, a, fields_dev, c->stream));
  if (st != LBM_OK) return st;
  c->steps = 0;
  c->window = 0;
  return finish_step_outputs(c);  // mass of f~(0); residual snapshot := f~(0)
}

int create_common(lbm_lattice lattice, lbm_grid grid, double tau, const lbm_wall* bottom,
                  const lbm_wall* top, lbm_precision prec, void* hip_stream, void* dev_buf,
                  size_t bytes, lbm_ctx** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  Layout lay;
  if (!layout(int(lattice), grid, int(prec), &lay)) return LBM_EINVAL;
  if (!(tau > 0) || !wall_ok(bottom) || !wall_ok(top)) return LBM_EINVAL;
  int Q, D, N, EQ;
  double r;
  host_lattice(int(lattice), &Q, &D, &N, &EQ, &r, nullptr, nullptr);
  const bool thermal = lattice == LBM_D3Q121;
  if (!thermal && (bottom->T != 1.0 || top->T != 1.0)) return LBM_EINVAL;
  if (D == 2 && (bottom->uz != 0.0 || top->uz != 0.0)) return LBM_EINVAL;
  if (dev_buf && (bytes < lay.total || (reinterpret_cast<uintptr_t>(dev_buf) & 255)))
    return LBM_ENOMEM;

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->lattice = int(lattice);
  c->prec = int(prec);
  c->nx = grid.nx;
  c->ny = grid.ny;
  c->Q = Q;
  c->N = N;
  c->D = D;
  c->tau = tau;
  c->r = r;
  c->wb = *bottom;
  c->wt = *top;
  c->alpha_b = c->alpha_t = 1.0;
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->plane = lay.plane;
  c->elem = elem_bytes(int(prec));
  c->uref = std::fmax(std::hypot(bottom->ux, bottom->uz), std::hypot(top->ux, top->uz));
  if (!(c->uref > 0)) c->uref = 1.0;

  Tables host_tab;
  if (!fill_tables(c, &host_tab)) {
    delete c;
    return LBM_ENEGATIVE;
  }
  if (dev_buf) {
    c->base = static_cast<char*>(dev_buf);
    c->owns = false;
  } else {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, lay.total);
    if (e != hipSuccess || !p) {
      g_last_hip = e;
      (void)hipGetLastError();
      delete c;
      return LBM_ENOMEM;
    }
    c->base = static_cast<char*>(p);
    c->owns = true;
  }
  c->bytes = lay.total;
  const size_t pop_bytes = align256(size_t(Q) * lay.plane * c->elem);
  c->f[0] = c->base + lay.pop;
  c->f[1] = c->base + lay.pop + pop_bytes;
  c->ratio = reinterpret_cast<double*>(c->base + lay.ratio);
  c->tab = reinterpret_cast<Tables*>(c->base + lay.tab);
  c->mom = reinterpret_cast<double*>(c->base + lay.mom);
  c->snap = reinterpret_cast<double*>(c->base + lay.snap);
  c->partial = reinterpret_cast<double*>(c->base + lay.partial);
  c->result = reinterpret_cast<double*>(c->base + lay.result);
  c->status = LBM_OK;

  int st = device_status(
      c, hipMemcpyAsync(c->tab, &host_tab, sizeof(Tables), hipMemcpyHostToDevice, c->stream));
  // zero both population buffers once, so that the padding at the end of
  // each plane (never written by the kernels) holds no stale bytes and a
  // checkpoint is a pure function of the state
  if (st == LBM_OK) st = device_status(c, hipMemsetAsync(c->f[0], 0, 2 * pop_bytes, c->stream));
  if (st == LBM_OK) st = device_status(c, hipStreamSynchronize(c->stream));
  if (st == LBM_OK) st = run_init(c, nullptr);
  if (st != LBM_OK) {
    lbm_destroy(c);
    return st;
  }
  *out = c;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_lattice_info(lbm_lattice lattice, int* Q, int* D, int* N, int* eq_order, double* r,
                     int* e, double* w) {
  int q, d, n, eq;
  double rr;
  if (host_lattice(int(lattice), &q, &d, &n, &eq, &rr, e, w) != 0) return LBM_EINVAL;
  if (Q) *Q = q;
  if (D) *D = d;
  if (N) *N = n;
  if (eq_order) *eq_order = eq;
  if (r) *r = rr;
  return LBM_OK;
}

double lbm_tau_from_kn(lbm_lattice lattice, int32_t ny, double kn) {
  int Q, D, N, EQ;
  double r;
  if (host_lattice(int(lattice), &Q, &D, &N, &EQ, &r, nullptr, nullptr) != 0 || ny < 1 ||
      !(kn > 0))
    return NAN;
  return std::sqrt(2.0 / M_PI) * kn * r * double(ny);
}

size_t lbm_required_bytes(lbm_lattice lattice, lbm_grid grid, lbm_precision prec) {
  Layout lay;
  if (!layout(int(lattice), grid, int(prec), &lay)) return 0;
  return lay.total;
}

int lbm_create(lbm_lattice lattice, lbm_grid grid, double tau, const lbm_wall* bottom,
               const lbm_wall* top, lbm_precision prec, void* hip_stream, lbm_ctx** out) {
  return create_common(lattice, grid, tau, bottom, top, prec, hip_stream, nullptr, 0, out);
}

int lbm_create_in(lbm_lattice lattice, lbm_grid grid, double tau, const lbm_wall* bottom,
                  const lbm_wall* top, lbm_precision prec, void* hip_stream, void* dev_buf,
                  size_t bytes, lbm_ctx** out) {
  if (!dev_buf) return LBM_EINVAL;
  return create_common(lattice, grid, tau, bottom, top, prec, hip_stream, dev_buf, bytes, out);
}

int lbm_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy,
             const double* T) {
  if (!c) return LBM_EINVAL;
  if (c->status != LBM_OK) return c->status;
  if (!rho && !ux && !uy && !T) return run_init(c, nullptr);
  const long long nodes = (long long)c->nx * c->ny;
  std::vector<double> h(size_t(5) * nodes);
  for (long long i = 0; i < nodes; ++i) {
    h[i] = rho ? rho[i] : 1.0;
    h[nodes + i] = ux ? ux[i] : 0.0;
    h[2 * nodes + i] = uy ? uy[i] : 0.0;
    h[3 * nodes + i] = 0.0;
    h[4 * nodes + i] = T ? T[i] : 1.0;
    if (!std::isfinite(h[i]) || !(h[i] > 0) || !std::isfinite(h[nodes + i]) ||
        !std::isfinite(h[2 * nodes + i]) || !std::isfinite(h[4 * nodes + i]) ||
        !(h[4 * nodes + i] > 0))
      return LBM_EINVAL;
  }
  // stage the fields in the output-field area; the init kernel reads a
  // node's inputs before it overwrites them with that node's outputs
  if (!hip_ok(hipMemcpyAsync(c->mom, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                     c->stream)))
    return fail(c, LBM_EDEVICE);
  int st = run_init(c, c->mom);
  if (st == LBM_OK && !hip_ok(hipStreamSynchronize(c->stream))) st = fail(c, LBM_EDEVICE);
  return st;
}

static constexpr int kTimingChunk = 1024;

static int collect_times(lbm_ctx* c, int used) {
  if (used == 0) return LBM_OK;
  if (!hip_ok(hipEventSynchronize(c->ev[3 * used - 1]))) return fail(c, LBM_EDEVICE);
  for (int k = 0; k < used; ++k) {
    float w = 0, u = 0;
    if (!hip_ok(hipEventElapsedTime(&w, c->ev[3 * k], c->ev[3 * k + 1])) ||
        !hip_ok(hipEventElapsedTime(&u, c->ev[3 * k + 1], c->ev[3 * k + 2])))
      return fail(c, LBM_EDEVICE);
    c->t_wall_ms += w;
    c->t_update_ms += u;
    c->n_wall += 1;
    c->n_update += 1;
  }
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c || n < 0) return LBM_EINVAL;
  if (c->status != LBM_OK) return c->status;
  if (n == 0) return LBM_OK;
  int used = 0;
  // rows that are a multiple of the block width take the row-tiled update
  // with the wall sums fused in; other shapes take wall_kernel + update
  const bool rows = c->nx % kBlock == 0;
  for (int64_t i = 0; i < n; ++i) {
    StepArgs a = make_args(c, c->f[c->cur], c->f[c->cur ^ 1], c->mom);
    a.step = uint32_t(c->steps + i + 1);
    if (c->timing && !hip_ok(hipEventRecord(c->ev[3 * used], c->stream)))
      return fail(c, LBM_EDEVICE);
    int st = rows ? LBM_OK : device_status(c, launch_wall(c->lattice, c->prec, a, c->stream));
    if (c->timing && !hip_ok(hipEventRecord(c->ev[3 * used + 1], c->stream)))
      return fail(c, LBM_EDEVICE);
    if (st == LBM_OK)
      st = device_status(c, rows ? launch_step_rows(c->lattice, c->prec, a, i == n - 1, c->stream)
                                 : launch_step(c->lattice, c->prec, a, i == n - 1, c->stream));
    if (c->timing && !hip_ok(hipEventRecord(c->ev[3 * used + 2], c->stream)))
      return fail(c, LBM_EDEVICE);
    if (st != LBM_OK) return st;
    c->cur ^= 1;
    if (c->timing && ++used == kTimingChunk) {
      st = collect_times(c, used);
      if (st != LBM_OK) return st;
      used = 0;
    }
  }
  if (c->timing) {
    const int st = collect_times(c, used);
    if (st != LBM_OK) return st;
  }
  c->steps += n;
  c->window = n;
  return finish_step_outputs(c);
}

int lbm_field(lbm_ctx* c, lbm_field_id id, double* host_out) {
  if (!c || !host_out || int(id) < 0 || int(id) >= kFields) return LBM_EINVAL;
  if (c->status != LBM_OK) return c->status;
  const long long nodes = (long long)c->nx * c->ny;
  if (!hip_ok(hipMemcpyAsync(host_out, c->mom + (long long)id * nodes, sizeof(double) * nodes,
                     hipMemcpyDeviceToHost, c->stream)) ||
      !hip_ok(hipStreamSynchronize(c->stream)))
    return fail(c, LBM_EDEVICE);
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* T, double* sxy,
                double* qx, double* qy) {
  if (!c) return LBM_EINVAL;
  double* outs[7] = {rho, ux, uy, T, sxy, qx, qy};
  const lbm_field_id ids[7] = {LBM_RHO, LBM_UX, LBM_UY, LBM_T, LBM_SXY, LBM_QX, LBM_QY};
  for (int k = 0; k < 7; ++k) {
    if (!outs[k]) continue;
    const int st = lbm_field(c, ids[k], outs[k]);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

static int read_result(lbm_ctx* c, double* res) {
  if (c->status != LBM_OK) return c->status;
  if (!hip_ok(hipMemcpyAsync(res, c->result, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream)) ||
      !hip_ok(hipStreamSynchronize(c->stream)))
    return fail(c, LBM_EDEVICE);
  if (res[3] != 0.0) return fail(c, LBM_ENONFINITE);
  return LBM_OK;
}

int lbm_residual(lbm_ctx* c, double* r) {
  if (!c || !r) return LBM_EINVAL;
  double res[4];
  const int st = read_result(c, res);
  if (st != LBM_OK) return st;
  if (c->window == 0) {
    *r = INFINITY;
    return LBM_OK;
  }
  const double n = double(c->nx) * c->ny;
  const double ru = std::sqrt(res[1]) / (double(c->window) * c->uref * std::sqrt(n));
  const double rt = std::sqrt(res[2]) / (double(c->window) * std::sqrt(n));
  *r = std::fmax(ru, rt);
  return LBM_OK;
}

int lbm_mass(lbm_ctx* c, double* m) {
  if (!c || !m) return LBM_EINVAL;
  double res[4];
  const int st = read_result(c, res);
  if (st != LBM_OK) return st;
  *m = res[0];
  return LBM_OK;
}

int lbm_steps_done(lbm_ctx* c, int64_t* steps) {
  if (!c || !steps) return LBM_EINVAL;
  *steps = c->steps;
  return LBM_OK;
}

// Checkpoint layout: [int64 steps][int64 window][populations f*][fields]
// [residual snapshot]; everything needed to continue bit-identically.
size_t lbm_state_bytes(lbm_ctx* c) {
  if (!c) return 0;
  const size_t nodes = size_t(c->nx) * c->ny;
  return 16 + size_t(c->Q) * c->plane * c->elem + sizeof(double) * (kFields + 4) * nodes;
}

int lbm_save(lbm_ctx* c, void* host, size_t bytes) {
  if (!c || !host || bytes < lbm_state_bytes(c)) return LBM_EINVAL;
  if (c->status != LBM_OK) return c->status;
  char* p = static_cast<char*>(host);
  std::memcpy(p, &c->steps, 8);
  std::memcpy(p + 8, &c->window, 8);
  const size_t pop = size_t(c->Q) * c->plane * c->elem;
  const size_t nodes = size_t(c->nx) * c->ny;
  if (!hip_ok(hipMemcpyAsync(p + 16, c->f[c->cur], pop, hipMemcpyDeviceToHost, c->stream)) ||
      !hip_ok(hipMemcpyAsync(p + 16 + pop, c->mom, sizeof(double) * kFields * nodes,
                     hipMemcpyDeviceToHost, c->stream)) ||
      !hip_ok(hipMemcpyAsync(p + 16 + pop + sizeof(double) * kFields * nodes, c->snap,
                     sizeof(double) * 4 * nodes, hipMemcpyDeviceToHost, c->stream)) ||
      !hip_ok(hipStreamSynchronize(c->stream)))
    return fail(c, LBM_EDEVICE);
  return LBM_OK;
}

int lbm_load(lbm_ctx* c, const void* host, size_t bytes) {
  if (!c || !host || bytes < lbm_state_bytes(c)) return LBM_EINVAL;
  if (c->status != LBM_OK) return c->status;
  const char* p = static_cast<const char*>(host);
  int64_t steps, window;
  std::memcpy(&steps, p, 8);
  std::memcpy(&window, p + 8, 8);
  const size_t pop = size_t(c->Q) * c->plane * c->elem;
  const size_t nodes = size_t(c->nx) * c->ny;
  c->cur = 0;
  if (!hip_ok(hipMemcpyAsync(c->f[0], p + 16, pop, hipMemcpyHostToDevice, c->stream)) ||
      !hip_ok(hipMemcpyAsync(c->mom, p + 16 + pop, sizeof(double) * kFields * nodes,
                     hipMemcpyHostToDevice, c->stream)) ||
      !hip_ok(hipMemcpyAsync(c->snap, p + 16 + pop + sizeof(double) * kFields * nodes,
                     sizeof(double) * 4 * nodes, hipMemcpyHostToDevice, c->stream)) ||
      !hip_ok(hipStreamSynchronize(c->stream)))
    return fail(c, LBM_EDEVICE);
  c->steps = steps;
  c->window = 0;
  (void)window;
  return LBM_OK;
}

// Device scratch of lbm_batch_step (case descriptors + outputs), grown on
// demand and kept for the life of the process; guarded by a mutex.
static std::mutex g_batch_mu;
static char* g_batch_dev = nullptr;
static size_t g_batch_cap = 0;

int lbm_batch_run(lbm_ctx* const* ctxs, int n_ctx, const int64_t* budgets, int64_t window,
                  double tol, double* residuals_out, int64_t* steps_out, int* state_out) {
  if (!ctxs || n_ctx <= 0 || !budgets || window <= 0 || window > INT_MAX) return LBM_EINVAL;
  if (!ctxs[0]) return LBM_EINVAL;
  const hipStream_t stream = ctxs[0]->stream;
  for (int i = 0; i < n_ctx; ++i) {
    lbm_ctx* c = ctxs[i];
    if (!c || c->stream != stream) return LBM_EINVAL;
    if (c->status != LBM_OK) return c->status;
    if (c->nx > kBatchMaxNx) return LBM_EUNSUPPORTED;
    if (budgets[i] < window || budgets[i] > INT_MAX) return LBM_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return LBM_EINVAL;  // one context twice would race
  }
  // group the cases by storage format, force variant and, for the formats
  // whose large set has its own kernel instance, set class: one launch per
  // group present (group = format + kPrecCount * (has_force + 2 * large))
  constexpr int kGroups = 4 * kPrecCount;
  std::vector<CaseDesc> desc(n_ctx);
  std::vector<int> pos(n_ctx), fmt(n_ctx);
  int start[kGroups + 1] = {};
  for (int i = 0; i < n_ctx; ++i) {
    const lbm_ctx* c = ctxs[i];
    const bool force = c->acc[0] != 0.0 || c->acc[1] != 0.0 || c->acc[2] != 0.0;
    const bool large = batch_splits_sets(c->prec) && c->lattice == LBM_D3Q121;
    fmt[i] = c->prec + kPrecCount * ((force ? 1 : 0) + (large ? 2 : 0));
  }
  if (!plan_groups(fmt.data(), n_ctx, kGroups, start, pos.data())) return LBM_EINVAL;
  for (int i = 0; i < n_ctx; ++i) {
    lbm_ctx* c = ctxs[i];
    CaseDesc& d = desc[pos[i]];
    d.a = make_args(c, nullptr, nullptr, c->mom);
    d.f[0] = c->f[0];
    d.f[1] = c->f[1];
    d.cur = c->cur;
    d.snap = c->snap;
    d.result = c->result;
    d.uref = c->uref;
    d.tol = tol;
    d.lattice = c->lattice;
    d.window = int(window);
    d.budget = int(budgets[i] / window * window);
  }
  const size_t desc_bytes = align256(sizeof(CaseDesc) * size_t(n_ctx));
  const size_t need = desc_bytes + sizeof(CaseOut) * size_t(n_ctx);
  std::vector<CaseOut> out(n_ctx);
  std::lock_guard<std::mutex> lock(g_batch_mu);
  if (need > g_batch_cap) {
    if (g_batch_dev) (void)hipFree(g_batch_dev);
    g_batch_dev = nullptr;
    g_batch_cap = 0;
    void* p = nullptr;
    if (!hip_ok(hipMalloc(&p, need))) return LBM_ENOMEM;
    g_batch_dev = static_cast<char*>(p);
    g_batch_cap = need;
  }
  CaseDesc* ddesc = reinterpret_cast<CaseDesc*>(g_batch_dev);
  CaseOut* dout = reinterpret_cast<CaseOut*>(g_batch_dev + desc_bytes);
  if (!hip_ok(hipMemcpyAsync(ddesc, desc.data(), sizeof(CaseDesc) * size_t(n_ctx),
                             hipMemcpyHostToDevice, stream)))
    return LBM_EDEVICE;
  for (int p = 0; p < kGroups; ++p) {
    const int cnt = start[p + 1] - start[p];
    if (cnt == 0) continue;
    if (cnt < 0 || start[p] + cnt > n_ctx) return LBM_EINVAL;  // grouping is inconsistent
    const int v = p / kPrecCount;
    if (!hip_ok(launch_batch(p % kPrecCount, (v & 1) != 0, (v & 2) != 0, ddesc + start[p], cnt,
                             dout + start[p], stream)))
      return LBM_EDEVICE;
  }
  if (!hip_ok(hipMemcpyAsync(out.data(), dout, sizeof(CaseOut) * out.size(),
                             hipMemcpyDeviceToHost, stream)) ||
      !hip_ok(hipStreamSynchronize(stream)))
    return LBM_EDEVICE;
  for (int i = 0; i < n_ctx; ++i) {
    lbm_ctx* c = ctxs[i];
    const CaseOut& o = out[pos[i]];
    const int64_t done = int64_t(o.steps);
    c->cur ^= int(done & 1);
    c->steps += done;
    c->window = window;
    if (residuals_out) residuals_out[i] = o.residual;
    if (steps_out) steps_out[i] = done;
    if (state_out) state_out[i] = int(o.state);
  }
  return LBM_OK;
}

int lbm_batch_step(lbm_ctx* const* ctxs, int n_ctx, int64_t k_steps, double* residuals_out) {
  if (!ctxs || n_ctx <= 0 || k_steps <= 0) return LBM_EINVAL;
  std::vector<int64_t> budgets(n_ctx, k_steps);
  return lbm_batch_run(ctxs, n_ctx, budgets.data(), k_steps, -1.0, residuals_out, nullptr,
                       nullptr);
}

int lbm_set_accommodation(lbm_ctx* c, double alpha_bottom, double alpha_top) {
  if (!c || !(alpha_bottom >= 0.0 && alpha_bottom <= 1.0) ||
      !(alpha_top >= 0.0 && alpha_top <= 1.0))
    return LBM_EINVAL;
  c->alpha_b = alpha_bottom;
  c->alpha_t = alpha_top;
  Tables host_tab;
  (void)fill_tables(c, &host_tab);  // walls unchanged: already checked at creation
  int st = device_status(
      c, hipMemcpyAsync(c->tab, &host_tab, sizeof(Tables), hipMemcpyHostToDevice, c->stream));
  if (st == LBM_OK) st = device_status(c, hipStreamSynchronize(c->stream));
  return st;
}

int lbm_set_viscosity_law(lbm_ctx* c, int enable, double exponent) {
  if (!c) return LBM_EINVAL;
  if (enable) {
    if (c->lattice != LBM_D3Q121 || !std::isfinite(c->tau) || !std::isfinite(exponent) ||
        std::fabs(exponent) > 4.0)
      return LBM_EINVAL;
    c->law = 1;
    c->vexp = exponent;
  } else {
    c->law = 0;
    c->vexp = 0.0;
  }
  return LBM_OK;
}

int lbm_set_body_force(lbm_ctx* c, double ax, double ay, double az) {
  if (!c) return LBM_EINVAL;
  const double v[3] = {ax, ay, az};
  for (double x : v)
    if (!std::isfinite(x) || std::fabs(x) > 1.0) return LBM_EINVAL;
  if (c->D == 2 && az != 0.0) return LBM_EINVAL;
  for (int i = 0; i < 3; ++i) c->acc[i] = v[i];
  return LBM_OK;
}

int lbm_set_timing(lbm_ctx* c, int enable) {
  if (!c) return LBM_EINVAL;
  if (enable && c->ev.empty()) {
    c->ev.resize(3 * kTimingChunk, nullptr);
    for (auto& e : c->ev)
      if (!hip_ok(hipEventCreate(&e))) return fail(c, LBM_EDEVICE);
  }
  c->timing = enable != 0;
  c->t_update_ms = c->t_wall_ms = 0.0;
  c->n_update = c->n_wall = 0;
  return LBM_OK;
}

int lbm_kernel_time(lbm_ctx* c, double* update_ms, int64_t* update_launches, double* wall_ms,
                    int64_t* wall_launches) {
  if (!c) return LBM_EINVAL;
  if (update_ms) *update_ms = c->t_update_ms;
  if (update_launches) *update_launches = c->n_update;
  if (wall_ms) *wall_ms = c->t_wall_ms;
  if (wall_launches) *wall_launches = c->n_wall;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->owns && c->base) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->base);
  }
  delete c;
}

const char* lbm_last_device_error(void) {
  if (g_last_hip == hipSuccess) return "none";
  std::snprintf(g_last_msg, sizeof(g_last_msg), "%s: %s", hipGetErrorName(g_last_hip),
                hipGetErrorString(g_last_hip));
  return g_last_msg;
}

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of device memory or buffer too small";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite value in the fields";
    case LBM_ENEGATIVE: return "wall Maxwellian not positive for an outgoing velocity";
    case LBM_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
