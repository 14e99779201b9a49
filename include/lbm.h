/*
 * lbm.h - C ABI of the MI355X (gfx950) implementation of the high-order
 * multi-speed lattice Boltzmann BGK scheme with the kinetic diffuse-reflection
 * wall of Meng & Zhang, "Kinetic diffuse boundary condition for high-order
 * lattice Boltzmann model with streaming-collision mechanism"
 * (arXiv:1209.5201).
 *
 * Problem (Sec. IV): a channel of nx periodic columns by ny fluid rows between
 * two planar walls.  The bottom wall lies half a spacing below row 0 (normal
 * +y), the top wall half a spacing above row ny-1 (normal -y) (Sec. III).
 * Walls move tangentially with velocity (ux, 0, uz) at temperature T.  Three
 * velocity sets (Sec. IV): D2Q16, D2Q17 (isothermal) and D3Q121 (thermal; the
 * z direction is a single periodic plane, so c_z enters the equilibrium and
 * the moments but not the streaming).
 *
 * One step is Eq. (eq:scheme): BGK relaxation of f~ (the variable of Sec. II)
 * towards the truncated Maxwellian of Eq. (eq:feq) with rate 1/(tau + 1/2),
 * streaming along the integer velocities, and, for populations that cross a
 * wall, the diffuse re-emission of Eq. (eq:dkboundary): all mass arriving in
 * the N ghost layers of a ghost column is pooled and sent back along every
 * outgoing velocity of every layer in proportion to the wall Maxwellian.
 *
 * Conventions shared by every call:
 *  - Every call returns an lbm_status (LBM_OK = 0, negative on error) unless
 *    stated otherwise; the library never aborts and never prints.
 *  - Host arrays are caller-owned.  Fields are nx*ny doubles, row-major with
 *    x fastest (index y*nx + x).
 *  - Device work is queued on the context's HIP stream.  Calls that return
 *    data to the host synchronize that stream; lbm_step does not.
 *  - A context is not thread-safe; use one context per host thread/stream.
 *  - A device error makes the context's status sticky: later calls return it.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Velocity sets (Sec. IV).  The paper omits the tables; the library uses
 * D2Q17 on the shells (0,0),(1,0),(1,1),(2,2),(3,0) (degree 7), D3Q121 on the
 * shells (000),(100),(111),(210),(220),(222),(300),(311),(320),(333)
 * (degree 9), and D2Q16 = tensor product of {+-1: 9/20, +-3: 1/20} with
 * r = sqrt(5)/3 and the 2nd-order equilibrium (a labelled construction). */
typedef enum { LBM_D2Q16 = 0, LBM_D2Q17 = 1, LBM_D3Q121 = 2 } lbm_lattice;

/* Storage / arithmetic of the populations.  FP64: everything in double.
 * FP32: populations, moments, f^eq and relaxation in float.
 * BF16_DEV / FP16_DEV: populations stored as 16-bit (f - w_a) * S with a
 * per-format power-of-two S, decoded to float for all arithmetic.
 * FP32_STORE: populations stored as float deviations f - w_a, rounded
 * stochastically (a counter-based hash of node, velocity and step picks one
 * of the two neighbouring floats, so results are reproducible); every
 * arithmetic step in double.  The FP32 traffic, with single precision only
 * in the stored values.
 * In every precision the wall sums, the wall ratio M/D, the output fields and
 * the mass / residual reductions are double. */
typedef enum {
  LBM_FP64 = 0,
  LBM_FP32 = 1,
  LBM_BF16_DEV = 2,
  LBM_FP16_DEV = 3,
  LBM_FP32_STORE = 4
} lbm_precision;

typedef struct { int32_t nx, ny; } lbm_grid;

/* Wall velocity (tangential only: the normal component is zero by
 * construction) and temperature, non-dimensional (Sec. II). */
typedef struct { double ux, uz, T; } lbm_wall;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,        /* invalid argument */
    LBM_ENOMEM = -2,        /* device allocation failed / buffer too small */
    LBM_EDEVICE = -3,       /* HIP runtime error */
    LBM_ENONFINITE = -4,    /* a NaN/Inf appeared in the moments */
    LBM_ENEGATIVE = -5,     /* negative wall Maxwellian (positivity lost) */
    LBM_EUNSUPPORTED = -6   /* valid request this library does not provide */
} lbm_status;

/* Output fields of lbm_field (Eq. (eq:summac)): density, velocity,
 * temperature, shear stress sigma_xy and heat flux q.  Stress and heat flux
 * are those of f, obtained from f~ by the conversion of Sec. II:
 * X[f] = X[f^eq] + tau/(tau+1/2) (X[f~] - X[f^eq]).  Isothermal lattices
 * report T = 1. */
typedef enum {
    LBM_RHO = 0, LBM_UX = 1, LBM_UY = 2, LBM_UZ = 3, LBM_T = 4,
    LBM_SXY = 5, LBM_QX = 6, LBM_QY = 7, LBM_QZ = 8
} lbm_field_id;
#define LBM_NUM_FIELDS 9

/* Describe a velocity set (Sec. II, the set xi = {c_a, w_a}).  Outputs may
 * be NULL.  e receives Q rows of 3 integers (c_a = r e_a), w receives Q
 * weights, N the number of ghost layers per wall (largest |e_y|, Sec. III),
 * eq_order the truncation order of Eq. (eq:feq).  Host-only; no GPU needed. */
int lbm_lattice_info(lbm_lattice lattice, int *Q, int *D, int *N, int *eq_order,
                     double *r, int *e, double *w);

/* Relaxation time in time steps for a channel of ny rows at Knudsen number
 * kn: sqrt(2/pi) * kn * r * ny (Sec. II tau = mu/p in reference units with
 * the Kn definition of Sec. IV; dx = 1/ny, dt = dx/r).  Returns NaN on
 * invalid input.  Host-only. */
double lbm_tau_from_kn(lbm_lattice lattice, int32_t ny, double kn);

/* Bytes of device memory a context needs (populations x2, wall ratios,
 * tables, output fields, residual snapshot, reduction scratch).  0 on invalid
 * input.  Host-only; use it to admit work by HBM footprint. */
size_t lbm_required_bytes(lbm_lattice lattice, lbm_grid grid, lbm_precision prec);

/* Create a context, allocate its device memory (owned; freed by
 * lbm_destroy) and initialise it to the rest state rho = 1, u = 0, T = 1.
 * tau > 0 is the relaxation time in time steps (+INFINITY: no collisions).
 * Requires nx >= 1, ny >= 2N, finite walls with T > 0, T = 1 on isothermal
 * lattices, and g^eq(u_w, T_w) > 0 for every velocity leaving each wall
 * (positivity of the diffuse wall, Sec. I) else LBM_ENEGATIVE.
 * hip_stream: a hipStream_t, or NULL for the null stream. */
int lbm_create(lbm_lattice lattice, lbm_grid grid, double tau,
               const lbm_wall *bottom, const lbm_wall *top, lbm_precision prec,
               void *hip_stream, lbm_ctx **out);

/* Same as lbm_create, but all device memory is carved from the caller's
 * buffer dev_buf of `bytes` >= lbm_required_bytes(...) bytes (256-byte
 * aligned).  The caller keeps ownership and must keep it alive until
 * lbm_destroy. */
int lbm_create_in(lbm_lattice lattice, lbm_grid grid, double tau,
                  const lbm_wall *bottom, const lbm_wall *top, lbm_precision prec,
                  void *hip_stream, void *dev_buf, size_t bytes, lbm_ctx **out);

/* Set f~ = f^eq(rho, u, T) at every node from host fields (NULL: rho = 1,
 * u = 0, T = 1); resets the step count and the residual window.  uz = 0. */
int lbm_init(lbm_ctx *ctx, const double *rho, const double *ux,
             const double *uy, const double *T);

/* Advance n >= 0 steps (asynchronous).  After the last step the output
 * fields, the total mass and the residual (below) are refreshed. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* Copy one output field at the current time to host (nx*ny doubles). */
int lbm_field(lbm_ctx *ctx, lbm_field_id id, double *host_out);

/* Convenience: several fields at once; NULL pointers are skipped. */
int lbm_moments(lbm_ctx *ctx, double *rho, double *ux, double *uy, double *T,
                double *sxy, double *qx, double *qy);

/* Convergence rate over the last lbm_step call of K steps:
 *   max(|u - u_prev|_2 / (K U_ref sqrt(n)), |T - T_prev|_2 / (K sqrt(n)))
 * with n = nx*ny and U_ref the largest wall speed (1 if both are at rest).
 * The paper gives no criterion; this per-step rate is the reading used.
 * Returns LBM_ENONFINITE if the fields contain NaN/Inf. */
int lbm_residual(lbm_ctx *ctx, double *r);

/* Total mass sum f~ over the fluid (FP64 reduction, fixed order). */
int lbm_mass(lbm_ctx *ctx, double *m);

/* Number of steps taken since creation / lbm_init. */
int lbm_steps_done(lbm_ctx *ctx, int64_t *steps);

/* Checkpoint: the current populations and step count.  lbm_state_bytes gives
 * the size; save/load copy to/from caller host memory of that size.  A run
 * resumed from a saved state continues bit-identically. */
size_t lbm_state_bytes(lbm_ctx *ctx);
int lbm_save(lbm_ctx *ctx, void *host, size_t bytes);
int lbm_load(lbm_ctx *ctx, const void *host, size_t bytes);

/* Serving: advance several contexts by k_steps in one persistent launch per
 * storage format present (one workgroup per context; the whole k-step
 * window runs inside the launch), then refresh each context's fields, mass
 * and residual exactly as lbm_step(ctx, k_steps) would.  A context's result
 * does not depend on which other contexts share the batch.  All contexts
 * must use the same HIP stream and device and appear once; nx <= 64
 * (LBM_EUNSUPPORTED otherwise: use lbm_step for wide grids).
 * residuals_out (may be NULL): n_ctx residuals as lbm_residual reports them,
 * NaN for a context whose fields became non-finite.  Synchronizes the stream.
 * Not thread-safe against concurrent lbm_batch_step calls on other threads
 * for the same contexts. */
int lbm_batch_step(lbm_ctx *const *ctxs, int n_ctx, int64_t k_steps, double *residuals_out);

/* Serving with convergence inside the launch: context i advances in windows
 * of `window` steps, at most budgets[i] steps (rounded down to a multiple of
 * the window; >= window), and stops after the first window whose residual
 * (as lbm_residual defines it, over that window) is below tol.  A context's
 * stopping step depends only on its own data, not on the batch or on its
 * budget.  Outputs (each may be NULL): the residual of each context's last
 * window (NaN: non-finite), the steps it advanced, and its state (1
 * converged, 0 budget used up, -1 non-finite fields).  Same conventions as
 * lbm_batch_step. */
int lbm_batch_run(lbm_ctx *const *ctxs, int n_ctx, const int64_t *budgets, int64_t window,
                  double tol, double *residuals_out, int64_t *steps_out, int *state_out);

/* Accommodation of each wall: the wall scatters with Maxwell's kernel
 * R = alpha R_D + (1 - alpha) R_S, built on the generic scattering kernel
 * of Sec. III: the fraction alpha of the incoming mass is re-emitted
 * diffusely (R_D, Eq. (eq:dkboundary)), the rest is reflected specularly
 * (normal velocity reversed, from the mirror-image ghost cell).  alpha = 1
 * (the default after lbm_create) is the paper's wall, alpha = 0 a specular
 * wall.  Applies to every later step of the context.  Requires
 * 0 <= alpha <= 1 for both walls, else LBM_EINVAL and nothing changes.
 * Synchronizes the context stream. */
int lbm_set_accommodation(lbm_ctx *ctx, double alpha_bottom, double alpha_top);

/* Local relaxation time for thermal problems (end of Sec. II: tau may
 * follow the local gas temperature).  With enable != 0 every node relaxes
 * with tau_node = tau * T^(w - 1) / rho, the non-dimensional tau = mu / p
 * of Sec. II for p = rho T and a power-law viscosity mu = T^w (w = exponent;
 * 1/2 hard spheres, 1 Maxwell molecules), tau being the value given to
 * lbm_create (its value at rho = T = 1); the stress and heat flux
 * conversion uses each node's tau.  enable = 0 restores constant tau (the
 * default, the paper's runs).  Requires the thermal set (LBM_D3Q121), a
 * finite tau and |w| <= 4, else LBM_EINVAL and nothing changes.  Host-only.
 * The state after lbm_step holds the populations after the collision of
 * the last step, so the law governs the collisions of later steps. */
int lbm_set_viscosity_law(lbm_ctx *ctx, int enable, double exponent);

/* Body force: a constant acceleration (ax, ay, az) of every node, in
 * velocity units (those of the wall velocities) gained per time step; for a
 * force-driven (Poiseuille) channel take ax != 0 with walls at rest.  Not in
 * the paper: its Boltzmann force term -a . grad_c f is projected on the
 * Hermite polynomials up to the equilibrium's order, which gives
 * F = a . d f^eq / du, and the change of variable of Sec. II applied to the
 * collision and this term gives
 *   f*~ = f~ - (f~ - f^eq)/(tau + 1/2) + tau/(tau + 1/2) F,
 * f^eq and F taken at the moments of f: u = u[f~] + a/2 and
 * T = T[f~] + |a|^2/(4D) (these are the reported u and T).  (0, 0, 0), the
 * default, is the force-free scheme.  Requires finite |a_i| <= 1 and
 * az = 0 on the 2-D sets, else LBM_EINVAL and nothing changes.  Host-only;
 * governs the collisions of later steps. */
int lbm_set_body_force(lbm_ctx *ctx, double ax, double ay, double az);

/* Kernel timing with HIP events (profiling aid).  While enabled, lbm_step
 * brackets every launch of the wall-sum kernel and of the fused update kernel
 * with events on the context stream and accumulates their durations; the
 * call then synchronizes the stream every 1024 steps.  Enabling resets the
 * accumulators. */
int lbm_set_timing(lbm_ctx *ctx, int enable);
int lbm_kernel_time(lbm_ctx *ctx, double *update_ms, int64_t *update_launches,
                    double *wall_ms, int64_t *wall_launches);

/* Release the context (and its device memory if it owns it). */
void lbm_destroy(lbm_ctx *ctx);

/* Static string for a status code. */
const char *lbm_strerror(int status);

/* Name and description of the last HIP runtime error the library saw on the
 * calling thread ("none" if there was none); valid until the next call on
 * this thread.  Explains an LBM_EDEVICE / LBM_ENOMEM status. */
const char *lbm_last_device_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
