/*
 * FP64 reference implementation of the high-order lattice Boltzmann BGK
 * update with the kinetic diffuse-reflection wall of Meng & Zhang
 * (arXiv:1209.5201).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle: a plain, slow,
 * literal rendering of the paper's equations, used to check the product
 * path.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg may load it.  It shares no code, header or table with the product.
 *
 * Geometry (the paper's Couette set-up, Sec. IV, with the wall placed half a
 * grid spacing outside the first fluid row, Sec. III):
 *   - nx periodic columns x, ny fluid rows y = 0..ny-1;
 *   - bottom wall below row 0, normal +y; ghost layer l (l = 0..N-1) is the
 *     row -(l+1);
 *   - top wall above row ny-1, normal -y; ghost layer l is the row ny+l;
 *   - z is a single periodic plane, so z-streaming is the identity while c_z
 *     still enters the equilibrium and the moments (3-D velocity sets).
 *
 * State: f~ of Sec. II (the variable that removes the implicitness of the
 * trapezoidal scheme), stored per node as Q consecutive doubles,
 * f[(y*nx + x)*Q + a].
 *
 * One step (Eq. (eq:scheme) with Sec. III):
 *   1. moments of f~ (Eq. (eq:summac)), f^eq from Eq. (eq:feq);
 *   2. post-collision f* = f~ - (f~ - f^eq)/(tau + 1/2)   (dt = 1);
 *   3. stream every f* along its integer velocity; what leaves the fluid
 *      lands in an explicit ghost array as the incoming f^I (Sec. III);
 *   4. the wall turns incoming into outgoing populations through the
 *      scattering kernel R of Sec. III, taken of Maxwell's form
 *      R = alpha R_D + (1 - alpha) R_S per wall:
 *        - diffuse part R_D (the paper's wall, alpha = 1): per ghost column,
 *          pool all incoming mass over all layers and re-emit the fraction
 *          alpha of it along every outgoing velocity of every layer in
 *          proportion to the wall Maxwellian, Eq. (eq:dkboundary);
 *        - specular part R_S: the fraction 1 - alpha of each incoming
 *          population is sent back with its normal velocity reversed, from
 *          the ghost cell where a mirror at the wall plane would put it;
 *   5. the outgoing f^O stream into the fluid in the same step.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int Q, D, eq_order, thermal;
    const int *e;      /* Q rows of (ex, ey, ez) */
    const double *w;   /* Q weights */
    double r;          /* c_a = r * e_a */
} olat;

/* Eq. (eq:feq): g^eq_a(u, T), truncated after the requested order.
 * The terms are grouped exactly as printed in the paper. */
static double geq(const olat *L, int a, const double u[3], double T)
{
    double c[3], cu = 0.0, uu = 0.0, cc = 0.0;
    double D = (double)L->D;
    double th = T - 1.0;
    double g;
    int i;
    for (i = 0; i < 3; ++i) {
        c[i] = L->r * (double)L->e[3 * a + i];
        cu += c[i] * u[i];
        uu += u[i] * u[i];
        cc += c[i] * c[i];
    }
    g = 1.0 + cu;
    if (L->eq_order >= 2)
        g += 0.5 * (cu * cu - uu + th * (cc - D));
    if (L->eq_order >= 3)
        g += cu / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2.0));
    if (L->eq_order >= 4) {
        g += (cu * cu * cu * cu - 6.0 * cu * cu * uu + 3.0 * uu * uu) / 24.0;
        g += th / 4.0 * ((cc - D - 2.0) * (cu * cu - uu) - 2.0 * cu * cu);
        g += th * th / 8.0 * (cc * cc - 2.0 * (D + 2.0) * cc + D * (D + 2.0));
    }
    return L->w[a] * g;
}

/* Body force (not in the paper; a constant acceleration a of every node).
 * The force term of the Boltzmann equation, -a . grad_c f, projected on the
 * Hermite polynomials up to the equilibrium's order N equals the
 * directional derivative of the truncated equilibrium in u at fixed rho and
 * T: F_a = a . d f^eq_a / du.  Here the printed terms of Eq. (eq:feq) are
 * differentiated one by one (d(c.u) = a.c, d(u.u) = 2 a.u); unit density. */
static double force_term(const olat *L, int a, const double u[3], double T,
                         const double acc[3])
{
    double c[3], cu = 0.0, uu = 0.0, cc = 0.0, ca = 0.0, au = 0.0;
    double D = (double)L->D;
    double th = T - 1.0;
    double d;
    int i;
    for (i = 0; i < 3; ++i) {
        c[i] = L->r * (double)L->e[3 * a + i];
        cu += c[i] * u[i];
        uu += u[i] * u[i];
        cc += c[i] * c[i];
        ca += c[i] * acc[i];
        au += acc[i] * u[i];
    }
    d = ca;
    if (L->eq_order >= 2)
        d += 0.5 * (2.0 * cu * ca - 2.0 * au);
    if (L->eq_order >= 3)
        d += ca / 6.0 * (cu * cu - 3.0 * uu + 3.0 * th * (cc - D - 2.0)) +
             cu / 6.0 * (2.0 * cu * ca - 6.0 * au);
    if (L->eq_order >= 4) {
        d += (4.0 * cu * cu * cu * ca - 6.0 * (2.0 * cu * ca * uu + cu * cu * 2.0 * au) +
              3.0 * 2.0 * uu * 2.0 * au) / 24.0;
        d += th / 4.0 * ((cc - D - 2.0) * (2.0 * cu * ca - 2.0 * au) - 4.0 * cu * ca);
    }
    return L->w[a] * d;
}

/* Eq. (eq:summac): density, velocity and temperature of one node.
 * Isothermal lattices use T = 1 (Sec. II, after Eq. (eq:feq)). */
static void node_moments(const olat *L, const double *f, double *rho,
                         double u[3], double *T)
{
    double m0 = 0.0, m1[3] = {0.0, 0.0, 0.0};
    int a, i;
    for (a = 0; a < L->Q; ++a) {
        m0 += f[a];
        for (i = 0; i < 3; ++i)
            m1[i] += f[a] * L->r * (double)L->e[3 * a + i];
    }
    *rho = m0;
    for (i = 0; i < 3; ++i)
        u[i] = m1[i] / m0;
    if (L->thermal) {
        double e2 = 0.0;
        for (a = 0; a < L->Q; ++a) {
            double C2 = 0.0;
            for (i = 0; i < 3; ++i) {
                double Ci = L->r * (double)L->e[3 * a + i] - u[i];
                C2 += Ci * Ci;
            }
            e2 += f[a] * C2;
        }
        *T = e2 / (m0 * (double)L->D);
    } else {
        *T = 1.0;
    }
}

/* Moments of the physical f from the stored f~ (Sec. II change of
 * variable, extended by the force: f = f~ + J/2 with J = -(f - f^eq)/tau + F,
 * whose mass and energy moments over J's collision part vanish):
 *   rho = sum f~,  rho u = sum f~ c + rho a / 2,
 *   rho D T = sum f~ |c|^2 + rho a.u - rho u^2, i.e. T = T[f~] + a^2/(4D).
 * acc == NULL: no force, the moments of f~ itself. */
static void phys_moments(const olat *L, const double *f, const double *acc,
                         double *rho, double u[3], double *T)
{
    int i;
    node_moments(L, f, rho, u, T);
    if (!acc)
        return;
    for (i = 0; i < 3; ++i)
        u[i] += 0.5 * acc[i];
    if (L->thermal)
        *T += (acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2]) /
              (4.0 * (double)L->D);
}

static int max_ey(const olat *L)
{
    int a, n = 0;
    for (a = 0; a < L->Q; ++a)
        if (abs(L->e[3 * a + 1]) > n)
            n = abs(L->e[3 * a + 1]);
    return n;
}

static int wrap(int x, int nx)
{
    int m = x % nx;
    return m < 0 ? m + nx : m;
}

/* Relaxation time of one node.  Constant tau (law == NULL) or, for thermal
 * problems (end of Sec. II: tau may follow the local temperature), the
 * non-dimensional tau = mu / p of Sec. II with p = rho T and a power-law
 * viscosity mu = T^omega_v: tau_node = tau * T^(omega_v - 1) / rho, tau
 * being the value at rho = T = 1.  law[0] = omega_v. */
static double node_tau(double tau, const double *law, double rho, double T)
{
    if (!law)
        return tau;
    return tau * pow(T, law[0] - 1.0) / rho;
}

/* One full step.  flux (may be NULL) receives, summed over all ghost
 * columns: incoming and outgoing mass of the bottom wall, then of the top. */
static void one_step(const olat *L, int nx, int ny, double tau, const double *law,
                     const double *acc,
                     const double *gb, const double *gt,
                     double alpha_b, double alpha_t, const int *mirror,
                     double *f, double *fs, double *fn,
                     double *ghb, double *ght, double *gob, double *got,
                     double *flux)
{
    const int Q = L->Q, N = max_ey(L);
    const size_t nodes = (size_t)nx * (size_t)ny;
    double Db = 0.0, Dt = 0.0;
    double in_b = 0.0, out_b = 0.0, in_t = 0.0, out_t = 0.0;
    size_t n;
    int x, y, a, l;

    /* 1-2. collision at every fluid node, Eq. (eq:scheme) with the node's
     * relaxation time; with a force, the trapezoidal rule of Sec. II applied
     * to J = -(f - f^eq)/tau + F gives
     *   f*~ = f~ - (f~ - f^eq)/(tau + 1/2) + tau/(tau + 1/2) F
     * with f^eq and F at the moments of f (phys_moments). */
    for (n = 0; n < nodes; ++n) {
        double rho, u[3], T, tn, omega;
        phys_moments(L, f + n * Q, acc, &rho, u, &T);
        tn = node_tau(tau, law, rho, T);
        omega = 1.0 / (tn + 0.5);
        for (a = 0; a < Q; ++a) {
            double feq = rho * geq(L, a, u, T);
            fs[n * Q + a] = f[n * Q + a] - omega * (f[n * Q + a] - feq);
            if (acc)
                fs[n * Q + a] += (isinf(tn) ? 1.0 : tn * omega) * rho *
                                 force_term(L, a, u, T, acc);
        }
    }

    /* 3. streaming: fluid -> fluid, or fluid -> ghost (incoming f^I) */
    memset(fn, 0, nodes * Q * sizeof(double));
    memset(ghb, 0, (size_t)N * nx * Q * sizeof(double));
    memset(ght, 0, (size_t)N * nx * Q * sizeof(double));
    for (y = 0; y < ny; ++y)
        for (x = 0; x < nx; ++x)
            for (a = 0; a < Q; ++a) {
                int xd = wrap(x + L->e[3 * a], nx);
                int yd = y + L->e[3 * a + 1];
                double v = fs[((size_t)y * nx + x) * Q + a];
                if (yd >= 0 && yd < ny)
                    fn[((size_t)yd * nx + xd) * Q + a] = v;
                else if (yd < 0)
                    ghb[((size_t)(-yd - 1) * nx + xd) * Q + a] = v;
                else
                    ght[((size_t)(yd - ny) * nx + xd) * Q + a] = v;
            }

    /* 4. denominators of Eq. (eq:dkboundary): sum over layers l and over the
     * velocities that leave the wall at layer l, (c - u_w).n > l. */
    for (l = 0; l < N; ++l)
        for (a = 0; a < Q; ++a) {
            if (L->e[3 * a + 1] > l)      /* bottom: n = +y */
                Db += gb[a];
            if (-L->e[3 * a + 1] > l)     /* top: n = -y */
                Dt += gt[a];
        }

    /* 4. outgoing ghost populations f^O from the generic scattering closure
     * of Sec. III, f^O = sum over incoming of R f^I, with
     *   R = alpha R_D + (1 - alpha) R_S:
     * R_D (Eq. (eq:dkboundary)) pools all incoming mass of a ghost column and
     * re-emits it in proportion to the wall Maxwellian; R_S (specular) sends
     * each incoming particle back with its normal velocity reversed, from the
     * mirror-image ghost position, so that it continues its straight path
     * reflected at the wall (half a spacing outside the first fluid row). */
    memset(gob, 0, (size_t)N * nx * Q * sizeof(double));
    memset(got, 0, (size_t)N * nx * Q * sizeof(double));
    for (x = 0; x < nx; ++x) {
        double Mb = 0.0, Mt = 0.0;
        for (l = 0; l < N; ++l)
            for (a = 0; a < Q; ++a) {
                if (L->e[3 * a + 1] < -l)     /* (c'-u_w).n < -l, n = +y */
                    Mb += ghb[((size_t)l * nx + x) * Q + a];
                if (-L->e[3 * a + 1] < -l)    /* n = -y */
                    Mt += ght[((size_t)l * nx + x) * Q + a];
            }
        in_b += Mb;
        in_t += Mt;
        for (l = 0; l < N; ++l)
            for (a = 0; a < Q; ++a) {
                if (L->e[3 * a + 1] > l)
                    gob[((size_t)l * nx + x) * Q + a] += alpha_b * Mb / Db * gb[a];
                if (-L->e[3 * a + 1] > l)
                    got[((size_t)l * nx + x) * Q + a] += alpha_t * Mt / Dt * gt[a];
            }
    }
    for (x = 0; x < nx; ++x)
        for (l = 0; l < N; ++l)
            for (a = 0; a < Q; ++a) {
                /* a particle of velocity (ex, ey, ez) that landed in ghost
                 * (x, layer l) came from fluid row -ey - l - 1; reflected, it
                 * leaves ghost (x - ex, that layer) with velocity (ex, -ey, ez) */
                int ey = L->e[3 * a + 1];
                if (ey < -l) {
                    int lm = -ey - l - 1, xm = wrap(x - L->e[3 * a], nx);
                    gob[((size_t)lm * nx + xm) * Q + mirror[a]] +=
                        (1.0 - alpha_b) * ghb[((size_t)l * nx + x) * Q + a];
                }
                if (-ey < -l) {
                    int lm = ey - l - 1, xm = wrap(x - L->e[3 * a], nx);
                    got[((size_t)lm * nx + xm) * Q + mirror[a]] +=
                        (1.0 - alpha_t) * ght[((size_t)l * nx + x) * Q + a];
                }
            }

    /* 5. the outgoing populations stream into the fluid in the same step */
    for (x = 0; x < nx; ++x)
        for (l = 0; l < N; ++l)
            for (a = 0; a < Q; ++a) {
                if (L->e[3 * a + 1] > l) {
                    double fo = gob[((size_t)l * nx + x) * Q + a];
                    int xd = wrap(x + L->e[3 * a], nx);
                    int yd = -(l + 1) + L->e[3 * a + 1];
                    fn[((size_t)yd * nx + xd) * Q + a] = fo;
                    out_b += fo;
                }
                if (-L->e[3 * a + 1] > l) {
                    double fo = got[((size_t)l * nx + x) * Q + a];
                    int xd = wrap(x + L->e[3 * a], nx);
                    int yd = ny + l + L->e[3 * a + 1];
                    fn[((size_t)yd * nx + xd) * Q + a] = fo;
                    out_t += fo;
                }
            }
    memcpy(f, fn, nodes * Q * sizeof(double));
    if (flux) {
        flux[0] = in_b;
        flux[1] = out_b;
        flux[2] = in_t;
        flux[3] = out_t;
    }
}

/* ---------------------------------------------------------------- API --- */

/* g^eq_a(u, T) for all a (rho = 1), Eq. (eq:feq). */
void orc_geq(int Q, int D, int eq_order, int thermal, const int *e,
             const double *w, double r, const double *u, double T,
             double *out)
{
    olat L = {Q, D, eq_order, thermal, e, w, r};
    int a;
    for (a = 0; a < Q; ++a)
        out[a] = geq(&L, a, u, thermal ? T : 1.0);
}

/* f~(0) = f^eq(rho0, u0, T0) at every node (fields of nx*ny values,
 * row-major with x fastest; u0 holds three such fields x, y, z). */
void orc_init(int Q, int D, int eq_order, int thermal, const int *e,
              const double *w, double r, int nx, int ny, const double *rho0,
              const double *u0, const double *T0, double *f)
{
    olat L = {Q, D, eq_order, thermal, e, w, r};
    size_t nodes = (size_t)nx * (size_t)ny, n;
    int a;
    for (n = 0; n < nodes; ++n) {
        double u[3] = {u0[n], u0[nodes + n], u0[2 * nodes + n]};
        double T = thermal ? T0[n] : 1.0;
        for (a = 0; a < Q; ++a)
            f[n * Q + a] = rho0[n] * geq(&L, a, u, T);
    }
}

/* Advance f~ by nsteps.  wall_b/wall_t = {ux, uz, T} of each wall
 * (tangential velocities only); alpha_b/alpha_t their accommodation (1:
 * diffuse, Eq. (eq:dkboundary); 0: specular).  tau is the relaxation time in
 * time steps; +inf gives the collisionless limit.  flux (may be NULL): 4
 * doubles per step, see one_step().  law (may be NULL): the viscosity law
 * of node_tau().  acc (may be NULL): body force, 3 components of the
 * acceleration per time step (see force_term()).  Returns 0, -1 on allocation failure,
 * -2 if a velocity has no mirror image in the set. */
int orc_run(int Q, int D, int eq_order, int thermal, const int *e,
            const double *w, double r, int nx, int ny, double tau,
            const double *wall_b, const double *wall_t, double alpha_b,
            double alpha_t, double *f, long nsteps, double *flux,
            const double *law, const double *acc)
{
    olat L = {Q, D, eq_order, thermal, e, w, r};
    const int N = max_ey(&L);
    const size_t nodes = (size_t)nx * (size_t)ny;
    double ub[3] = {wall_b[0], 0.0, wall_b[1]};
    double ut[3] = {wall_t[0], 0.0, wall_t[1]};
    double *gb = malloc(Q * sizeof(double));
    double *gt = malloc(Q * sizeof(double));
    double *fs = malloc(nodes * Q * sizeof(double));
    double *fn = malloc(nodes * Q * sizeof(double));
    double *ghb = malloc((size_t)N * nx * Q * sizeof(double));
    double *ght = malloc((size_t)N * nx * Q * sizeof(double));
    double *gob = malloc((size_t)N * nx * Q * sizeof(double));
    double *got = malloc((size_t)N * nx * Q * sizeof(double));
    int *mirror = malloc(Q * sizeof(int));
    long s;
    int a, b, rc = 0;
    if (!gb || !gt || !fs || !fn || !ghb || !ght || !gob || !got || !mirror) {
        rc = -1;
        goto done;
    }
    /* wall Maxwellians at (u_w, T_w) with unit density (Sec. III, R_D) */
    for (a = 0; a < Q; ++a) {
        gb[a] = geq(&L, a, ub, thermal ? wall_b[2] : 1.0);
        gt[a] = geq(&L, a, ut, thermal ? wall_t[2] : 1.0);
    }
    /* mirror[a]: the velocity with the normal component reversed */
    for (a = 0; a < Q; ++a) {
        mirror[a] = -1;
        for (b = 0; b < Q; ++b)
            if (e[3 * b] == e[3 * a] && e[3 * b + 1] == -e[3 * a + 1] &&
                e[3 * b + 2] == e[3 * a + 2])
                mirror[a] = b;
        if (mirror[a] < 0) {
            rc = -2;
            goto done;
        }
    }
    for (s = 0; s < nsteps; ++s)
        one_step(&L, nx, ny, tau, law, acc, gb, gt, alpha_b, alpha_t, mirror, f, fs, fn,
                 ghb, ght, gob, got, flux ? flux + 4 * s : NULL);
done:
    free(gb);
    free(gt);
    free(fs);
    free(fn);
    free(ghb);
    free(ght);
    free(gob);
    free(got);
    free(mirror);
    return rc;
}

/* Output fields of f~ at one time level (Eq. (eq:summac)).  The stress and
 * heat flux of the original f follow from f - f^eq = (f~ - f^eq) tau/(tau+1/2),
 * tau the node's relaxation time (node_tau), with f~ + F/2 in place of f~
 * under a body force
 * (the change of variable of Sec. II); the moments are linear in f, so
 *   X[f] = X[f^eq] + tau/(tau + 1/2) (X[f~] - X[f^eq]).
 * out: 9 fields of nx*ny: rho, ux, uy, uz, T, sigma_xy, q_x, q_y, q_z. */
void orc_moments(int Q, int D, int eq_order, int thermal, const int *e,
                 const double *w, double r, int nx, int ny, double tau,
                 const double *f, double *out, const double *law,
                 const double *acc)
{
    olat L = {Q, D, eq_order, thermal, e, w, r};
    const size_t nodes = (size_t)nx * (size_t)ny;
    size_t n;
    int a, i;
    for (n = 0; n < nodes; ++n) {
        const double *fn = f + n * Q;
        double rho, u[3], T, tn, k;
        double sig_t = 0.0, sig_e = 0.0, q_t[3] = {0, 0, 0}, q_e[3] = {0, 0, 0};
        phys_moments(&L, fn, acc, &rho, u, &T);
        tn = node_tau(tau, law, rho, T);
        k = isinf(tn) ? 1.0 : tn / (tn + 0.5);
        for (a = 0; a < Q; ++a) {
            double C[3], C2 = 0.0, feq = rho * geq(&L, a, u, T);
            /* with a force, f - f^eq = tau/(tau+1/2) (f~ + F/2 - f^eq) */
            double ft = fn[a] + (acc ? 0.5 * rho * force_term(&L, a, u, T, acc) : 0.0);
            for (i = 0; i < 3; ++i) {
                C[i] = L.r * (double)L.e[3 * a + i] - u[i];
                C2 += C[i] * C[i];
            }
            /* the xy entry of the trace-free tensor C<i C j> is C_x C_y */
            sig_t += ft * C[0] * C[1];
            sig_e += feq * C[0] * C[1];
            for (i = 0; i < 3; ++i) {
                q_t[i] += 0.5 * ft * C2 * C[i];
                q_e[i] += 0.5 * feq * C2 * C[i];
            }
        }
        out[0 * nodes + n] = rho;
        out[1 * nodes + n] = u[0];
        out[2 * nodes + n] = u[1];
        out[3 * nodes + n] = u[2];
        out[4 * nodes + n] = T;
        out[5 * nodes + n] = sig_e + k * (sig_t - sig_e);
        out[6 * nodes + n] = q_e[0] + k * (q_t[0] - q_e[0]);
        out[7 * nodes + n] = q_e[1] + k * (q_t[1] - q_e[1]);
        out[8 * nodes + n] = q_e[2] + k * (q_t[2] - q_e[2]);
    }
}
