/*
 * FP64 CPU oracle for one time step of the phase-field lattice Boltzmann model of
 * Liang, Xu, Chen, Wang, Chai & Shi, "Phase-field-based lattice Boltzmann modeling of
 * large-density-ratio two-phase flows" (arXiv:1710.09541).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the HIP library
 * is checked against.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Everything is double precision, plain loops over a [9][ny][nx] array per distribution
 * set, two copies (current / next).  Per-node work is independent, so the OpenMP loop
 * over rows gives bit-identical results for any thread count.
 *
 * Notation follows the paper: f_i is the phase-field (conservative Allen-Cahn)
 * distribution with relaxation time tau_f (called tau_phi here), g_i is the flow
 * distribution with relaxation time tau_g.  Lattice units: dx = dt = 1, c_s^2 = 1/3.
 * The phase field runs on D2Q9 (the paper's choice) or on D2Q5 (which Sec. 2.2 also
 * admits); the flow lattice and the stencils of Eqs. 27-28 are always D2Q9.
 *
 * One step n -> n+1 (state = post-streaming f, g and Q = (phi u) of the previous step):
 *   S1  phi = sum_i f_i                                    (Sec. 2.2, Eq. 12)
 *   S2  grad phi, lap phi, isotropic central stencils      (Sec. 2.3, Eqs. 27-28)
 *   S3  rho (Eq. 13), mu_phi (Eqs. 6-7), lambda (Eq. 3), n (Eq. 2),
 *       nu by the chosen law (Eqs. 24-26), tau_g (Eq. 23), F = mu_phi grad phi + G (Eqs. 5, 19)
 *   S4  u from Eq. 22a
 *   S5  p from Eq. 22b (u first, then p)
 *   S6  D = phi u - Q (backward difference for d_t(phi u) in Eq. 11); Q <- phi u
 *   S7  collide f: BGK + source F_i                        (Eqs. 8, 9, 11); with the local
 *       scheme of Eq. 29 the normal in F_i comes from the non-equilibrium first moment
 *   S8  collide g: BGK + forcing G_i                       (Eqs. 15-17, 20)
 *   S9  stream, with periodic / half-way bounce-back / open (pressure outlet) boundaries.
 * Readings where the paper is silent are listed next to the code that takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- lattice (Eq. 10) */
/* D2Q9 velocities: i = 0 rest; 1..4 axis directions at angles (i-1) pi/2;
 * 5..8 diagonals at angles (i-5) pi/2 + pi/4 (length sqrt 2).  Weights 4/9, 1/9, 1/36. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* opposite direction: c_opp(i) = -c_i */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* D2Q5 for the phase field (Sec. 2.2 allows it): the rest and the four axis velocities,
 * i = 0..4 as above, weights 1/3 and 1/6, the same c_s^2 = 1/3 (sum w_i c_i c_i = I/3). */
static const double WGT5[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};

/* weights of the phase-field lattice with qf velocities (9 or 5) */
static const double* fweights(int qf) { return qf == 5 ? WGT5 : WGT; }
/* c_s^2 = 1/3 (c = 1); its reciprocal 3 and the derived factors 1/(2 c_s^4) = 9/2,
 * 1/(2 c_s^2) = 3/2 and c_s^2/(1 - w_0) = 3/5 are written as exact constants, so no rounded
 * 1/3 enters the arithmetic. */
static const double INV_CS2 = 3.0;
/* ambient pressure of an open side: the reference pressure p = 0 of the initial state */
static const double P_AMBIENT = 0.0;

enum { ORC_PERIODIC = 0, ORC_WALL = 1, ORC_OPEN = 2 };
enum { ORC_NU_LINEAR = 0, ORC_NU_INVERSE = 1, ORC_MU_STEP = 2 };
enum { ORC_GRAD_ISOTROPIC = 0, ORC_GRAD_LOCAL_NEQ = 1 };

typedef struct {
    int32_t nx, ny;
    int32_t bc_ylo, bc_yhi;  /* ORC_PERIODIC on both sides or on neither */
    int32_t visc_law;        /* ORC_NU_LINEAR (Eq. 24), ORC_NU_INVERSE (Eq. 25), ORC_MU_STEP (Eq. 26) */
    int32_t grad_scheme;     /* normal n in F_i: ORC_GRAD_ISOTROPIC (Eq. 2 with Eq. 27) or
                                ORC_GRAD_LOCAL_NEQ (Eq. 29); everything else always uses
                                Eqs. 27-28 */
    double rho_l, rho_g;     /* phase densities (Eq. 13) */
    double nu_l, nu_g;       /* phase kinematic viscosities */
    double sigma, W, M;      /* surface tension, interface width, mobility */
    double Gx, Gy;           /* body-force density G (Eq. 4b) */
    int32_t f_lattice;       /* velocities of the phase-field lattice: 9 (D2Q9) or 5 (D2Q5) */
    int32_t reserved;
} orc_params;

typedef struct {
    orc_params p;
    double tau_f;            /* M = c_s^2 (tau_f - 0.5)  (Eq. 14) */
    double kappa, beta;      /* k = 1.5 sigma W, beta = 12 sigma / W  (Eq. 7) */
    int64_t n;               /* nx * ny */
    int64_t steps;
    double *f, *g;           /* current post-streaming state, [9][ny][nx] */
    double *fn, *gn;         /* next state */
    double *q;               /* (phi u) of the previous step, [2][ny][nx] */
    double *phi;             /* scratch: phi of the current step */
    double *p_edge;          /* p of the first [0][nx] and last [1][nx] rows at collision */
} orc_sim;

#define AT(i, y, x, nx, ny) (((int64_t)(i) * (ny) + (y)) * (nx) + (x))

/* --------------------------------------------------------------- local formulas */

/* f_i^eq = w_i phi (1 + c_i.u / c_s^2)  (Eq. 9), i < qf */
static void feq_node(int qf, double phi, double ux, double uy, double out[9]) {
    const double* w = fweights(qf);
    for (int i = 0; i < qf; ++i) {
        double cu = CX[i] * ux + CY[i] * uy;
        out[i] = w[i] * phi * (1.0 + cu * INV_CS2);
    }
}

/* s_i(u) = w_i [c_i.u / c_s^2 + (c_i.u)^2 / (2 c_s^4) - u.u / (2 c_s^2)]  (Eq. 17) */
static double s_i(int i, double ux, double uy) {
    double cu = CX[i] * ux + CY[i] * uy;
    double uu = ux * ux + uy * uy;
    return WGT[i] * (cu * INV_CS2 + cu * cu * 4.5 - uu * 1.5);
}

/* g_i^eq: p/c_s^2 (w_0 - 1) + rho s_0 for i = 0, p/c_s^2 w_i + rho s_i otherwise  (Eq. 16) */
static void geq_node(double p, double rho, double ux, double uy, double out[9]) {
    out[0] = p * INV_CS2 * (WGT[0] - 1.0) + rho * s_i(0, ux, uy);
    for (int i = 1; i < 9; ++i) out[i] = p * INV_CS2 * WGT[i] + rho * s_i(i, ux, uy);
}

/* F_i = (1 - 1/(2 tau_f)) w_i c_i.[d_t(phi u) + c_s^2 lambda n] / c_s^2  (Eq. 11),
 * i.e. (1 - 1/(2 tau_f)) w_i c_i.[d_t(phi u) / c_s^2 + lambda n] */
static void fsource_node(int qf, double tau_f, double dtx, double dty, double lambda,
                         double nx_, double ny_, double out[9]) {
    const double* w = fweights(qf);
    double vx = dtx * INV_CS2 + lambda * nx_;
    double vy = dty * INV_CS2 + lambda * ny_;
    for (int i = 0; i < qf; ++i)
        out[i] = (1.0 - 1.0 / (2.0 * tau_f)) * w[i] * (CX[i] * vx + CY[i] * vy);
}

/* G_i = (1 - 1/(2 tau_g)) w_i [c_i.F / c_s^2 + (rho_l - rho_g) u grad(phi) : c_i c_i / c_s^2]
 * (Eq. 20, the form of Eq. 18 after substituting Eqs. 5 and 13) */
static void gforce_node(double tau_g, double Fx, double Fy, double drho, double ux, double uy,
                        double dpx, double dpy, double out[9]) {
    for (int i = 0; i < 9; ++i) {
        double cF = CX[i] * Fx + CY[i] * Fy;
        double cu = CX[i] * ux + CY[i] * uy;
        double cgp = CX[i] * dpx + CY[i] * dpy;
        out[i] = (1.0 - 1.0 / (2.0 * tau_g)) * WGT[i] * (cF * INV_CS2 + drho * cu * cgp * INV_CS2);
    }
}

/* kinematic viscosity by the chosen law (Sec. 2.3: Eq. 24 linear in phi, Eq. 25 inverse
 * linear, Eq. 26 step in the dynamic viscosity with nu = mu / rho and the tie phi = 0.5
 * going to the liquid) */
static double viscosity(const orc_params* p, double phi, double rho) {
    switch (p->visc_law) {
        case ORC_NU_INVERSE:
            return 1.0 / (phi * (1.0 / p->nu_l - 1.0 / p->nu_g) + 1.0 / p->nu_g);
        case ORC_MU_STEP: {
            double mu = (phi >= 0.5) ? p->rho_l * p->nu_l : p->rho_g * p->nu_g;
            return mu / rho;
        }
        default:
            return phi * (p->nu_l - p->nu_g) + p->nu_g;
    }
}

/* --------------------------------------------------------------- boundaries */

static int wrap(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

/* Row index of phi used by the stencil at row y + dy.  Periodic in y wraps; at a wall or
 * an open side the ghost row mirrors the first interior row (zero normal gradient).  The
 * paper does not state the ghost values; this is the reading used throughout. */
static int ghost_row(const orc_params* p, int y) {
    if (y < 0) return p->bc_ylo == ORC_PERIODIC ? y + p->ny : 0;
    if (y >= p->ny) return p->bc_yhi == ORC_PERIODIC ? y - p->ny : p->ny - 1;
    return y;
}

/* isotropic gradient and Laplacian of a scalar field at (x, y)  (Eqs. 27-28; the index of
 * the shifted position in Eq. 27 is c_i, the same as the weight's) */
static void stencil_node(const orc_params* p, const double* phi, int x, int y, double* gx,
                         double* gy, double* lap) {
    int nx = p->nx;
    double c = phi[(int64_t)y * nx + x];
    double sx = 0.0, sy = 0.0, sl = 0.0;
    for (int i = 1; i < 9; ++i) {
        int xx = wrap(x + CX[i], nx);
        int yy = ghost_row(p, y + CY[i]);
        double v = phi[(int64_t)yy * nx + xx];
        sx += WGT[i] * CX[i] * v;
        sy += WGT[i] * CY[i] * v;
        sl += 2.0 * WGT[i] * (v - c);
    }
    *gx = sx * INV_CS2;
    *gy = sy * INV_CS2;
    *lap = sl * INV_CS2;
}

/* Normal vector from the local non-equilibrium scheme (Sec. 2.3, Eq. 29).  With
 * A = -c_s^2 tau_f, B = M lambda (dt = 1) and
 *     C = sum_i c_i (f_i - f_i^eq) + 0.5 d_t(phi u)
 * (the time derivative in C is the one of Eq. 11: it is what the Chapman-Enskog expansion
 * of Eq. 8 leaves in the first moment of f - f^eq, C = (A + B/|grad phi|) grad phi),
 * Eq. 29a gives |grad phi| = (|C| + B)/(c_s^2 tau_f) and then A + B/|grad phi| =
 * -c_s^2 tau_f |C| / (|C| + B) < 0, so Eq. 29b followed by n = grad phi / |grad phi|
 * (Eq. 2) is exactly
 *     n = -C / |C|.
 * That closed form is evaluated here: the printed two-step form divides 0 by 0 where
 * C = 0 (every node of an equilibrium state) and cancels badly where |C| << B.  Where
 * |C| does not exceed 1e-12 the direction is undefined and n is taken as zero, as for the
 * isotropic scheme. */
static void normal_local_neq(int qf, const double f[9], const double fe[9], double dtx,
                             double dty, double* nx_, double* ny_) {
    double cx = 0.0, cy = 0.0;
    for (int i = 0; i < qf; ++i) {
        cx += CX[i] * (f[i] - fe[i]);
        cy += CY[i] * (f[i] - fe[i]);
    }
    cx += 0.5 * dtx;
    cy += 0.5 * dty;
    double cmag = sqrt(cx * cx + cy * cy);
    if (cmag > 1e-12) {
        *nx_ = -cx / cmag;
        *ny_ = -cy / cmag;
    } else {
        *nx_ = 0.0;
        *ny_ = 0.0;
    }
}

/* --------------------------------------------------------------- node closure */

typedef struct {
    double phi, rho, p, ux, uy;
    double dpx, dpy, lap, mu_phi, lambda, nx, ny, tau_g, Fx, Fy;
} orc_node;

/* S3-S5 at one node, from phi, its stencil values and the node's g_i */
static void closure_node(const orc_sim* s, double phi, double dpx, double dpy, double lap,
                         const double g[9], orc_node* o) {
    const orc_params* p = &s->p;
    o->phi = phi;
    o->dpx = dpx;
    o->dpy = dpy;
    o->lap = lap;
    o->rho = phi * (p->rho_l - p->rho_g) + p->rho_g;                          /* Eq. 13 */
    o->mu_phi = 4.0 * s->beta * phi * (phi - 1.0) * (phi - 0.5) - s->kappa * lap;  /* Eq. 6 */
    o->lambda = 4.0 * phi * (1.0 - phi) / p->W;                               /* Eq. 3 */
    double mag = sqrt(dpx * dpx + dpy * dpy);
    /* Eq. 2; where the gradient vanishes the normal is taken as zero (lambda n is then
     * negligible anyway).  Threshold 1e-12. */
    if (mag > 1e-12) {
        o->nx = dpx / mag;
        o->ny = dpy / mag;
    } else {
        o->nx = 0.0;
        o->ny = 0.0;
    }
    double nu = viscosity(p, phi, o->rho);
    o->tau_g = nu * INV_CS2 + 0.5;                                            /* Eq. 23 */
    o->Fx = o->mu_phi * dpx + p->Gx;                                          /* Eqs. 5, 19 */
    o->Fy = o->mu_phi * dpy + p->Gy;
    /* Eq. 22a: rho u = sum_i c_i g_i + 0.5 F */
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < 9; ++i) {
        mx += CX[i] * g[i];
        my += CY[i] * g[i];
    }
    o->ux = (mx + 0.5 * o->Fx) / o->rho;
    o->uy = (my + 0.5 * o->Fy) / o->rho;
    /* Eq. 22b: p = c_s^2/(1 - w_0) [sum_{i!=0} g_i + 0.5 (rho_l - rho_g) u.grad phi + rho s_0(u)] */
    double sg = 0.0;
    for (int i = 1; i < 9; ++i) sg += g[i];
    double ugp = o->ux * dpx + o->uy * dpy;
    o->p = 0.6 * (sg + 0.5 * (p->rho_l - p->rho_g) * ugp + o->rho * s_i(0, o->ux, o->uy));
}

static void compute_phi(orc_sim* s) {
    const int64_t n = s->n;
    const int qf = s->p.f_lattice;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int i = 0; i < qf; ++i) acc += s->f[(int64_t)i * n + k];
        s->phi[k] = acc;                                                      /* Eq. 12 */
    }
}

/* gather the 9 g values of one node from the state */
static void gather(const double* a, int64_t n, int64_t k, double out[9]) {
    for (int i = 0; i < 9; ++i) out[i] = a[(int64_t)i * n + k];
}

/* --------------------------------------------------------------- one step */

static void step_once(orc_sim* s) {
    const orc_params* p = &s->p;
    const int nx = p->nx, ny = p->ny;
    const int qf = p->f_lattice;
    const int64_t n = s->n;
    compute_phi(s);                                                           /* S1 */

#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            int64_t k = (int64_t)y * nx + x;
            double f[9], g[9];
            gather(s->f, n, k, f);
            gather(s->g, n, k, g);
            double dpx, dpy, lap;
            stencil_node(p, s->phi, x, y, &dpx, &dpy, &lap);                  /* S2 */
            orc_node o;
            closure_node(s, s->phi[k], dpx, dpy, lap, g, &o);                 /* S3-S5 */
            if (y == 0) s->p_edge[x] = o.p;          /* kept for an open side (below) */
            if (y == ny - 1) s->p_edge[nx + x] = o.p;

            /* S6: d_t(phi u) by a backward difference over one step */
            double pux = o.phi * o.ux, puy = o.phi * o.uy;
            double dtx = pux - s->q[k], dty = puy - s->q[n + k];
            s->q[k] = pux;
            s->q[n + k] = puy;

            /* S7: f_i* = f_i - (f_i - f_i^eq)/tau_f + F_i  (Eq. 8) */
            double fe[9], fs[9], fpost[9];
            feq_node(qf, o.phi, o.ux, o.uy, fe);
            if (p->grad_scheme == ORC_GRAD_LOCAL_NEQ)                        /* Eq. 29 */
                normal_local_neq(qf, f, fe, dtx, dty, &o.nx, &o.ny);
            fsource_node(qf, s->tau_f, dtx, dty, o.lambda, o.nx, o.ny, fs);
            for (int i = 0; i < qf; ++i) fpost[i] = f[i] - (f[i] - fe[i]) / s->tau_f + fs[i];

            /* S8: g_i* = g_i - (g_i - g_i^eq)/tau_g + G_i  (Eq. 15) */
            double ge[9], gf[9], gpost[9];
            geq_node(o.p, o.rho, o.ux, o.uy, ge);
            gforce_node(o.tau_g, o.Fx, o.Fy, p->rho_l - p->rho_g, o.ux, o.uy, dpx, dpy, gf);
            for (int i = 0; i < 9; ++i) gpost[i] = g[i] - (g[i] - ge[i]) / o.tau_g + gf[i];

            /* S9: push to x + c_i.  x is periodic.  In y: periodic wrap; a wall half a cell
             * beyond the first / last row reflects the population back into the node it
             * left, reversed (half-way bounce-back); an open side lets it leave. */
            for (int i = 0; i < 9; ++i) {
                int xd = wrap(x + CX[i], nx);
                int yd = y + CY[i];
                int side = yd < 0 ? p->bc_ylo : (yd >= ny ? p->bc_yhi : -1);
                if (side == -1 || side == ORC_PERIODIC) {
                    yd = wrap(yd, ny);
                    if (i < qf) s->fn[AT(i, yd, xd, nx, ny)] = fpost[i];
                    s->gn[AT(i, yd, xd, nx, ny)] = gpost[i];
                } else if (side == ORC_WALL) {
                    if (i < qf) s->fn[AT(OPP[i], y, x, nx, ny)] = fpost[i];
                    s->gn[AT(OPP[i], y, x, nx, ny)] = gpost[i];
                } /* ORC_OPEN: the population leaves the domain */
            }
        }
    }

    /* Open side.  The paper names an open boundary at the top of the impact domain and
     * gives no formula; the reading taken is a pressure outlet: one node beyond the edge
     * row the pressure is the ambient one, p = 0 (the reference pressure of the initial
     * state), and every other field has zero normal gradient.  It is imposed by
     * non-equilibrium extrapolation (Guo, Zheng & Shi, 2002): the ghost node beyond the
     * edge sends what the edge node below it sent, with the pressure part of the flow
     * equilibrium (Eq. 16) taken at the ambient pressure instead of the node's own.  For a
     * population i entering through the side, with s = (x - c_ix, edge row) its source,
     *     f_i(x, edge) = f*_i(s)
     *     g_i(x, edge) = g*_i(s) + (p_amb - p(s)) w_i / c_s^2      (i != 0; Eq. 16)
     * where f*, g* are post-collision values and p(s) the pressure of the source node's
     * collision.  f*_i(s) and g*_i(s) are what streamed into the adjacent interior row,
     * same x, from s.  (A zero-gradient copy of g alone leaves the pressure level of the
     * side free; with liquid or a fast splash at the side it then drifts and blows up.) */
    if (p->bc_yhi == ORC_OPEN) {
        for (int i = 0; i < 9; ++i) {
            if (CY[i] >= 0) continue;
            for (int x = 0; x < nx; ++x) {
                int xs = wrap(x - CX[i], nx);
                if (i < qf) s->fn[AT(i, ny - 1, x, nx, ny)] = s->fn[AT(i, ny - 2, x, nx, ny)];
                s->gn[AT(i, ny - 1, x, nx, ny)] =
                    s->gn[AT(i, ny - 2, x, nx, ny)] + (P_AMBIENT - s->p_edge[nx + xs]) * INV_CS2 * WGT[i];
            }
        }
    }
    if (p->bc_ylo == ORC_OPEN) {
        for (int i = 0; i < 9; ++i) {
            if (CY[i] <= 0) continue;
            for (int x = 0; x < nx; ++x) {
                int xs = wrap(x - CX[i], nx);
                if (i < qf) s->fn[AT(i, 0, x, nx, ny)] = s->fn[AT(i, 1, x, nx, ny)];
                s->gn[AT(i, 0, x, nx, ny)] =
                    s->gn[AT(i, 1, x, nx, ny)] + (P_AMBIENT - s->p_edge[xs]) * INV_CS2 * WGT[i];
            }
        }
    }

    double* t = s->f;
    s->f = s->fn;
    s->fn = t;
    t = s->g;
    s->g = s->gn;
    s->gn = t;
    s->steps += 1;
}

/* --------------------------------------------------------------- exported API */

/* Validates the parameters; returns 0 if usable, a negative code otherwise. */
int orc_check(const orc_params* p) {
    if (!p || p->nx < 3 || p->ny < 3) return -1;
    if ((p->bc_ylo == ORC_PERIODIC) != (p->bc_yhi == ORC_PERIODIC)) return -2;
    if (p->bc_ylo < 0 || p->bc_ylo > 2 || p->bc_yhi < 0 || p->bc_yhi > 2) return -3;
    if (p->visc_law < 0 || p->visc_law > 2) return -4;
    if (p->grad_scheme < 0 || p->grad_scheme > 1) return -7;
    if (p->f_lattice != 9 && p->f_lattice != 5) return -8;
    if (!(p->rho_l > 0) || !(p->rho_g > 0) || !(p->nu_l > 0) || !(p->nu_g > 0)) return -5;
    if (!(p->W > 0) || !(p->M > 0) || !(p->sigma >= 0)) return -6;
    return 0;
}

/* Creates a simulation at step 0 (reading of the unstated initial state: the
 * distributions start at their equilibria, f = f^eq(phi0, u0), g = g^eq(p = 0, u0) with
 * rho = rho(phi0), and Q = phi0 u0 so that the first backward difference sees no jump
 * from before t = 0).  phi0, ux0, uy0 are [ny][nx] row-major; they are copied. */
orc_sim* orc_create(const orc_params* p, const double* phi0, const double* ux0,
                    const double* uy0) {
    if (orc_check(p) != 0) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->p = *p;
    s->n = (int64_t)p->nx * p->ny;
    s->tau_f = p->M * INV_CS2 + 0.5;             /* Eq. 14 */
    s->kappa = 1.5 * p->sigma * p->W;            /* Eq. 7 */
    s->beta = 12.0 * p->sigma / p->W;
    size_t n9 = (size_t)(9 * s->n);
    s->f = (double*)malloc(n9 * sizeof(double));
    s->g = (double*)malloc(n9 * sizeof(double));
    s->fn = (double*)calloc(n9, sizeof(double));
    s->gn = (double*)calloc(n9, sizeof(double));
    s->q = (double*)malloc((size_t)(2 * s->n) * sizeof(double));
    s->phi = (double*)malloc((size_t)s->n * sizeof(double));
    s->p_edge = (double*)calloc((size_t)(2 * p->nx), sizeof(double));
    if (!s->f || !s->g || !s->fn || !s->gn || !s->q || !s->phi || !s->p_edge) {
        free(s->f); free(s->g); free(s->fn); free(s->gn); free(s->q); free(s->phi);
        free(s->p_edge); free(s);
        return NULL;
    }
    for (int64_t k = 0; k < s->n; ++k) {
        double ph = phi0[k], ux = ux0[k], uy = uy0[k];
        double rho = ph * (p->rho_l - p->rho_g) + p->rho_g;
        double fe[9] = {0.0}, ge[9];
        feq_node(p->f_lattice, ph, ux, uy, fe);
        geq_node(0.0, rho, ux, uy, ge);
        for (int i = 0; i < 9; ++i) {
            s->f[(int64_t)i * s->n + k] = fe[i];   /* planes qf..8 unused (zero) for D2Q5 */
            s->g[(int64_t)i * s->n + k] = ge[i];
        }
        s->q[k] = ph * ux;
        s->q[s->n + k] = ph * uy;
    }
    return s;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->f); free(s->g); free(s->fn); free(s->gn); free(s->q); free(s->phi);
    free(s->p_edge); free(s);
}

void orc_step(orc_sim* s, int64_t nsteps) {
    for (int64_t t = 0; t < nsteps; ++t) step_once(s);
}

int64_t orc_steps_done(const orc_sim* s) { return s->steps; }

/* Macroscopic fields of the current state, exactly the values the next collision uses
 * (S1-S5).  Each output is [ny][nx]; any pointer may be NULL. */
void orc_moments(orc_sim* s, double* phi, double* rho, double* pr, double* ux, double* uy) {
    const orc_params* p = &s->p;
    compute_phi(s);
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y) {
        for (int x = 0; x < p->nx; ++x) {
            int64_t k = (int64_t)y * p->nx + x;
            double g[9], dpx, dpy, lap;
            gather(s->g, s->n, k, g);
            stencil_node(p, s->phi, x, y, &dpx, &dpy, &lap);
            orc_node o;
            closure_node(s, s->phi[k], dpx, dpy, lap, g, &o);
            if (phi) phi[k] = o.phi;
            if (rho) rho[k] = o.rho;
            if (pr) pr[k] = o.p;
            if (ux) ux[k] = o.ux;
            if (uy) uy[k] = o.uy;
        }
    }
}

/* Raw state: f and g are [9][ny][nx] post-streaming distributions, q is [2][ny][nx]. */
void orc_get_state(const orc_sim* s, double* f, double* g, double* q) {
    if (f) memcpy(f, s->f, (size_t)(9 * s->n) * sizeof(double));
    if (g) memcpy(g, s->g, (size_t)(9 * s->n) * sizeof(double));
    if (q) memcpy(q, s->q, (size_t)(2 * s->n) * sizeof(double));
}

void orc_set_state(orc_sim* s, const double* f, const double* g, const double* q) {
    if (f) memcpy(s->f, f, (size_t)(9 * s->n) * sizeof(double));
    if (g) memcpy(s->g, g, (size_t)(9 * s->n) * sizeof(double));
    if (q) memcpy(s->q, q, (size_t)(2 * s->n) * sizeof(double));
}

/* ------------------------------------------- single-node entry points for unit pins */

void orc_lattice(int32_t* cx, int32_t* cy, double* w, int32_t* opp) {
    for (int i = 0; i < 9; ++i) {
        cx[i] = CX[i];
        cy[i] = CY[i];
        w[i] = WGT[i];
        opp[i] = OPP[i];
    }
}

void orc_feq(int32_t qf, double phi, double ux, double uy, double* out) {
    feq_node(qf, phi, ux, uy, out);
}

void orc_geq(double p, double rho, double ux, double uy, double* out) {
    geq_node(p, rho, ux, uy, out);
}

void orc_fsource(int32_t qf, double tau_f, double dtx, double dty, double lambda, double nx_,
                 double ny_, double* out) {
    fsource_node(qf, tau_f, dtx, dty, lambda, nx_, ny_, out);
}

/* weights of the phase-field lattice with qf velocities (its velocities are c_0..c_{qf-1}) */
void orc_fweights(int32_t qf, double* w) {
    const double* src = fweights(qf);
    for (int i = 0; i < qf; ++i) w[i] = src[i];
}

void orc_gforce(double tau_g, double Fx, double Fy, double drho, double ux, double uy,
                double dpx, double dpy, double* out) {
    gforce_node(tau_g, Fx, Fy, drho, ux, uy, dpx, dpy, out);
}

/* Stencils of Eqs. 27-28 over a whole [ny][nx] field with the boundary rules above. */
int orc_stencil(const orc_params* p, const double* phi, double* gx, double* gy, double* lap) {
    if (orc_check(p) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            int64_t k = (int64_t)y * p->nx + x;
            stencil_node(p, phi, x, y, &gx[k], &gy[k], &lap[k]);
        }
    return 0;
}

/* Moment step (S3-S5) at one node given phi, its stencil values and the node's g_i.
 * out = {rho, mu_phi, lambda, n_x, n_y, tau_g, F_x, F_y, u_x, u_y, p}. */
void orc_closure(const orc_params* p, double phi, double dpx, double dpy, double lap,
                 const double* g, double* out) {
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.p = *p;
    s.tau_f = p->M * INV_CS2 + 0.5;
    s.kappa = 1.5 * p->sigma * p->W;
    s.beta = 12.0 * p->sigma / p->W;
    orc_node o;
    closure_node(&s, phi, dpx, dpy, lap, g, &o);
    double v[11] = {o.rho, o.mu_phi, o.lambda, o.nx, o.ny, o.tau_g, o.Fx, o.Fy, o.ux, o.uy, o.p};
    memcpy(out, v, sizeof(v));
}

/* Eq. 29 normal at one node from its f_i, phi, u and d_t(phi u); out = {n_x, n_y}. */
void orc_normal_local_neq(int32_t qf, const double* f, double phi, double ux, double uy,
                          double dtx, double dty, double* out) {
    double fe[9];
    feq_node(qf, phi, ux, uy, fe);
    normal_local_neq(qf, f, fe, dtx, dty, &out[0], &out[1]);
}
