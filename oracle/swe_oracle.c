/*
 * FP64 reference checker for the explicit 2-D shallow-water RK3 step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the bench's
 * CPU-baseline leg load it.  It shares no header, helper or table with the
 * HIP path.
 *
 * It is written to be read against the paper (Madden, Marras & Suckale,
 * "Leveraging Google's Tensor Processing Units for tsunami-risk mitigation
 * planning in the Pacific Northwest and beyond"):
 *   - Methods, Eqs. (1)-(3): the nonlinear shallow-water system with the
 *     1/2 g (h^2 - b^2) pressure flux, bed source -g (h+b) grad b (taken
 *     relative to the datum, R2) and the explicit Manning friction
 *     -g n^2 |q| q / h^(7/3);
 *   - Methods, Eq. (4): the vector form u_t + F_x + G_y = S, u = (h, hu, hv);
 *   - Methods, WENO paragraph and Eq. (5): fifth-order WENO reconstruction,
 *     one value for each characteristic direction at every half-step face;
 *   - Methods, Lax-Friedrichs paragraph, Eq. (6): global-maximum wave-speed
 *     Lax-Friedrichs splitting;
 *   - Methods, Eq. (7): the explicit update operator T with the source taken
 *     explicitly at the cell centre;
 *   - Methods, Eq. (8): the three-stage TVD Runge-Kutta combination.
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes):
 *   R1  WENO acts on the split fluxes F+- = (F +- alpha u~)/2 at the faces
 *       (finite-difference flux splitting); the printed LF formula, which
 *       multiplies alpha by a flux difference, is read as this split form.
 *   R2  The bed enters relative to the datum (the still-water level, 0):
 *       with m = min(b, 0) the pressure flux is 1/2 g (h^2 - m^2), the bed
 *       source -g (h + m) db/dx, and u~ = (h + m, hu, hv), so the mass
 *       component of the LF viscosity acts on h + m.  Below the datum m = b
 *       and this is the printed form (Eqs. (1)-(3)): 1/2 g (h^2 - b^2),
 *       -g (h + b) grad b, viscosity on the surface h + b.  On land m = 0 and
 *       it is 1/2 g h^2, -g h grad b, viscosity on the depth.  Both forms
 *       are the same differential system (d(m^2)/dx = 2 m db/dx wherever m
 *       is not constant), but the printed one, read literally on dry land
 *       (h = 0), has the flux -1/2 g b^2 and a viscosity on b between dry
 *       cells, which the clamp of R7 turns into water appearing on land.
 *       The face value of b used by the bed source is reconstructed with the
 *       nonlinear weights of the hu (x) or hv (y) split flux.  Together these
 *       make still water at any level over a bed below the datum, and still
 *       water at the datum next to any dry land, exact discrete steady
 *       states (the bed treatment the paper takes from Xing & Shu).
 *   R3  alpha_x = max(|u| + sqrt(g h+)), alpha_y = max(|v| + sqrt(g h+)) over
 *       the interior cells of each stage's input, one per scenario.
 *   R4  dt = cfl / (alpha_x/dx + alpha_y/dy) from u^n, held over the three
 *       stages (0 when both speeds vanish); cfl <= 0 selects dt_fixed.
 *   R5  WENO5-JS constants: linear weights (1/10, 6/10, 3/10), epsilon
 *       weno_eps added to beta, power 2.
 *   R6  The y-momentum bed term uses db/dy (the printed db/dx is a typo).
 *   R7  wet <=> h > h_dry; dry cells have zero velocity and no friction.
 *       After every stage h < 0 is clamped to 0 (the added mass is recorded,
 *       weighted by how much of it reaches u^(n+1): 1/6, 2/3, 1) and the
 *       momentum is zeroed where h <= h_dry.
 *   R8  Friction stiffness cap: kappa <= kappa_cap/dt when kappa_cap > 0.
 *   R9  Boundaries: REFLECT mirrors three ghost layers (normal momentum odd);
 *       FIXED freezes the ghost (h, hu, hv) at the create-time values of the
 *       nearest interior cell and extends b linearly.
 *   R10 Variant, off by default (oracle_set_friction): point-implicit
 *       friction.  The paper keeps friction explicit and names an implicit
 *       treatment as the alternative it did not take (Methods); this reading
 *       takes each stage's friction term backward in time with kappa frozen
 *       at the stage input w and not capped:
 *         q_out = [a_n q^n + a_w (q_w + dt L'(w))] / (1 + a_w dt kappa(w)),
 *       L' the right-hand side without friction, (a_n, a_w) = (0, 1),
 *       (3/4, 1/4), (1/3, 2/3) for the three stages.
 *   R11 Variant, off by default (oracle_set_split): local Lax-Friedrichs
 *       splitting.  The paper splits with one global maximum speed per
 *       stage (Methods, Lax-Friedrichs paragraph); this variant takes, for
 *       each face, the largest normal speed |u_n| + sqrt(g h+) over the six
 *       cells that the face's two reconstructions read, and splits those six
 *       cells' fluxes with it.  Each face flux stays single-valued
 *       (conservative), and a constant h + m gives no mass flux
 *       (well-balanced as R2).  The time step stays global (R4).
 *
 * Build: gcc -O2 -std=c11 -fopenmp -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HALO 3

typedef struct {
    int32_t nx, ny;
    double dx, dy, g, cfl, dt_fixed, h_dry, weno_eps, kappa_cap;
    int32_t bc[4]; /* west, east, south, north */
} oracle_params;

enum { BC_REFLECT = 0, BC_FIXED = 1 };
enum { WEST = 0, EAST = 1, SOUTH = 2, NORTH = 3 };

typedef struct {
    oracle_params p;
    int NX, NY;                   /* extended sizes nx + 6, ny + 6 */
    double *b;                    /* extended; ghosts set once at create */
    double *gn2;                  /* interior: g n^2 */
    double *h, *hu, *hv;          /* u^n (extended) */
    double *h1, *hu1, *hv1;       /* u^(1) (extended) */
    double *h2, *hu2, *hv2;       /* u^(2) (extended) */
    double *Lh, *Lhu, *Lhv;       /* interior right-hand side */
    double *fx[3], *gy[3];        /* interior -dF/dx and -dG/dy per component */
    double *bedx, *bedy;          /* interior bed terms */
    double *ghost[4][3];          /* frozen FIXED ghosts: [side][field][layer*len + k] */
    double t, mass, clamp_mass, runup, alpha_x, alpha_y, dt_last;
    double *kap;                  /* interior friction rate of the stage input (implicit mode) */
    int64_t step;
    int nonfinite;
    int friction_implicit;        /* R10 */
    int local_alpha;              /* R11 */
} oracle_ctx;

static inline size_t IX(const oracle_ctx *c, int i, int j)
{
    return (size_t)(j + HALO) * (size_t)c->NX + (size_t)(i + HALO);
}

static inline size_t II(const oracle_ctx *c, int i, int j)
{
    return (size_t)j * (size_t)c->p.nx + (size_t)i;
}

/* ------------------------------------------------------------------------ */
/* WENO5-JS (Jiang & Shu), Methods: WENO paragraph.                          */
/* v[0..4] is the five-point stencil read in the upwind direction; the       */
/* return value is the reconstruction at the face between v[2] and v[3].     */
/* ------------------------------------------------------------------------ */

static void weno5_candidates(const double v[5], double q[3])
{
    q[0] = (2.0 * v[0] - 7.0 * v[1] + 11.0 * v[2]) / 6.0;
    q[1] = (-v[1] + 5.0 * v[2] + 2.0 * v[3]) / 6.0;
    q[2] = (2.0 * v[2] + 5.0 * v[3] - v[4]) / 6.0;
}

static double weno5(const double v[5], double eps, double w[3])
{
    static const double d[3] = {0.1, 0.6, 0.3};
    double q[3], beta[3], a[3];
    weno5_candidates(v, q);
    const double s0 = v[0] - 2.0 * v[1] + v[2], t0 = v[0] - 4.0 * v[1] + 3.0 * v[2];
    const double s1 = v[1] - 2.0 * v[2] + v[3], t1 = v[1] - v[3];
    const double s2 = v[2] - 2.0 * v[3] + v[4], t2 = 3.0 * v[2] - 4.0 * v[3] + v[4];
    beta[0] = 13.0 / 12.0 * s0 * s0 + 0.25 * t0 * t0;
    beta[1] = 13.0 / 12.0 * s1 * s1 + 0.25 * t1 * t1;
    beta[2] = 13.0 / 12.0 * s2 * s2 + 0.25 * t2 * t2;
    double sum = 0.0;
    for (int k = 0; k < 3; k++) {
        a[k] = d[k] / ((eps + beta[k]) * (eps + beta[k]));
        sum += a[k];
    }
    double r = 0.0;
    for (int k = 0; k < 3; k++) {
        w[k] = a[k] / sum;
        r += w[k] * q[k];
    }
    return r;
}

/* Reconstruction of another sequence with given (already normalised) weights. */
static double weno5_with_weights(const double v[5], const double w[3])
{
    double q[3];
    weno5_candidates(v, q);
    return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

/* ------------------------------------------------------------------------ */
/* Boundary ghosts (R9)                                                       */
/* ------------------------------------------------------------------------ */

static void fill_ghosts(oracle_ctx *c, double *h, double *hu, double *hv)
{
    const int nx = c->p.nx, ny = c->p.ny;
    for (int j = 0; j < ny; j++) {
        for (int k = 0; k < HALO; k++) {
            size_t g = IX(c, -1 - k, j), s = IX(c, k, j);
            if (c->p.bc[WEST] == BC_REFLECT) {
                h[g] = h[s]; hu[g] = -hu[s]; hv[g] = hv[s];
            } else {
                h[g] = c->ghost[WEST][0][k * ny + j];
                hu[g] = c->ghost[WEST][1][k * ny + j];
                hv[g] = c->ghost[WEST][2][k * ny + j];
            }
            g = IX(c, nx + k, j); s = IX(c, nx - 1 - k, j);
            if (c->p.bc[EAST] == BC_REFLECT) {
                h[g] = h[s]; hu[g] = -hu[s]; hv[g] = hv[s];
            } else {
                h[g] = c->ghost[EAST][0][k * ny + j];
                hu[g] = c->ghost[EAST][1][k * ny + j];
                hv[g] = c->ghost[EAST][2][k * ny + j];
            }
        }
    }
    for (int i = 0; i < nx; i++) {
        for (int k = 0; k < HALO; k++) {
            size_t g = IX(c, i, -1 - k), s = IX(c, i, k);
            if (c->p.bc[SOUTH] == BC_REFLECT) {
                h[g] = h[s]; hu[g] = hu[s]; hv[g] = -hv[s];
            } else {
                h[g] = c->ghost[SOUTH][0][k * nx + i];
                hu[g] = c->ghost[SOUTH][1][k * nx + i];
                hv[g] = c->ghost[SOUTH][2][k * nx + i];
            }
            g = IX(c, i, ny + k); s = IX(c, i, ny - 1 - k);
            if (c->p.bc[NORTH] == BC_REFLECT) {
                h[g] = h[s]; hu[g] = hu[s]; hv[g] = -hv[s];
            } else {
                h[g] = c->ghost[NORTH][0][k * nx + i];
                hu[g] = c->ghost[NORTH][1][k * nx + i];
                hv[g] = c->ghost[NORTH][2][k * nx + i];
            }
        }
    }
}

/* Static bed ghosts: mirror for REFLECT, linear extension for FIXED. */
static void fill_bed_ghosts(oracle_ctx *c)
{
    const int nx = c->p.nx, ny = c->p.ny;
    double *b = c->b;
    for (int j = 0; j < ny; j++) {
        for (int k = 0; k < HALO; k++) {
            if (c->p.bc[WEST] == BC_REFLECT)
                b[IX(c, -1 - k, j)] = b[IX(c, k, j)];
            else
                b[IX(c, -1 - k, j)] = b[IX(c, 0, j)] + (k + 1) * (b[IX(c, 0, j)] - b[IX(c, 1, j)]);
            if (c->p.bc[EAST] == BC_REFLECT)
                b[IX(c, nx + k, j)] = b[IX(c, nx - 1 - k, j)];
            else
                b[IX(c, nx + k, j)] = b[IX(c, nx - 1, j)] + (k + 1) * (b[IX(c, nx - 1, j)] - b[IX(c, nx - 2, j)]);
        }
    }
    for (int i = 0; i < nx; i++) {
        for (int k = 0; k < HALO; k++) {
            if (c->p.bc[SOUTH] == BC_REFLECT)
                b[IX(c, i, -1 - k)] = b[IX(c, i, k)];
            else
                b[IX(c, i, -1 - k)] = b[IX(c, i, 0)] + (k + 1) * (b[IX(c, i, 0)] - b[IX(c, i, 1)]);
            if (c->p.bc[NORTH] == BC_REFLECT)
                b[IX(c, i, ny + k)] = b[IX(c, i, ny - 1 - k)];
            else
                b[IX(c, i, ny + k)] = b[IX(c, i, ny - 1)] + (k + 1) * (b[IX(c, i, ny - 1)] - b[IX(c, i, ny - 2)]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Global wave speeds (R3)                                                    */
/* ------------------------------------------------------------------------ */

static void wave_speeds(oracle_ctx *c, const double *h, const double *hu, const double *hv,
                        double *ax, double *ay)
{
    const int nx = c->p.nx, ny = c->p.ny;
    double mx = 0.0, my = 0.0;
    int bad = 0;
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            const size_t e = IX(c, i, j);
            const double hp = h[e] > 0.0 ? h[e] : 0.0;
            const double cel = sqrt(c->p.g * hp);
            double u = 0.0, v = 0.0;
            if (h[e] > c->p.h_dry) {
                u = hu[e] / h[e];
                v = hv[e] / h[e];
            }
            const double sx = fabs(u) + cel, sy = fabs(v) + cel;
            if (!isfinite(sx) || !isfinite(sy) || !isfinite(h[e]))
                bad = 1;
            if (sx > mx) mx = sx;
            if (sy > my) my = sy;
        }
    }
    if (bad) {
        c->nonfinite = 1;
        mx = my = NAN;
    }
    *ax = mx;
    *ay = my;
}

static double time_step(const oracle_ctx *c, double ax, double ay)
{
    if (c->p.cfl <= 0.0)
        return c->p.dt_fixed;
    const double den = ax / c->p.dx + ay / c->p.dy;
    if (!(den > 0.0))
        return isnan(den) ? NAN : 0.0;
    return c->p.cfl / den;
}

/* ------------------------------------------------------------------------ */
/* Right-hand side L(w), Eq. (7): flux divergence plus sources.               */
/* w is extended with ghosts filled.                                          */
/* ------------------------------------------------------------------------ */

/* The bed relative to the datum (R2): b below it, 0 on land. */
static inline double datum_bed(double b)
{
    return b < 0.0 ? b : 0.0;
}

/* Cell flux F (x) or G (y) and the LF-split vector u~ of one cell.  dir 0 = x. */
static void cell_flux(const oracle_ctx *c, int dir, double h, double hu, double hv, double b,
                      double F[3], double U[3])
{
    double u = 0.0, v = 0.0;
    if (h > c->p.h_dry) {
        u = hu / h;
        v = hv / h;
    }
    const double m = datum_bed(b);
    const double pres = 0.5 * c->p.g * (h * h - m * m);
    if (dir == 0) {
        F[0] = hu;
        F[1] = hu * u + pres;
        F[2] = hu * v;
    } else {
        F[0] = hv;
        F[1] = hv * u;
        F[2] = hv * v + pres;
    }
    U[0] = h + m;
    U[1] = hu;
    U[2] = hv;
}

/* Speed of the fastest wave along direction dir in one cell (R3, R11). */
static double normal_speed(const oracle_ctx *c, int dir, double h, double hu, double hv)
{
    const double hp = h > 0.0 ? h : 0.0;
    double un = 0.0;
    if (h > c->p.h_dry)
        un = (dir == 0 ? hu : hv) / h;
    return fabs(un) + sqrt(c->p.g * hp);
}

/* One line of faces along direction dir.  n = number of interior cells on the
 * line; val(k) for k in [-3, n+3) reads the extended line.  Outputs
 * div[m][k] = -(Fhat_{k+1/2} - Fhat_{k-1/2}) / ds and dbh[k] = bhat_{k+1/2} - bhat_{k-1/2}
 * for the interior cells k in [0, n).  alpha is the stage's global speed;
 * with R11 each face takes its own from sp. */
static void line_faces(const oracle_ctx *c, int dir, int n, double alpha, double ds,
                       const double *lh, const double *lhu, const double *lhv, const double *lb,
                       double *div0, double *div1, double *div2, double *dbh,
                       double *Fc, double *Uc, double *sp, double *Fhat, double *bhat)
{
    /* cell fluxes and LF split vectors at every cell of the extended line:
     * Fc/Uc[(k+3)*3 + m]; normal wave speeds sp[k+3] for R11 */
    for (int k = -HALO; k < n + HALO; k++) {
        cell_flux(c, dir, lh[k], lhu[k], lhv[k], lb[k], &Fc[(k + HALO) * 3], &Uc[(k + HALO) * 3]);
        sp[k + HALO] = normal_speed(c, dir, lh[k], lhu[k], lhv[k]);
    }
    /* the momentum component normal to the faces owns the bed weights */
    const int mb = dir == 0 ? 1 : 2;
    /* face f = k + 1/2 for k in [-1, n): stored at index k + 1 */
    for (int k = -1; k < n; k++) {
        double a = alpha;
        if (c->local_alpha) {
            a = 0.0;
            for (int s = -2; s <= 3; s++)  /* cells k-2 .. k+3 */
                if (sp[k + s + HALO] > a)
                    a = sp[k + s + HALO];
        }
        double wp[3], wm[3], vp[5], vm[5];
        for (int m = 0; m < 3; m++) {
            for (int s = 0; s < 5; s++) {
                const int ip = (k - 2 + s + HALO) * 3 + m;  /* cells k-2 .. k+2 */
                const int im = (k + 3 - s + HALO) * 3 + m;  /* cells k+3 .. k-1 */
                vp[s] = 0.5 * (Fc[ip] + a * Uc[ip]);
                vm[s] = 0.5 * (Fc[im] - a * Uc[im]);
            }
            double w0[3], w1[3];
            const double rp = weno5(vp, c->p.weno_eps, w0);
            const double rm = weno5(vm, c->p.weno_eps, w1);
            Fhat[(k + 1) * 3 + m] = rp + rm;
            if (m == mb) {
                memcpy(wp, w0, sizeof wp);
                memcpy(wm, w1, sizeof wm);
            }
        }
        double bp[5], bm[5];
        for (int s = 0; s < 5; s++) {
            bp[s] = lb[k - 2 + s];
            bm[s] = lb[k + 3 - s];
        }
        bhat[k + 1] = 0.5 * (weno5_with_weights(bp, wp) + weno5_with_weights(bm, wm));
    }
    for (int k = 0; k < n; k++) {
        div0[k] = -(Fhat[(k + 1) * 3 + 0] - Fhat[k * 3 + 0]) / ds;
        div1[k] = -(Fhat[(k + 1) * 3 + 1] - Fhat[k * 3 + 1]) / ds;
        div2[k] = -(Fhat[(k + 1) * 3 + 2] - Fhat[k * 3 + 2]) / ds;
        dbh[k] = bhat[k + 1] - bhat[k];
    }
}

static void rhs(oracle_ctx *c, const double *h, const double *hu, const double *hv,
                double ax, double ay, double dt)
{
    const int nx = c->p.nx, ny = c->p.ny;
    const double g = c->p.g;

    /* x faces, one row at a time */
#pragma omp parallel
    {
        const int nmax = (nx > ny ? nx : ny) + 2 * HALO;
        double *lh = malloc(sizeof(double) * nmax * 4);
        double *lhu = lh + nmax, *lhv = lh + 2 * nmax, *lb = lh + 3 * nmax;
        double *Fc = malloc(sizeof(double) * nmax * 7);
        double *Uc = Fc + nmax * 3, *sp = Fc + nmax * 6;
        double *Fhat = malloc(sizeof(double) * (nmax + 1) * 3);
        double *bhat = malloc(sizeof(double) * (nmax + 1));
        double *d0 = malloc(sizeof(double) * nmax * 4);
        double *d1 = d0 + nmax, *d2 = d0 + 2 * nmax, *db = d0 + 3 * nmax;

#pragma omp for schedule(static)
        for (int j = 0; j < ny; j++) {
            for (int k = -HALO; k < nx + HALO; k++) {
                const size_t e = IX(c, k, j);
                lh[k + HALO] = h[e]; lhu[k + HALO] = hu[e];
                lhv[k + HALO] = hv[e]; lb[k + HALO] = c->b[e];
            }
            line_faces(c, 0, nx, ax, c->p.dx, lh + HALO, lhu + HALO, lhv + HALO, lb + HALO,
                       d0, d1, d2, db, Fc, Uc, sp, Fhat, bhat);
            for (int i = 0; i < nx; i++) {
                const size_t o = II(c, i, j);
                const double eta = h[IX(c, i, j)] + datum_bed(c->b[IX(c, i, j)]);
                c->fx[0][o] = d0[i];
                c->fx[1][o] = d1[i];
                c->fx[2][o] = d2[i];
                c->bedx[o] = -g * eta * db[i] / c->p.dx;
            }
        }

#pragma omp for schedule(static)
        for (int i = 0; i < nx; i++) {
            for (int k = -HALO; k < ny + HALO; k++) {
                const size_t e = IX(c, i, k);
                lh[k + HALO] = h[e]; lhu[k + HALO] = hu[e];
                lhv[k + HALO] = hv[e]; lb[k + HALO] = c->b[e];
            }
            line_faces(c, 1, ny, ay, c->p.dy, lh + HALO, lhu + HALO, lhv + HALO, lb + HALO,
                       d0, d1, d2, db, Fc, Uc, sp, Fhat, bhat);
            for (int j = 0; j < ny; j++) {
                const size_t o = II(c, i, j);
                const double eta = h[IX(c, i, j)] + datum_bed(c->b[IX(c, i, j)]);
                c->gy[0][o] = d0[j];
                c->gy[1][o] = d1[j];
                c->gy[2][o] = d2[j];
                c->bedy[o] = -g * eta * db[j] / c->p.dy;
            }
        }
        free(lh); free(Fc); free(Fhat); free(bhat); free(d0);
    }

    /* sources and assembly: L = ((-dF/dx) + (-dG/dy)) + S */
    const int implicit = c->friction_implicit;
    const double cap = (!implicit && c->p.kappa_cap > 0.0 && dt > 0.0) ? c->p.kappa_cap / dt : INFINITY;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            const size_t e = IX(c, i, j), o = II(c, i, j);
            double kappa = 0.0;
            if (h[e] > c->p.h_dry && c->gn2[o] > 0.0) {
                const double qn = sqrt(hu[e] * hu[e] + hv[e] * hv[e]);
                kappa = c->gn2[o] * qn / pow(h[e], 7.0 / 3.0);
                if (kappa > cap)
                    kappa = cap;
            }
            c->kap[o] = kappa;
            if (implicit)
                kappa = 0.0; /* R10: taken in the combination instead */
            c->Lh[o] = c->fx[0][o] + c->gy[0][o];
            c->Lhu[o] = (c->fx[1][o] + c->gy[1][o]) + (c->bedx[o] - kappa * hu[e]);
            c->Lhv[o] = (c->fx[2][o] + c->gy[2][o]) + (c->bedy[o] - kappa * hv[e]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* TVD-RK3 stage combination, Eq. (8), and the wet/dry fix-up (R7).          */
/* out = an * un + aw * (w + dt L(w))                                         */
/* ------------------------------------------------------------------------ */

static void combine(oracle_ctx *c, double an, double aw, double weight, double dt,
                    const double *hn, const double *hun, const double *hvn,
                    const double *hw, const double *huw, const double *hvw,
                    double *ho, double *huo, double *hvo)
{
    const int nx = c->p.nx, ny = c->p.ny;
    double added = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : added)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            const size_t e = IX(c, i, j), o = II(c, i, j);
            double nh = hw[e] + dt * c->Lh[o];
            double nhu = huw[e] + dt * c->Lhu[o];
            double nhv = hvw[e] + dt * c->Lhv[o];
            if (an != 0.0) {
                nh = an * hn[e] + aw * nh;
                nhu = an * hun[e] + aw * nhu;
                nhv = an * hvn[e] + aw * nhv;
            }
            if (c->friction_implicit) {
                const double den = 1.0 + aw * dt * c->kap[o];
                nhu /= den;
                nhv /= den;
            }
            if (nh < 0.0) {
                added += -nh;
                nh = 0.0;
            }
            if (nh <= c->p.h_dry) {
                nhu = 0.0;
                nhv = 0.0;
            }
            ho[e] = nh;
            huo[e] = nhu;
            hvo[e] = nhv;
        }
    }
    c->clamp_mass += weight * added * c->p.dx * c->p.dy;
}

static void diagnostics(oracle_ctx *c)
{
    const int nx = c->p.nx, ny = c->p.ny;
    double m = 0.0, r = c->runup;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            const size_t e = IX(c, i, j);
            m += c->h[e];
            if (c->b[e] > 0.0 && c->h[e] > c->p.h_dry && c->b[e] > r)
                r = c->b[e];
        }
    c->mass = m * c->p.dx * c->p.dy;
    c->runup = r;
}

/* ------------------------------------------------------------------------ */
/* Public entry points                                                        */
/* ------------------------------------------------------------------------ */

void oracle_destroy(oracle_ctx *c)
{
    if (!c)
        return;
    double **arrs[] = {&c->b, &c->gn2, &c->h, &c->hu, &c->hv, &c->h1, &c->hu1, &c->hv1,
                       &c->h2, &c->hu2, &c->hv2, &c->Lh, &c->Lhu, &c->Lhv,
                       &c->fx[0], &c->fx[1], &c->fx[2], &c->gy[0], &c->gy[1], &c->gy[2],
                       &c->bedx, &c->bedy, &c->kap};
    for (size_t k = 0; k < sizeof arrs / sizeof arrs[0]; k++)
        free(*arrs[k]);
    for (int s = 0; s < 4; s++)
        for (int f = 0; f < 3; f++)
            free(c->ghost[s][f]);
    free(c);
}

/* Returns NULL on invalid input (sizes < 3, non-positive spacing, negative or
 * non-finite fields, unknown boundary kind) or allocation failure. */
oracle_ctx *oracle_create(const oracle_params *p, const double *b, const double *n,
                          const double *h, const double *hu, const double *hv)
{
    if (!p || !b || !n || !h || !hu || !hv)
        return NULL;
    if (p->nx < 3 || p->ny < 3 || !(p->dx > 0.0) || !(p->dy > 0.0) || !(p->g > 0.0))
        return NULL;
    if (p->cfl <= 0.0 && !(p->dt_fixed > 0.0))
        return NULL;
    for (int s = 0; s < 4; s++)
        if (p->bc[s] != BC_REFLECT && p->bc[s] != BC_FIXED)
            return NULL;
    const size_t N = (size_t)p->nx * (size_t)p->ny;
    for (size_t k = 0; k < N; k++) {
        if (!isfinite(b[k]) || !isfinite(n[k]) || !isfinite(h[k]) || !isfinite(hu[k]) ||
            !isfinite(hv[k]) || h[k] < 0.0 || n[k] < 0.0)
            return NULL;
    }
    oracle_ctx *c = calloc(1, sizeof *c);
    if (!c)
        return NULL;
    c->p = *p;
    c->NX = p->nx + 2 * HALO;
    c->NY = p->ny + 2 * HALO;
    const size_t E = (size_t)c->NX * (size_t)c->NY;
    double **ext[] = {&c->b, &c->h, &c->hu, &c->hv, &c->h1, &c->hu1, &c->hv1,
                      &c->h2, &c->hu2, &c->hv2};
    for (size_t k = 0; k < sizeof ext / sizeof ext[0]; k++)
        if (!(*ext[k] = calloc(E, sizeof(double)))) {
            oracle_destroy(c);
            return NULL;
        }
    double **in[] = {&c->gn2, &c->Lh, &c->Lhu, &c->Lhv, &c->fx[0], &c->fx[1], &c->fx[2],
                     &c->gy[0], &c->gy[1], &c->gy[2], &c->bedx, &c->bedy, &c->kap};
    for (size_t k = 0; k < sizeof in / sizeof in[0]; k++)
        if (!(*in[k] = calloc(N, sizeof(double)))) {
            oracle_destroy(c);
            return NULL;
        }
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            const size_t e = IX(c, i, j), o = II(c, i, j);
            c->b[e] = b[o];
            c->h[e] = h[o];
            c->hu[e] = hu[o];
            c->hv[e] = hv[o];
            c->gn2[o] = p->g * n[o] * n[o];
        }
    fill_bed_ghosts(c);
    /* frozen ghosts for FIXED sides: nearest interior cell at create time */
    for (int s = 0; s < 4; s++) {
        const int len = (s < 2) ? p->ny : p->nx;
        for (int f = 0; f < 3; f++)
            if (!(c->ghost[s][f] = calloc((size_t)HALO * len, sizeof(double)))) {
                oracle_destroy(c);
                return NULL;
            }
        for (int k = 0; k < HALO; k++)
            for (int q = 0; q < len; q++) {
                int i, j;
                if (s == WEST) { i = 0; j = q; }
                else if (s == EAST) { i = p->nx - 1; j = q; }
                else if (s == SOUTH) { i = q; j = 0; }
                else { i = q; j = p->ny - 1; }
                const size_t e = IX(c, i, j);
                c->ghost[s][0][k * len + q] = c->h[e];
                c->ghost[s][1][k * len + q] = c->hu[e];
                c->ghost[s][2][k * len + q] = c->hv[e];
            }
    }
    c->runup = 0.0;
    diagnostics(c);
    fill_ghosts(c, c->h, c->hu, c->hv);
    wave_speeds(c, c->h, c->hu, c->hv, &c->alpha_x, &c->alpha_y);
    return c;
}

/* Advance nsteps full RK3 steps.  Returns 0, or -4 once a wave speed became
 * non-finite (the state is then left as it was when that was detected). */
int oracle_step(oracle_ctx *c, int nsteps)
{
    if (!c)
        return -1;
    for (int s = 0; s < nsteps; s++) {
        if (c->nonfinite)
            return -4;
        double ax, ay;
        /* stage 1: u1 = u^n + dt L(u^n) */
        fill_ghosts(c, c->h, c->hu, c->hv);
        wave_speeds(c, c->h, c->hu, c->hv, &ax, &ay);
        const double dt = time_step(c, ax, ay);
        if (c->nonfinite || !isfinite(dt)) {
            c->nonfinite = 1;
            return -4;
        }
        rhs(c, c->h, c->hu, c->hv, ax, ay, dt);
        combine(c, 0.0, 1.0, 1.0 / 6.0, dt, c->h, c->hu, c->hv, c->h, c->hu, c->hv,
                c->h1, c->hu1, c->hv1);
        /* stage 2: u2 = 3/4 u^n + 1/4 (u1 + dt L(u1)) */
        fill_ghosts(c, c->h1, c->hu1, c->hv1);
        wave_speeds(c, c->h1, c->hu1, c->hv1, &ax, &ay);
        if (c->nonfinite)
            return -4;
        rhs(c, c->h1, c->hu1, c->hv1, ax, ay, dt);
        combine(c, 0.75, 0.25, 2.0 / 3.0, dt, c->h, c->hu, c->hv, c->h1, c->hu1, c->hv1,
                c->h2, c->hu2, c->hv2);
        /* stage 3: u^{n+1} = 1/3 u^n + 2/3 (u2 + dt L(u2)), written over u1 then swapped */
        fill_ghosts(c, c->h2, c->hu2, c->hv2);
        wave_speeds(c, c->h2, c->hu2, c->hv2, &ax, &ay);
        if (c->nonfinite)
            return -4;
        rhs(c, c->h2, c->hu2, c->hv2, ax, ay, dt);
        combine(c, 1.0 / 3.0, 2.0 / 3.0, 1.0, dt, c->h, c->hu, c->hv, c->h2, c->hu2, c->hv2,
                c->h1, c->hu1, c->hv1);
        double *t;
        t = c->h; c->h = c->h1; c->h1 = t;
        t = c->hu; c->hu = c->hu1; c->hu1 = t;
        t = c->hv; c->hv = c->hv1; c->hv1 = t;
        c->t += dt;
        c->dt_last = dt;
        c->step += 1;
        diagnostics(c);
        fill_ghosts(c, c->h, c->hu, c->hv);
        wave_speeds(c, c->h, c->hu, c->hv, &c->alpha_x, &c->alpha_y);
    }
    return c->nonfinite ? -4 : 0;
}

/* R11: 1 selects local Lax-Friedrichs splitting, 0 (default) the global speed. */
void oracle_set_split(oracle_ctx *c, int local)
{
    if (c)
        c->local_alpha = local ? 1 : 0;
}

/* R10: 1 selects point-implicit friction, 0 (default) the explicit term. */
void oracle_set_friction(oracle_ctx *c, int implicit)
{
    if (c)
        c->friction_implicit = implicit ? 1 : 0;
}

/* Copy the interior state (any pointer may be NULL). */
void oracle_read(const oracle_ctx *c, double *h, double *hu, double *hv)
{
    for (int j = 0; j < c->p.ny; j++)
        for (int i = 0; i < c->p.nx; i++) {
            const size_t e = IX(c, i, j), o = II(c, i, j);
            if (h) h[o] = c->h[e];
            if (hu) hu[o] = c->hu[e];
            if (hv) hv[o] = c->hv[e];
        }
}

/* out[0..7] = t, step, mass, clamp_mass, runup, alpha_x, alpha_y, dt of last step */
void oracle_scalars(const oracle_ctx *c, double *out)
{
    out[0] = c->t;
    out[1] = (double)c->step;
    out[2] = c->mass;
    out[3] = c->clamp_mass;
    out[4] = c->runup;
    out[5] = c->alpha_x;
    out[6] = c->alpha_y;
    out[7] = c->dt_last;
}

/* L(u^n) of the current state, with alpha and dt taken from u^n. */
void oracle_rhs(oracle_ctx *c, double *Lh, double *Lhu, double *Lhv)
{
    double ax, ay;
    fill_ghosts(c, c->h, c->hu, c->hv);
    wave_speeds(c, c->h, c->hu, c->hv, &ax, &ay);
    rhs(c, c->h, c->hu, c->hv, ax, ay, time_step(c, ax, ay));
    const size_t N = (size_t)c->p.nx * (size_t)c->p.ny;
    memcpy(Lh, c->Lh, N * sizeof(double));
    memcpy(Lhu, c->Lhu, N * sizeof(double));
    memcpy(Lhv, c->Lhv, N * sizeof(double));
}

/* One stage of the scheme applied to the current state as w = u^n (stage 1:
 * u1 = u^n + dt L(u^n) with the fix-up), written to the outputs; the context
 * is left unchanged apart from its scratch arrays.  Returns dt. */
double oracle_stage1(oracle_ctx *c, double *h, double *hu, double *hv)
{
    double ax, ay;
    fill_ghosts(c, c->h, c->hu, c->hv);
    wave_speeds(c, c->h, c->hu, c->hv, &ax, &ay);
    const double dt = time_step(c, ax, ay);
    rhs(c, c->h, c->hu, c->hv, ax, ay, dt);
    const double keep = c->clamp_mass;
    combine(c, 0.0, 1.0, 1.0 / 6.0, dt, c->h, c->hu, c->hv, c->h, c->hu, c->hv,
            c->h1, c->hu1, c->hv1);
    c->clamp_mass = keep;
    for (int j = 0; j < c->p.ny; j++)
        for (int i = 0; i < c->p.nx; i++) {
            const size_t e = IX(c, i, j), o = II(c, i, j);
            h[o] = c->h1[e];
            hu[o] = c->hu1[e];
            hv[o] = c->hv1[e];
        }
    return dt;
}

/* WENO5-JS reconstruction of one five-point stencil; w receives the weights. */
double oracle_weno5(const double *v, double eps, double *w)
{
    double ww[3];
    const double r = weno5(v, eps, ww);
    if (w)
        memcpy(w, ww, sizeof ww);
    return r;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
