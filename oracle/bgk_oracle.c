/*
 * bgk_oracle.c -- plain FP64 CPU reference of the BGK discrete-velocity step.
 *
 * TEST INFRASTRUCTURE.  This is the oracle the HIP library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark load it.  The library never links, imports or calls it and
 * the two share no code: no header, helper, table or constant generator.
 *
 * What it computes follows Frezzotti, Ghiroldi and Gibelli, "Solving Kinetic
 * Equations on GPUs I: Model Kinetic Equations" (arXiv:0903.4044):
 *   BGKW equation, local Maxwellian ............ Sec. 2, Eqs. (BGKW), (Maxw)
 *   macroscopic moments ........................ Sec. 2, Eq. (macroscopic)
 *   collision frequency ........................ Sec. 2, Eq. (frequency), Sec. 4.1
 *   phase-space grid of point values ........... Sec. 2.1
 *   splitting, exact homogeneous relaxation .... Sec. 2.1, Eq. (relaxation)
 *   upwind free streaming (first-order base) ... Sec. 2.1, Eq. (upwind)
 *   shock far-field states ..................... Sec. 4.1, Eqs. (bc_shock), (RH)
 *   diffuse (fully accommodating) walls ........ Sec. 5.1, Eq. (bc_cavity)
 *
 * Units are the normalised ones of Sec. 4.1: velocity in sqrt(2 R T_r), so
 * that 2RT becomes T and the Maxwellian reads
 *     Phi_j = n (pi T)^(-3/2) exp(-|v_j - V|^2 / T),
 * the temperature moment reads T = (2 / 3n) sum_j |v_j - V|^2 f_j dV, and the
 * collision frequency (Eq. frequency with mu ~ T^omega) is nu = n T^(1-omega)/Kn.
 *
 * Readings of points the paper leaves open (all restated where used):
 *   - streaming is the one-step minmod-limited upwind scheme in flux form;
 *     with the limiter off it is Eq. (upwind) exactly; the paper's own
 *     large-time-step form (Sec. 2.1, below Eq. (exact)) translates each
 *     v_x by the integer part of its Courant number and applies Eq. (upwind)
 *     to the fraction left ("shift" streaming, one-dimensional problems);
 *   - a time step is R_{dt/2} S_dt R_{dt/2} (Strang) or R_dt S_dt (Lie,
 *     the paper's order), every R using the moments of its own input;
 *   - two ghost layers per side: the far-field Maxwellians for the shock,
 *     the diffuse-wall rule of Eq. (bc_cavity) for the cavity;
 *   - dt = CFL / max_j sum_d |v_d(j)| / dx_d over velocity cell centres;
 *   - the reduced velocity space for two-dimensional problems (the
 *     projection the paper cites in Sec. 3 and Sec. 6): f is replaced by
 *     g = int f dv_z and h = int v_z^2 f dv_z on the (v_x, v_y) grid, with
 *     the v_z integrals of Eq. (Maxw) taken exactly and V_z = 0;
 *   - the conservative variant (Sec. 2.1, the remark after Eq. (exact)) takes
 *     the effective (n~, V~, T~) as the exact root of "grid moments of the
 *     discretized Maxwellian = the cell's n, V, T"; the collision frequency
 *     keeps the cell's own n and T; far-field and wall Maxwellians stay point
 *     values (their densities already come from Eq. (RH) and from the
 *     zero-mass-flux rule).
 *
 *   - the three-dimensional extension (Sec. 2.1: the method carries over to
 *     two and three spatial dimensions, one upwind stencil per direction):
 *     a cube with six diffuse walls, the lid (y = y1) moving along x.
 *
 * Storage: f[cell][jz][jy][jx] (velocity fastest), cell = (iz * ny + iy) * nx + ix.
 * Everything is double precision.  Loops are plain; OpenMP only splits the
 * loop over spatial cells.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SHOCK 0
#define ORC_CAVITY 1
#define ORC_PERIODIC1 2
#define ORC_PERIODIC2 3
#define ORC_CAVITY3 4
#define ORC_PERIODIC3 5

typedef struct {
    int kind;
    int nx, ny;
    double x0, x1, y0, y1;
    int nv[3];
    double vlo[3], vhi[3];
    double kn, omega;
    double cfl, dt;
    double mach;
    double lid_mach;
    double t_wall;
    int strang; /* 1: R_{dt/2} S R_{dt/2}; 0: R_dt S (Lie) */
    int minmod; /* 1: minmod slopes; 0: first-order upwind; 2: shift + first-order upwind */
    int conservative; /* 1: relaxations use the effective Maxwellian parameters */
    int reduced; /* 1: the velocity components the problem does not stream along are
                    integrated out: v_z for two-dimensional kinds (nv[2] = 2; plane jz = 0
                    holds g = int f dv_z, plane 1 h = int v_z^2 f dv_z), v_y and v_z for
                    one-dimensional kinds (nv[1] = 1, nv[2] = 2; g = int f dv_y dv_z,
                    h = int (v_y^2 + v_z^2) f dv_y dv_z) */
    int nz;         /* three-dimensional kinds: cells along z */
    double z0, z1;  /* and the box along z */
} orc_problem;

static const double GAMMA = 5.0 / 3.0;

/* ------------------------------------------------------------------ grid */

static int is3d(const orc_problem *p) { return p->kind == ORC_CAVITY3 || p->kind == ORC_PERIODIC3; }
static int is2d(const orc_problem *p) { return p->kind == ORC_CAVITY || p->kind == ORC_PERIODIC2; }
/* streaming directions of the problem */
static int ndim(const orc_problem *p) { return is3d(p) ? 3 : is2d(p) ? 2 : 1; }
static long ncell(const orc_problem *p)
{
    return (long)p->nx * (ndim(p) >= 2 ? p->ny : 1) * (ndim(p) == 3 ? p->nz : 1);
}
static long nvel(const orc_problem *p) { return (long)p->nv[0] * p->nv[1] * p->nv[2]; }
/* number of velocity components integrated out (0: full velocity space) */
static int nred(const orc_problem *p) { return p->reduced ? (is2d(p) ? 1 : 2) : 0; }

static double dvel(const orc_problem *p, int a)
{
    if (a == 2 && nred(p) >= 1) return 1.0; /* the two planes are integrals over v_z */
    if (a == 1 && nred(p) == 2) return 1.0; /* and over v_y */
    return (p->vhi[a] - p->vlo[a]) / p->nv[a];
}
static double dvol(const orc_problem *p) { return dvel(p, 0) * dvel(p, 1) * dvel(p, 2); }
static double dxs(const orc_problem *p) { return (p->x1 - p->x0) / p->nx; }
static double dys(const orc_problem *p) { return (p->y1 - p->y0) / p->ny; }
static double dzs(const orc_problem *p) { return (p->z1 - p->z0) / p->nz; }

/* Velocity of every node, Sec. 2.1: cell centres of a box cut into equal
 * cells, v_a(k) = lo_a + (k + 1/2) dv_a.  Returned as three arrays of Nv,
 * with two weights per node: m, the node's share in mass and momentum, and
 * e, an energy term beyond m |v|^2.  Full velocity space: m = 1, e = 0.
 * Reduced (v_z integrated out, the projection the paper cites in Sec. 3 and
 * Sec. 6): v_z = 0 on both planes; the g plane has m = 1, e = 0 and the h
 * plane m = 0, e = 1 (h already is the v_z^2 moment). */
typedef struct { double *vx, *vy, *vz, *m, *e; long nv; int reduced; } velgrid; /* reduced: components out */

static velgrid make_velgrid(const orc_problem *p)
{
    velgrid g;
    g.nv = nvel(p);
    g.reduced = nred(p);
    g.vx = malloc(sizeof(double) * g.nv);
    g.vy = malloc(sizeof(double) * g.nv);
    g.vz = malloc(sizeof(double) * g.nv);
    g.m = malloc(sizeof(double) * g.nv);
    g.e = malloc(sizeof(double) * g.nv);
    for (int jz = 0; jz < p->nv[2]; ++jz)
        for (int jy = 0; jy < p->nv[1]; ++jy)
            for (int jx = 0; jx < p->nv[0]; ++jx) {
                long j = ((long)jz * p->nv[1] + jy) * p->nv[0] + jx;
                g.vx[j] = p->vlo[0] + (jx + 0.5) * dvel(p, 0);
                g.vy[j] = nred(p) == 2 ? 0.0 : p->vlo[1] + (jy + 0.5) * dvel(p, 1);
                if (p->reduced) {
                    g.vz[j] = 0.0;
                    g.m[j] = jz == 0 ? 1.0 : 0.0;
                    g.e[j] = jz == 0 ? 0.0 : 1.0;
                } else {
                    g.vz[j] = p->vlo[2] + (jz + 0.5) * dvel(p, 2);
                    g.m[j] = 1.0;
                    g.e[j] = 0.0;
                }
            }
    return g;
}

static void free_velgrid(velgrid *g) { free(g->vx); free(g->vy); free(g->vz); free(g->m); free(g->e); }

void orc_velocity_nodes(const orc_problem *p, double *vx, double *vy, double *vz)
{
    velgrid g = make_velgrid(p);
    memcpy(vx, g.vx, sizeof(double) * g.nv);
    memcpy(vy, g.vy, sizeof(double) * g.nv);
    memcpy(vz, g.vz, sizeof(double) * g.nv);
    free_velgrid(&g);
}

/* Time step.  The paper fixes dt as a fraction of the collision time and
 * handles Courant numbers above one by shifting (Sec. 2.1); the workloads
 * here fix a Courant number instead: dt = CFL / max_j sum_d |v_d(j)|/dx_d. */
double orc_dt(const orc_problem *p)
{
    if (p->dt > 0.0) return p->dt;
    double m = 0.0;
    for (int jx = 0; jx < p->nv[0]; ++jx) {
        double ax = fabs(p->vlo[0] + (jx + 0.5) * dvel(p, 0)) / dxs(p);
        if (ndim(p) == 1) { if (ax > m) m = ax; continue; }
        for (int jy = 0; jy < p->nv[1]; ++jy) {
            double ay = fabs(p->vlo[1] + (jy + 0.5) * dvel(p, 1)) / dys(p);
            if (ndim(p) == 2) { if (ax + ay > m) m = ax + ay; continue; }
            for (int jz = 0; jz < p->nv[2]; ++jz) {
                double az = fabs(p->vlo[2] + (jz + 0.5) * dvel(p, 2)) / dzs(p);
                if (ax + ay + az > m) m = ax + ay + az;
            }
        }
    }
    return p->cfl / m;
}

/* ------------------------------------------------------------- physics */

/* Local Maxwellian, Eq. (Maxw), in normalised units. */
/* Reduced velocity space: the integrals of Eq. (Maxw) over the components
 * taken out (V = 0 along them),
 *   over v_z:      int Phi dv_z = n (pi T)^-1 exp(-((v_x - V_x)^2 + (v_y - V_y)^2) / T),
 *                  int v_z^2 Phi dv_z = (T / 2) times that;
 *   over v_y, v_z: int Phi = n (pi T)^-1/2 exp(-(v_x - V_x)^2 / T),
 *                  int (v_y^2 + v_z^2) Phi = T times that. */
static void maxwellian_on(const velgrid *g, double n, const double V[3], double T, double *phi)
{
    if (g->reduced) {
        const double pre = g->reduced == 1 ? n / (M_PI * T) : n / sqrt(M_PI * T);
        const double hfac = g->reduced == 1 ? 0.5 * T : T;
        for (long j = 0; j < g->nv; ++j) {
            double cx = g->vx[j] - V[0], cy = g->vy[j] - V[1];
            phi[j] = pre * exp(-(cx * cx + cy * cy) / T) * (g->m[j] != 0.0 ? 1.0 : hfac);
        }
        return;
    }
    double pre = n * pow(M_PI * T, -1.5);
    for (long j = 0; j < g->nv; ++j) {
        double cx = g->vx[j] - V[0], cy = g->vy[j] - V[1], cz = g->vz[j] - V[2];
        phi[j] = pre * exp(-(cx * cx + cy * cy + cz * cz) / T);
    }
}

void orc_maxwellian(const orc_problem *p, double n, const double V[3], double T, double *phi)
{
    velgrid g = make_velgrid(p);
    maxwellian_on(&g, n, V, T, phi);
    free_velgrid(&g);
}

/* Macroscopic moments of one cell, Eq. (macroscopic), as velocity sums over
 * the piecewise-constant f of Sec. 2.1:  n = sum f dV,  V = sum v f dV / n,
 * T = (2/3) sum |v - V|^2 f dV / n  (second pass about the mean). */
static void cell_moments(const velgrid *g, double dV, const double *f, double *n, double V[3], double *T)
{
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    for (long j = 0; j < g->nv; ++j) {
        s0 += g->m[j] * f[j];
        sx += g->m[j] * g->vx[j] * f[j];
        sy += g->m[j] * g->vy[j] * f[j];
        sz += g->m[j] * g->vz[j] * f[j];
    }
    *n = s0 * dV;
    V[0] = sx * dV / *n;
    V[1] = sy * dV / *n;
    V[2] = sz * dV / *n;
    double s2 = 0.0;
    for (long j = 0; j < g->nv; ++j) {
        double cx = g->vx[j] - V[0], cy = g->vy[j] - V[1], cz = g->vz[j] - V[2];
        s2 += (g->m[j] * (cx * cx + cy * cy + cz * cz) + g->e[j]) * f[j];
    }
    *T = 2.0 / 3.0 * s2 * dV / *n;
}

/* mom[cell][5] = (n, Vx, Vy, Vz, T). */
void orc_moments(const orc_problem *p, const double *f, double *mom)
{
    velgrid g = make_velgrid(p);
    const long nc = ncell(p), nv = nvel(p);
    const double dV = dvol(p);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c)
        cell_moments(&g, dV, f + c * nv, &mom[5 * c], &mom[5 * c + 1], &mom[5 * c + 4]);
    free_velgrid(&g);
}

/* Collision frequency, Eq. (frequency) with a power-law viscosity
 * (Eq. viscosity, exponent omega), normalised as in Sec. 4.1. */
double orc_collision_frequency(const orc_problem *p, double n, double T)
{
    return n * pow(T, 1.0 - p->omega) / p->kn;
}

/* ------------------------------------------ effective Maxwellian parameters */

/* Solves the 5x5 system A x = b in place (Gaussian elimination with partial
 * pivoting); returns 0, or -1 for a singular matrix. */
static int solve5(double A[5][5], double b[5])
{
    for (int k = 0; k < 5; ++k) {
        int piv = k;
        for (int r = k + 1; r < 5; ++r)
            if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
        if (A[piv][k] == 0.0) return -1;
        if (piv != k) {
            for (int c = 0; c < 5; ++c) {
                double t = A[k][c];
                A[k][c] = A[piv][c];
                A[piv][c] = t;
            }
            double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int r = k + 1; r < 5; ++r) {
            double m = A[r][k] / A[k][k];
            for (int c = k; c < 5; ++c) A[r][c] -= m * A[k][c];
            b[r] -= m * b[k];
        }
    }
    for (int k = 4; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < 5; ++c) s -= A[k][c] * b[c];
        b[k] = s / A[k][k];
    }
    return 0;
}

/* Effective Maxwellian parameters (Sec. 2.1, the remark on conservation
 * after Eq. (exact)).  The point values of Eq. (Maxw) taken with a cell's
 * (n, V, T) do not have exactly those moments on the velocity grid.  The
 * effective values q = (n~, V~, T~) are the ones whose discretized Maxwellian
 * has them:   M(Phi(q)) = (n, V, T),   M being the grid moments of
 * Eq. (macroscopic) (cell_moments above).  The root is found by Newton's
 * method started at (n, V, T), with the Jacobian of M(Phi(q)) from the chain
 * rule over the grid nodes, at Phi(q)'s own moments (nd, Vd, Td):
 *   d nd / d Phi_j   = dV,
 *   d Vd_a / d Phi_j = dV (v_a - Vd_a) / nd,
 *   d Td / d Phi_j   = (2/3) dV (|v - Vd|^2 - 3 Td / 2) / nd,
 *   d Phi_j / d n~   = Phi_j / n~,
 *   d Phi_j / d V~_a = Phi_j 2 (v_a - V~_a) / T~,
 *   d Phi_j / d T~   = Phi_j (|v - V~|^2 / T~^2 - 3 / (2 T~)).
 * The iteration stops once a step changes no parameter by more than 1e-14 of
 * its scale (n~, sqrt(T~), T~), after one more step, or after 60 steps.
 * phi is scratch of nv doubles.  Returns the number of Newton steps taken. */
static int effective_parameters(const velgrid *g, double dV, double n, const double V[3], double T, double q[5],
                                double *phi)
{
    q[0] = n;
    q[1] = V[0];
    q[2] = V[1];
    q[3] = V[2];
    q[4] = T;
    int it = 0, polish = 0;
    while (it < 60) {
        double nd, Vd[3], Td;
        maxwellian_on(g, q[0], q + 1, q[4], phi);
        cell_moments(g, dV, phi, &nd, Vd, &Td);
        double J[5][5] = {{0}}, r[5] = {nd - n, Vd[0] - V[0], Vd[1] - V[1], Vd[2] - V[2], Td - T};
        for (long j = 0; j < g->nv; ++j) {
            const double v[3] = {g->vx[j], g->vy[j], g->vz[j]}, m = g->m[j];
            double dM[5], dP[5], cd2 = 0.0, ct2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                cd2 += (v[a] - Vd[a]) * (v[a] - Vd[a]);
                ct2 += (v[a] - q[1 + a]) * (v[a] - q[1 + a]);
            }
            dM[0] = m * dV;
            for (int a = 0; a < 3; ++a) dM[1 + a] = m * dV * (v[a] - Vd[a]) / nd;
            dM[4] = 2.0 / 3.0 * dV * (m * cd2 + g->e[j] - 1.5 * Td * m) / nd;
            dP[0] = phi[j] / q[0];
            for (int a = 0; a < 3; ++a) dP[1 + a] = phi[j] * 2.0 * (v[a] - q[1 + a]) / q[4];
            /* T~ enters the prefactor as T~^(-3/2); in the reduced spaces as
             * T~^(-1) (g) and T~^0 (h = (T~/2) g) with v_z out, T~^(-1/2)
             * (g) and T~^(1/2) (h = T~ g) with v_y and v_z out */
            const double k = g->reduced == 1 ? (m != 0.0 ? 1.0 : 0.0)
                           : g->reduced == 2 ? (m != 0.0 ? 0.5 : -0.5) : 1.5;
            dP[4] = phi[j] * (ct2 / (q[4] * q[4]) - k / q[4]);
            for (int row = 0; row < 5; ++row)
                for (int col = 0; col < 5; ++col) J[row][col] += dM[row] * dP[col];
        }
        for (int a = 3 - g->reduced; a < 3 && g->reduced; ++a) { /* V = 0 along the components out */
            for (int k = 0; k < 5; ++k) J[1 + a][k] = J[k][1 + a] = 0.0;
            J[1 + a][1 + a] = 1.0;
            r[1 + a] = 0.0;
        }
        if (solve5(J, r) != 0) break;
        for (int k = 0; k < 5; ++k) q[k] -= r[k];
        ++it;
        const double vs = sqrt(q[4]);
        int small = fabs(r[0]) <= 1e-14 * q[0] && fabs(r[4]) <= 1e-14 * q[4];
        for (int a = 0; a < 3; ++a) small = small && fabs(r[1 + a]) <= 1e-14 * vs;
        if (polish) break;
        if (small) polish = 1;
    }
    return it;
}

/* Effective parameters of the cell moments (n, V, T); q = (n~, V~, T~).
 * Returns the number of Newton steps. */
int orc_effective_parameters(const orc_problem *p, double n, const double V[3], double T, double *q)
{
    velgrid g = make_velgrid(p);
    double *phi = malloc(sizeof(double) * g.nv);
    int it = effective_parameters(&g, dvol(p), n, V, T, q, phi);
    free(phi);
    free_velgrid(&g);
    return it;
}

/* Homogeneous relaxation over a time tau, solved exactly (Eq. relaxation):
 * out = Phi + (f - Phi) exp(-nu tau), Phi and nu from the moments of f.  With
 * p->conservative, Phi is the Maxwellian of the effective parameters (the
 * collision frequency keeps the cell's own n and T), so that Phi, and with it
 * out, has exactly the grid moments of f. */
void orc_relax(const orc_problem *p, const double *f, double *out, double tau)
{
    velgrid g = make_velgrid(p);
    const long nc = ncell(p), nv = nvel(p);
    const double dV = dvol(p);
#pragma omp parallel
    {
        double *phi = malloc(sizeof(double) * nv);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            const double *fc = f + c * nv;
            double n, V[3], T;
            cell_moments(&g, dV, fc, &n, V, &T);
            if (p->conservative) {
                double q[5];
                effective_parameters(&g, dV, n, V, T, q, phi);
                maxwellian_on(&g, q[0], q + 1, q[4], phi);
            } else {
                maxwellian_on(&g, n, V, T, phi);
            }
            double decay = exp(-orc_collision_frequency(p, n, T) * tau);
            for (long j = 0; j < nv; ++j)
                out[c * nv + j] = phi[j] + (fc[j] - phi[j]) * decay;
        }
        free(phi);
    }
    free_velgrid(&g);
}

/* -------------------------------------------------------- boundary states */

/* Rankine-Hugoniot states, Eq. (RH), with upstream n = T = 1 and the Mach
 * number defined below Eq. (RH); V^- = M sqrt(gamma/2) in sqrt(2RT^-) units. */
void orc_rankine_hugoniot(double mach, double up[3], double down[3])
{
    double m2 = mach * mach;
    double r = 4.0 * m2 / (m2 + 3.0);
    up[0] = 1.0;
    up[1] = mach * sqrt(GAMMA / 2.0);
    up[2] = 1.0;
    down[0] = up[0] * r;
    down[1] = up[1] / r;
    down[2] = up[2] * (5.0 * m2 - 1.0) * (m2 + 3.0) / (16.0 * m2);
}

/* Lid speed: the lid Mach number taken at the reference temperature T_r,
 * U_W = Ma sqrt(gamma R T_r) = Ma sqrt(gamma / 2) in sqrt(2RT_r) units.  It
 * does not change with the wall temperature. */
static double lid_speed(const orc_problem *p)
{
    return p->lid_mach * sqrt(GAMMA / 2.0);
}

/* Unit-density wall Maxwellian (pi T_w)^(-3/2) exp(-|v - V_W|^2 / T_w). */
static void wall_maxwellian(const orc_problem *p, const velgrid *g, double uw, double *phi)
{
    double V[3] = {uw, 0.0, 0.0};
    maxwellian_on(g, 1.0, V, p->t_wall, phi);
}

/* Walls are numbered 0 left (x = x0, inward normal +x), 1 right (-x),
 * 2 bottom (y = y0, +y), 3 top / lid (-y, moving with speed U_W along x),
 * and in three dimensions 4 back (z = z0, +z) and 5 front (-z): wall w lies
 * across axis w / 2, on the low side for even w. */
static void wall_normal(int w, int *axis, double *sign)
{
    *axis = w / 2;
    *sign = (w % 2 == 0) ? 1.0 : -1.0;
}

/* Wall density of Eq. (bc_cavity): the emitted Maxwellian carries the mass
 * flux that the gas brings to the wall, so the net flux through the wall is
 * zero.  Both fluxes are the discrete sums over the velocity grid:
 *   n_W = sum_{v.n<0} |v.n| g0 / sum_{v.n>0} (v.n) Phi_W,
 * g0 being the wall-adjacent cell. */
static double wall_density(const velgrid *g, int axis, double sign, const double *g0, const double *phiw)
{
    const double *va = axis == 0 ? g->vx : axis == 1 ? g->vy : g->vz;
    double num = 0.0, den = 0.0;
    for (long j = 0; j < g->nv; ++j) {
        double vn = sign * va[j];
        if (vn < 0.0) num += -vn * g->m[j] * g0[j];
        else if (vn > 0.0) den += vn * g->m[j] * phiw[j];
    }
    return num / den;
}

/* n_W for every wall face of a cavity state g: nw[w * L + k] with
 * L = max(nx, ny), k the cell index along the wall. */
void orc_wall_density(const orc_problem *p, const double *gs, double *nw)
{
    velgrid g = make_velgrid(p);
    const int nx = p->nx, ny = p->ny;
    const long nv = nvel(p);
    const int L = nx > ny ? nx : ny;
    double *rest = malloc(sizeof(double) * nv), *lid = malloc(sizeof(double) * nv);
    wall_maxwellian(p, &g, 0.0, rest);
    wall_maxwellian(p, &g, lid_speed(p), lid);
    for (int w = 0; w < 4; ++w) {
        int axis; double sign;
        wall_normal(w, &axis, &sign);
        int len = axis == 0 ? ny : nx;
        for (int k = 0; k < len; ++k) {
            long c;
            if (w == 0) c = (long)k * nx;
            else if (w == 1) c = (long)k * nx + nx - 1;
            else if (w == 2) c = k;
            else c = (long)(ny - 1) * nx + k;
            nw[w * L + k] = wall_density(&g, axis, sign, gs + c * nv, w == 3 ? lid : rest);
        }
    }
    free(rest); free(lid);
    free_velgrid(&g);
}

/* --------------------------------------------------------------- streaming */

static double minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* Upwind value at the face between u0 and u1 for Courant number C, given the
 * four values (um1, u0, u1, u2) along the direction.  For C > 0 the face takes
 * u0 plus half its limited slope scaled by (1 - C); for C < 0 it mirrors onto
 * u1.  Without the limiter this is the donor cell value of Eq. (upwind). */
static double face_value(double um1, double u0, double u1, double u2, double C, int limit)
{
    if (C > 0.0) return u0 + (limit ? 0.5 * (1.0 - C) * minmod(u1 - u0, u0 - um1) : 0.0);
    if (C < 0.0) return u1 - (limit ? 0.5 * (1.0 + C) * minmod(u2 - u1, u1 - u0) : 0.0);
    return 0.0;
}

/* Free streaming over dt along x by translation (Sec. 2.1, Eq. (exact) and
 * the text below it): the exact solution moves f by v_x dt.  With the
 * Courant number C = v_x dt / dx, |C| = m + th (m its integer part), the
 * value is first taken m cells upwind and Eq. (upwind) is then applied over
 * the fraction th:
 *     out_i = (1 - th) g_{i - s m} + th g_{i - s (m + 1)},   s = sign(v_x).
 * Positions outside [0, nx) hold the far-field Maxwellians of Eq. (bc_shock)
 * (upstream for x < 0) or the periodic images.  One-dimensional problems. */
static void stream_shift(const orc_problem *p, const double *gs, double *out, double dt)
{
    velgrid g = make_velgrid(p);
    const int nx = p->nx;
    const long nv = nvel(p);
    const double dx = dxs(p);
    double *up = 0, *dn = 0;
    if (p->kind == ORC_SHOCK) {
        double su[3], sd[3];
        orc_rankine_hugoniot(p->mach, su, sd);
        double Vu[3] = {su[1], 0, 0}, Vd[3] = {sd[1], 0, 0};
        up = malloc(sizeof(double) * nv);
        dn = malloc(sizeof(double) * nv);
        maxwellian_on(&g, su[0], Vu, su[2], up);
        maxwellian_on(&g, sd[0], Vd, sd[2], dn);
    }
#pragma omp parallel for schedule(static)
    for (int ix = 0; ix < nx; ++ix) {
        double *o = out + (long)ix * nv;
        for (long j = 0; j < nv; ++j) {
            const double C = g.vx[j] * dt / dx;
            const long s = C > 0.0 ? 1 : -1;
            const double a = fabs(C);
            const long m = (long)floor(a);
            const double th = a - (double)m;
            double val[2];
            for (int k = 0; k < 2; ++k) {
                long pos = ix - s * (m + k);
                if (pos >= 0 && pos < nx) val[k] = gs[pos * nv + j];
                else if (p->kind == ORC_SHOCK) val[k] = pos < 0 ? up[j] : dn[j];
                else val[k] = gs[(((pos % nx) + nx) % nx) * nv + j];
            }
            o[j] = (1.0 - th) * val[0] + th * val[1];
        }
    }
    free(up);
    free(dn);
    free_velgrid(&g);
}

/* Free streaming over dt, Eq. (freestreaming), in flux form:
 *   out_i = g_i - sum_d C_d (face_{i+1/2} - face_{i-1/2}),  C_d = v_d dt / dx_d,
 * every face built from the same input g.  g is first copied into an array
 * with two ghost layers on each side of each streaming direction. */
void orc_stream(const orc_problem *p, const double *gs, double *out, double dt)
{
    if (p->minmod == 2) {
        stream_shift(p, gs, out, dt);
        return;
    }
    velgrid g = make_velgrid(p);
    const int dim = ndim(p);
    const int nx = p->nx, ny = dim >= 2 ? p->ny : 1, nz = dim == 3 ? p->nz : 1;
    const long nv = nvel(p);
    /* two ghost layers on each side of each streaming direction */
    const int px = nx + 4, py = dim >= 2 ? ny + 4 : 1, pz = dim == 3 ? nz + 4 : 1;
    const int oy = dim >= 2 ? 2 : 0, oz = dim == 3 ? 2 : 0;
    double *G = malloc(sizeof(double) * (long)px * py * pz * nv);
#define PAD(ix, iy, iz) (G + ((((long)(iz) + oz) * py + (iy) + oy) * px + (ix) + 2) * nv)
#define SRC(ix, iy, iz) (gs + (((long)(iz) * ny + (iy)) * nx + (ix)) * nv)

    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix)
                memcpy(PAD(ix, iy, iz), SRC(ix, iy, iz), sizeof(double) * nv);

    if (p->kind == ORC_SHOCK) {
        /* Far-field states of Eq. (bc_shock) fill both ghost layers. */
        double up[3], dn[3];
        orc_rankine_hugoniot(p->mach, up, dn);
        double Vu[3] = {up[1], 0, 0}, Vd[3] = {dn[1], 0, 0};
        maxwellian_on(&g, up[0], Vu, up[2], PAD(-2, 0, 0));
        maxwellian_on(&g, up[0], Vu, up[2], PAD(-1, 0, 0));
        maxwellian_on(&g, dn[0], Vd, dn[2], PAD(nx, 0, 0));
        maxwellian_on(&g, dn[0], Vd, dn[2], PAD(nx + 1, 0, 0));
    } else if (p->kind == ORC_PERIODIC1 || p->kind == ORC_PERIODIC2 || p->kind == ORC_PERIODIC3) {
        /* periodic images; each direction's stencil only reaches the ghosts
         * along that direction, so no edge or corner ghosts are needed */
        for (int iz = 0; iz < nz; ++iz)
            for (int iy = 0; iy < ny; ++iy) {
                memcpy(PAD(-2, iy, iz), SRC(nx - 2, iy, iz), sizeof(double) * nv);
                memcpy(PAD(-1, iy, iz), SRC(nx - 1, iy, iz), sizeof(double) * nv);
                memcpy(PAD(nx, iy, iz), SRC(0, iy, iz), sizeof(double) * nv);
                memcpy(PAD(nx + 1, iy, iz), SRC(1, iy, iz), sizeof(double) * nv);
            }
        if (dim >= 2)
            for (int iz = 0; iz < nz; ++iz)
                for (int ix = 0; ix < nx; ++ix) {
                    memcpy(PAD(ix, -2, iz), SRC(ix, ny - 2, iz), sizeof(double) * nv);
                    memcpy(PAD(ix, -1, iz), SRC(ix, ny - 1, iz), sizeof(double) * nv);
                    memcpy(PAD(ix, ny, iz), SRC(ix, 0, iz), sizeof(double) * nv);
                    memcpy(PAD(ix, ny + 1, iz), SRC(ix, 1, iz), sizeof(double) * nv);
                }
        if (dim == 3)
            for (int iy = 0; iy < ny; ++iy)
                for (int ix = 0; ix < nx; ++ix) {
                    memcpy(PAD(ix, iy, -2), SRC(ix, iy, nz - 2), sizeof(double) * nv);
                    memcpy(PAD(ix, iy, -1), SRC(ix, iy, nz - 1), sizeof(double) * nv);
                    memcpy(PAD(ix, iy, nz), SRC(ix, iy, 0), sizeof(double) * nv);
                    memcpy(PAD(ix, iy, nz + 1), SRC(ix, iy, 1), sizeof(double) * nv);
                }
    } else {
        /* Diffuse walls, Eq. (bc_cavity).  For velocities leaving the wall
         * (v.n > 0) both ghosts hold n_W Phi_W; for velocities arriving at it
         * both ghosts repeat the wall-adjacent cell, so the wall face takes
         * that cell's value and the net mass flux through it is exactly zero. */
        double *rest = malloc(sizeof(double) * nv), *lid = malloc(sizeof(double) * nv);
        wall_maxwellian(p, &g, 0.0, rest);
        wall_maxwellian(p, &g, lid_speed(p), lid);
        const int N[3] = {nx, ny, nz};
        for (int w = 0; w < 2 * dim; ++w) {
            int axis; double sign;
            wall_normal(w, &axis, &sign);
            const double *va = axis == 0 ? g.vx : axis == 1 ? g.vy : g.vz;
            const double *phiw = w == 3 ? lid : rest;
            /* the face's cells run over the two other coordinates */
            const int b1 = axis == 0 ? 1 : 0, b2 = axis == 2 ? 1 : 2;
            for (int k2 = 0; k2 < N[b2]; ++k2)
                for (int k1 = 0; k1 < N[b1]; ++k1) {
                    int a[3], d1[3], d2[3];
                    a[b1] = d1[b1] = d2[b1] = k1;
                    a[b2] = d1[b2] = d2[b2] = k2;
                    a[axis] = sign > 0.0 ? 0 : N[axis] - 1;
                    d1[axis] = sign > 0.0 ? -1 : N[axis];
                    d2[axis] = sign > 0.0 ? -2 : N[axis] + 1;
                    const double *g0 = SRC(a[0], a[1], a[2]);
                    double nW = wall_density(&g, axis, sign, g0, phiw);
                    double *q1 = PAD(d1[0], d1[1], d1[2]), *q2 = PAD(d2[0], d2[1], d2[2]);
                    for (long j = 0; j < nv; ++j) {
                        double v = sign * va[j] > 0.0 ? nW * phiw[j] : g0[j];
                        q1[j] = v;
                        q2[j] = v;
                    }
                }
        }
        free(rest); free(lid);
    }

    const double dx = dxs(p), dy = dim >= 2 ? dys(p) : 1.0, dz = dim == 3 ? dzs(p) : 1.0;
    const int limit = p->minmod;
#pragma omp parallel for collapse(3) schedule(static)
    for (int iz = 0; iz < nz; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                const double *xm2 = PAD(ix - 2, iy, iz), *xm1 = PAD(ix - 1, iy, iz), *c0 = PAD(ix, iy, iz),
                             *xp1 = PAD(ix + 1, iy, iz), *xp2 = PAD(ix + 2, iy, iz);
                double *o = out + (((long)iz * ny + iy) * nx + ix) * nv;
                for (long j = 0; j < nv; ++j) {
                    double Cx = g.vx[j] * dt / dx;
                    double r = c0[j] - Cx * (face_value(xm1[j], c0[j], xp1[j], xp2[j], Cx, limit) -
                                             face_value(xm2[j], xm1[j], c0[j], xp1[j], Cx, limit));
                    if (dim >= 2) {
                        const double *ym2 = PAD(ix, iy - 2, iz), *ym1 = PAD(ix, iy - 1, iz),
                                     *yp1 = PAD(ix, iy + 1, iz), *yp2 = PAD(ix, iy + 2, iz);
                        double Cy = g.vy[j] * dt / dy;
                        r -= Cy * (face_value(ym1[j], c0[j], yp1[j], yp2[j], Cy, limit) -
                                   face_value(ym2[j], ym1[j], c0[j], yp1[j], Cy, limit));
                    }
                    if (dim == 3) {
                        const double *zm2 = PAD(ix, iy, iz - 2), *zm1 = PAD(ix, iy, iz - 1),
                                     *zp1 = PAD(ix, iy, iz + 1), *zp2 = PAD(ix, iy, iz + 2);
                        double Cz = g.vz[j] * dt / dz;
                        r -= Cz * (face_value(zm1[j], c0[j], zp1[j], zp2[j], Cz, limit) -
                                   face_value(zm2[j], zm1[j], c0[j], zp1[j], Cz, limit));
                    }
                    o[j] = r;
                }
            }
#undef PAD
#undef SRC
    free(G);
    free_velgrid(&g);
}

/* ------------------------------------------------------------ time step */

/* One time step (Sec. 2.1).  Strang: out = R_{dt/2}(S_dt(R_{dt/2}(f))).
 * Lie (the paper's order): out = R_dt(S_dt(f)). */
void orc_step(const orc_problem *p, const double *f, double *out)
{
    const double dt = orc_dt(p);
    const long n = ncell(p) * nvel(p);
    double *a = malloc(sizeof(double) * n);
    if (p->strang) {
        double *b = malloc(sizeof(double) * n);
        orc_relax(p, f, a, 0.5 * dt);
        orc_stream(p, a, b, dt);
        orc_relax(p, b, out, 0.5 * dt);
        free(b);
    } else {
        orc_stream(p, f, a, dt);
        orc_relax(p, a, out, dt);
    }
    free(a);
}

/* nsteps steps in place on f. */
void orc_run(const orc_problem *p, double *f, int nsteps)
{
    const long n = ncell(p) * nvel(p);
    double *t = malloc(sizeof(double) * n);
    for (int s = 0; s < nsteps; ++s) {
        orc_step(p, f, t);
        memcpy(f, t, sizeof(double) * n);
    }
    free(t);
}

/* Initial states: the Rankine-Hugoniot step of Sec. 4.1 (upstream state for
 * x < 0, downstream for x >= 0); the gas at rest, n = T = 1, otherwise. */
void orc_initial_state(const orc_problem *p, double *f)
{
    velgrid g = make_velgrid(p);
    const long nc = ncell(p), nv = nvel(p);
    if (p->kind == ORC_SHOCK) {
        double up[3], dn[3];
        orc_rankine_hugoniot(p->mach, up, dn);
        double Vu[3] = {up[1], 0, 0}, Vd[3] = {dn[1], 0, 0};
        for (long c = 0; c < nc; ++c) {
            double x = p->x0 + (c + 0.5) * dxs(p);
            if (x < 0.0) maxwellian_on(&g, up[0], Vu, up[2], f + c * nv);
            else maxwellian_on(&g, dn[0], Vd, dn[2], f + c * nv);
        }
    } else {
        double V[3] = {0, 0, 0};
        for (long c = 0; c < nc; ++c) maxwellian_on(&g, 1.0, V, 1.0, f + c * nv);
    }
    free_velgrid(&g);
}

/* ------------------------------------------------------------ diagnostics */

/* Domain totals of mass, momentum (3) and energy sum |v|^2 f, and the
 * entropy functional sum f ln f, all times dV and the cell size. */
void orc_totals(const orc_problem *p, const double *f, double *tot /* [6] */)
{
    velgrid g = make_velgrid(p);
    const long nc = ncell(p), nv = nvel(p);
    const double w = dvol(p) * dxs(p) * (ndim(p) >= 2 ? dys(p) : 1.0) * (ndim(p) == 3 ? dzs(p) : 1.0);
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (long c = 0; c < nc; ++c)
        for (long j = 0; j < nv; ++j) {
            double v = f[c * nv + j], mv = g.m[j] * v;
            s[0] += mv;
            s[1] += g.vx[j] * mv;
            s[2] += g.vy[j] * mv;
            s[3] += g.vz[j] * mv;
            s[4] += (g.vx[j] * g.vx[j] + g.vy[j] * g.vy[j] + g.vz[j] * g.vz[j]) * mv + g.e[j] * v;
            if (mv > 0.0) s[5] += mv * log(mv);
        }
    for (int k = 0; k < 6; ++k) tot[k] = s[k] * w;
    free_velgrid(&g);
}

/* Lid shear: the flux of x-momentum through the lid face, built with the
 * same ghost rule as the streaming step (gas leaving the top row for
 * v_y > 0, wall Maxwellian n_W Phi_W entering for v_y < 0), summed along
 * the lid: L = sum_i dx [sum_{vy>0} vx vy f dV + n_W,i sum_{vy<0} vx vy Phi_W dV]. */
double orc_lid_shear(const orc_problem *p, const double *f)
{
    if (ndim(p) == 3) return NAN; /* defined for the two-dimensional cavity */
    velgrid g = make_velgrid(p);
    const int nx = p->nx, ny = p->ny;
    const long nv = nvel(p);
    const double dV = dvol(p), dx = dxs(p);
    double *lid = malloc(sizeof(double) * nv);
    wall_maxwellian(p, &g, lid_speed(p), lid);
    double L = 0.0;
    for (int ix = 0; ix < nx; ++ix) {
        const double *ft = f + ((long)(ny - 1) * nx + ix) * nv;
        double nW = wall_density(&g, 1, -1.0, ft, lid);
        double s_in = 0.0, s_out = 0.0;
        for (long j = 0; j < nv; ++j) {
            if (g.vy[j] > 0.0) s_in += g.m[j] * g.vx[j] * g.vy[j] * ft[j];
            else if (g.vy[j] < 0.0) s_out += g.m[j] * g.vx[j] * g.vy[j] * lid[j];
        }
        L += dx * (s_in + nW * s_out) * dV;
    }
    free(lid);
    free_velgrid(&g);
    return L;
}

/* Steady-cavity metrics compared in the Table of Sec. 5.2, for a lid speed
 * U_W and a gas initially at rest with n = T = 1 (pressure p0 = nT/2 = 1/2 in
 * these units):
 *   D, the mean shear stress on the lid in units of p0 U_W:
 *        D = -L / (p0 U_W W), L = orc_lid_shear (the lid's xy-momentum
 *        flux integrated over the lid width W);
 *   G, the flow rate of the main vortex: the integral of u = V_x / U_W along
 *        the vertical line through the middle of the cavity (the middle
 *        column, or the mean of the two middle columns for even nx), from
 *        the vortex centre (the zero of u met first going down from the lid)
 *        up to the lid, in units of the height H, as Sec. 5.2 defines it (the
 *        paper gives no further normalisation).
 * u is taken as linear between cell centres (the zero by linear
 * interpolation) and extrapolated linearly over the half cell next to the
 * lid; with no zero the integral starts at the bottom wall. */
void orc_cavity_metrics(const orc_problem *p, const double *f, double *out /* [2] */)
{
    const int nx = p->nx, ny = p->ny;
    const double uw = lid_speed(p), W = p->x1 - p->x0, H = p->y1 - p->y0, dy = H / ny;
    if (p->kind != ORC_CAVITY || uw == 0.0) { /* defined for a cavity with a moving lid */
        out[0] = out[1] = NAN;
        return;
    }
    out[0] = -orc_lid_shear(p, f) / (0.5 * uw * W);
    double *mom = malloc(sizeof(double) * 5 * ncell(p));
    double *u = malloc(sizeof(double) * ny);
    orc_moments(p, f, mom);
    for (int iy = 0; iy < ny; ++iy) {
        double vx;
        if (nx % 2) vx = mom[5 * ((long)iy * nx + nx / 2) + 1];
        else vx = 0.5 * (mom[5 * ((long)iy * nx + nx / 2 - 1) + 1] + mom[5 * ((long)iy * nx + nx / 2) + 1]);
        u[iy] = vx / uw;
    }
    int top = ny - 1;
    while (top > 0 && u[top - 1] > 0.0) --top; /* u > 0 on rows top .. ny-1 */
    double G = 0.0;
    if (top > 0 && u[top] > 0.0) {
        /* zero between the centres of rows top-1 and top */
        double frac = u[top] / (u[top] - u[top - 1]);
        G += 0.5 * u[top] * frac * dy;
    } else if (top == 0) {
        /* no zero: from the bottom wall, u extrapolated over its half cell */
        double ub = ny > 1 ? u[0] - 0.5 * (u[1] - u[0]) : u[0];
        G += 0.25 * dy * (ub + u[0]);
    }
    for (int iy = top; iy < ny - 1; ++iy) G += 0.5 * (u[iy] + u[iy + 1]) * dy;
    double ulid = ny > 1 ? u[ny - 1] + 0.5 * (u[ny - 1] - u[ny - 2]) : u[ny - 1];
    G += 0.25 * dy * (u[ny - 1] + ulid);
    out[1] = G / H;
    free(u);
    free(mom);
}


/* ================================================================ adjoint
 *
 * Reverse sweep of the discrete map above, derived by hand.  For a scalar
 * loss L of f^N the adjoint state lambda^n = dL/df^n obeys
 *     lambda^n = (d f^{n+1} / d f^n)^T lambda^{n+1},
 * with the plain sum over all (cell, velocity) entries as inner product.
 * Parameter gradients (Kn and the wall temperature T_w) accumulate the
 * partial derivatives of every sub-step.  The minmod slope is differentiated
 * on the branch the forward step takes (zero where the two differences
 * disagree in sign, else the difference of smaller magnitude, the second one
 * on a tie).
 */

/* Relaxation R_tau (Eq. relaxation) of one cell, y = (1 - E) Phi + E x with
 * E = exp(-nu tau), Phi and nu from the moments of x.  Given mu = dL/dy,
 * writes xbar = (dy/dx)^T mu and adds dL/dKn to *gkn. */
static void relax_adjoint_cell(const orc_problem *p, const velgrid *g, double dV, const double *x,
                               const double *mu, double tau, double *xbar, double *gkn, double *phi)
{
    double n, V[3], T;
    cell_moments(g, dV, x, &n, V, &T);
    maxwellian_on(g, n, V, T, phi);
    const double nu = orc_collision_frequency(p, n, T), E = exp(-nu * tau);
    double A = 0, B[3] = {0, 0, 0}, C = 0, D = 0;
    for (long j = 0; j < g->nv; ++j) {
        const double c[3] = {g->vx[j] - V[0], g->vy[j] - V[1], g->vz[j] - V[2]};
        const double w = mu[j] * phi[j];
        A += w;
        for (int a = 0; a < 3; ++a) B[a] += w * c[a];
        C += w * (c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        D += mu[j] * (x[j] - phi[j]);
    }
    /* adjoints of n, V, T:  dPhi/dn = Phi/n, dPhi/dV = 2 Phi (v - V)/T,
     * dPhi/dT = Phi (|v - V|^2/T^2 - 3/(2T)), dE/dn = -tau E nu/n,
     * dE/dT = -tau E (1 - omega) nu/T, and dy/dE = x - Phi. */
    const double Gn = (1.0 - E) * A / n - tau * E * nu / n * D;
    double GV[3];
    for (int a = 0; a < 3; ++a) GV[a] = (1.0 - E) * 2.0 * B[a] / T;
    const double GT = (1.0 - E) * (C / (T * T) - 1.5 * A / T) - tau * E * (1.0 - p->omega) * nu / T * D;
    *gkn += tau * E * nu / p->kn * D;  /* dE/dKn = tau E nu / Kn */
    /* chain to the raw sums M0 = n, M1 = n V, M2 = n (|V|^2 + 3T/2), whose
     * derivatives with respect to x_k are dV (1, v_k, |v_k|^2) */
    const double V2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    double G0 = Gn + GT * (2.0 / 3.0) * (V2 - 1.5 * T) / n;
    double G1[3];
    for (int a = 0; a < 3; ++a) {
        G0 -= GV[a] * V[a] / n;
        G1[a] = GV[a] / n - GT * (4.0 / 3.0) * V[a] / n;
    }
    const double G2 = GT * (2.0 / 3.0) / n;
    for (long j = 0; j < g->nv; ++j)
        xbar[j] = E * mu[j] + dV * (G0 + G1[0] * g->vx[j] + G1[1] * g->vy[j] + G1[2] * g->vz[j] +
                                    G2 * (g->vx[j] * g->vx[j] + g->vy[j] * g->vy[j] + g->vz[j] * g->vz[j]));
}

void orc_relax_adjoint(const orc_problem *p, const double *x, const double *mu, double *xbar, double tau, double *gkn)
{
    velgrid g = make_velgrid(p);
    const long nc = ncell(p), nv = nvel(p);
    const double dV = dvol(p);
    double total = 0.0;
#pragma omp parallel reduction(+ : total)
    {
        double *phi = malloc(sizeof(double) * nv);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double gk = 0.0;
            relax_adjoint_cell(p, &g, dV, x + c * nv, mu + c * nv, tau, xbar + c * nv, &gk, phi);
            total += gk;
        }
        free(phi);
    }
    *gkn += total;
    free_velgrid(&g);
}

/* Branch the minmod of (a, b) takes: 0 (slope zero), 1 (a), 2 (b). */
static int minmod_branch(double a, double b)
{
    if (a * b <= 0.0) return 0;
    return fabs(a) < fabs(b) ? 1 : 2;
}

/* Adjoint of one face value (see face_value) for Courant number C: the
 * face depends on (um1, u0, u1, u2) = padded cells (m-1, m, m+1, m+2); w is
 * the adjoint of the face value, accumulated into the padded adjoint. */
static void face_adjoint(double *Gb_m1, double *Gb_0, double *Gb_1, double *Gb_2, double um1, double u0, double u1,
                         double u2, double C, int limit, double w)
{
    if (C > 0.0) {
        *Gb_0 += w;
        if (!limit) return;
        const double s = 0.5 * (1.0 - C) * w;
        const int br = minmod_branch(u1 - u0, u0 - um1);
        if (br == 1) { *Gb_1 += s; *Gb_0 -= s; }
        else if (br == 2) { *Gb_0 += s; *Gb_m1 -= s; }
    } else if (C < 0.0) {
        *Gb_1 += w;
        if (!limit) return;
        const double s = -0.5 * (1.0 + C) * w;
        const int br = minmod_branch(u2 - u1, u1 - u0);
        if (br == 1) { *Gb_2 += s; *Gb_1 -= s; }
        else if (br == 2) { *Gb_1 += s; *Gb_0 -= s; }
    }
}

/* Adjoint of orc_stream at input gs: given mu = dL/d(out), writes
 * gbar = dL/dgs and adds dL/dT_w (through the wall Maxwellian and n_W) to
 * *gtw.  Scatter form over a padded adjoint array, then the transpose of the
 * ghost construction. */
void orc_stream_adjoint(const orc_problem *p, const double *gs, const double *mu, double *gbar, double dt, double *gtw)
{
    velgrid g = make_velgrid(p);
    const int two = is2d(p);
    const int nx = p->nx, ny = two ? p->ny : 1;
    const long nv = nvel(p);
    const int px = nx + 4, py = two ? ny + 4 : 1, oy = two ? 2 : 0;
    const long npad = (long)px * py * nv;
    double *G = malloc(sizeof(double) * npad);
    double *Gb = calloc(npad, sizeof(double));
#define PAD(A, ix, iy) ((A) + ((long)((iy) + oy) * px + (ix) + 2) * nv)
#define SRC(ix, iy) (gs + ((long)(iy) * nx + (ix)) * nv)
    /* forward padded input, built exactly as in orc_stream */
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) memcpy(PAD(G, ix, iy), SRC(ix, iy), sizeof(double) * nv);
    double *rest = malloc(sizeof(double) * nv), *lid = malloc(sizeof(double) * nv);
    const int Lw = nx > ny ? nx : ny;
    double *nW_store = malloc(sizeof(double) * 4 * Lw);
    if (p->kind == ORC_SHOCK) {
        double up[3], dn[3];
        orc_rankine_hugoniot(p->mach, up, dn);
        double Vu[3] = {up[1], 0, 0}, Vd[3] = {dn[1], 0, 0};
        maxwellian_on(&g, up[0], Vu, up[2], PAD(G, -2, 0));
        maxwellian_on(&g, up[0], Vu, up[2], PAD(G, -1, 0));
        maxwellian_on(&g, dn[0], Vd, dn[2], PAD(G, nx, 0));
        maxwellian_on(&g, dn[0], Vd, dn[2], PAD(G, nx + 1, 0));
    } else if (p->kind == ORC_PERIODIC1 || p->kind == ORC_PERIODIC2) {
        for (int iy = 0; iy < ny; ++iy) {
            memcpy(PAD(G, -2, iy), SRC(nx - 2, iy), sizeof(double) * nv);
            memcpy(PAD(G, -1, iy), SRC(nx - 1, iy), sizeof(double) * nv);
            memcpy(PAD(G, nx, iy), SRC(0, iy), sizeof(double) * nv);
            memcpy(PAD(G, nx + 1, iy), SRC(1, iy), sizeof(double) * nv);
        }
        if (two)
            for (int ix = 0; ix < nx; ++ix) {
                memcpy(PAD(G, ix, -2), SRC(ix, ny - 2), sizeof(double) * nv);
                memcpy(PAD(G, ix, -1), SRC(ix, ny - 1), sizeof(double) * nv);
                memcpy(PAD(G, ix, ny), SRC(ix, 0), sizeof(double) * nv);
                memcpy(PAD(G, ix, ny + 1), SRC(ix, 1), sizeof(double) * nv);
            }
    } else {
        wall_maxwellian(p, &g, 0.0, rest);
        wall_maxwellian(p, &g, lid_speed(p), lid);
        for (int w = 0; w < 4; ++w) {
            int axis; double sign;
            wall_normal(w, &axis, &sign);
            const double *va = axis == 0 ? g.vx : g.vy;
            const double *phiw = w == 3 ? lid : rest;
            int len = axis == 0 ? ny : nx;
            for (int k = 0; k < len; ++k) {
                int ax, ay, gx1, gy1, gx2, gy2;
                if (w == 0) { ax = 0; ay = k; gx1 = -1; gx2 = -2; gy1 = gy2 = k; }
                else if (w == 1) { ax = nx - 1; ay = k; gx1 = nx; gx2 = nx + 1; gy1 = gy2 = k; }
                else if (w == 2) { ax = k; ay = 0; gy1 = -1; gy2 = -2; gx1 = gx2 = k; }
                else { ax = k; ay = ny - 1; gy1 = ny; gy2 = ny + 1; gx1 = gx2 = k; }
                const double *g0 = SRC(ax, ay);
                double nW = wall_density(&g, axis, sign, g0, phiw);
                nW_store[w * Lw + k] = nW;
                double *d1 = PAD(G, gx1, gy1), *d2 = PAD(G, gx2, gy2);
                for (long j = 0; j < nv; ++j) {
                    double v = sign * va[j] > 0.0 ? nW * phiw[j] : g0[j];
                    d1[j] = v;
                    d2[j] = v;
                }
            }
        }
    }

    /* transpose of the stencil: out_i = G_i - C (face_{i+1/2} - face_{i-1/2}) */
    const double dx = dxs(p), dy = two ? dys(p) : 1.0;
    const int limit = p->minmod;
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const double *m = mu + ((long)iy * nx + ix) * nv;
            for (long j = 0; j < nv; ++j) {
                PAD(Gb, ix, iy)[j] += m[j];
                const double Cx = g.vx[j] * dt / dx;
                /* face i+1/2 from padded (ix-1, ix, ix+1, ix+2), face i-1/2 from (ix-2 .. ix+1) */
                face_adjoint(&PAD(Gb, ix - 1, iy)[j], &PAD(Gb, ix, iy)[j], &PAD(Gb, ix + 1, iy)[j],
                             &PAD(Gb, ix + 2, iy)[j], PAD(G, ix - 1, iy)[j], PAD(G, ix, iy)[j], PAD(G, ix + 1, iy)[j],
                             PAD(G, ix + 2, iy)[j], Cx, limit, -Cx * m[j]);
                face_adjoint(&PAD(Gb, ix - 2, iy)[j], &PAD(Gb, ix - 1, iy)[j], &PAD(Gb, ix, iy)[j],
                             &PAD(Gb, ix + 1, iy)[j], PAD(G, ix - 2, iy)[j], PAD(G, ix - 1, iy)[j], PAD(G, ix, iy)[j],
                             PAD(G, ix + 1, iy)[j], Cx, limit, Cx * m[j]);
                if (two) {
                    const double Cy = g.vy[j] * dt / dy;
                    face_adjoint(&PAD(Gb, ix, iy - 1)[j], &PAD(Gb, ix, iy)[j], &PAD(Gb, ix, iy + 1)[j],
                                 &PAD(Gb, ix, iy + 2)[j], PAD(G, ix, iy - 1)[j], PAD(G, ix, iy)[j],
                                 PAD(G, ix, iy + 1)[j], PAD(G, ix, iy + 2)[j], Cy, limit, -Cy * m[j]);
                    face_adjoint(&PAD(Gb, ix, iy - 2)[j], &PAD(Gb, ix, iy - 1)[j], &PAD(Gb, ix, iy)[j],
                                 &PAD(Gb, ix, iy + 1)[j], PAD(G, ix, iy - 2)[j], PAD(G, ix, iy - 1)[j],
                                 PAD(G, ix, iy)[j], PAD(G, ix, iy + 1)[j], Cy, limit, Cy * m[j]);
                }
            }
        }

    /* interior adjoint */
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) memcpy(gbar + ((long)iy * nx + ix) * nv, PAD(Gb, ix, iy), sizeof(double) * nv);
    /* transpose of the ghost construction */
    if (p->kind == ORC_PERIODIC1 || p->kind == ORC_PERIODIC2) {
        for (int iy = 0; iy < ny; ++iy)
            for (long j = 0; j < nv; ++j) {
                gbar[((long)iy * nx + nx - 2) * nv + j] += PAD(Gb, -2, iy)[j];
                gbar[((long)iy * nx + nx - 1) * nv + j] += PAD(Gb, -1, iy)[j];
                gbar[((long)iy * nx + 0) * nv + j] += PAD(Gb, nx, iy)[j];
                gbar[((long)iy * nx + 1) * nv + j] += PAD(Gb, nx + 1, iy)[j];
            }
        if (two)
            for (int ix = 0; ix < nx; ++ix)
                for (long j = 0; j < nv; ++j) {
                    gbar[((long)(ny - 2) * nx + ix) * nv + j] += PAD(Gb, ix, -2)[j];
                    gbar[((long)(ny - 1) * nx + ix) * nv + j] += PAD(Gb, ix, -1)[j];
                    gbar[((long)0 * nx + ix) * nv + j] += PAD(Gb, ix, ny)[j];
                    gbar[((long)1 * nx + ix) * nv + j] += PAD(Gb, ix, ny + 1)[j];
                }
    } else if (p->kind == ORC_CAVITY) {
        /* ghost(j) = g0(j) for incident j; n_W Phi_W(j) for emitted j, with
         * n_W = sum_inc |v.n| g0 / D_W, D_W = sum_em (v.n) Phi_W(T_w). */
        for (int w = 0; w < 4; ++w) {
            int axis; double sign;
            wall_normal(w, &axis, &sign);
            const double *va = axis == 0 ? g.vx : g.vy;
            const double *phiw = w == 3 ? lid : rest;
            const double uw = w == 3 ? lid_speed(p) : 0.0;
            const double Tw = p->t_wall;
            double D = 0.0, Dp = 0.0;
            for (long j = 0; j < nv; ++j) {
                const double vn = sign * va[j];
                if (vn > 0.0) {
                    const double c2 = (g.vx[j] - uw) * (g.vx[j] - uw) + g.vy[j] * g.vy[j] + g.vz[j] * g.vz[j];
                    D += vn * phiw[j];
                    Dp += vn * phiw[j] * (c2 / (Tw * Tw) - 1.5 / Tw);
                }
            }
            int len = axis == 0 ? ny : nx;
            for (int k = 0; k < len; ++k) {
                int ax, ay, gx1, gy1, gx2, gy2;
                if (w == 0) { ax = 0; ay = k; gx1 = -1; gx2 = -2; gy1 = gy2 = k; }
                else if (w == 1) { ax = nx - 1; ay = k; gx1 = nx; gx2 = nx + 1; gy1 = gy2 = k; }
                else if (w == 2) { ax = k; ay = 0; gy1 = -1; gy2 = -2; gx1 = gx2 = k; }
                else { ax = k; ay = ny - 1; gy1 = ny; gy2 = ny + 1; gx1 = gx2 = k; }
                const double nW = nW_store[w * Lw + k];
                double *gb0 = gbar + ((long)ay * nx + ax) * nv;
                const double *b1 = PAD(Gb, gx1, gy1), *b2 = PAD(Gb, gx2, gy2);
                double nWbar = 0.0;
                for (long j = 0; j < nv; ++j) {
                    const double gam = b1[j] + b2[j];
                    const double vn = sign * va[j];
                    if (vn > 0.0) {
                        const double c2 = (g.vx[j] - uw) * (g.vx[j] - uw) + g.vy[j] * g.vy[j] + g.vz[j] * g.vz[j];
                        const double dphi = phiw[j] * (c2 / (Tw * Tw) - 1.5 / Tw);
                        nWbar += gam * phiw[j];
                        *gtw += gam * nW * (dphi - phiw[j] * Dp / D);
                    } else {
                        gb0[j] += gam;
                    }
                }
                for (long j = 0; j < nv; ++j) {
                    const double vn = sign * va[j];
                    if (vn < 0.0) gb0[j] += nWbar * (-vn) / D;
                }
            }
        }
    }
#undef PAD
#undef SRC
    free(rest); free(lid); free(nW_store);
    free(G); free(Gb);
    free_velgrid(&g);
}

/* Adjoint of one time step at f (Strang: R_{dt/2} S R_{dt/2}; Lie: R_dt S):
 * lam_n = (d step / d f)^T lam_next; grad[0] += dL/dKn, grad[1] += dL/dT_w. */
void orc_step_adjoint(const orc_problem *p, const double *f, const double *lam_next, double *lam_n, double *grad)
{
    const double dt = orc_dt(p);
    const long n = ncell(p) * nvel(p);
    double *a = malloc(sizeof(double) * n), *h = malloc(sizeof(double) * n), *t = malloc(sizeof(double) * n);
    if (p->strang) {
        orc_relax(p, f, a, 0.5 * dt);
        orc_stream(p, a, h, dt);
        orc_relax_adjoint(p, h, lam_next, t, 0.5 * dt, &grad[0]);
        double *u = malloc(sizeof(double) * n);
        orc_stream_adjoint(p, a, t, u, dt, &grad[1]);
        orc_relax_adjoint(p, f, u, lam_n, 0.5 * dt, &grad[0]);
        free(u);
    } else {
        orc_stream(p, f, h, dt);
        orc_relax_adjoint(p, h, lam_next, t, dt, &grad[0]);
        orc_stream_adjoint(p, f, t, lam_n, dt, &grad[1]);
    }
    free(a); free(h); free(t);
}

/* Gradient of orc_lid_shear: lam = dL/df (zero outside the top row),
 * grad[1] += dL/dT_w.  With N_i = sum_{vy>0} vy f_top,i, K = sum_{vy<0} vx vy Phi_W,
 * D = sum_{vy<0} |vy| Phi_W:  L = sum_i dx dV [sum_{vy>0} vx vy f_top,i + N_i K / D]. */
void orc_lid_shear_grad(const orc_problem *p, const double *f, double *lam, double *grad)
{
    velgrid g = make_velgrid(p);
    const int nx = p->nx, ny = p->ny;
    const long nv = nvel(p);
    const double dV = dvol(p), dx = dxs(p), Tw = p->t_wall, uw = lid_speed(p);
    double *lid = malloc(sizeof(double) * nv);
    wall_maxwellian(p, &g, uw, lid);
    double K = 0, D = 0, Kp = 0, Dp = 0;
    for (long j = 0; j < nv; ++j)
        if (g.vy[j] < 0.0) {
            const double c2 = (g.vx[j] - uw) * (g.vx[j] - uw) + g.vy[j] * g.vy[j] + g.vz[j] * g.vz[j];
            const double dphi = lid[j] * (c2 / (Tw * Tw) - 1.5 / Tw);
            K += g.vx[j] * g.vy[j] * lid[j];
            D += -g.vy[j] * lid[j];
            Kp += g.vx[j] * g.vy[j] * dphi;
            Dp += -g.vy[j] * dphi;
        }
    memset(lam, 0, sizeof(double) * ncell(p) * nv);
    for (int ix = 0; ix < nx; ++ix) {
        const long c = (long)(ny - 1) * nx + ix;
        double N = 0.0;
        for (long j = 0; j < nv; ++j)
            if (g.vy[j] > 0.0) {
                lam[c * nv + j] = dx * dV * (g.vx[j] * g.vy[j] + g.vy[j] * K / D);
                N += g.vy[j] * f[c * nv + j];
            }
        grad[1] += dx * dV * N * (Kp / D - K * Dp / (D * D));
    }
    free(lid);
    free_velgrid(&g);
}
