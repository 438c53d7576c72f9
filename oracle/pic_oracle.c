/*
 * pic_oracle.c -- slow, plain FP64 CPU oracle for the SDMD particle-in-cell step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Derouillat & Beck, "Single Domain Multiple Decompositions
 * for Particle-in-Cell simulations"):
 *
 *   * SDSD mode (section 2.1): one undecomposed periodic grid holding every
 *     macro-particle.  This is the plain definition of one PIC iteration:
 *     field interpolation, push, deposition (section 3.3, "Particles" timer),
 *     then the Maxwell solve (section 3.3, "Fields" timer).
 *   * SDMD mode (section 2.2): the same iteration with two decompositions of
 *     the same domain -- small patches own the particles, large regions own the
 *     fields -- and the two extra transfers the section lists: (i) patch
 *     currents are summed into regions after deposition, (ii) region fields are
 *     copied to the patches after the Maxwell solve.  Regions exchange ghost
 *     layers with their neighbours.
 *
 * The paper names but does not define the sub-algorithms; they are written
 * here from the published methods it cites (section 3.2):
 *   * Yee staggered finite-difference Maxwell solver;
 *   * Esirkepov charge-conserving deposition with the second-order (quadratic
 *     B-spline, 5-point frame) shape function;
 *   * the pusher is not named; the Boris scheme is used.
 *
 * Units are normalised (c = 1).  Equations: dE/dt = curl B - J,
 * dB/dt = -curl E, du/dt = (q/m)(E + u x B / gamma), dx/dt = u / gamma.
 *
 * Staggering (index (i,j,k) of a component sits at the listed position, in
 * units of the cell size):
 *     Ex (i+1/2, j, k)      Bx (i, j+1/2, k+1/2)      Jx like Ex
 *     Ey (i, j+1/2, k)      By (i+1/2, j, k+1/2)      Jy like Ey
 *     Ez (i, j, k+1/2)      Bz (i+1/2, j+1/2, k)      Jz like Ez
 * In 2D3V the z axis has one cell and no derivative; Ez, Jz sit on (i, j).
 *
 * Field storage: one array of 12 components, each n[2]*n[1]*n[0] doubles,
 * x fastest.  Components: Ex Ey Ez | Bx By Bz (B at t^{n+1/2}) |
 * Bmx Bmy Bmz (B time-centred at t^n) | Jx Jy Jz (J at t^{n-1/2}).
 *
 * State at the start of step n: positions x^n, momenta u^{n-1/2}, weights w,
 * E^n, B^{n+1/2}, Bm^n.
 *
 * Readings where the paper is silent (listed again in the design notes):
 *   - nearest-node tie X+1/2 integer takes floor (delta = -1/2);
 *   - the cell of a position is floor(x/dx) clamped to [0, n-1];
 *   - positions wrap periodically after deposition: x -= L if x >= L,
 *     x += L if x < 0, then x = 0 if x == L;
 *   - B for the push is Bm^n = (B^{n-1/2} + B^{n+1/2}) / 2;
 *   - the initial momenta are taken as u^{-1/2}; B^{1/2} = B^0 - dt/2 curl E^0
 *     and Bm^0 = B^0 unless all three are given.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t dims;        /* 2 (2D3V) or 3 (3D3V) */
    int32_t n[3];        /* cells per axis; n[2] == 1 in 2D */
    double  d[3];        /* cell size per axis; d[2] unused in 2D */
    double  dt;
    double  q, m;        /* species charge and mass (electrons: -1, 1) */
    int32_t patch[3];    /* SDMD: cells per patch per axis */
    int32_t nreg[3];     /* SDMD: regions per axis */
    int32_t filter;      /* passes of the binomial current filter (0 = none) */
} ocfg;

typedef struct {
    int64_t n;
    double *x, *y, *z;   /* z unused in 2D */
    double *ux, *uy, *uz;
    double *w;
} oparts;

enum { EX, EY, EZ, BX, BY, BZ, BMX, BMY, BMZ, JX, JY, JZ, NCOMP };

/* staggering per component: 1 = dual (half-integer) along that axis */
static const int STAG[NCOMP][3] = {
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},   /* E */
    {0, 1, 1}, {1, 0, 1}, {1, 1, 0},   /* B */
    {0, 1, 1}, {1, 0, 1}, {1, 1, 0},   /* Bm */
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},   /* J */
};

static int64_t ncells(const ocfg* c) { return (int64_t)c->n[0] * c->n[1] * c->n[2]; }

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static int64_t gidx(const ocfg* c, int64_t i, int64_t j, int64_t k)
{
    return wrapi(i, c->n[0]) + (int64_t)c->n[0] * (wrapi(j, c->n[1]) + (int64_t)c->n[1] * wrapi(k, c->n[2]));
}

/* ------------------------------------------------------------------------ */
/* Shape function: quadratic B-spline (second order, section 3.2).           */
/* S(s) = 3/4 - s^2 for |s| <= 1/2; (3/2 - |s|)^2 / 2 for 1/2 < |s| <= 3/2.  */
/* ------------------------------------------------------------------------ */
double oracle_S(double s)
{
    double a = fabs(s);
    if (a <= 0.5) return 0.75 - s * s;
    if (a <= 1.5) {
        double t = 1.5 - a;
        return 0.5 * t * t;
    }
    return 0.0;
}

/* ------------------------------------------------------------------------ */
/* Field interpolation (section 3.3, "Particles": interpolation).            */
/* F(X) = sum over nodes of prod_axes S(X_a - node_a) F(node), node_a being   */
/* i or i + 1/2 according to the staggering.  E from E^n, B from Bm^n.       */
/* ------------------------------------------------------------------------ */
static double interp_comp(const ocfg* c, const double* F, int comp, const double X[3])
{
    const double* A = F + (int64_t)comp * ncells(c);
    double s = 0.0;
    int64_t fx = (int64_t)floor(X[0]), fy = (int64_t)floor(X[1]);
    int64_t fz = (c->dims == 3) ? (int64_t)floor(X[2]) : 0;
    int kz0 = (c->dims == 3) ? -2 : 0, kz1 = (c->dims == 3) ? 2 : 0;
    for (int kz = kz0; kz <= kz1; ++kz) {
        double wz = 1.0;
        int64_t k = fz + kz;
        if (c->dims == 3) wz = oracle_S(X[2] - (double)k - 0.5 * STAG[comp][2]);
        for (int ky = -2; ky <= 2; ++ky) {
            int64_t j = fy + ky;
            double wy = oracle_S(X[1] - (double)j - 0.5 * STAG[comp][1]);
            for (int kx = -2; kx <= 2; ++kx) {
                int64_t i = fx + kx;
                double wx = oracle_S(X[0] - (double)i - 0.5 * STAG[comp][0]);
                s += wx * wy * wz * A[gidx(c, i, j, k)];
            }
        }
    }
    return s;
}

/* out[0..2] = E^n, out[3..5] = Bm^n at position (x, y, z) */
void oracle_interp(const ocfg* c, const double* F, double x, double y, double z, double out[6])
{
    double X[3] = {x / c->d[0], y / c->d[1], (c->dims == 3) ? z / c->d[2] : 0.0};
    out[0] = interp_comp(c, F, EX, X);
    out[1] = interp_comp(c, F, EY, X);
    out[2] = interp_comp(c, F, EZ, X);
    out[3] = interp_comp(c, F, BMX, X);
    out[4] = interp_comp(c, F, BMY, X);
    out[5] = interp_comp(c, F, BMZ, X);
}

/* ------------------------------------------------------------------------ */
/* Boris push (the paper's "push"; the scheme is a reading): half electric   */
/* kick, magnetic rotation, half electric kick.  u is updated in place.      */
/* ------------------------------------------------------------------------ */
void oracle_boris(double qm, double dt, const double EB[6], double u[3])
{
    double h = 0.5 * qm * dt;
    double um[3] = {u[0] + h * EB[0], u[1] + h * EB[1], u[2] + h * EB[2]};
    double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {h * EB[3] / g, h * EB[4] / g, h * EB[5] / g};
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
    /* u' = u- + u- x t */
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    /* u+ = u- + u' x s */
    double upl[3] = {um[0] + (up[1] * s[2] - up[2] * s[1]),
                     um[1] + (up[2] * s[0] - up[0] * s[2]),
                     um[2] + (up[0] * s[1] - up[1] * s[0])};
    u[0] = upl[0] + h * EB[0];
    u[1] = upl[1] + h * EB[1];
    u[2] = upl[2] + h * EB[2];
}

double oracle_gamma(const double u[3])
{
    return sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

/* ------------------------------------------------------------------------ */
/* Esirkepov charge-conserving deposition, order 2 (section 3.2).            */
/* One particle moving from X0 to X1 (cell units, unwrapped).  The 5-point   */
/* frame is centred on the primal node nearest X0.  DS = S(X1-.) - S(X0-.).  */
/* The W weights split the change of the shape product between the axes;    */
/* Jx on the dual x nodes is the running sum of -q w (dx/dt) Wx along x, and */
/* likewise for y (and z in 3D).  In 2D3V, Jz = q w vz Wz on primal nodes.  */
/* `add` receives (component, i, j, k, value) with global unwrapped indices. */
/* ------------------------------------------------------------------------ */
typedef void (*add_fn)(void* ctx, int comp, int64_t i, int64_t j, int64_t k, double v);

static void esirkepov(const ocfg* c, const double X0[3], const double X1[3], double w, double vz,
                      add_fn add, void* actx)
{
    const double q = c->q, dt = c->dt;
    int dims = c->dims;
    int64_t i0[3];
    double S0[3][5], DS[3][5];
    for (int a = 0; a < dims; ++a) {
        i0[a] = (int64_t)floor(X0[a] + 0.5);
        for (int k = 0; k < 5; ++k) {
            double node = (double)(i0[a] + k - 2);
            S0[a][k] = oracle_S(X0[a] - node);
            DS[a][k] = oracle_S(X1[a] - node) - S0[a][k];
        }
    }
    const double third = 1.0 / 3.0;
    if (dims == 2) {
        double Wx[5][5], Wy[5][5], Wz[5][5];
        for (int k = 0; k < 5; ++k)
            for (int l = 0; l < 5; ++l) {
                Wx[k][l] = DS[0][k] * (S0[1][l] + 0.5 * DS[1][l]);
                Wy[k][l] = DS[1][l] * (S0[0][k] + 0.5 * DS[0][k]);
                Wz[k][l] = S0[0][k] * S0[1][l] + 0.5 * DS[0][k] * S0[1][l] + 0.5 * S0[0][k] * DS[1][l] +
                           third * DS[0][k] * DS[1][l];
            }
        double cx = -q * w * c->d[0] / dt, cy = -q * w * c->d[1] / dt, cz = q * w * vz;
        for (int l = 0; l < 5; ++l) {
            double acc = 0.0;
            for (int k = 0; k < 5; ++k) {
                acc += Wx[k][l];
                add(actx, 0, i0[0] + k - 2, i0[1] + l - 2, 0, cx * acc);
            }
        }
        for (int k = 0; k < 5; ++k) {
            double acc = 0.0;
            for (int l = 0; l < 5; ++l) {
                acc += Wy[k][l];
                add(actx, 1, i0[0] + k - 2, i0[1] + l - 2, 0, cy * acc);
            }
        }
        for (int k = 0; k < 5; ++k)
            for (int l = 0; l < 5; ++l) add(actx, 2, i0[0] + k - 2, i0[1] + l - 2, 0, cz * Wz[k][l]);
        return;
    }
    /* 3D */
    double Wx[5][5][5], Wy[5][5][5], Wz[5][5][5];
    for (int k = 0; k < 5; ++k)
        for (int l = 0; l < 5; ++l)
            for (int m = 0; m < 5; ++m) {
                Wx[k][l][m] = DS[0][k] * (S0[1][l] * S0[2][m] + 0.5 * DS[1][l] * S0[2][m] +
                                          0.5 * S0[1][l] * DS[2][m] + third * DS[1][l] * DS[2][m]);
                Wy[k][l][m] = DS[1][l] * (S0[0][k] * S0[2][m] + 0.5 * DS[0][k] * S0[2][m] +
                                          0.5 * S0[0][k] * DS[2][m] + third * DS[0][k] * DS[2][m]);
                Wz[k][l][m] = DS[2][m] * (S0[0][k] * S0[1][l] + 0.5 * DS[0][k] * S0[1][l] +
                                          0.5 * S0[0][k] * DS[1][l] + third * DS[0][k] * DS[1][l]);
            }
    double cx = -q * w * c->d[0] / dt, cy = -q * w * c->d[1] / dt, cz = -q * w * c->d[2] / dt;
    for (int l = 0; l < 5; ++l)
        for (int m = 0; m < 5; ++m) {
            double acc = 0.0;
            for (int k = 0; k < 5; ++k) {
                acc += Wx[k][l][m];
                add(actx, 0, i0[0] + k - 2, i0[1] + l - 2, i0[2] + m - 2, cx * acc);
            }
        }
    for (int k = 0; k < 5; ++k)
        for (int m = 0; m < 5; ++m) {
            double acc = 0.0;
            for (int l = 0; l < 5; ++l) {
                acc += Wy[k][l][m];
                add(actx, 1, i0[0] + k - 2, i0[1] + l - 2, i0[2] + m - 2, cy * acc);
            }
        }
    for (int k = 0; k < 5; ++k)
        for (int l = 0; l < 5; ++l) {
            double acc = 0.0;
            for (int m = 0; m < 5; ++m) {
                acc += Wz[k][l][m];
                add(actx, 2, i0[0] + k - 2, i0[1] + l - 2, i0[2] + m - 2, cz * acc);
            }
        }
}

/* deposit straight into a global periodic J (3 components) */
typedef struct { const ocfg* c; double* J; } global_add_ctx;

static void global_add(void* p, int comp, int64_t i, int64_t j, int64_t k, double v)
{
    global_add_ctx* g = (global_add_ctx*)p;
    g->J[(int64_t)comp * ncells(g->c) + gidx(g->c, i, j, k)] += v;
}

/* Public: deposit one particle's move X0 -> X1 (physical positions, 3 each)  */
/* into J (3 components, global grid, accumulated).                           */
void oracle_deposit_one(const ocfg* c, double* J, const double x0[3], const double x1[3], double w, double vz)
{
    double X0[3], X1[3];
    for (int a = 0; a < 3; ++a) {
        double d = (a < c->dims) ? c->d[a] : 1.0;
        X0[a] = (a < c->dims) ? x0[a] / d : 0.0;
        X1[a] = (a < c->dims) ? x1[a] / d : 0.0;
    }
    global_add_ctx g = {c, J};
    esirkepov(c, X0, X1, w, vz, global_add, &g);
}

/* ------------------------------------------------------------------------ */
/* Yee solver (section 3.2) on the undecomposed periodic grid.               */
/* Ampere: E += dt (curl B - J) with B^{n+1/2}, J^{n+1/2}.                   */
/* Faraday: B^{n+3/2} = B^{n+1/2} - dt curl E^{n+1}.                         */
/* Bm^{n+1} = (B^{n+1/2} + B^{n+3/2}) / 2.                                   */
/* In 2D the z differences vanish (one periodic cell).                       */
/* ------------------------------------------------------------------------ */
static void ampere(const ocfg* c, double* F, double dt)
{
    int64_t N = ncells(c);
    double *Ex = F + EX * N, *Ey = F + EY * N, *Ez = F + EZ * N;
    const double *Bx = F + BX * N, *By = F + BY * N, *Bz = F + BZ * N;
    const double *Jx = F + JX * N, *Jy = F + JY * N, *Jz = F + JZ * N;
    double dx = c->d[0], dy = c->d[1], dz = (c->dims == 3) ? c->d[2] : 1.0;
    for (int64_t k = 0; k < c->n[2]; ++k)
        for (int64_t j = 0; j < c->n[1]; ++j)
            for (int64_t i = 0; i < c->n[0]; ++i) {
                int64_t p = gidx(c, i, j, k);
                Ex[p] += dt * ((Bz[p] - Bz[gidx(c, i, j - 1, k)]) / dy - (By[p] - By[gidx(c, i, j, k - 1)]) / dz - Jx[p]);
                Ey[p] += dt * ((Bx[p] - Bx[gidx(c, i, j, k - 1)]) / dz - (Bz[p] - Bz[gidx(c, i - 1, j, k)]) / dx - Jy[p]);
                Ez[p] += dt * ((By[p] - By[gidx(c, i - 1, j, k)]) / dx - (Bx[p] - Bx[gidx(c, i, j - 1, k)]) / dy - Jz[p]);
            }
}

static void faraday(const ocfg* c, double* F, double dt)
{
    int64_t N = ncells(c);
    const double *Ex = F + EX * N, *Ey = F + EY * N, *Ez = F + EZ * N;
    double *Bx = F + BX * N, *By = F + BY * N, *Bz = F + BZ * N;
    double dx = c->d[0], dy = c->d[1], dz = (c->dims == 3) ? c->d[2] : 1.0;
    for (int64_t k = 0; k < c->n[2]; ++k)
        for (int64_t j = 0; j < c->n[1]; ++j)
            for (int64_t i = 0; i < c->n[0]; ++i) {
                int64_t p = gidx(c, i, j, k);
                Bx[p] -= dt * ((Ez[gidx(c, i, j + 1, k)] - Ez[p]) / dy - (Ey[gidx(c, i, j, k + 1)] - Ey[p]) / dz);
                By[p] -= dt * ((Ex[gidx(c, i, j, k + 1)] - Ex[p]) / dz - (Ez[gidx(c, i + 1, j, k)] - Ez[p]) / dx);
                Bz[p] -= dt * ((Ey[gidx(c, i + 1, j, k)] - Ey[p]) / dx - (Ex[gidx(c, i, j + 1, k)] - Ex[p]) / dy);
            }
}

void oracle_yee(const ocfg* c, double* F)
{
    int64_t N = ncells(c);
    double* Bold = (double*)malloc(sizeof(double) * 3 * N);
    memcpy(Bold, F + BX * N, sizeof(double) * 3 * N);
    ampere(c, F, c->dt);
    faraday(c, F, c->dt);
    for (int a = 0; a < 3; ++a)
        for (int64_t p = 0; p < N; ++p) F[(BMX + a) * N + p] = 0.5 * (Bold[a * N + p] + F[(BX + a) * N + p]);
    free(Bold);
}

/* Initial half step: B^{1/2} = B^0 - (dt/2) curl E^0 and Bm^0 = B^0.        */
/* On entry the B slot holds B^0.                                            */
void oracle_init_fields(const ocfg* c, double* F)
{
    int64_t N = ncells(c);
    memcpy(F + BMX * N, F + BX * N, sizeof(double) * 3 * N);
    faraday(c, F, 0.5 * c->dt);
}

/* ------------------------------------------------------------------------ */
/* Binomial current filter (section 3.2: a two-pass binomial filter smooths  */
/* the current densities every iteration; Birdsall & Langdon).  One pass     */
/* smooths a component along x, then y, then z (3D) with the 1-2-1 kernel,   */
/* out(i) = (in(i-1) + 2 in(i) + in(i+1)) / 4, periodic, on the component's  */
/* own lattice (the kernel is shift invariant, so the staggering of Jx, Jy,  */
/* Jz needs no special treatment).  Applied to J after deposition (and, in   */
/* SDMD, after the patch -> region sum), before Ampere.                      */
/* ------------------------------------------------------------------------ */
static void binomial_sweep(const ocfg* c, double* a, double* tmp, int axis)
{
    for (int64_t k = 0; k < c->n[2]; ++k)
        for (int64_t j = 0; j < c->n[1]; ++j)
            for (int64_t i = 0; i < c->n[0]; ++i) {
                int64_t lo, hi;
                if (axis == 0) {
                    lo = gidx(c, i - 1, j, k);
                    hi = gidx(c, i + 1, j, k);
                } else if (axis == 1) {
                    lo = gidx(c, i, j - 1, k);
                    hi = gidx(c, i, j + 1, k);
                } else {
                    lo = gidx(c, i, j, k - 1);
                    hi = gidx(c, i, j, k + 1);
                }
                int64_t p = gidx(c, i, j, k);
                tmp[p] = (a[lo] + 2.0 * a[p] + a[hi]) * 0.25;
            }
    memcpy(a, tmp, sizeof(double) * ncells(c));
}

/* `passes` passes over `ncomp` consecutive global arrays */
void oracle_filter(const ocfg* c, double* a, int32_t ncomp, int32_t passes)
{
    int64_t N = ncells(c);
    double* tmp = (double*)malloc(sizeof(double) * N);
    for (int comp = 0; comp < ncomp; ++comp)
        for (int pass = 0; pass < passes; ++pass)
            for (int axis = 0; axis < c->dims; ++axis) binomial_sweep(c, a + comp * N, tmp, axis);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Position wrap and cell / patch binning.                                   */
/* ------------------------------------------------------------------------ */
double oracle_wrap(double x, double L)
{
    if (x >= L) x -= L;
    if (x < 0.0) x += L;
    if (x == L) x = 0.0;
    return x;
}

int64_t oracle_cell(double x, double d, int64_t n)
{
    double f = floor(x / d);
    int64_t i = (int64_t)f;
    if (i > n - 1) i = n - 1;
    if (i < 0) i = 0;
    return i;
}

/* patch index of every particle (x fastest over patches) */
void oracle_bin(const ocfg* c, const oparts* P, int32_t* patch)
{
    int64_t np[3] = {c->n[0] / c->patch[0], c->n[1] / c->patch[1], 1};
    if (c->dims == 3) np[2] = c->n[2] / c->patch[2];
    for (int64_t p = 0; p < P->n; ++p) {
        int64_t ci = oracle_cell(P->x[p], c->d[0], c->n[0]);
        int64_t cj = oracle_cell(P->y[p], c->d[1], c->n[1]);
        int64_t ck = (c->dims == 3) ? oracle_cell(P->z[p], c->d[2], c->n[2]) : 0;
        int64_t pk = (c->dims == 3) ? ck / c->patch[2] : 0;
        patch[p] = (int32_t)(ci / c->patch[0] + np[0] * (cj / c->patch[1] + np[1] * pk));
    }
}

/* Split position form (the GPU's FP32 form): cell i and in-cell offset      */
/* xi in [0,1) as float.  xi rounding up to 1 moves to the next cell.        */
void oracle_split(double x, double d, int64_t n, int32_t* cell, float* xi)
{
    int64_t i = oracle_cell(x, d, n);
    float f = (float)(x / d - (double)i);
    if (f < 0.0f) f = 0.0f;
    if (f >= 1.0f) {
        f = 0.0f;
        i += 1;
        if (i >= n) i -= n;
    }
    *cell = (int32_t)i;
    *xi = f;
}

/* ------------------------------------------------------------------------ */
/* SDSD step: one undecomposed grid (section 2.1).                           */
/* ------------------------------------------------------------------------ */
static void push_one(const ocfg* c, const double* F, double* x, double* y, double* z, double* ux, double* uy,
                     double* uz, double X0[3], double X1[3], double* vz_out)
{
    double EB[6];
    oracle_interp(c, F, *x, *y, (c->dims == 3) ? *z : 0.0, EB);
    double u[3] = {*ux, *uy, *uz};
    oracle_boris(c->q / c->m, c->dt, EB, u);
    double g = oracle_gamma(u);
    double nx = *x + c->dt * u[0] / g;
    double ny = *y + c->dt * u[1] / g;
    double nz = (c->dims == 3) ? *z + c->dt * u[2] / g : 0.0;
    X0[0] = *x / c->d[0];
    X0[1] = *y / c->d[1];
    X0[2] = (c->dims == 3) ? *z / c->d[2] : 0.0;
    X1[0] = nx / c->d[0];
    X1[1] = ny / c->d[1];
    X1[2] = (c->dims == 3) ? nz / c->d[2] : 0.0;
    *vz_out = u[2] / g;
    *ux = u[0];
    *uy = u[1];
    *uz = u[2];
    *x = oracle_wrap(nx, c->n[0] * c->d[0]);
    *y = oracle_wrap(ny, c->n[1] * c->d[1]);
    if (c->dims == 3) *z = oracle_wrap(nz, c->n[2] * c->d[2]);
}

/* Interpolate, push, move and deposit every particle (stored order) into a  */
/* zeroed J; no field update.  Returns the largest |displacement| in cells.  */
double oracle_particles_sdsd(const ocfg* c, double* F, oparts* P)
{
    int64_t N = ncells(c);
    memset(F + JX * N, 0, sizeof(double) * 3 * N);
    global_add_ctx g = {c, F + JX * N};
    double maxd = 0.0;
    double dummy = 0.0;
    for (int64_t p = 0; p < P->n; ++p) {
        double X0[3], X1[3], vz;
        push_one(c, F, &P->x[p], &P->y[p], c->dims == 3 ? &P->z[p] : &dummy, &P->ux[p], &P->uy[p], &P->uz[p], X0,
                 X1, &vz);
        for (int a = 0; a < c->dims; ++a)
            if (fabs(X1[a] - X0[a]) > maxd) maxd = fabs(X1[a] - X0[a]);
        esirkepov(c, X0, X1, P->w[p], vz, global_add, &g);
    }
    return maxd;
}

/* Push a set of particles through the given fields without depositing      */
/* (used to check sampled particles one by one).                            */
void oracle_push_only(const ocfg* c, const double* F, oparts* P)
{
    double dummy = 0.0;
    for (int64_t p = 0; p < P->n; ++p) {
        double X0[3], X1[3], vz;
        push_one(c, F, &P->x[p], &P->y[p], c->dims == 3 ? &P->z[p] : &dummy, &P->ux[p], &P->uy[p], &P->uz[p], X0,
                 X1, &vz);
    }
}

double oracle_step_sdsd(const ocfg* c, double* F, oparts* P)
{
    double maxd = oracle_particles_sdsd(c, F, P);
    if (c->filter > 0) oracle_filter(c, F + JX * ncells(c), 3, c->filter);
    oracle_yee(c, F);
    return maxd;
}

/* ------------------------------------------------------------------------ */
/* SDMD step (section 2.2): patches own particles, regions own fields.       */
/* ------------------------------------------------------------------------ */
#define GH 2 /* ghost layers around each region */

typedef struct {
    const ocfg* c;
    int64_t o[3];     /* origin (global cell index) */
    int64_t s[3];     /* interior size */
    int64_t a[3];     /* allocated size = s + 2*GH (1 in 2D z) */
    double* f;        /* 12 components */
} region;

static int64_t ridx(const region* r, int64_t li, int64_t lj, int64_t lk)
{
    int g2 = (r->c->dims == 3) ? GH : 0;
    return (li + GH) + r->a[0] * ((lj + GH) + r->a[1] * (lk + g2));
}

static int64_t rsize(const region* r) { return r->a[0] * r->a[1] * r->a[2]; }

/* region that owns global cell index (i,j,k) (already wrapped) */
static int region_of(const ocfg* c, const int64_t rs[3], int64_t i, int64_t j, int64_t k)
{
    int64_t ri = i / rs[0], rj = j / rs[1], rk = (c->dims == 3) ? k / rs[2] : 0;
    return (int)(ri + c->nreg[0] * (rj + c->nreg[1] * rk));
}

/* Fill all ghost nodes of `comp` in every region from the interior of the  */
/* region owning the (periodically wrapped) global node: the region-region  */
/* synchronisation.                                                         */
static void exchange_ghosts(const ocfg* c, region* R, int nR, const int64_t rs[3], int comp)
{
    for (int r = 0; r < nR; ++r) {
        region* g = &R[r];
        int gz = (c->dims == 3) ? GH : 0;
        for (int64_t lk = -gz; lk < g->s[2] + gz; ++lk)
            for (int64_t lj = -GH; lj < g->s[1] + GH; ++lj)
                for (int64_t li = -GH; li < g->s[0] + GH; ++li) {
                    int inside = li >= 0 && li < g->s[0] && lj >= 0 && lj < g->s[1] && lk >= 0 && lk < g->s[2];
                    if (inside) continue;
                    int64_t gi = wrapi(g->o[0] + li, c->n[0]);
                    int64_t gj = wrapi(g->o[1] + lj, c->n[1]);
                    int64_t gk = wrapi(g->o[2] + lk, c->n[2]);
                    region* src = &R[region_of(c, rs, gi, gj, gk)];
                    g->f[comp * rsize(g) + ridx(g, li, lj, lk)] =
                        src->f[comp * rsize(src) + ridx(src, gi - src->o[0], gj - src->o[1], gk - src->o[2])];
                }
    }
}

/* Tile of one patch: J contributions on nodes [p0-2, p0+P+2] per axis.     */
typedef struct {
    const ocfg* c;
    int64_t o[3];     /* tile origin = patch origin - 2 */
    int64_t a[3];     /* tile size = P + 5 */
    double* t;        /* 3 components */
} tile;

static void tile_add(void* p, int comp, int64_t i, int64_t j, int64_t k, double v)
{
    tile* T = (tile*)p;
    int64_t li = i - T->o[0], lj = j - T->o[1], lk = (T->c->dims == 3) ? k - T->o[2] : 0;
    int64_t sz = T->a[0] * T->a[1] * T->a[2];
    /* the 5-point frame of a particle of the patch always lies in the tile */
    if (li < 0 || li >= T->a[0] || lj < 0 || lj >= T->a[1] || lk < 0 || lk >= T->a[2]) abort();
    T->t[comp * sz + li + T->a[0] * (lj + T->a[1] * lk)] += v;
}

/* Window of one patch: E and Bm on nodes [p0-1, p0+P+1] per axis, copied   */
/* from the patch's region (transfer (ii)).                                 */
typedef struct {
    ocfg lc;          /* a periodic-free local view used for interpolation */
    int64_t o[3];
    int64_t a[3];
    double* f;        /* 12 components, only E and Bm filled */
} window;

static double window_interp(const window* W, int comp, const double Xg[3])
{
    /* same loop structure as interp_comp, indices relative to the window */
    const ocfg* c = &W->lc;
    int64_t sz = W->a[0] * W->a[1] * W->a[2];
    const double* A = W->f + (int64_t)comp * sz;
    double s = 0.0;
    int64_t fx = (int64_t)floor(Xg[0]), fy = (int64_t)floor(Xg[1]);
    int64_t fz = (c->dims == 3) ? (int64_t)floor(Xg[2]) : 0;
    int kz0 = (c->dims == 3) ? -2 : 0, kz1 = (c->dims == 3) ? 2 : 0;
    for (int kz = kz0; kz <= kz1; ++kz) {
        double wz = 1.0;
        int64_t k = fz + kz;
        if (c->dims == 3) wz = oracle_S(Xg[2] - (double)k - 0.5 * STAG[comp][2]);
        for (int ky = -2; ky <= 2; ++ky) {
            int64_t j = fy + ky;
            double wy = oracle_S(Xg[1] - (double)j - 0.5 * STAG[comp][1]);
            for (int kx = -2; kx <= 2; ++kx) {
                int64_t i = fx + kx;
                double wx = oracle_S(Xg[0] - (double)i - 0.5 * STAG[comp][0]);
                double wt = wx * wy * wz;
                int64_t li = i - W->o[0], lj = j - W->o[1], lk = (c->dims == 3) ? k - W->o[2] : 0;
                int in = li >= 0 && li < W->a[0] && lj >= 0 && lj < W->a[1] && lk >= 0 && lk < W->a[2];
                if (!in) {
                    /* outside the window the weight must be exactly zero */
                    if (wt != 0.0) abort();
                    s += wt * 0.0;
                    continue;
                }
                s += wt * A[li + W->a[0] * (lj + W->a[1] * lk)];
            }
        }
    }
    return s;
}

static int check_decomp(const ocfg* c)
{
    for (int a = 0; a < c->dims; ++a) {
        if (c->patch[a] < 4 || c->n[a] % c->patch[a]) return -1;
        if (c->nreg[a] < 1 || c->n[a] % c->nreg[a]) return -1;
        if ((c->n[a] / c->nreg[a]) % c->patch[a]) return -1;
    }
    return 0;
}

/* One SDMD step.  F is the assembled global state on entry and exit; the    */
/* step itself only touches region, window and tile copies of it.           */
/* Returns 0, or -1 for an invalid decomposition.                            */
int oracle_step_sdmd(const ocfg* c, double* F, oparts* P, int32_t fields_only)
{
    if (check_decomp(c)) return -1;
    const int dims = c->dims;
    const int64_t NC = ncells(c);
    int64_t rs[3] = {c->n[0] / c->nreg[0], c->n[1] / c->nreg[1], (dims == 3) ? c->n[2] / c->nreg[2] : 1};
    int nR = c->nreg[0] * c->nreg[1] * ((dims == 3) ? c->nreg[2] : 1);
    region* R = (region*)calloc(nR, sizeof(region));

    /* 1. regions hold the fields: copy interiors, then synchronise ghosts */
    for (int r = 0; r < nR; ++r) {
        int64_t ri = r % c->nreg[0], rj = (r / c->nreg[0]) % c->nreg[1], rk = r / (c->nreg[0] * c->nreg[1]);
        R[r].c = c;
        R[r].o[0] = ri * rs[0];
        R[r].o[1] = rj * rs[1];
        R[r].o[2] = (dims == 3) ? rk * rs[2] : 0;
        for (int a = 0; a < 3; ++a) {
            R[r].s[a] = rs[a];
            R[r].a[a] = (a < dims) ? rs[a] + 2 * GH : 1;
        }
        R[r].f = (double*)calloc((size_t)NCOMP * rsize(&R[r]), sizeof(double));
        for (int comp = 0; comp < NCOMP; ++comp)
            for (int64_t lk = 0; lk < rs[2]; ++lk)
                for (int64_t lj = 0; lj < rs[1]; ++lj)
                    for (int64_t li = 0; li < rs[0]; ++li)
                        R[r].f[comp * rsize(&R[r]) + ridx(&R[r], li, lj, lk)] =
                            F[comp * NC + gidx(c, R[r].o[0] + li, R[r].o[1] + lj, R[r].o[2] + lk)];
    }
    for (int comp = EX; comp <= BMZ; ++comp) exchange_ghosts(c, R, nR, rs, comp);

    int64_t np[3] = {c->n[0] / c->patch[0], c->n[1] / c->patch[1], (dims == 3) ? c->n[2] / c->patch[2] : 1};
    int64_t nP = np[0] * np[1] * np[2];

    if (!fields_only) {
        /* 2. patches own the particles: stable counting sort of indices */
        int32_t* pid = (int32_t*)malloc(sizeof(int32_t) * (P->n ? P->n : 1));
        oracle_bin(c, P, pid);
        int64_t* off = (int64_t*)calloc(nP + 1, sizeof(int64_t));
        for (int64_t p = 0; p < P->n; ++p) off[pid[p] + 1]++;
        for (int64_t q = 0; q < nP; ++q) off[q + 1] += off[q];
        int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (P->n ? P->n : 1));
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * nP);
        for (int64_t q = 0; q < nP; ++q) fill[q] = off[q];
        for (int64_t p = 0; p < P->n; ++p) order[fill[pid[p]]++] = p;

        /* 3. per patch: window copy (transfer ii), push, deposit into tile */
        int64_t tA[3], wA[3];
        for (int a = 0; a < 3; ++a) {
            tA[a] = (a < dims) ? c->patch[a] + 5 : 1;
            wA[a] = (a < dims) ? c->patch[a] + 3 : 1;
        }
        int64_t tsz = tA[0] * tA[1] * tA[2], wsz = wA[0] * wA[1] * wA[2];
        double* tiles = (double*)calloc((size_t)3 * tsz * nP, sizeof(double));
        double dummy = 0.0;
        /* Patches are independent here: each reads the regions, writes its */
        /* own tile and updates its own particles.  The timing build of the  */
        /* CPU baseline takes them in parallel with dynamic scheduling (the  */
        /* paper's thread model, section 4); the parity build is compiled   */
        /* without OpenMP and ignores the pragma.  Either way the result is  */
        /* the same bit for bit: step 4 sums the tiles in patch order.       */
#pragma omp parallel for schedule(dynamic)
        for (int64_t q = 0; q < nP; ++q) {
            int64_t pq[3] = {q % np[0], (q / np[0]) % np[1], q / (np[0] * np[1])};
            int64_t p0[3];
            for (int a = 0; a < 3; ++a) p0[a] = (a < dims) ? pq[a] * c->patch[a] : 0;
            const region* rg = &R[region_of(c, rs, p0[0], p0[1], p0[2])];
            window W;
            W.lc = *c;
            for (int a = 0; a < 3; ++a) {
                W.o[a] = (a < dims) ? p0[a] - 1 : 0;
                W.a[a] = wA[a];
            }
            W.f = (double*)calloc((size_t)NCOMP * wsz, sizeof(double));
            int comps[6] = {EX, EY, EZ, BMX, BMY, BMZ};
            for (int ci = 0; ci < 6; ++ci)
                for (int64_t lk = 0; lk < wA[2]; ++lk)
                    for (int64_t lj = 0; lj < wA[1]; ++lj)
                        for (int64_t li = 0; li < wA[0]; ++li) {
                            int64_t gi = W.o[0] + li - rg->o[0], gj = W.o[1] + lj - rg->o[1];
                            int64_t gk = (dims == 3) ? W.o[2] + lk - rg->o[2] : 0;
                            W.f[comps[ci] * wsz + li + wA[0] * (lj + wA[1] * lk)] =
                                rg->f[comps[ci] * rsize(rg) + ridx(rg, gi, gj, gk)];
                        }
            tile T;
            T.c = c;
            for (int a = 0; a < 3; ++a) {
                T.o[a] = (a < dims) ? p0[a] - 2 : 0;
                T.a[a] = tA[a];
            }
            T.t = tiles + 3 * tsz * q;
            for (int64_t s = off[q]; s < off[q + 1]; ++s) {
                int64_t p = order[s];
                double* zp = (dims == 3) ? &P->z[p] : &dummy;
                double Xg[3] = {P->x[p] / c->d[0], P->y[p] / c->d[1], (dims == 3) ? *zp / c->d[2] : 0.0};
                /* positions in the unwrapped frame of this patch: a particle */
                /* of the last patch can sit exactly at the clamped edge      */
                double EB[6];
                EB[0] = window_interp(&W, EX, Xg);
                EB[1] = window_interp(&W, EY, Xg);
                EB[2] = window_interp(&W, EZ, Xg);
                EB[3] = window_interp(&W, BMX, Xg);
                EB[4] = window_interp(&W, BMY, Xg);
                EB[5] = window_interp(&W, BMZ, Xg);
                double u[3] = {P->ux[p], P->uy[p], P->uz[p]};
                oracle_boris(c->q / c->m, c->dt, EB, u);
                double g = oracle_gamma(u);
                double nx = P->x[p] + c->dt * u[0] / g;
                double ny = P->y[p] + c->dt * u[1] / g;
                double nz = (dims == 3) ? *zp + c->dt * u[2] / g : 0.0;
                double X1[3] = {nx / c->d[0], ny / c->d[1], (dims == 3) ? nz / c->d[2] : 0.0};
                esirkepov(c, Xg, X1, P->w[p], u[2] / g, tile_add, &T);
                P->ux[p] = u[0];
                P->uy[p] = u[1];
                P->uz[p] = u[2];
                P->x[p] = oracle_wrap(nx, c->n[0] * c->d[0]);
                P->y[p] = oracle_wrap(ny, c->n[1] * c->d[1]);
                if (dims == 3) *zp = oracle_wrap(nz, c->n[2] * c->d[2]);
            }
            free(W.f);
        }

        /* 4. transfer (i): region J = sum of the patch tiles, patch order */
        for (int r = 0; r < nR; ++r)
            for (int comp = JX; comp <= JZ; ++comp)
                for (int64_t s = 0; s < rsize(&R[r]); ++s) R[r].f[comp * rsize(&R[r]) + s] = 0.0;
        for (int64_t q = 0; q < nP; ++q) {
            int64_t pq[3] = {q % np[0], (q / np[0]) % np[1], q / (np[0] * np[1])};
            int64_t to[3];
            for (int a = 0; a < 3; ++a) to[a] = (a < dims) ? pq[a] * c->patch[a] - 2 : 0;
            for (int comp = 0; comp < 3; ++comp)
                for (int64_t lk = 0; lk < tA[2]; ++lk)
                    for (int64_t lj = 0; lj < tA[1]; ++lj)
                        for (int64_t li = 0; li < tA[0]; ++li) {
                            double v = tiles[3 * tsz * q + comp * tsz + li + tA[0] * (lj + tA[1] * lk)];
                            int64_t gi = wrapi(to[0] + li, c->n[0]), gj = wrapi(to[1] + lj, c->n[1]);
                            int64_t gk = (dims == 3) ? wrapi(to[2] + lk, c->n[2]) : 0;
                            region* rg = &R[region_of(c, rs, gi, gj, gk)];
                            rg->f[(JX + comp) * rsize(rg) + ridx(rg, gi - rg->o[0], gj - rg->o[1], gk - rg->o[2])] +=
                                v;
                        }
        }
        free(tiles);
        free(pid);
        free(off);
        free(order);
        free(fill);

        /* 4b. binomial filter on the regions: before each pass the regions  */
        /*     synchronise their J ghosts; a sweep along an axis runs on the */
        /*     interior along that axis and one ghost node further along the */
        /*     axes still to be swept, so the next sweep finds its inputs.   */
        for (int pass = 0; pass < c->filter; ++pass) {
            for (int comp = JX; comp <= JZ; ++comp) exchange_ghosts(c, R, nR, rs, comp);
            for (int r = 0; r < nR; ++r) {
                region* g = &R[r];
                int64_t S = rsize(g);
                double* tmp = (double*)malloc(sizeof(double) * S);
                for (int comp = JX; comp <= JZ; ++comp) {
                    double* f = g->f + comp * S;
                    for (int axis = 0; axis < dims; ++axis) {
                        int64_t lo[3], hi[3];
                        for (int b = 0; b < 3; ++b) {
                            int ext = (b < dims && b > axis) ? 1 : 0;
                            lo[b] = -ext;
                            hi[b] = g->s[b] + ext;
                        }
                        memcpy(tmp, f, sizeof(double) * S);
                        for (int64_t lk = lo[2]; lk < hi[2]; ++lk)
                            for (int64_t lj = lo[1]; lj < hi[1]; ++lj)
                                for (int64_t li = lo[0]; li < hi[0]; ++li) {
                                    int64_t p = ridx(g, li, lj, lk);
                                    int64_t m = ridx(g, li - (axis == 0), lj - (axis == 1), lk - (axis == 2));
                                    int64_t q = ridx(g, li + (axis == 0), lj + (axis == 1), lk + (axis == 2));
                                    tmp[p] = (f[m] + 2.0 * f[p] + f[q]) * 0.25;
                                }
                        memcpy(f, tmp, sizeof(double) * S);
                    }
                }
                free(tmp);
            }
        }
    } else {
        /* currents are taken as given in F */
        for (int r = 0; r < nR; ++r)
            for (int comp = JX; comp <= JZ; ++comp)
                for (int64_t lk = 0; lk < rs[2]; ++lk)
                    for (int64_t lj = 0; lj < rs[1]; ++lj)
                        for (int64_t li = 0; li < rs[0]; ++li)
                            R[r].f[comp * rsize(&R[r]) + ridx(&R[r], li, lj, lk)] =
                                F[comp * NC + gidx(c, R[r].o[0] + li, R[r].o[1] + lj, R[r].o[2] + lk)];
    }

    /* 5. Maxwell on each region: Ampere on the interior, E ghost exchange,  */
    /*    Faraday on the interior, B ghost exchange, Bm.                     */
    double dx = c->d[0], dy = c->d[1], dz = (dims == 3) ? c->d[2] : 1.0, dt = c->dt;
    for (int r = 0; r < nR; ++r) {
        region* g = &R[r];
        int64_t S = rsize(g);
        double* f = g->f;
        int zs = (dims == 3) ? 1 : 0; /* z neighbour offset exists only in 3D */
        for (int64_t lk = 0; lk < g->s[2]; ++lk)
            for (int64_t lj = 0; lj < g->s[1]; ++lj)
                for (int64_t li = 0; li < g->s[0]; ++li) {
                    int64_t p = ridx(g, li, lj, lk);
                    int64_t pjm = ridx(g, li, lj - 1, lk), pim = ridx(g, li - 1, lj, lk);
                    int64_t pkm = zs ? ridx(g, li, lj, lk - 1) : p;
                    f[EX * S + p] += dt * ((f[BZ * S + p] - f[BZ * S + pjm]) / dy - (f[BY * S + p] - f[BY * S + pkm]) / dz -
                                           f[JX * S + p]);
                    f[EY * S + p] += dt * ((f[BX * S + p] - f[BX * S + pkm]) / dz - (f[BZ * S + p] - f[BZ * S + pim]) / dx -
                                           f[JY * S + p]);
                    f[EZ * S + p] += dt * ((f[BY * S + p] - f[BY * S + pim]) / dx - (f[BX * S + p] - f[BX * S + pjm]) / dy -
                                           f[JZ * S + p]);
                }
    }
    for (int comp = EX; comp <= EZ; ++comp) exchange_ghosts(c, R, nR, rs, comp);
    for (int r = 0; r < nR; ++r) {
        region* g = &R[r];
        int64_t S = rsize(g);
        double* f = g->f;
        int zs = (dims == 3) ? 1 : 0;
        for (int64_t lk = 0; lk < g->s[2]; ++lk)
            for (int64_t lj = 0; lj < g->s[1]; ++lj)
                for (int64_t li = 0; li < g->s[0]; ++li) {
                    int64_t p = ridx(g, li, lj, lk);
                    int64_t pjp = ridx(g, li, lj + 1, lk), pip = ridx(g, li + 1, lj, lk);
                    int64_t pkp = zs ? ridx(g, li, lj, lk + 1) : p;
                    double bx = f[BX * S + p], by = f[BY * S + p], bz = f[BZ * S + p];
                    f[BX * S + p] -= dt * ((f[EZ * S + pjp] - f[EZ * S + p]) / dy - (f[EY * S + pkp] - f[EY * S + p]) / dz);
                    f[BY * S + p] -= dt * ((f[EX * S + pkp] - f[EX * S + p]) / dz - (f[EZ * S + pip] - f[EZ * S + p]) / dx);
                    f[BZ * S + p] -= dt * ((f[EY * S + pip] - f[EY * S + p]) / dx - (f[EX * S + pjp] - f[EX * S + p]) / dy);
                    f[BMX * S + p] = 0.5 * (bx + f[BX * S + p]);
                    f[BMY * S + p] = 0.5 * (by + f[BY * S + p]);
                    f[BMZ * S + p] = 0.5 * (bz + f[BZ * S + p]);
                }
    }

    /* 6. assemble the global state from the region interiors */
    for (int r = 0; r < nR; ++r) {
        for (int comp = 0; comp < NCOMP; ++comp)
            for (int64_t lk = 0; lk < rs[2]; ++lk)
                for (int64_t lj = 0; lj < rs[1]; ++lj)
                    for (int64_t li = 0; li < rs[0]; ++li)
                        F[comp * NC + gidx(c, R[r].o[0] + li, R[r].o[1] + lj, R[r].o[2] + lk)] =
                            R[r].f[comp * rsize(&R[r]) + ridx(&R[r], li, lj, lk)];
        free(R[r].f);
    }
    free(R);
    return 0;
}

/* Deposit prescribed moves (x0 -> x1) without pushing: mode 0 straight into */
/* the global grid (SDSD), mode 1 into patch tiles summed into regions in    */
/* patch order (SDMD transfer (i)).  J (3 components) is overwritten.         */
int oracle_deposit_moves(const ocfg* c, int32_t mode, int64_t n, const double* x0, const double* y0,
                         const double* z0, const double* x1, const double* y1, const double* z1, const double* w,
                         const double* vz, double* J)
{
    int dims = c->dims;
    int64_t NC = ncells(c);
    memset(J, 0, sizeof(double) * 3 * NC);
    if (mode == 0) {
        global_add_ctx g = {c, J};
        for (int64_t p = 0; p < n; ++p) {
            double X0[3] = {x0[p] / c->d[0], y0[p] / c->d[1], dims == 3 ? z0[p] / c->d[2] : 0.0};
            double X1[3] = {x1[p] / c->d[0], y1[p] / c->d[1], dims == 3 ? z1[p] / c->d[2] : 0.0};
            esirkepov(c, X0, X1, w[p], vz ? vz[p] : 0.0, global_add, &g);
        }
        return 0;
    }
    if (check_decomp(c)) return -1;
    int64_t np[3] = {c->n[0] / c->patch[0], c->n[1] / c->patch[1], (dims == 3) ? c->n[2] / c->patch[2] : 1};
    int64_t nP = np[0] * np[1] * np[2];
    int64_t tA[3];
    for (int a = 0; a < 3; ++a) tA[a] = (a < dims) ? c->patch[a] + 5 : 1;
    int64_t tsz = tA[0] * tA[1] * tA[2];
    double* tiles = (double*)calloc((size_t)3 * tsz * nP, sizeof(double));
    /* particles grouped by patch of x0, stored order inside a patch */
    oparts P0 = {n, (double*)x0, (double*)y0, (double*)z0, NULL, NULL, NULL, NULL};
    int32_t* pid = (int32_t*)malloc(sizeof(int32_t) * (n ? n : 1));
    oracle_bin(c, &P0, pid);
    for (int64_t q = 0; q < nP; ++q) {
        int64_t pq[3] = {q % np[0], (q / np[0]) % np[1], q / (np[0] * np[1])};
        tile T;
        T.c = c;
        for (int a = 0; a < 3; ++a) {
            T.o[a] = (a < dims) ? pq[a] * c->patch[a] - 2 : 0;
            T.a[a] = tA[a];
        }
        T.t = tiles + 3 * tsz * q;
        for (int64_t p = 0; p < n; ++p) {
            if (pid[p] != q) continue;
            double X0[3] = {x0[p] / c->d[0], y0[p] / c->d[1], dims == 3 ? z0[p] / c->d[2] : 0.0};
            double X1[3] = {x1[p] / c->d[0], y1[p] / c->d[1], dims == 3 ? z1[p] / c->d[2] : 0.0};
            esirkepov(c, X0, X1, w[p], vz ? vz[p] : 0.0, tile_add, &T);
        }
    }
    for (int64_t q = 0; q < nP; ++q) {
        int64_t pq[3] = {q % np[0], (q / np[0]) % np[1], q / (np[0] * np[1])};
        int64_t to[3];
        for (int a = 0; a < 3; ++a) to[a] = (a < dims) ? pq[a] * c->patch[a] - 2 : 0;
        for (int comp = 0; comp < 3; ++comp)
            for (int64_t lk = 0; lk < tA[2]; ++lk)
                for (int64_t lj = 0; lj < tA[1]; ++lj)
                    for (int64_t li = 0; li < tA[0]; ++li) {
                        double v = tiles[3 * tsz * q + comp * tsz + li + tA[0] * (lj + tA[1] * lk)];
                        J[comp * NC + gidx(c, to[0] + li, to[1] + lj, (dims == 3) ? to[2] + lk : 0)] += v;
                    }
    }
    free(tiles);
    free(pid);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                              */
/* ------------------------------------------------------------------------ */
/* charge density on primal nodes: rho = sum q w prod S (ions not included) */
void oracle_rho(const ocfg* c, const oparts* P, double* rho)
{
    int64_t NC = ncells(c);
    memset(rho, 0, sizeof(double) * NC);
    for (int64_t p = 0; p < P->n; ++p) {
        double X[3] = {P->x[p] / c->d[0], P->y[p] / c->d[1], (c->dims == 3) ? P->z[p] / c->d[2] : 0.0};
        int64_t f[3] = {(int64_t)floor(X[0]), (int64_t)floor(X[1]), (int64_t)floor(X[2])};
        int kz0 = (c->dims == 3) ? -2 : 0, kz1 = (c->dims == 3) ? 2 : 0;
        for (int kz = kz0; kz <= kz1; ++kz) {
            double wz = (c->dims == 3) ? oracle_S(X[2] - (double)(f[2] + kz)) : 1.0;
            for (int ky = -2; ky <= 2; ++ky) {
                double wy = oracle_S(X[1] - (double)(f[1] + ky));
                for (int kx = -2; kx <= 2; ++kx) {
                    double wx = oracle_S(X[0] - (double)(f[0] + kx));
                    rho[gidx(c, f[0] + kx, f[1] + ky, (c->dims == 3) ? f[2] + kz : 0)] += c->q * P->w[p] * wx * wy * wz;
                }
            }
        }
    }
}

/* discrete divergence of E on primal nodes (backward differences of the    */
/* dual-staggered components)                                               */
void oracle_divE(const ocfg* c, const double* F, double* div)
{
    int64_t N = ncells(c);
    const double *Ex = F + EX * N, *Ey = F + EY * N, *Ez = F + EZ * N;
    for (int64_t k = 0; k < c->n[2]; ++k)
        for (int64_t j = 0; j < c->n[1]; ++j)
            for (int64_t i = 0; i < c->n[0]; ++i) {
                int64_t p = gidx(c, i, j, k);
                double v = (Ex[p] - Ex[gidx(c, i - 1, j, k)]) / c->d[0] + (Ey[p] - Ey[gidx(c, i, j - 1, k)]) / c->d[1];
                if (c->dims == 3) v += (Ez[p] - Ez[gidx(c, i, j, k - 1)]) / c->d[2];
                div[p] = v;
            }
}

/* out: U_E = 1/2 sum E^2 dV, U_B = 1/2 sum Bm^2 dV, K = sum m w (gamma-1) dV */
void oracle_energy(const ocfg* c, const double* F, const oparts* P, double out[3])
{
    int64_t N = ncells(c);
    double dV = c->d[0] * c->d[1] * ((c->dims == 3) ? c->d[2] : 1.0);
    double ue = 0.0, ub = 0.0, k = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int64_t p = 0; p < N; ++p) {
            ue += F[(EX + a) * N + p] * F[(EX + a) * N + p];
            ub += F[(BMX + a) * N + p] * F[(BMX + a) * N + p];
        }
    for (int64_t p = 0; p < P->n; ++p) {
        double u[3] = {P->ux[p], P->uy[p], P->uz[p]};
        k += c->m * P->w[p] * (oracle_gamma(u) - 1.0);
    }
    out[0] = 0.5 * ue * dV;
    out[1] = 0.5 * ub * dV;
    out[2] = k * dV;
}
