/*
 * sanitize_check.c -- drives every entry point of the oracle under the
 * address and undefined-behaviour sanitizers (test infrastructure, like the
 * oracle itself; built and run by the CPU test suite with gcc).
 *
 * It includes pic_oracle.c into one translation unit and runs, on small
 * seeded 2D and 3D cases with particles crossing patch, region and periodic
 * boundaries:
 *   - SDSD and SDMD steps (with and without the binomial filter), checking
 *     that the two decompositions give the same fields and particles
 *     (section 2.2: SDMD re-decomposes one domain), to round-off;
 *   - the per-patch and the global deposition of the same moves
 *     (oracle_deposit_moves, both modes), which must agree;
 *   - interpolation, Boris, binning, the split position form, charge
 *     density, the discrete divergence and the energies.
 * Any out-of-bounds access, leak, overflow or other undefined behaviour
 * aborts the run with the sanitizer's report; a failed check exits 1.
 */
#include "pic_oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x243F6A8885A308D3ull;

/* splitmix64: a seeded uniform in [0, 1) */
static double urand(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

typedef struct {
    double *x, *y, *z, *ux, *uy, *uz, *w;
} pbuf;

static oparts make_parts(const ocfg* c, int64_t n, pbuf* b)
{
    double** arr[7] = {&b->x, &b->y, &b->z, &b->ux, &b->uy, &b->uz, &b->w};
    for (int k = 0; k < 7; ++k) *arr[k] = (double*)malloc(sizeof(double) * (size_t)n);
    double L[3] = {c->n[0] * c->d[0], c->n[1] * c->d[1], c->dims == 3 ? c->n[2] * c->d[2] : 1.0};
    for (int64_t p = 0; p < n; ++p) {
        b->x[p] = urand() * L[0];
        b->y[p] = urand() * L[1];
        b->z[p] = c->dims == 3 ? urand() * L[2] : 0.0;
        /* fast enough that many particles change cell, patch and region */
        b->ux[p] = 1.5 * (urand() - 0.5);
        b->uy[p] = 1.5 * (urand() - 0.5);
        b->uz[p] = 1.5 * (urand() - 0.5);
        b->w[p] = 0.01 + 0.02 * urand();
    }
    oparts P = {n, b->x, b->y, b->z, b->ux, b->uy, b->uz, b->w};
    return P;
}

static oparts copy_parts(const oparts* s, pbuf* b)
{
    const double* src[7] = {s->x, s->y, s->z, s->ux, s->uy, s->uz, s->w};
    double** dst[7] = {&b->x, &b->y, &b->z, &b->ux, &b->uy, &b->uz, &b->w};
    for (int k = 0; k < 7; ++k) {
        *dst[k] = (double*)malloc(sizeof(double) * (size_t)s->n);
        memcpy(*dst[k], src[k], sizeof(double) * (size_t)s->n);
    }
    oparts P = {s->n, b->x, b->y, b->z, b->ux, b->uy, b->uz, b->w};
    return P;
}

static void free_parts(pbuf* b)
{
    free(b->x);
    free(b->y);
    free(b->z);
    free(b->ux);
    free(b->uy);
    free(b->uz);
    free(b->w);
}

static double maxabs_diff(const double* a, const double* b, int64_t n)
{
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (fabs(a[i] - b[i]) > m) m = fabs(a[i] - b[i]);
    return m;
}

static int fails = 0;

static void expect(int ok, const char* what, double v)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s (%g)\n", what, v);
        fails++;
    }
}

static void run_case(ocfg c, int64_t n, int steps)
{
    const int64_t NC = (int64_t)c.n[0] * c.n[1] * c.n[2];
    double* F0 = (double*)calloc((size_t)NCOMP * NC, sizeof(double));
    for (int64_t i = 0; i < 6 * NC; ++i) F0[i] = 0.05 * (urand() - 0.5);
    oracle_init_fields(&c, F0);
    pbuf ba, bb;
    oparts PA = make_parts(&c, n, &ba);
    oparts PB = copy_parts(&PA, &bb);
    double* FA = (double*)malloc(sizeof(double) * (size_t)NCOMP * NC);
    double* FB = (double*)malloc(sizeof(double) * (size_t)NCOMP * NC);
    memcpy(FA, F0, sizeof(double) * (size_t)NCOMP * NC);
    memcpy(FB, F0, sizeof(double) * (size_t)NCOMP * NC);

    for (int s = 0; s < steps; ++s) {
        oracle_step_sdsd(&c, FA, &PA);
        expect(oracle_step_sdmd(&c, FB, &PB, 0) == 0, "sdmd step accepted", 0.0);
    }
    const double dF = maxabs_diff(FA, FB, NCOMP * NC);
    expect(dF < 1e-12, "SDMD fields == SDSD fields", dF);
    double dP = 0.0;
    const double* pa[6] = {PA.x, PA.y, PA.z, PA.ux, PA.uy, PA.uz};
    const double* pb[6] = {PB.x, PB.y, PB.z, PB.ux, PB.uy, PB.uz};
    for (int k = 0; k < 6; ++k) {
        const double d = maxabs_diff(pa[k], pb[k], n);
        if (d > dP) dP = d;
    }
    expect(dP < 1e-12, "SDMD particles == SDSD particles", dP);

    /* diagnostics on the final state */
    double* rho = (double*)malloc(sizeof(double) * (size_t)NC);
    double* div = (double*)malloc(sizeof(double) * (size_t)NC);
    oracle_rho(&c, &PA, rho);
    oracle_divE(&c, FA, div);
    double en[3];
    oracle_energy(&c, FA, &PA, en);
    expect(isfinite(en[0]) && isfinite(en[1]) && isfinite(en[2]), "finite energies", en[0]);
    int32_t* pid = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    oracle_bin(&c, &PA, pid);
    int64_t np = (int64_t)(c.n[0] / c.patch[0]) * (c.n[1] / c.patch[1]) * (c.dims == 3 ? c.n[2] / c.patch[2] : 1);
    int bad = 0;
    for (int64_t p = 0; p < n; ++p) bad += pid[p] < 0 || pid[p] >= np;
    expect(bad == 0, "patch ids in range", bad);
    for (int64_t p = 0; p < n; p += 7) {
        int32_t cell;
        float xi;
        oracle_split(PA.x[p], c.d[0], c.n[0], &cell, &xi);
        expect(cell >= 0 && cell < c.n[0] && xi >= 0.0f && xi < 1.0f, "split form in range", xi);
        double eb[6];
        oracle_interp(&c, FA, PA.x[p], PA.y[p], PA.z[p], eb);
        double u[3] = {PA.ux[p], PA.uy[p], PA.uz[p]};
        oracle_boris(c.q / c.m, c.dt, eb, u);
        expect(isfinite(u[0] + u[1] + u[2]), "finite Boris momentum", u[0]);
    }
    free(pid);
    free(rho);
    free(div);
    free_parts(&ba);
    free_parts(&bb);
    free(FA);
    free(FB);
    free(F0);
}

/* oracle_deposit_moves: per-patch tiles summed into the grid (mode 1) equal
   the global deposition (mode 0) of the same moves */
static void deposit_case(ocfg c, int64_t n)
{
    const int64_t NC = (int64_t)c.n[0] * c.n[1] * c.n[2];
    const double L[3] = {c.n[0] * c.d[0], c.n[1] * c.d[1], c.dims == 3 ? c.n[2] * c.d[2] : 1.0};
    double* b[8];
    for (int k = 0; k < 8; ++k) b[k] = (double*)malloc(sizeof(double) * (size_t)n);
    double *x0 = b[0], *y0 = b[1], *z0 = b[2], *x1 = b[3], *y1 = b[4], *z1 = b[5], *w = b[6], *vz = b[7];
    for (int64_t p = 0; p < n; ++p) {
        x0[p] = urand() * L[0];
        y0[p] = urand() * L[1];
        z0[p] = c.dims == 3 ? urand() * L[2] : 0.0;
        /* moves of up to 0.9 cell, across patch and periodic boundaries */
        x1[p] = x0[p] + 0.9 * (2.0 * urand() - 1.0) * c.d[0];
        y1[p] = y0[p] + 0.9 * (2.0 * urand() - 1.0) * c.d[1];
        z1[p] = c.dims == 3 ? z0[p] + 0.9 * (2.0 * urand() - 1.0) * c.d[2] : 0.0;
        w[p] = 0.01 + urand();
        vz[p] = urand() - 0.5;
    }
    double* Jg = (double*)malloc(sizeof(double) * 3 * (size_t)NC);
    double* Jt = (double*)malloc(sizeof(double) * 3 * (size_t)NC);
    expect(oracle_deposit_moves(&c, 0, n, x0, y0, z0, x1, y1, z1, w, vz, Jg) == 0, "global deposit", 0.0);
    expect(oracle_deposit_moves(&c, 1, n, x0, y0, z0, x1, y1, z1, w, vz, Jt) == 0, "tile deposit", 0.0);
    double m = 0.0;
    for (int64_t i = 0; i < 3 * NC; ++i)
        if (fabs(Jg[i]) > m) m = fabs(Jg[i]);
    const double d = maxabs_diff(Jg, Jt, 3 * NC);
    expect(m > 0.0 && d <= 1e-12 * m, "tiles summed == global deposition", d);
    for (int k = 0; k < 8; ++k) free(b[k]);
    free(Jg);
    free(Jt);
    double f[64];
    for (int i = 0; i < 64; ++i) f[i] = urand();
    ocfg c1 = c;
    c1.dims = 2;
    c1.n[0] = 8;
    c1.n[1] = 8;
    c1.n[2] = 1;
    oracle_filter(&c1, f, 1, 2);
}

int main(void)
{
    ocfg c2 = {2, {32, 16, 1}, {0.2, 0.25, 1.0}, 0.0, -1.0, 1.0, {8, 4, 1}, {2, 2, 1}, 0};
    c2.dt = 0.9 / sqrt(1.0 / (c2.d[0] * c2.d[0]) + 1.0 / (c2.d[1] * c2.d[1]));
    run_case(c2, 2000, 4);
    c2.filter = 2;
    run_case(c2, 2000, 3);
    ocfg c3 = {3, {8, 8, 12}, {0.2, 0.2, 0.2}, 0.0, -1.0, 1.0, {4, 4, 4}, {2, 1, 3}, 0};
    c3.dt = 0.9 / sqrt(3.0 / (0.2 * 0.2));
    run_case(c3, 1500, 2);
    c3.filter = 1;
    run_case(c3, 1500, 2);
    deposit_case(c2, 3000);
    deposit_case(c3, 2000);
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
