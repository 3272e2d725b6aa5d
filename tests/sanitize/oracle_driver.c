/* Driver for a sanitizer build of the oracle (test infrastructure): two steps
 * of every reconstruction on small ragged grids with periodic, outflow and
 * mixed boundaries, plus each unit entry point, so that AddressSanitizer and
 * UndefinedBehaviorSanitizer see every loop of the oracle's source.  Exits 0
 * when every call returns VREF_OK and every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "vlct_ref.h"

static int finite_all(const double *a, size_t n)
{
    for (size_t q = 0; q < n; ++q)
        if (!isfinite(a[q])) return 0;
    return 1;
}

static int run_grid(int nx, int ny, int nz, int recon, const int bc[3])
{
    vref_grid g = {nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, 5.0 / 3.0, 0.4, recon,
                   {bc[0], bc[1], bc[2]}};
    const size_t nc = (size_t)nx * ny * nz;
    const size_t len[8] = {nc, nc, nc, nc, nc, (size_t)(nx + 1) * ny * nz,
                           (size_t)nx * (ny + 1) * nz, (size_t)nx * ny * (nz + 1)};
    double *st[8], *out[8];
    for (int f = 0; f < 8; ++f) {
        st[f] = malloc(len[f] * sizeof(double));
        out[f] = malloc(len[f] * sizeof(double));
        if (!st[f] || !out[f]) return 1;
    }
    const double pi = 3.14159265358979323846;
    /* smooth state; B = (1, 0.3 + 0.1 sin(2 pi x), 0.2) is divergence-free */
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = ((size_t)k * ny + j) * nx + i;
                const double x = (i + 0.5) / nx, y = (j + 0.5) / ny, z = (k + 0.5) / nz;
                const double rho = 1.0 + 0.2 * sin(2 * pi * (x + y)) * cos(2 * pi * z);
                const double vx = 0.5 * sin(2 * pi * y), vy = 0.4 * cos(2 * pi * z),
                             vz = 0.3 * sin(2 * pi * x);
                const double by = 0.3 + 0.1 * sin(2 * pi * x);
                st[0][c] = rho;
                st[1][c] = rho * vx;
                st[2][c] = rho * vy;
                st[3][c] = rho * vz;
                st[4][c] = 0.6 / (5.0 / 3.0 - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz) +
                           0.5 * (1.0 + by * by + 0.04);
            }
    for (size_t q = 0; q < len[5]; ++q) st[5][q] = 1.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i)
                st[6][((size_t)k * (ny + 1) + j) * nx + i] = 0.3 + 0.1 * sin(2 * pi * (i + 0.5) / nx);
    for (size_t q = 0; q < len[7]; ++q) st[7][q] = 0.2;
    double dt = 0.0;
    int rc = vref_cfl_dt(&g, (const double *const *)st, &dt, 1);
    for (int s = 0; s < 2 && rc == VREF_OK; ++s) {
        double next = 0.0;
        uint32_t status = 0;
        rc = vref_step(&g, (const double *const *)st, out, dt, &next, &status, 1);
        for (int f = 0; f < 8 && rc == VREF_OK; ++f)
            if (!finite_all(out[f], len[f])) rc = 99;
        for (int f = 0; f < 8; ++f) {
            double *t = st[f];
            st[f] = out[f];
            out[f] = t;
        }
        dt = next;
    }
    if (rc == VREF_OK) {
        /* the stage hooks and diagnostics on the final state */
        const size_t ne = (size_t)(nx + 1) * (ny + 1) * (nz + 1);
        double *ex = malloc(ne * sizeof(double)), *ey = malloc(ne * sizeof(double)),
               *ez = malloc(ne * sizeof(double));
        rc = vref_edge_emfs(&g, (const double *const *)st, recon, ex, ey, ez, 1);
        double *bo[3] = {out[5], out[6], out[7]};
        const double *bi[3] = {st[5], st[6], st[7]};
        if (rc == VREF_OK) vref_ct_update(&g, bi, bo, ex, ey, ez, dt);
        if (rc == VREF_OK) rc = vref_half_step(&g, (const double *const *)st, out, dt, 1);
        if (rc == VREF_OK && !isfinite(vref_divb_norm(&g, (const double *const *)st))) rc = 98;
        free(ex);
        free(ey);
        free(ez);
    }
    for (int f = 0; f < 8; ++f) {
        free(st[f]);
        free(out[f]);
    }
    return rc;
}

int main(void)
{
    const int bcs[3][3] = {{0, 0, 0}, {1, 1, 1}, {1, 0, 1}};
    int bad = 0;
    for (int recon = 1; recon <= 5; ++recon)
        for (int b = 0; b < 3; ++b) {
            const int rc = run_grid(7, 6, 5, recon, bcs[b]);
            if (rc) {
                printf("recon %d bc set %d: rc %d\n", recon, b, rc);
                ++bad;
            }
        }
    /* unit entry points */
    const double w[35] = {1.0, 0.3, -0.2, 0.1, 0.6, 0.4, -0.3, 1.1, 0.2, -0.1, 0.2, 0.65, 0.35, -0.25,
                          1.2, 0.1, 0.0, 0.3, 0.7, 0.3, -0.2, 1.15, 0.0, 0.1, 0.35, 0.68, 0.25, -0.15,
                          1.05, -0.1, 0.2, 0.4, 0.62, 0.2, -0.1};
    double fl[8], fm[7], fp[7], R[49], L[49], lam[7], cf, cs;
    vref_wave_speeds(1.0, 0.6, 1.0, 0.4, -0.3, 5.0 / 3.0, &cf, &cs);
    vref_hlld(w, w + 7, 0.8, 5.0 / 3.0, fl);
    vref_phys_flux(w, 0.8, 5.0 / 3.0, fl);
    vref_eigen(w, 0.8, 5.0 / 3.0, R, L, lam);
    vref_plmc(w, 0.8, 5.0 / 3.0, fm, fp);
    vref_ppmc(w, 0.8, 5.0 / 3.0, fm, fp);
    vref_plmp(w, fm, fp);
    vref_ppmp(w, 0.8, 5.0 / 3.0, fm, fp);
    if (!finite_all(fm, 7) || !finite_all(fp, 7) || !isfinite(cf) || !isfinite(cs)) ++bad;
    printf("oracle sanitizer driver: %d failures\n", bad);
    return bad != 0;
}
