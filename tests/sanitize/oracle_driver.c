/* Test driver: runs every entry point of the CPU oracle on small 1-D, 2-D and
 * 3-D grids (periodic and outflow faces, every option) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer can check the oracle's
 * memory accesses and arithmetic.  Exit status 0 when every call returns
 * and every result is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include "wombat_oracle.h"

static int bad = 0;
static void check(const char *what, double x)
{
    if (!isfinite(x)) { fprintf(stderr, "non-finite %s\n", what); bad = 1; }
}

/* a smooth magnetised state: rho, p > 0 everywhere */
static void fill_state(const orc_grid *g, double *u)
{
    long n = orc_state_size(g), i;
    for (i = 0; i < n; ++i) u[i] = 0.0;
    int nx = g->nx, ny = g->ny, nz = g->nz;
    int gx = nx > 1 ? 3 : 0, gy = ny > 1 ? 3 : 0, gz = nz > 1 ? 3 : 0;
    long sx = 1, sy = nx + 2 * gx, sz = (long)(nx + 2 * gx) * (ny + 2 * gy);
    long sv = sz * (nz + 2 * gz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int ii = 0; ii < nx; ++ii) {
                double x = (ii + 0.5) / nx, y = (j + 0.5) / ny, z = (k + 0.5) / nz;
                double W[8] = { 1.0 + 0.3 * sin(6.28318 * (x + y)), 0.3 * cos(6.28318 * z), -0.2, 0.1 * sin(6.28318 * y),
                                0.7, 0.4 * cos(6.28318 * x), -0.3, 1.0 + 0.2 * cos(6.28318 * (y + z)) };
                double U[8];
                orc_prim_to_cons(W, g->gamma, U);
                long id = (ii + gx) * sx + (j + gy) * sy + (k + gz) * sz;
                for (int v = 0; v < 8; ++v) u[v * sv + id] = U[v];
            }
}

static void run_grid(int nx, int ny, int nz, int outflow)
{
    orc_grid g = { nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz, 5.0 / 3.0, 0.4, 1e-6,
                   { 0, 0, 0, 0, 0, 0 }, 0, 0 };
    if (outflow) for (int f = 0; f < 6; ++f) g.bc[f] = 1;
    long n = orc_state_size(&g);
    double *u = malloc(sizeof(double) * n), *d = malloc(sizeof(double) * n), a[7], s[8], mx, l1;
    for (int weights = 0; weights < 2; ++weights)
        for (int lf = 0; lf < 2; ++lf) {
            g.weights = weights;
            g.lf_global = lf;
            fill_state(&g, u);
            orc_fill_ghosts(&g, u);
            if (orc_rhs(&g, u, d)) bad = 1;
            if (orc_rhs_nofill(&g, u, d)) bad = 1;
            if (orc_rhs_linear(&g, u, d)) bad = 1;
            for (int dir = 0; dir < 3; ++dir) orc_lf_global(&g, u, dir, a);
            double dt = orc_cfl_dt(&g, u);
            check("dt", dt);
            if (orc_rk4_step(&g, u, dt)) bad = 1;
            if (orc_ssprk3_step(&g, u, orc_cfl_dt(&g, u))) bad = 1;
            orc_sums(&g, u, s);
            orc_divb(&g, u, &mx, &l1);
            for (int v = 0; v < 8; ++v) check("sum", s[v]);
            check("divb", mx);
        }
    free(u);
    free(d);
}

int main(void)
{
    double Us[48], F[8], L[64], R[64], lam[8], om[3], is[3], dev, a7[7] = { 1, 1, 1, 1, 1, 1, 1 };
    for (int j = 0; j < 6; ++j) {
        double W[8] = { 1.0 + 0.1 * j, 0.2, -0.1, 0.3, 0.5, 0.2 * j, -0.4, 1.0 };
        orc_prim_to_cons(W, 5.0 / 3.0, Us + 8 * j);
    }
    orc_interface_flux(Us, 5.0 / 3.0, 1e-6, F);
    orc_interface_flux_ex(Us, 5.0 / 3.0, 1e-6, 1, F, &dev);
    orc_interface_flux_z(Us, 5.0 / 3.0, 1e-6, F);
    orc_interface_flux_alpha(Us, 5.0 / 3.0, 1e-6, 1, a7, F);
    orc_linear_flux(Us, 5.0 / 3.0, F);
    for (int c = 0; c < 8; ++c) check("flux", F[c]);
    double Wn[8] = { 1.0, 0.1, 0.2, -0.3, 0.0, 0.0, 0.0, 0.6 };      /* B = 0: degenerate */
    orc_eigensystem(Wn, 5.0 / 3.0, lam, L, R);
    orc_weno_weights(0, 0, 1, 0, 1e-6, om, is);
    orc_weno_weights_z(0, 0, 1, 0, 1e-6, om, is);
    check("phi", orc_weno_phi(0.1, 0.2, -0.3, 0.4, 1e-6));
    double f6[6] = { 1, 2, 3, 2, 1, 0 }, u6[6] = { 0, 1, 0, 1, 0, 1 };
    check("field", orc_weno_field_flux(f6, u6, 1.5, 1e-6));
    check("field_z", orc_weno_field_flux_z(f6, u6, 1.5, 1e-6));
    run_grid(16, 1, 1, 1);
    run_grid(12, 9, 1, 0);
    run_grid(1, 10, 8, 1);
    run_grid(9, 8, 7, 0);
    printf(bad ? "FAILED\n" : "ok\n");
    return bad;
}
