/*
 * Drives every entry point of the FP64 oracle on small grids, for the
 * sanitizer check in tests/test_oracle_sanitized.py (built with gcc and
 * -fsanitize=address,undefined; no GPU involved).  Every collision form,
 * both z modes, the alternative readings, the free energy-moment rate and a
 * gravity ramp; exit status 0 when every result is finite and the phase mass
 * is conserved to rounding.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/axi_oracle.h"

static int run_case(int nr, int nz, int zper, int collision, int alt, int free_s1, double g_ramp)
{
    ora_params p;
    memset(&p, 0, sizeof p);
    p.nr = nr;
    p.nz = nz;
    p.z_periodic = zper;
    p.dispersed_gas = zper ? 0 : 1;
    p.collision = collision;
    p.alt = alt;
    p.free_s1 = free_s1;
    p.W = 4.0;
    p.mobility = 0.1;
    p.sigma = 1e-3;
    p.rho_l = 1.0;
    p.rho_g = 0.1;
    p.nu_l = 0.1;
    p.nu_g = 0.1;
    p.g_z = zper ? 0.0 : -1e-5;
    p.g_ramp = g_ramp;
    for (int i = 0; i < 9; ++i) {
        p.s_f[i] = 1.0;
        p.s_g[i] = 1.0;
    }
    if (free_s1) p.s_g[1] = 1.2;
    const size_t nn = (size_t)nr * nz;
    double *phi0 = malloc(nn * sizeof(double));
    const double R = 0.3 * (nr < nz ? nr : nz), zc = 0.5 * nz;
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            const double r = j + 0.5, dz = k - zc, d = R - sqrt(r * r + dz * dz);
            phi0[(size_t)j * nz + k] = 0.5 + 0.5 * tanh(2.0 * d / p.W);
        }
    ora_case *c = ora_create(&p, phi0);
    if (!c) return 1;
    double *f = malloc(9 * nn * sizeof(double)), *g = malloc(9 * nn * sizeof(double));
    double *aux = malloc(3 * nn * sizeof(double));
    double *fp = malloc(9 * nn * sizeof(double)), *gp = malloc(9 * nn * sizeof(double));
    double *Fz = malloc(nn * sizeof(double)), *Fr = malloc(nn * sizeof(double));
    double *fld = malloc(5 * nn * sizeof(double));
    ora_diag d0, d1;
    ora_diagnostics(c, &d0);
    ora_step(c, 7);
    ora_step_debug(c, fp, gp, Fz, Fr);
    ora_get_state(c, f, g, aux);
    ora_set_state(c, f, g, aux, ora_time(c));
    ora_step(c, 5);
    ora_moments(c, fld, fld + nn, fld + 2 * nn, fld + 3 * nn, fld + 4 * nn);
    ora_diagnostics(c, &d1);
    double sf[9], sg[9];
    ora_rates(c, sf, sg);
    int bad = d1.nonfinite != 0 || ora_time(c) != 13;
    for (size_t n = 0; n < 5 * nn; ++n) bad |= !isfinite(fld[n]);
    for (size_t n = 0; n < 9 * nn; ++n) bad |= !isfinite(fp[n]) || !isfinite(gp[n]);
    /* the specular axis image and bounce-back conserve the phase mass; the
       odd axis image (alt bit 2) does not */
    if (!(alt & 2)) bad |= fabs(d1.phase_mass - d0.phase_mass) > 1e-11 * fabs(d0.phase_mass);
    ora_destroy(c);
    free(phi0); free(f); free(g); free(aux); free(fp); free(gp); free(Fz); free(Fr); free(fld);
    if (bad) fprintf(stderr, "case nr=%d nz=%d zper=%d collision=%d alt=%d free_s1=%d failed\n", nr, nz, zper,
                     collision, alt, free_s1);
    return bad;
}

int main(void)
{
    int fails = 0;
    /* the lattice, the stencil and the propagation pieces */
    int32_t cz[9], cr[9];
    double w[9], M[81], Minv[81];
    ora_lattice(cz, cr, w, M, Minv);
    const int nr = 9, nz = 13;
    double *chi = malloc((size_t)nr * nz * sizeof(double)), *dz = malloc((size_t)nr * nz * sizeof(double));
    double *dr = malloc((size_t)nr * nz * sizeof(double)), *lap = malloc((size_t)nr * nz * sizeof(double));
    double *post = malloc(9 * (size_t)nr * nz * sizeof(double)), *out = malloc(9 * (size_t)nr * nz * sizeof(double));
    for (int n = 0; n < nr * nz; ++n) chi[n] = sin(0.3 * n);
    for (int n = 0; n < 9 * nr * nz; ++n) post[n] = cos(0.1 * n);
    for (int zper = 0; zper < 2; ++zper) {
        ora_stencil(nr, nz, zper, chi, dz, dr, lap);
        ora_stream(nr, nz, zper, post, out);
    }
    free(chi); free(dz); free(dr); free(lap); free(post); free(out);
    /* whole cases: 4 x 4 (the smallest grid), a ragged grid, both z modes */
    const int grids[3][2] = {{4, 4}, {11, 17}, {16, 24}};
    for (int gi = 0; gi < 3; ++gi)
        for (int zper = 0; zper < 2; ++zper)
            for (int col = 0; col < 3; ++col) {
                fails += run_case(grids[gi][0], grids[gi][1], zper, col, 0, 0, 0.0);
                if (col != 1) fails += run_case(grids[gi][0], grids[gi][1], zper, col, 0, 1, 6.0);
            }
    for (int alt = 1; alt < 8; ++alt) fails += run_case(11, 17, 1, 0, alt, 0, 0.0);
    printf("oracle sanitizer run: %d failing cases\n", fails);
    return fails != 0;
}
