/*
 * Plain FP64 CPU oracle for the axisymmetric Allen-Cahn MRT lattice Boltzmann
 * model (Liang, Li, Chen & Xu, "Axisymmetric lattice Boltzmann model for
 * multiphase flows with large density ratio", arXiv:1810.09299).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plainly written reference that
 * the HIP library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the HIP library, and the HIP library never calls it.
 *
 * Layout of every field: [nr][nz] with z fastest; population arrays are
 * [9][nr][nz].  Row j sits at r_j = j + 1/2, column k at z_k = k.
 */
#ifndef AXI_ORACLE_H
#define AXI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nr, nz;
    int32_t z_periodic;               /* 1: periodic in z, 0: no-slip walls at both z ends */
    int32_t dispersed_gas;            /* diagnostics only: 0 tracks phi (drop), 1 tracks 1-phi (bubble) */
    int32_t collision;                /* 0: MRT (Eqs. 9-10, 24); 1: SRT, every rate 1/tau (Sec. 2.2);
                                         2: non-orthogonal (raw-moment) MRT (Sec. 4) */
    int32_t alt;                      /* alternative readings, ORA_ALT_* bits; 0 = the adopted ones */
    int32_t free_s1;                  /* 1: s_1^g = s_g[1] instead of 1/tau_g (an extension) */
    int32_t reserved;                 /* 0 */
    double W, mobility, sigma;        /* interface width, mobility M, surface tension */
    double rho_l, rho_g, nu_l, nu_g;  /* bulk densities and kinematic viscosities */
    double g_z;                       /* axial acceleration of the buoyancy force */
    double g_ramp;                    /* steps over which g_z is reached linearly (0: at once) */
    double s_f[9], s_g[9];            /* relaxation rates; s_f[3..6] and s_g[1,7,8] are derived */
} ora_params;

/* Alternative readings where the paper is silent, for the tests that compare
 * them with the adopted readings (see axi_oracle.c); never set otherwise. */
#define ORA_ALT_JOINT_PU 1   /* Eqs. 32-33 solved together within the step        */
#define ORA_ALT_ODD_AXIS 2   /* odd (sign-flipped) axis image of the populations   */
#define ORA_ALT_FREE_S1 4    /* s_1^g from s_g[1], not tied to 1/tau_g              */

typedef struct {
    int64_t t;
    double phase_mass, fluid_mass, mom_z, umax;
    double p_in, p_out, dp, R_eq, semi_z, semi_r, centroid_z, rise_u, min_axis_phi;
    int64_t nonfinite;
} ora_diag;

typedef struct ora_case ora_case;

ora_case *ora_create(const ora_params *p, const double *phi0);
void ora_destroy(ora_case *c);
void ora_step(ora_case *c, int64_t nsteps);
/* one step that also returns the post-collision populations and the total force */
void ora_step_debug(ora_case *c, double *f_post, double *g_post, double *Fz, double *Fr);
int64_t ora_time(const ora_case *c);
void ora_moments(const ora_case *c, double *phi, double *rho, double *uz, double *ur, double *p);
void ora_diagnostics(const ora_case *c, ora_diag *d);
void ora_get_state(const ora_case *c, double *f, double *g, double *aux);
void ora_set_state(ora_case *c, const double *f, const double *g, const double *aux, int64_t t);

/* pieces exported for the pins */
void ora_lattice(int32_t *cz, int32_t *cr, double *w, double *Mmat, double *Minv);
void ora_stencil(int32_t nr, int32_t nz, int32_t z_periodic, const double *chi,
                 double *dz, double *dr, double *lap);
void ora_stream(int32_t nr, int32_t nz, int32_t z_periodic, const double *post, double *out);
void ora_rates(const ora_case *c, double *s_f, double *s_g_nonnu);

#ifdef __cplusplus
}
#endif
#endif
