/*
 * Plain FP64 CPU oracle for the axisymmetric Allen-Cahn MRT lattice Boltzmann
 * model of Liang, Li, Chen & Xu (arXiv:1810.09299).
 *
 * TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the HIP library never calls it and shares no code
 * with it.  It is written for checking by eye against the paper, not for speed:
 * every node is visited with plain loops, every equation is evaluated in the
 * form the paper prints it, and all arithmetic is IEEE double without
 * contraction (built with -O2 -ffp-contract=off, no fast-math).
 *
 * One time step, in the paper's order (Sec. 2.2-2.3):
 *   phase field (Eq. 16) -> isotropic gradient/Laplacian (Eqs. 39-40, ghost
 *   rules of Sec. 2.3) -> density/viscosity (Eqs. 17, 35) -> chemical
 *   potential and surface force (Eqs. 2, 4 and the axisymmetric mu~ of
 *   Sec. 2.1) -> pressure (Eq. 33) -> velocity (Eq. 32) -> total force
 *   (Eq. 30) -> MRT collision of f in moment space (Eqs. 19, 21-23) and of g
 *   (Eqs. 24, 27-28, 36-37) -> propagation (Eq. 20) with the axis and wall
 *   conditions of Sec. 2.3.
 *
 * Readings taken where the paper is silent (each marked "reading:" below):
 *   R-axis   x of Eq. 12 is z, y is r (Eq. 21 puts u_z in moment 3, u_r in 5).
 *   R-nodes  node (k, j) sits at z = k, r = j + 1/2; the r-wall is half-way
 *            beyond the last row.
 *   R-dt     the first step takes d_t J = 0 (previous state = initial state).
 *   R-n      n = 0 where |grad phi| <= 1e-12.
 *   R-pu     pressure (Eq. 33) uses the previous step's velocity; velocity
 *            (Eq. 32) then uses that pressure; force, equilibria and source
 *            all use the new (p, u).
 *   R-rates  s_f[3..6] = 1/tau_f (Eq. 18 and the relations of Sec. 3.1);
 *            s_g[1] = s_g[7] = s_g[8] = 1/tau_g(phi) (Eqs. 34-35).
 *   R-grad   grad rho comes from Eq. 39 applied to rho; d(r rho) is
 *            r d(rho) + rho delta_{beta r} (product rule).
 *   R-ghost  stencil ghosts: mirror about the axis and about every wall,
 *            periodic wrap in z when periodic.
 *   R-bc     pull propagation: a source inside the grid is read directly;
 *            a source beyond a wall (r-wall, z-wall, or a corner that also
 *            touches the axis) gives half-way bounce-back of the node's own
 *            opposite population; a source beyond the axis only is the
 *            specular image (c_r flipped) of the axis-row node it mirrors.
 *   R-grav   G = ((rho - rho_l) g_z, 0): buoyancy relative to the liquid.
 *   R-init   u = 0, p = 0, g = 0, f = f^eq(phi0, 0) + h with h the exact
 *            discrete non-equilibrium part of a uniform phi (see ora_create).
 *   R-region diagnostics: sums weighted by psi = phi (or 1 - phi for a
 *            bubble) over the nodes with psi > 1/100, so that a bulk phase
 *            field slightly off 0 or 1 on a large grid does not count:
 *            R_eq = (1.5 sum r psi)^(1/3) (volume 2 pi sum r psi), centroid
 *            and rise velocity the psi-weighted means of z and u_z.
 *
 * SRT (collision = 1): the special case the paper notes at the end of
 * Sec. 2.2, every rate equal, here 1/tau_f for f and 1/tau_g(phi) for g (so
 * s_2^g = 1/tau_g in s_p too).  It is evaluated in population space from the
 * paper's population-space forms -- equilibria Eqs. 11 and 25-26, sources
 * Eqs. 14-15 and 27-30 with M^-1 (I - S/2) M = (1 - s/2) I -- not through the
 * moment-space route of the MRT collision, so that the two can be checked
 * against each other.
 *
 * Two parameters beyond the paper's statement of the problem:
 *   g_ramp    the acceleration g_z is reached linearly over the first g_ramp
 *             steps: the step from time t uses g_z (t + 1) / g_ramp while
 *             t + 1 < g_ramp (the paper's G is any external force; its bubble
 *             test, whose start this is for, is missing from the text).
 *   free_s1   an extension: the energy moment relaxes at s_g[1] as given, in
 *             the collision and in s_p of Eq. 33, instead of the 1/tau_g that
 *             Sec. 2.3 ties it to (that constraint limits tau_g to about
 *             (0.65, 1.15); see the stability tests).  Not the paper's method.
 *
 * Alternative readings (ora_params.alt, a bit mask, 0 for every check of the
 * HIP library), only for the tests that compare a reading with its
 * alternatives where the paper leaves the choice open:
 *   ORA_ALT_JOINT_PU  pressure (Eq. 33) and velocity (Eq. 32) solved together:
 *                     alternated within the step until neither changes (at
 *                     most 200 rounds), instead of Eq. 33 with the previous
 *                     step's velocity (R-pu).
 *   ORA_ALT_ODD_AXIS  a population arriving across the axis is minus the c_r-
 *                     mirrored population of the axis-row node (the odd
 *                     continuation of r-weighted values) instead of plus
 *                     (R-bc); propagation then no longer conserves sum f.
 *   ORA_ALT_FREE_S1   the rate of the energy moment e is s_g[1] as given
 *                     instead of 1/tau_g (the constraint s1 = s7 = s8 of
 *                     Eq. 34 dropped for s1), in the collision and in s_p.
 *
 * Non-orthogonal MRT (collision = 2): the extension the paper names in Sec. 4,
 * with M replaced by the raw-moment basis N of the lattice (rows 1, c_z, c_r,
 * c_z^2 + c_r^2, c_z^2 - c_r^2, c_z c_r, c_z^2 c_r, c_z c_r^2, c_z^2 c_r^2) in
 * Eqs. 9-10 and 24.  Readings:
 *   R-nbasis  the equilibria and sources are the paper's population-space ones
 *             (Eqs. 11, 15, 25-26, 29) taken into raw moments: N f^eq, N R, N T.
 *   R-nrates  each raw row relaxes with the rate of the orthogonal moment it
 *             stands for: 1 <- s0, c_z <- s3, c_r <- s5, c^2 <- s1 (e),
 *             c_z^2 - c_r^2 <- s7, c_z c_r <- s8, c_z^2 c_r <- s6 (q_r),
 *             c_z c_r^2 <- s4 (q_z), c_z^2 c_r^2 <- s2 (eps).
 *   R-nsp     s_p of Eq. 33 comes from the same Chapman-Enskog step as
 *             Eq. (C.7): the rho u_r coefficient of g_0 - g_0^eq, which for
 *             the raw basis is w_0 (3/s_c - 1/s_q - 1) / 2 with s_c the rate
 *             of c^2 (= 1/tau_g) and s_q that of c_z^2 c_r^2 (= s_2^g);
 *             for the orthogonal basis the same step gives the paper's
 *             (s1 + s2 - s1 s2) / (2 s1 s2).
 */
#include "axi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- lattice (Eq. 12), with the paper's x axis along z and y along r ---- */
static const int CZ[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CR[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WGT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2 = c^2/3 with c = dx/dt = 1 */

/* transformation matrix M exactly as printed in Sec. 2.2 */
static const double MMAT[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

struct ora_case {
    ora_params prm;
    int64_t t;
    double *f, *g;                  /* post-propagation populations at time t */
    double *phi_prev, *uz_prev, *ur_prev;
    double Minv[9][9];
    double N[9][9], Ninv[9][9];     /* raw-moment basis (collision = 2) */
};

/* raw-moment basis of the non-orthogonal MRT (reading R-nbasis), from c_i */
static void raw_basis(double N[9][9])
{
    for (int i = 0; i < 9; ++i) {
        double z = CZ[i], r = CR[i];
        N[0][i] = 1.0;
        N[1][i] = z;
        N[2][i] = r;
        N[3][i] = z * z + r * r;
        N[4][i] = z * z - r * r;
        N[5][i] = z * r;
        N[6][i] = z * z * r;
        N[7][i] = z * r * r;
        N[8][i] = z * z * r * r;
    }
}

/* orthogonal rate that each raw row relaxes with (reading R-nrates) */
static const int RAW_RATE[9] = {0, 3, 5, 1, 7, 8, 6, 4, 2};

/* inverse of a 9x9 matrix by Gauss-Jordan elimination with partial pivoting */
static void invert9(const double A[9][9], double inv[9][9])
{
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c)
            a[r][c] = (c < 9) ? A[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col]))
                piv = r;
        if (piv != col)
            for (int c = 0; c < 18; ++c) {
                double tmp = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = tmp;
            }
        double d = a[col][col];
        for (int c = 0; c < 18; ++c)
            a[col][c] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == col)
                continue;
            double m = a[r][col];
            for (int c = 0; c < 18; ++c)
                a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c)
            inv[r][c] = a[r][c + 9];
}

static size_t node(int nz, int j, int k) { return (size_t)j * nz + k; }
static size_t pop(int nr, int nz, int i, int j, int k) { return ((size_t)i * nr + j) * nz + k; }

/* r of row j (Sec. 2.3: the first lattice line lies at r = dx/2) */
static double radius(int j) { return j + 0.5; }

/* ---- stencil ghosts (Sec. 2.3, reading R-ghost) ---- */
static double ghost(int nr, int nz, int zper, const double *chi, int k, int j)
{
    if (j < 0)
        j = -1 - j;               /* axis: axisymmetric image */
    if (j >= nr)
        j = 2 * nr - 1 - j;       /* wall: mirror image */
    if (zper) {
        k %= nz;
        if (k < 0)
            k += nz;
    } else {
        if (k < 0)
            k = -1 - k;
        if (k >= nz)
            k = 2 * nz - 1 - k;
    }
    return chi[node(nz, j, k)];
}

/* Eqs. 39 and 40 at node (k, j), dt = 1 */
static void iso_stencil(int nr, int nz, int zper, const double *chi, int k, int j,
                        double *dz, double *dr, double *lap)
{
    double c0 = chi[node(nz, j, k)];
    double sz = 0.0, sr = 0.0, sl = 0.0;
    for (int i = 1; i < 9; ++i) {
        double a = ghost(nr, nz, zper, chi, k + CZ[i], j + CR[i]);
        double b = ghost(nr, nz, zper, chi, k + 2 * CZ[i], j + 2 * CR[i]);
        sz += WGT[i] * CZ[i] * (8.0 * a - b);
        sr += WGT[i] * CR[i] * (8.0 * a - b);
        sl += WGT[i] * (16.0 * a - b - 15.0 * c0);
    }
    *dz = sz / (6.0 * CS2);
    *dr = sr / (6.0 * CS2);
    *lap = sl / (6.0 * CS2);
}

void ora_stencil(int32_t nr, int32_t nz, int32_t z_periodic, const double *chi,
                 double *dz, double *dr, double *lap)
{
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            iso_stencil(nr, nz, z_periodic, chi, k, j, &dz[n], &dr[n], &lap[n]);
        }
}

/* ---- propagation, Eq. 20, with the boundary rules of Sec. 2.3 (R-bc) ---- */
static int opposite(int i)
{
    for (int q = 0; q < 9; ++q)
        if (CZ[q] == -CZ[i] && CR[q] == -CR[i])
            return q;
    return -1;
}

static int r_mirror(int i)
{
    for (int q = 0; q < 9; ++q)
        if (CZ[q] == CZ[i] && CR[q] == -CR[i])
            return q;
    return -1;
}

static void stream_alt(int32_t nr, int32_t nz, int32_t zper, int odd_axis, const double *post, double *out);

void ora_stream(int32_t nr, int32_t nz, int32_t zper, const double *post, double *out)
{
    stream_alt(nr, nz, zper, 0, post, out);
}

static void stream_alt(int32_t nr, int32_t nz, int32_t zper, int odd_axis, const double *post, double *out)
{
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < nr; ++j)
            for (int k = 0; k < nz; ++k) {
                int sk = k - CZ[i], sj = j - CR[i];
                int cross_z = 0;
                if (zper)
                    sk = (sk % nz + nz) % nz;
                else if (sk < 0 || sk >= nz)
                    cross_z = 1;
                double v;
                if (sj >= nr || cross_z) {
                    v = post[pop(nr, nz, opposite(i), j, k)];         /* bounce-back */
                } else if (sj < 0) {
                    v = post[pop(nr, nz, r_mirror(i), 0, sk)];        /* specular at the axis */
                    if (odd_axis)
                        v = -v;                                       /* ORA_ALT_ODD_AXIS */
                } else {
                    v = post[pop(nr, nz, i, sj, sk)];
                }
                out[pop(nr, nz, i, j, k)] = v;
            }
}

/* ---- equilibrium pieces ---- */

/* s_i(u) of Eq. 26 */
static double s_of_u(int i, double uz, double ur)
{
    double cu = CZ[i] * uz + CR[i] * ur;
    double uu = uz * uz + ur * ur;
    return WGT[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

static double tau_f_of(const ora_params *p) { return p->mobility / CS2 + 0.5; } /* Eq. 18 */

/* macroscopic state of one node at time t (the prefix shared by step and moments) */
typedef struct {
    double r, phi, rho, nu, dphi_z, dphi_r, lap;
    double drho_z, drho_r, fs_z, fs_r, G_z, G_r;
    double s_nu, s_p, p, uz, ur, Fz, Fr;
} macro;

/* phi of every node, Eq. 16 */
static void phase_field(const ora_case *c, double *phi)
{
    int nr = c->prm.nr, nz = c->prm.nz;
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            double s = 0.0;
            for (int i = 0; i < 9; ++i)
                s += c->f[pop(nr, nz, i, j, k)];
            phi[node(nz, j, k)] = s / radius(j);
        }
}

/* Eq. 17 */
static double density(const ora_params *p, double phi) { return phi * p->rho_l + (1.0 - phi) * p->rho_g; }

static void compute_macro(const ora_case *c, const double *phi, const double *rhof, int k, int j, macro *m)
{
    const ora_params *P = &c->prm;
    int nr = P->nr, nz = P->nz;
    size_t n = node(nz, j, k);
    double r = radius(j);
    m->r = r;
    m->phi = phi[n];
    m->rho = rhof[n];
    m->nu = m->phi * P->nu_l + (1.0 - m->phi) * P->nu_g;                 /* Eq. 35 */
    iso_stencil(nr, nz, P->z_periodic, phi, k, j, &m->dphi_z, &m->dphi_r, &m->lap);
    double unused;
    iso_stencil(nr, nz, P->z_periodic, rhof, k, j, &m->drho_z, &m->drho_r, &unused);

    /* chemical potential (Eq. 4 with k and beta of Sec. 2.1) and its
       axisymmetric correction mu~ = mu - k d_r(phi)/r (Sec. 2.1) */
    double kap = 1.5 * P->sigma * P->W;
    double beta = 12.0 * P->sigma / P->W;
    double mu = 4.0 * beta * m->phi * (m->phi - 1.0) * (m->phi - 0.5) - kap * m->lap;
    double mut = mu - kap * m->dphi_r / r;
    m->fs_z = mut * m->dphi_z;
    m->fs_r = mut * m->dphi_r;
    double gz = P->g_z;
    if (P->g_ramp > 0.0 && (double)(c->t + 1) < P->g_ramp)
        gz = P->g_z * ((double)(c->t + 1) / P->g_ramp);                  /* g_ramp */
    m->G_z = (m->rho - P->rho_l) * gz;       /* reading R-grav */
    m->G_r = 0.0;

    /* relaxation rates for the viscous moments (Eq. 34) and s_p (Eq. 33) */
    double tau_g = m->nu / CS2 + 0.5;
    m->s_nu = 1.0 / tau_g;
    double s1 = ((P->alt & ORA_ALT_FREE_S1) || P->free_s1) ? P->s_g[1] : m->s_nu;
    double s2 = P->collision == 1 ? m->s_nu : P->s_g[2];
    if (P->collision == 2)
        m->s_p = 0.5 * (3.0 / s1 - 1.0 / s2 - 1.0);       /* reading R-nsp */
    else
        m->s_p = (s1 + s2 - s1 * s2) / (2.0 * s1 * s2);

    /* pressure, Eq. 33, with the previous step's velocity (reading R-pu) */
    double uzp = c->uz_prev[n], urp = c->ur_prev[n];
    double sum_g = 0.0;
    for (int i = 1; i < 9; ++i)
        sum_g += c->g[pop(nr, nz, i, j, k)];
    double jz = 0.0, jr = 0.0;
    for (int i = 0; i < 9; ++i) {
        jz += CZ[i] * c->g[pop(nr, nz, i, j, k)];
        jr += CR[i] * c->g[pop(nr, nz, i, j, k)];
    }
    int rounds = (P->alt & ORA_ALT_JOINT_PU) ? 200 : 1;
    for (int it = 0; it < rounds; ++it) {
        double u_grad_rho = uzp * m->drho_z + urp * m->drho_r;
        m->p = CS2 / (1.0 - WGT[0]) *
               (sum_g / r + 0.5 * u_grad_rho + m->rho * s_of_u(0, uzp, urp) -
                m->s_p * WGT[0] * m->rho * urp / r);

        /* velocity, Eq. 32 */
        m->uz = (jz + 0.5 * (r * (m->fs_z + m->G_z))) / (r * m->rho);
        m->ur = (jr + 0.5 * (r * (m->fs_r + m->G_r) + m->p)) / (r * m->rho + m->nu * m->rho / r);
        if (m->uz == uzp && m->ur == urp)
            break;
        uzp = m->uz;                                  /* ORA_ALT_JOINT_PU: again with this velocity */
        urp = m->ur;
    }

    /* total force, Eq. 30 */
    m->Fz = r * (m->fs_z + m->G_z);
    m->Fr = r * (m->fs_r + m->G_r) + (m->p - 2.0 * m->rho * m->nu / r * m->ur);
}

/* moment-space MRT relaxation with a source: Eq. 19 (and its g analogue,
   Eqs. 24 and 27) written as m+ = m - S(m - m_eq) + (I - S/2) m_src */
static void mrt(const ora_case *c, const double s[9], const double meq[9], const double msrc[9],
                double popv[9])
{
    double m[9], mp[9];
    for (int a = 0; a < 9; ++a) {
        m[a] = 0.0;
        for (int i = 0; i < 9; ++i)
            m[a] += MMAT[a][i] * popv[i];
    }
    for (int a = 0; a < 9; ++a)
        mp[a] = m[a] - s[a] * (m[a] - meq[a]) + (1.0 - 0.5 * s[a]) * msrc[a];
    for (int i = 0; i < 9; ++i) {
        popv[i] = 0.0;
        for (int a = 0; a < 9; ++a)
            popv[i] += c->Minv[i][a] * mp[a];
    }
}

static void rates_f(const ora_params *P, double s[9])
{
    double sf = 1.0 / tau_f_of(P);
    for (int a = 0; a < 9; ++a)
        s[a] = P->collision == 1 ? sf : P->s_f[a];
    s[3] = s[4] = s[5] = s[6] = sf;     /* reading R-rates */
}

/* population-space equilibrium (Eq. 11) and source (Eq. 15) of f at one node.
   dJz, dJr: d_t of r phi u + M phi e_r (Eq. 38). */
static void f_eq_src(const ora_params *P, double r, double phi, double uz, double ur, double dJz, double dJr,
                     double nz_, double nr_, double lambda, double feq[9], double R[9])
{
    for (int i = 0; i < 9; ++i) {
        double cJ = CZ[i] * (r * phi * uz) + CR[i] * (r * phi * ur + P->mobility * phi);
        feq[i] = WGT[i] * (r * phi + cJ / CS2);                                         /* Eq. 11 */
        R[i] = WGT[i] * (CZ[i] * (dJz + CS2 * r * nz_ * lambda) +
                         CR[i] * (dJr + CS2 * r * nr_ * lambda)) / CS2;                 /* Eq. 15 */
    }
}

/* population-space equilibrium (Eqs. 25-26) and forcing (Eq. 29) of g at one
   node.  drz, drr: d_z(r rho), d_r(r rho). */
static void g_eq_src(double r, double rho, double p, double uz, double ur, double Fz, double Fr, double drz,
                     double drr, double geq[9], double T[9])
{
    for (int i = 0; i < 9; ++i) {
        geq[i] = (i == 0 ? r * p / CS2 * (WGT[0] - 1.0) : r * p / CS2 * WGT[i]) +
                 r * rho * s_of_u(i, uz, ur);                                           /* Eqs. 25-26 */
        double cF = CZ[i] * Fz + CR[i] * Fr;
        /* u_alpha d_beta(r rho) c_ia c_ib */
        double cu = CZ[i] * uz + CR[i] * ur;
        double cd = CZ[i] * drz + CR[i] * drr;
        T[i] = WGT[i] * (cF / CS2 + cu * cd / CS2 - rho * ur);                          /* Eq. 29 */
    }
}

/* SRT collision at one node in population space: Eq. 9 (f) or Eq. 24 (g)
   with M^-1 S M = s I, and the source term Eq. 14 (or 27) with
   M^-1 (I - S/2) M = (1 - s/2) I. */
static void srt(double s, const double eq[9], const double src[9], double v[9])
{
    for (int i = 0; i < 9; ++i)
        v[i] = v[i] - s * (v[i] - eq[i]) + (1.0 - 0.5 * s) * src[i];
}

/* non-orthogonal MRT collision at one node: Eqs. 9-10 (or 24, 27) with the
   raw-moment basis N in place of M, equilibrium and source taken into raw
   moments (reading R-nbasis), raw row a relaxed with s_orth[RAW_RATE[a]]. */
static void nmrt(const ora_case *c, const double s_orth[9], const double eq[9], const double src[9],
                 double v[9])
{
    double m[9], meq[9], msrc[9], mp[9];
    for (int a = 0; a < 9; ++a) {
        m[a] = meq[a] = msrc[a] = 0.0;
        for (int i = 0; i < 9; ++i) {
            m[a] += c->N[a][i] * v[i];
            meq[a] += c->N[a][i] * eq[i];
            msrc[a] += c->N[a][i] * src[i];
        }
    }
    for (int a = 0; a < 9; ++a) {
        double s = s_orth[RAW_RATE[a]];
        mp[a] = m[a] - s * (m[a] - meq[a]) + (1.0 - 0.5 * s) * msrc[a];
    }
    for (int i = 0; i < 9; ++i) {
        v[i] = 0.0;
        for (int a = 0; a < 9; ++a)
            v[i] += c->Ninv[i][a] * mp[a];
    }
}

static void step_once(ora_case *c, double *f_post_out, double *g_post_out, double *Fz_out, double *Fr_out)
{
    const ora_params *P = &c->prm;
    int nr = P->nr, nz = P->nz;
    size_t nn = (size_t)nr * nz;
    double *phi = malloc(nn * sizeof(double));
    double *rhof = malloc(nn * sizeof(double));
    double *fp = malloc(9 * nn * sizeof(double));
    double *gp = malloc(9 * nn * sizeof(double));
    double *phi_new = malloc(nn * sizeof(double));
    double *uz_new = malloc(nn * sizeof(double));
    double *ur_new = malloc(nn * sizeof(double));

    phase_field(c, phi);
    for (size_t n = 0; n < nn; ++n)
        rhof[n] = density(P, phi[n]);

    double sf[9];
    rates_f(P, sf);

    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            macro m;
            compute_macro(c, phi, rhof, k, j, &m);
            double r = m.r;

            /* --- phase-field population f: Eqs. 19, 21-23 --- */
            double Jz = r * m.phi * m.uz;
            double Jr = r * m.phi * m.ur + P->mobility * m.phi;
            double php = c->phi_prev[n];
            double Jz_prev = r * php * c->uz_prev[n];
            double Jr_prev = r * php * c->ur_prev[n] + P->mobility * php;
            double lambda = -4.0 * (m.phi - 1.0) * m.phi / P->W;                 /* Eq. 2 */
            double gmag = sqrt(m.dphi_z * m.dphi_z + m.dphi_r * m.dphi_r);
            double nz_ = 0.0, nr_ = 0.0;
            if (gmag > 1e-12) {                                                /* reading R-n */
                nz_ = m.dphi_z / gmag;
                nr_ = m.dphi_r / gmag;
            }
            double mR1 = (Jz - Jz_prev) + CS2 * r * nz_ * lambda;              /* Eqs. 23, 38 */
            double mR2 = (Jr - Jr_prev) + CS2 * r * nr_ * lambda;
            double rphi = r * m.phi;
            double meq_f[9] = {rphi, -2.0 * rphi, rphi, Jz, -Jz, Jr, -Jr, 0.0, 0.0};   /* Eq. 21 */
            double mR[9] = {0.0, 0.0, 0.0, mR1, -mR1, mR2, -mR2, 0.0, 0.0};             /* Eq. 22 */
            double fv[9], feq[9], Rf[9];
            for (int i = 0; i < 9; ++i)
                fv[i] = c->f[pop(nr, nz, i, j, k)];
            if (P->collision == 0) {
                mrt(c, sf, meq_f, mR, fv);
            } else {
                f_eq_src(P, r, m.phi, m.uz, m.ur, Jz - Jz_prev, Jr - Jr_prev, nz_, nr_, lambda, feq, Rf);
                if (P->collision == 1)
                    srt(sf[0], feq, Rf, fv);
                else
                    nmrt(c, sf, feq, Rf, fv);
            }
            for (int i = 0; i < 9; ++i)
                fp[pop(nr, nz, i, j, k)] = fv[i];

            /* --- hydrodynamic population g: Eqs. 24, 27-28, 36-37 --- */
            double uz = m.uz, ur = m.ur, rho = m.rho;
            double u2 = uz * uz + ur * ur;
            double drz = r * m.drho_z;              /* d_z(r rho), reading R-grad */
            double drr = r * m.drho_r + rho;        /* d_r(r rho) */
            double meq_g[9] = {0.0,
                               r * (2.0 * m.p + rho * u2) / CS2,
                               -r * (3.0 * m.p + rho * u2) / CS2,
                               r * rho * uz, -r * rho * uz,
                               r * rho * ur, -r * rho * ur,
                               r * rho * (uz * uz - ur * ur),
                               r * rho * ur * uz};                                  /* Eq. 36 */
            double mT[9] = {r * (uz * m.drho_z + ur * m.drho_r),
                            2.0 * rho * ur,
                            -(uz * drz + ur * drr) - rho * ur,
                            m.Fz, -m.Fz, m.Fr, -m.Fr,
                            2.0 / 3.0 * (uz * drz - ur * drr),
                            1.0 / 3.0 * (uz * drr + ur * drz)};                     /* Eq. 37 */
            double sg[9];
            for (int a = 0; a < 9; ++a)
                sg[a] = P->s_g[a];
            sg[1] = sg[7] = sg[8] = m.s_nu;                                         /* Eq. 34 */
            if ((P->alt & ORA_ALT_FREE_S1) || P->free_s1)
                sg[1] = P->s_g[1];                                          /* free_s1 */
            double gv[9], geq[9], Tg[9];
            for (int i = 0; i < 9; ++i)
                gv[i] = c->g[pop(nr, nz, i, j, k)];
            if (P->collision == 0) {
                mrt(c, sg, meq_g, mT, gv);
            } else {
                g_eq_src(r, rho, m.p, uz, ur, m.Fz, m.Fr, drz, drr, geq, Tg);
                if (P->collision == 1)
                    srt(m.s_nu, geq, Tg, gv);
                else
                    nmrt(c, sg, geq, Tg, gv);
            }
            for (int i = 0; i < 9; ++i)
                gp[pop(nr, nz, i, j, k)] = gv[i];

            phi_new[n] = m.phi;
            uz_new[n] = uz;
            ur_new[n] = ur;
            if (Fz_out) {
                Fz_out[n] = m.Fz;
                Fr_out[n] = m.Fr;
            }
        }

    if (f_post_out) {
        memcpy(f_post_out, fp, 9 * nn * sizeof(double));
        memcpy(g_post_out, gp, 9 * nn * sizeof(double));
    }
    int odd = (P->alt & ORA_ALT_ODD_AXIS) != 0;
    stream_alt(nr, nz, P->z_periodic, odd, fp, c->f);   /* Eq. 20 */
    stream_alt(nr, nz, P->z_periodic, odd, gp, c->g);
    memcpy(c->phi_prev, phi_new, nn * sizeof(double));
    memcpy(c->uz_prev, uz_new, nn * sizeof(double));
    memcpy(c->ur_prev, ur_new, nn * sizeof(double));
    c->t += 1;

    free(phi); free(rhof); free(fp); free(gp);
    free(phi_new); free(uz_new); free(ur_new);
}

ora_case *ora_create(const ora_params *p, const double *phi0)
{
    ora_case *c = calloc(1, sizeof(ora_case));
    c->prm = *p;
    int nr = p->nr, nz = p->nz;
    size_t nn = (size_t)nr * nz;
    c->f = calloc(9 * nn, sizeof(double));
    c->g = calloc(9 * nn, sizeof(double));
    c->phi_prev = calloc(nn, sizeof(double));
    c->uz_prev = calloc(nn, sizeof(double));
    c->ur_prev = calloc(nn, sizeof(double));
    invert9(MMAT, c->Minv);
    raw_basis(c->N);
    invert9(c->N, c->Ninv);
    /* reading R-init: u = 0, p = 0, g = 0 (= g^eq, Eqs. 25-26) and
       f = f^eq(phi0, 0) of Eq. 11 plus h, where h is the non-equilibrium part
       that makes a uniform phase field an exact fixed point of collision
       (Eq. 19) and propagation (Eq. 20):  K h = b with K = M^-1 S^f M and
       b_i = -w_i c_ir phi0, the change of w_i r phi0 over one link in r.
       Without h the equilibrium flux M phi of Eq. 11 is unbalanced on the
       axis row in the first step.  The non-orthogonal form (collision = 2)
       takes K = N^-1 S^f N with its own basis and rates. */
    double sf[9], B[9][9], Binv[9][9], sb[9];
    rates_f(p, sf);
    for (int a = 0; a < 9; ++a)
        for (int i = 0; i < 9; ++i) {
            B[a][i] = p->collision == 2 ? c->N[a][i] : MMAT[a][i];
            Binv[i][a] = p->collision == 2 ? c->Ninv[i][a] : c->Minv[i][a];
        }
    for (int a = 0; a < 9; ++a)
        sb[a] = p->collision == 2 ? sf[RAW_RATE[a]] : sf[a];
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            double r = radius(j), ph = phi0[n];
            double uz0 = 0.0, ur0 = 0.0;
            double flux_z = r * ph * uz0;                      /* r phi u_z            */
            double flux_r = r * ph * ur0 + p->mobility * ph;   /* r phi u_r + M phi    */
            double b[9], mb[9], h[9];
            for (int i = 0; i < 9; ++i)
                b[i] = -WGT[i] * CR[i] * ph;
            for (int a = 0; a < 9; ++a) {
                mb[a] = 0.0;
                for (int i = 0; i < 9; ++i)
                    mb[a] += B[a][i] * b[i];
                mb[a] /= sb[a];                                /* S^-1 M b */
            }
            for (int i = 0; i < 9; ++i) {
                h[i] = 0.0;
                for (int a = 0; a < 9; ++a)
                    h[i] += Binv[i][a] * mb[a];
            }
            for (int i = 0; i < 9; ++i)                        /* Eq. 11 + h */
                c->f[pop(nr, nz, i, j, k)] =
                    WGT[i] * (r * ph + (CZ[i] * flux_z + CR[i] * flux_r) / CS2) + h[i];
            c->phi_prev[n] = ph;
        }
    return c;
}

void ora_destroy(ora_case *c)
{
    if (!c)
        return;
    free(c->f); free(c->g); free(c->phi_prev); free(c->uz_prev); free(c->ur_prev);
    free(c);
}

void ora_step(ora_case *c, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s)
        step_once(c, NULL, NULL, NULL, NULL);
}

void ora_step_debug(ora_case *c, double *f_post, double *g_post, double *Fz, double *Fr)
{
    step_once(c, f_post, g_post, Fz, Fr);
}

int64_t ora_time(const ora_case *c) { return c->t; }

void ora_moments(const ora_case *c, double *phi_o, double *rho_o, double *uz_o, double *ur_o, double *p_o)
{
    const ora_params *P = &c->prm;
    int nr = P->nr, nz = P->nz;
    size_t nn = (size_t)nr * nz;
    double *phi = malloc(nn * sizeof(double));
    double *rhof = malloc(nn * sizeof(double));
    phase_field(c, phi);
    for (size_t n = 0; n < nn; ++n)
        rhof[n] = density(P, phi[n]);
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            macro m;
            compute_macro(c, phi, rhof, k, j, &m);
            if (phi_o) phi_o[n] = m.phi;
            if (rho_o) rho_o[n] = m.rho;
            if (uz_o) uz_o[n] = m.uz;
            if (ur_o) ur_o[n] = m.ur;
            if (p_o) p_o[n] = m.p;
        }
    free(phi);
    free(rhof);
}

/* ---- diagnostics (not in the paper; definitions of this project) ----
 * psi is the dispersed phase: phi for a drop, 1 - phi for a bubble.
 * phase_mass  = sum of all f          (= sum r phi, the conserved quantity)
 * fluid_mass  = sum r rho,  mom_z = sum r rho u_z,  umax = max |u|
 * centroid_z  = sum r psi z / sum r psi,  rise_u = sum r psi u_z / sum r psi
 * R_eq        = (1.5 sum r psi)^(1/3)   (sphere volume = 2 pi sum r psi)
 * p_in        = mean p over nodes with d < R_eq - 2W, d = |(z - z_c, r)|
 * p_out       = mean p over nodes with d > R_eq + 2W at least 3 cells from
 *               every wall;  dp = p_in - p_out
 * semi_z      = half the distance between the psi = 1/2 crossings along the
 *               axis row that bracket the column nearest z_c
 * semi_r      = the psi = 1/2 crossing going up the column nearest z_c
 * min_axis_phi = min phi along the axis row;  nonfinite = count of nodes with
 *               a non-finite phi, u or p.
 */
static int wrapk(int k, int nz) { return ((k % nz) + nz) % nz; }

void ora_diagnostics(const ora_case *c, ora_diag *d)
{
    const ora_params *P = &c->prm;
    int nr = P->nr, nz = P->nz;
    size_t nn = (size_t)nr * nz;
    double *phi = malloc(nn * sizeof(double)), *rho = malloc(nn * sizeof(double));
    double *uz = malloc(nn * sizeof(double)), *ur = malloc(nn * sizeof(double));
    double *p = malloc(nn * sizeof(double));
    ora_moments(c, phi, rho, uz, ur, p);
    memset(d, 0, sizeof(*d));
    d->t = c->t;
    for (int i = 0; i < 9; ++i)
        for (size_t n = 0; n < nn; ++n)
            d->phase_mass += c->f[(size_t)i * nn + n];
    double spsi = 0.0, spz = 0.0, spu = 0.0;
    d->min_axis_phi = INFINITY;
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            double r = radius(j);
            double psi = P->dispersed_gas ? 1.0 - phi[n] : phi[n];
            d->fluid_mass += r * rho[n];
            d->mom_z += r * rho[n] * uz[n];
            double um = sqrt(uz[n] * uz[n] + ur[n] * ur[n]);
            if (um > d->umax)
                d->umax = um;
            if (psi > 0.01) {         /* the dispersed phase's region (reading R-region) */
                spsi += r * psi;
                spz += r * psi * k;
                spu += r * psi * uz[n];
            }
            if (j == 0 && phi[n] < d->min_axis_phi)
                d->min_axis_phi = phi[n];
            if (!isfinite(phi[n]) || !isfinite(uz[n]) || !isfinite(ur[n]) || !isfinite(p[n]))
                d->nonfinite += 1;
        }
    if (spsi > 0.0) {
        d->centroid_z = spz / spsi;
        d->rise_u = spu / spsi;
        d->R_eq = cbrt(1.5 * spsi);
    }
    double sin_ = 0.0, sout = 0.0;
    long cin = 0, cout = 0;
    for (int j = 0; j < nr; ++j)
        for (int k = 0; k < nz; ++k) {
            size_t n = node(nz, j, k);
            double dz = k - d->centroid_z, r = radius(j);
            double dist = sqrt(dz * dz + r * r);
            if (dist < d->R_eq - 2.0 * P->W) {
                sin_ += p[n];
                cin += 1;
            } else if (dist > d->R_eq + 2.0 * P->W) {
                int near_wall = (j > nr - 4) || (!P->z_periodic && (k < 3 || k > nz - 4));
                if (!near_wall) {
                    sout += p[n];
                    cout += 1;
                }
            }
        }
    d->p_in = cin ? sin_ / cin : 0.0;
    d->p_out = cout ? sout / cout : 0.0;
    d->dp = d->p_in - d->p_out;

    /* semi-axes from the psi = 1/2 crossings */
    int kc = (int)floor(d->centroid_z + 0.5);
    if (kc < 0) kc = 0;
    if (kc >= nz) kc = nz - 1;
#define PSI(jj, kk) (P->dispersed_gas ? 1.0 - phi[node(nz, (jj), (kk))] : phi[node(nz, (jj), (kk))])
    if (PSI(0, kc) > 0.5) {
        /* walk toward -z along the axis row (positions unwrapped) */
        double zlo = kc, zhi = kc;
        int pos = kc, kidx = kc;
        for (int s = 0; s < nz; ++s) {
            int mpos = pos - 1, midx = mpos;
            if (P->z_periodic) {
                midx = wrapk(mpos, nz);
            } else if (mpos < 0) {
                zlo = pos - 0.5;          /* reached the wall face */
                break;
            }
            double a = PSI(0, midx), b = PSI(0, kidx);
            if (a <= 0.5) {
                zlo = mpos + (0.5 - a) / (b - a);
                break;
            }
            pos = mpos;
            kidx = midx;
            zlo = pos;
        }
        pos = kc;
        kidx = kc;
        for (int s = 0; s < nz; ++s) {
            int ppos = pos + 1, pidx = ppos;
            if (P->z_periodic) {
                pidx = wrapk(ppos, nz);
            } else if (ppos >= nz) {
                zhi = pos + 0.5;
                break;
            }
            double a = PSI(0, kidx), b = PSI(0, pidx);
            if (b <= 0.5) {
                zhi = pos + (a - 0.5) / (a - b);
                break;
            }
            pos = ppos;
            kidx = pidx;
            zhi = pos;
        }
        d->semi_z = 0.5 * (zhi - zlo);

        double rc = nr;                   /* the r-wall if no crossing is found */
        for (int j = 0; j + 1 < nr; ++j) {
            double a = PSI(j, kc), b = PSI(j + 1, kc);
            if (b <= 0.5) {
                rc = radius(j) + (a - 0.5) / (a - b);
                break;
            }
        }
        d->semi_r = rc;
    }
#undef PSI
    free(phi); free(rho); free(uz); free(ur); free(p);
}

void ora_get_state(const ora_case *c, double *f, double *g, double *aux)
{
    size_t nn = (size_t)c->prm.nr * c->prm.nz;
    if (f) memcpy(f, c->f, 9 * nn * sizeof(double));
    if (g) memcpy(g, c->g, 9 * nn * sizeof(double));
    if (aux) {
        memcpy(aux, c->phi_prev, nn * sizeof(double));
        memcpy(aux + nn, c->uz_prev, nn * sizeof(double));
        memcpy(aux + 2 * nn, c->ur_prev, nn * sizeof(double));
    }
}

void ora_set_state(ora_case *c, const double *f, const double *g, const double *aux, int64_t t)
{
    size_t nn = (size_t)c->prm.nr * c->prm.nz;
    if (f) memcpy(c->f, f, 9 * nn * sizeof(double));
    if (g) memcpy(c->g, g, 9 * nn * sizeof(double));
    if (aux) {
        memcpy(c->phi_prev, aux, nn * sizeof(double));
        memcpy(c->uz_prev, aux + nn, nn * sizeof(double));
        memcpy(c->ur_prev, aux + 2 * nn, nn * sizeof(double));
    }
    c->t = t;
}

void ora_lattice(int32_t *cz, int32_t *cr, double *w, double *Mmat, double *Minv)
{
    double inv[9][9];
    invert9(MMAT, inv);
    for (int i = 0; i < 9; ++i) {
        cz[i] = CZ[i];
        cr[i] = CR[i];
        w[i] = WGT[i];
        for (int a = 0; a < 9; ++a) {
            Mmat[i * 9 + a] = MMAT[i][a];
            Minv[i * 9 + a] = inv[i][a];
        }
    }
}

void ora_rates(const ora_case *c, double *s_f, double *s_g_nonnu)
{
    rates_f(&c->prm, s_f);
    for (int a = 0; a < 9; ++a)
        s_g_nonnu[a] = c->prm.s_g[a];
}
