// Device-side building blocks of the lbm_axi step: lattice rules, the
// per-node collision of both populations, and the phase-field tile.
//
// Conventions (see include/lbm_axi.h): SoA population planes p*plane + j*nz + k
// with z fastest; row j at r = j + 1/2; population order of Eq. 12 with x -> z,
// y -> r.  The state between launches holds post-collision populations; a step
// pulls them across the links (Eq. 20 read backwards), collides and stores in
// place of the other ping-pong buffer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace axi {

// ---------------------------------------------------------------- lattice --
// D2Q9 links (Eq. 12): 0 rest, 1 +z, 2 +r, 3 -z, 4 -r, 5 (+z,+r), 6 (-z,+r),
// 7 (-z,-r), 8 (+z,-r).
__host__ __device__ constexpr int link_z(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int link_r(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int reverse_link(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5); }
__host__ __device__ constexpr int axis_image(int i) { return (i == 2) ? 4 : (i == 4) ? 2 : (i == 5) ? 8 : (i == 8) ? 5 : (i == 6) ? 7 : (i == 7) ? 6 : i; }

struct Geom {
    int nr, nz;
    int zper;          // 1 periodic in z, 0 walls
    int tiles_z;       // tiles along z
    int tiles;         // total tiles of the step launch
    int64_t plane;     // elements between population planes
};

// Source slot of population i arriving at (k, j) (Sec. 2.3 boundary rules):
// a source beyond the r-wall or a z-wall -- corners included -- is half-way
// bounce-back of the node's own reversed population; a source beyond the axis
// only is the mirror image (c_r flipped) on the axis row; periodic z wraps.
template <int I>
__device__ __forceinline__ int64_t pull_slot(const Geom &g, int k, int j)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    int sk = k - CZ, sj = j - CR;
    bool wall = (CR < 0) && (sj >= g.nr);
    if (CZ != 0) {
        if (g.zper) {
            sk = (sk < 0) ? sk + g.nz : (sk >= g.nz ? sk - g.nz : sk);
        } else if (sk < 0 || sk >= g.nz) {
            wall = true;
        }
    }
    if (wall)
        return (int64_t)reverse_link(I) * g.plane + (int64_t)j * g.nz + k;
    if (CR > 0 && sj < 0)
        return (int64_t)axis_image(I) * g.plane + sk;
    return (int64_t)I * g.plane + (int64_t)sj * g.nz + sk;
}

template <typename T, typename R>
__device__ __forceinline__ void pull9(const Geom &g, const T *__restrict__ src, int k, int j, R v[9])
{
    v[0] = (R)src[pull_slot<0>(g, k, j)];
    v[1] = (R)src[pull_slot<1>(g, k, j)];
    v[2] = (R)src[pull_slot<2>(g, k, j)];
    v[3] = (R)src[pull_slot<3>(g, k, j)];
    v[4] = (R)src[pull_slot<4>(g, k, j)];
    v[5] = (R)src[pull_slot<5>(g, k, j)];
    v[6] = (R)src[pull_slot<6>(g, k, j)];
    v[7] = (R)src[pull_slot<7>(g, k, j)];
    v[8] = (R)src[pull_slot<8>(g, k, j)];
}

// zeroth moment with a fixed summation order (used for every phi evaluation,
// so a node's phi is bit-identical wherever it is computed)
template <typename R>
__device__ __forceinline__ R sum9(const R v[9])
{
    return (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) + v[8];
}

// Quotients of smooth coefficients (the viscous rates, the interface normal):
// correctly rounded in double (the FP64 path is held to the oracle within
// 1e-12 per step), the hardware reciprocal and reciprocal square root (about
// 1 ulp) in float.  The phase field (1/r) and the velocity keep correctly
// rounded division in both precisions: the spurious currents are a small
// residual of large balancing forces and pick up any rounding bias there.
__device__ __forceinline__ double div_r(double a, double b) { return a / b; }
__device__ __forceinline__ float div_r(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }

template <typename R>
__device__ __forceinline__ R inv_radius(int j) { return (R)1 / ((R)j + (R)0.5); }

// stencil ghosts (Sec. 2.3): mirror about the axis and the walls, wrap if
// periodic; clamped so that cells no interior node reads stay in bounds
__device__ __forceinline__ int ghost_row(int j, int nr)
{
    if (j < 0) j = -1 - j;
    if (j >= nr) j = 2 * nr - 1 - j;
    return j < 0 ? 0 : (j >= nr ? nr - 1 : j);
}
__device__ __forceinline__ int ghost_col(int k, int nz, int zper)
{
    if (k >= 0 && k < nz) return k;   // the common case skips the division below
    if (zper) {
        k %= nz;
        return k < 0 ? k + nz : k;
    }
    if (k < 0) k = -1 - k;
    if (k >= nz) k = 2 * nz - 1 - k;
    return k < 0 ? 0 : (k >= nz ? nz - 1 : k);
}

template <typename T, typename R>
__device__ __forceinline__ R phase_at(const Geom &g, const T *__restrict__ f, int k, int j)
{
    R v[9];
    pull9<T, R>(g, f, k, j, v);
    return sum9(v) * inv_radius<R>(j);
}

// ---------------------------------------------------------------- physics --
template <typename R>
struct Phys {
    R rho_l, rho_g, drho;     // Eq. 17 as rho_g + phi*drho
    R nu_g, dnu;              // Eq. 35 as nu_g + phi*dnu
    R mob;                    // M
    R lam4W;                  // 4/W (Eq. 2)
    R beta4;                  // 4*beta = 48 sigma / W (Eq. 4)
    R kap;                    // k = 1.5 sigma W (Eq. 4)
    R g_z;                    // buoyancy acceleration
    R sf[9];                  // f rates with s3..s6 = 1/tau_f (Eq. 18)
    R sg[9];                  // g rates; [1], [7], [8] unused (per node, Eq. 34)
    R sg2;                    // s_2^g (enters s_p of Eq. 33)
    R isg2;                   // 1 / s_2^g (s_p of the non-orthogonal form)
    int free_s1;              // extension: e relaxes at sg[1] instead of 1/tau_g
    R isg1;                   // 1 / s_1^g when free_s1
    double g_full;            // g_z of the parameters (g_z above: this step's value)
    double g_ramp;            // steps over which g_full is reached (0: at once)
    int unit_rates;           // every free rate is 1 (the choice of all tests of Sec. 3)
    int srt;                  // SRT: every rate 1/tau_f (f), 1/tau_g(phi) (g, s_p too)
    int nmrt;                 // non-orthogonal (raw-moment) MRT (Sec. 4)
    int mode;                 // collision form of the kernel instance (COLLIDE_*)
    uint32_t round_key;       // FP16-deviation storage: mix32 of the step's time t
};

// The 32-bit finalizer of MurmurHash3 (Appleby): a bijection of 32-bit words
// in which every output bit depends on every input bit.
__host__ __device__ inline uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// The acceleration of the step from time t: g_full, reached linearly over
// the first g_ramp steps (g_full (t + 1) / g_ramp while t + 1 < g_ramp).
__host__ __device__ inline double ramp_accel(double g_full, double g_ramp, int64_t t)
{
    return (g_ramp > 0.0 && (double)(t + 1) < g_ramp) ? g_full * ((double)(t + 1) / g_ramp) : g_full;
}

// Collision forms, each a kernel instance of its own (see collide_node).
constexpr int COLLIDE_MRT = 0;      // free rates as given
constexpr int COLLIDE_MRT_UNIT = 1; // every free rate 1
constexpr int COLLIDE_SRT = 2;      // every rate equal (end of Sec. 2.2)
constexpr int COLLIDE_NMRT = 3;     // raw-moment basis in place of M (Sec. 4)

// Scales of the FP16-deviation storage (powers of two); see axi_half.hpp.
struct Codec {
    float sf, isf;   // f deviation scale and its inverse
    float sg, isg;   // g scale and its inverse
};

// Output planes of the macroscopic fields (double, [nr][nz], z fastest).
struct Fields {
    double *phi, *rho, *uz, *ur, *p;
};

// One node's fields at time t as the moments pass leaves them, with the sum
// of the f it pulls (its share of the phase mass); valid = the node is inside
// the grid.
struct NodeMoments {
    bool valid;
    int j, k;
    double phi, rho, uz, ur, p, mass;
};

// Phase-field stencil values around a node, read from the LDS tile.
template <typename R>
struct Stencil {
    R c;                                  // centre
    R e, w, n, s;                         // reach 1 along +z, -z, +r, -r
    R ee, ww, nn, ss;                     // reach 2
    R ne, nw, se, sw;                     // diagonals reach 1 (n = +r, e = +z)
    R nne, nnw, sse, ssw;                 // diagonals reach 2
};

// Eqs. 39-40 with c_s^2 = 1/3 and the D2Q9 weights expanded into coefficients.
template <typename R>
__device__ __forceinline__ void iso_derivatives(const Stencil<R> &s, R &dz, R &dr, R &lap)
{
    const R a1 = (R)(4.0 / 9.0), a2 = (R)(1.0 / 18.0), d1 = (R)(1.0 / 9.0), d2 = (R)(1.0 / 72.0);
    dz = a1 * (s.e - s.w) - a2 * (s.ee - s.ww) + d1 * ((s.ne + s.se) - (s.nw + s.sw)) -
         d2 * ((s.nne + s.sse) - (s.nnw + s.ssw));
    dr = a1 * (s.n - s.s) - a2 * (s.nn - s.ss) + d1 * ((s.ne + s.nw) - (s.se + s.sw)) -
         d2 * ((s.nne + s.nnw) - (s.sse + s.ssw));
    // the Laplacian's weights sum to zero: weigh differences from the centre
    // (exact for neighbouring values) instead of cancelling large sums
    const R c = s.c;
    lap = (R)(8.0 / 9.0) * (((s.e - c) + (s.w - c)) + ((s.n - c) + (s.s - c))) -
          a2 * (((s.ee - c) + (s.ww - c)) + ((s.nn - c) + (s.ss - c))) +
          (R)(2.0 / 9.0) * (((s.ne - c) + (s.nw - c)) + ((s.se - c) + (s.sw - c))) -
          d2 * (((s.nne - c) + (s.nnw - c)) + ((s.sse - c) + (s.ssw - c)));
}

// Macroscopic state of one node at time t: the part shared by the step and
// the moments pass.
template <typename R>
struct Macro {
    R phi, rho, nu, dz, dr, fsz, fsr, gzf, p, uz, ur, s_nu;
};

// Eqs. 16-17, 35, 2-4 (with mu~ of Sec. 2.1), 33, 32, with the pressure taken
// from the previous step's velocity (Eq. 33 needs u, Eq. 32 needs p).
template <typename R>
__device__ __forceinline__ void macro_state(const Phys<R> &P, R r, R ir, const Stencil<R> &st,
                                            const R gv[9], R uzp, R urp, Macro<R> &m)
{
    R phi = st.c;
    m.phi = phi;
    m.rho = P.rho_g + phi * P.drho;
    m.nu = P.nu_g + phi * P.dnu;
    R lap;
    iso_derivatives(st, m.dz, m.dr, lap);
    R mu = P.beta4 * phi * (phi - (R)1) * (phi - (R)0.5) - P.kap * lap;
    R mut = mu - P.kap * m.dr * ir;
    m.fsz = mut * m.dz;
    m.fsr = mut * m.dr;
    m.gzf = (m.rho - P.rho_l) * P.g_z;

    R tau_g = (R)3 * m.nu + (R)0.5;                 // Eq. 34, c_s^2 = 1/3
    m.s_nu = div_r((R)1, tau_g);
    R s2 = P.srt ? m.s_nu : P.sg2;
    // the energy moment's rate: 1/tau_g (Eq. 34), or its own with free_s1
    R s1 = P.free_s1 ? P.sg[1] : m.s_nu;
    R itau1 = P.free_s1 ? P.isg1 : tau_g;
    // Eq. 33's coefficient; for the raw-moment basis the same Chapman-Enskog
    // step (Appendix C) gives (3/s_c - 1/s_q - 1)/2, s_c = s_1 the rate of
    // c_z^2 + c_r^2 and s_q = s_2^g that of c_z^2 c_r^2
    R s_p = P.nmrt ? (R)0.5 * ((R)3 * itau1 - P.isg2 - (R)1)
                   : div_r(s1 + s2 - s1 * s2, (R)2 * s1 * s2);

    R g_moving = ((gv[1] + gv[2]) + (gv[3] + gv[4])) + ((gv[5] + gv[6]) + (gv[7] + gv[8]));
    R ugr = P.drho * (uzp * m.dz + urp * m.dr);
    // c_s^2/(1-w0) = 3/5;  rho s_0(u) = -(2/3) rho |u|^2;  w0 = 4/9
    m.p = (R)0.6 * (g_moving * ir + (R)0.5 * ugr - (R)(2.0 / 3.0) * m.rho * (uzp * uzp + urp * urp) -
                    s_p * (R)(4.0 / 9.0) * m.rho * urp * ir);

    R jz = (gv[1] - gv[3]) + ((gv[5] - gv[6]) + (gv[8] - gv[7]));
    R jr = (gv[2] - gv[4]) + ((gv[5] + gv[6]) - (gv[7] + gv[8]));
    m.uz = (jz + (R)0.5 * r * (m.fsz + m.gzf)) / (r * m.rho);
    m.ur = (jr + (R)0.5 * (r * m.fsr + m.p)) / (r * m.rho + m.rho * m.nu * ir);
}

// m = M v for the matrix of Sec. 2.2
template <typename R>
__device__ __forceinline__ void to_moments(const R v[9], R m[9])
{
    R axis = (v[1] + v[2]) + (v[3] + v[4]);
    R diag = (v[5] + v[6]) + (v[7] + v[8]);
    R qz = (v[5] - v[6]) - (v[7] - v[8]);
    R qr = (v[5] + v[6]) - (v[7] + v[8]);
    m[0] = v[0] + axis + diag;
    m[1] = (R)-4 * v[0] - axis + (R)2 * diag;
    m[2] = (R)4 * v[0] - (R)2 * axis + diag;
    m[3] = (v[1] - v[3]) + qz;
    m[4] = (R)-2 * (v[1] - v[3]) + qz;
    m[5] = (v[2] - v[4]) + qr;
    m[6] = (R)-2 * (v[2] - v[4]) + qr;
    m[7] = (v[1] - v[2]) + (v[3] - v[4]);
    m[8] = (v[5] - v[6]) + (v[7] - v[8]);
}

// v = M^-1 m, using M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
// (the rows of M are orthogonal)
template <typename R>
__device__ __forceinline__ void from_moments(const R m[9], R v[9])
{
    R n0 = m[0] * (R)(1.0 / 9.0), n1 = m[1] * (R)(1.0 / 36.0), n2 = m[2] * (R)(1.0 / 36.0);
    R n3 = m[3] * (R)(1.0 / 6.0), n4 = m[4] * (R)(1.0 / 12.0), n5 = m[5] * (R)(1.0 / 6.0);
    R n6 = m[6] * (R)(1.0 / 12.0), n7 = m[7] * (R)0.25, n8 = m[8] * (R)0.25;
    R base_a = n0 - n1 - (R)2 * n2;            // links 1-4
    R base_d = n0 + (R)2 * n1 + n2;            // links 5-8
    R xz = n3 - (R)2 * n4, xr = n5 - (R)2 * n6;
    R yz = n3 + n4, yr = n5 + n6;
    v[0] = n0 - (R)4 * n1 + (R)4 * n2;
    v[1] = base_a + xz + n7;
    v[2] = base_a + xr - n7;
    v[3] = base_a - xz + n7;
    v[4] = base_a - xr - n7;
    v[5] = base_d + yz + yr + n8;
    v[6] = base_d - yz + yr - n8;
    v[7] = base_d - yz - yr + n8;
    v[8] = base_d + yz - yr - n8;
}

// Raw moments of the non-orthogonal form (Sec. 4): rows 1, c_z, c_r,
// c_z^2 + c_r^2, c_z^2 - c_r^2, c_z c_r, c_z^2 c_r, c_z c_r^2, c_z^2 c_r^2
template <typename R>
__device__ __forceinline__ void to_raw(const R v[9], R m[9])
{
    R axis = (v[1] + v[2]) + (v[3] + v[4]);
    R diag = (v[5] + v[6]) + (v[7] + v[8]);
    R d56 = v[5] - v[6], d78 = v[7] - v[8];
    R up = v[5] + v[6], dn = v[7] + v[8];
    m[0] = v[0] + axis + diag;
    m[1] = (v[1] - v[3]) + (d56 - d78);
    m[2] = (v[2] - v[4]) + (up - dn);
    m[3] = axis + (R)2 * diag;
    m[4] = (v[1] + v[3]) - (v[2] + v[4]);
    m[5] = d56 + d78;
    m[6] = up - dn;
    m[7] = d56 - d78;
    m[8] = diag;
}

// v = N^-1 m for the raw basis (exact: coefficients 1, 1/2, 1/4)
template <typename R>
__device__ __forceinline__ void from_raw(const R m[9], R v[9])
{
    R h1 = (R)0.5 * m[1], h2 = (R)0.5 * m[2];
    R qp = (R)0.25 * (m[3] + m[4]), qm = (R)0.25 * (m[3] - m[4]);
    R h6 = (R)0.5 * m[6], h7 = (R)0.5 * m[7], h8 = (R)0.5 * m[8];
    R a = (R)0.25 * (m[8] + m[6]), b = (R)0.25 * (m[5] + m[7]);
    R c = (R)0.25 * (m[8] - m[6]), d = (R)0.25 * (m[5] - m[7]);
    v[0] = (m[0] - m[3]) + m[8];
    v[1] = (h1 + qp) - (h7 + h8);
    v[2] = (h2 + qm) - (h6 + h8);
    v[3] = (qp - h1) + (h7 - h8);
    v[4] = (qm - h2) + (h6 - h8);
    v[5] = a + b;
    v[6] = a - b;
    v[7] = c + d;
    v[8] = c - d;
}

// MRT relaxation with a source, in moment space: m+ = m - S(m - m_eq) + (1 - S/2) src
template <typename R>
__device__ __forceinline__ void relax(R m[9], const R s[9], const R meq[9], const R src[9])
{
#pragma unroll
    for (int a = 0; a < 9; ++a)
        m[a] = m[a] - s[a] * (m[a] - meq[a]) + ((R)1 - (R)0.5 * s[a]) * src[a];
}

// Collision of both populations at one node (Eqs. 19, 21-23 for f; 24, 27-30,
// 36-37 for g).  fv, gv: post-propagation values in, post-collision out.
// MODE selects the form (COLLIDE_*, Phys::mode); it is a template argument so
// that each kernel holds one collision form only and the register allocation
// is not the union of several.
template <int MODE, typename R>
__device__ __forceinline__ void collide_node(const Phys<R> &P, R r, R ir, const Macro<R> &m,
                                             R php, R uzp, R urp, R fv[9], R gv[9])
{
    // ---- f (phase field)
    R rphi = r * m.phi;                          // r phi for the fluxes
    R Jz = rphi * m.uz;
    R Jr = rphi * m.ur + P.mob * m.phi;
    R Jz_p = r * php * uzp;
    R Jr_p = r * php * urp + P.mob * php;
    R lam = P.lam4W * m.phi * ((R)1 - m.phi);
    R gsq = m.dz * m.dz + m.dr * m.dr;
    R nz = 0, nr = 0;
    if (gsq > (R)1e-24) {                       // |grad phi| > 1e-12
        R ig = rsqrt_r(gsq);
        nz = m.dz * ig;
        nr = m.dr * ig;
    }
    R src1 = (Jz - Jz_p) + (R)(1.0 / 3.0) * r * nz * lam;
    R src2 = (Jr - Jr_p) + (R)(1.0 / 3.0) * r * nr * lam;

    R uz = m.uz, ur = m.ur, rho = m.rho;
    R u2 = uz * uz + ur * ur;
    R dzr = r * P.drho * m.dz;                 // d_z (r rho)
    R drr = r * P.drho * m.dr + rho;           // d_r (r rho)
    R Fz = r * (m.fsz + m.gzf);
    R Fr = r * m.fsr + m.p - (R)2 * rho * m.nu * ur * ir;
    R rrho = r * rho;
    R udr = uz * dzr + ur * drr;               // u . grad(r rho)

    if constexpr (MODE == COLLIDE_SRT) {
        // Every rate equal: m+ = (1 - s) m + s m_eq + (1 - s/2) src for all
        // nine moments, so v+ = (1 - s) v + M^-1 (s m_eq + (1 - s/2) src)
        // and the populations need no forward transform.
        {
            R mass = sum9(fv);
            R s = P.sf[3], h = (R)1 - (R)0.5 * s, a = (R)1 - s;
            R qz = s * Jz + h * src1, qr = s * Jr + h * src2, sm = s * mass;
            R q[9] = {sm, (R)-2 * sm, sm, qz, -qz, qr, -qr, 0, 0};
            R w[9];
            from_moments(q, w);
#pragma unroll
            for (int i = 1; i < 9; ++i)
                fv[i] = a * fv[i] + w[i];
            fv[0] = mass - ((((fv[1] + fv[2]) + (fv[3] + fv[4])) + ((fv[5] + fv[6]) + (fv[7] + fv[8]))));
        }
        {
            R s = m.s_nu, h = (R)1 - (R)0.5 * s, a = (R)1 - s;
            R q[9], w[9];
            q[0] = h * (udr - rho * ur);
            q[1] = s * ((R)3 * r * ((R)2 * m.p + rho * u2)) + h * ((R)2 * rho * ur);
            q[2] = s * ((R)-3 * r * ((R)3 * m.p + rho * u2)) + h * (-udr - rho * ur);
            q[3] = s * (rrho * uz) + h * Fz;
            q[4] = -q[3];
            q[5] = s * (rrho * ur) + h * Fr;
            q[6] = -q[5];
            q[7] = s * (rrho * (uz * uz - ur * ur)) + h * ((R)(2.0 / 3.0) * (uz * dzr - ur * drr));
            q[8] = s * (rrho * uz * ur) + h * ((R)(1.0 / 3.0) * (uz * drr + ur * dzr));
            from_moments(q, w);
#pragma unroll
            for (int i = 0; i < 9; ++i)
                gv[i] = a * gv[i] + w[i];
        }
        return;
    }
    if constexpr (MODE == COLLIDE_NMRT) {
        // Eqs. 9-10 and 24 with the raw-moment basis N in place of M: the
        // equilibria and sources are the population forms (Eqs. 11, 15, 25-26,
        // 29) in raw moments; raw row a relaxes with the rate of the
        // orthogonal moment it stands for (1 <- s0, c_z <- s3, c_r <- s5,
        // c^2 <- s1, c_z^2 - c_r^2 <- s7, c_z c_r <- s8, c_z^2 c_r <- s6,
        // c_z c_r^2 <- s4, c_z^2 c_r^2 <- s2)
        {
            R mm[9], meq[9], srcv[9], s[9];
            to_raw(fv, mm);
            R mass = mm[0];
            meq[0] = mass; meq[1] = Jz; meq[2] = Jr;
            meq[3] = (R)(2.0 / 3.0) * mass; meq[4] = 0; meq[5] = 0;
            meq[6] = (R)(1.0 / 3.0) * Jr; meq[7] = (R)(1.0 / 3.0) * Jz; meq[8] = (R)(1.0 / 9.0) * mass;
            srcv[0] = 0; srcv[1] = src1; srcv[2] = src2; srcv[3] = 0; srcv[4] = 0; srcv[5] = 0;
            srcv[6] = (R)(1.0 / 3.0) * src2; srcv[7] = (R)(1.0 / 3.0) * src1; srcv[8] = 0;
            s[0] = P.sf[0]; s[1] = P.sf[3]; s[2] = P.sf[5]; s[3] = P.sf[1]; s[4] = P.sf[7];
            s[5] = P.sf[8]; s[6] = P.sf[6]; s[7] = P.sf[4]; s[8] = P.sf[2];
            relax(mm, s, meq, srcv);
            from_raw(mm, fv);
            fv[0] = mass - ((((fv[1] + fv[2]) + (fv[3] + fv[4])) + ((fv[5] + fv[6]) + (fv[7] + fv[8]))));
        }
        {
            R mm[9], meq[9], srcv[9], s[9];
            to_raw(gv, mm);
            R rp = r * m.p, ru2 = rrho * u2;
            meq[0] = 0; meq[1] = rrho * uz; meq[2] = rrho * ur;
            meq[3] = (R)2 * rp + ru2;
            meq[4] = rrho * (uz * uz - ur * ur);
            meq[5] = rrho * uz * ur;
            meq[6] = (R)(1.0 / 3.0) * (rrho * ur);
            meq[7] = (R)(1.0 / 3.0) * (rrho * uz);
            meq[8] = (R)(1.0 / 3.0) * (rp + ru2);
            R rur = rho * ur;
            srcv[0] = udr - rur;
            srcv[1] = Fz; srcv[2] = Fr;
            srcv[3] = (R)(4.0 / 3.0) * udr - (R)(2.0 / 3.0) * rur;
            srcv[4] = (R)(2.0 / 3.0) * (uz * dzr - ur * drr);
            srcv[5] = (R)(1.0 / 3.0) * (uz * drr + ur * dzr);
            srcv[6] = (R)(1.0 / 3.0) * Fr;
            srcv[7] = (R)(1.0 / 3.0) * Fz;
            srcv[8] = (R)(1.0 / 3.0) * udr - (R)(1.0 / 9.0) * rur;
            s[0] = P.sg[0]; s[1] = P.sg[3]; s[2] = P.sg[5]; s[3] = P.free_s1 ? P.sg[1] : m.s_nu; s[4] = m.s_nu;
            s[5] = m.s_nu; s[6] = P.sg[6]; s[7] = P.sg[4]; s[8] = P.sg[2];
            relax(mm, s, meq, srcv);
            from_raw(mm, gv);
        }
        return;
    }
    if constexpr (MODE == COLLIDE_MRT_UNIT) {
        // Every free rate is 1: a moment relaxed with rate 1 becomes its
        // equilibrium plus half its source whatever its value, so only the
        // moments with other rates are formed from the populations:
        // m3..m6 (rate 1/tau_f) of f, m1, m7, m8 (rate 1/tau_g) of g.
        {
            R mass = sum9(fv);                 // conserved: sum f+ = sum f
            R d13 = fv[1] - fv[3], d24 = fv[2] - fv[4];
            R qz = (fv[5] - fv[6]) - (fv[7] - fv[8]);
            R qr = (fv[5] + fv[6]) - (fv[7] + fv[8]);
            R m3 = d13 + qz, m4 = (R)-2 * d13 + qz;
            R m5 = d24 + qr, m6 = (R)-2 * d24 + qr;
            R s = P.sf[3], h = (R)1 - (R)0.5 * s;
            m3 = m3 - s * (m3 - Jz) + h * src1;
            m4 = m4 - s * (m4 + Jz) - h * src1;
            m5 = m5 - s * (m5 - Jr) + h * src2;
            m6 = m6 - s * (m6 + Jr) - h * src2;
            // M^-1 with m0 = mass, m1 = -2 mass, m2 = mass, m7 = m8 = 0
            R base_a = mass * (R)(1.0 / 9.0);
            R base_d = mass * (R)(1.0 / 36.0);
            R n3 = m3 * (R)(1.0 / 6.0), n4 = m4 * (R)(1.0 / 12.0);
            R n5 = m5 * (R)(1.0 / 6.0), n6 = m6 * (R)(1.0 / 12.0);
            R xz = n3 - (R)2 * n4, xr = n5 - (R)2 * n6, yz = n3 + n4, yr = n5 + n6;
            fv[1] = base_a + xz;
            fv[2] = base_a + xr;
            fv[3] = base_a - xz;
            fv[4] = base_a - xr;
            fv[5] = base_d + yz + yr;
            fv[6] = base_d - yz + yr;
            fv[7] = base_d - yz - yr;
            fv[8] = base_d + yz - yr;
            fv[0] = mass - ((((fv[1] + fv[2]) + (fv[3] + fv[4])) + ((fv[5] + fv[6]) + (fv[7] + fv[8]))));
        }
        {
            R axis = (gv[1] + gv[2]) + (gv[3] + gv[4]);
            R diag = (gv[5] + gv[6]) + (gv[7] + gv[8]);
            R mm[9];
            R m1 = (R)-4 * gv[0] - axis + (R)2 * diag;
            R m7 = (gv[1] - gv[2]) + (gv[3] - gv[4]);
            R m8 = (gv[5] - gv[6]) + (gv[7] - gv[8]);
            R s = m.s_nu, h = (R)1 - (R)0.5 * s;
            R meq1 = (R)3 * r * ((R)2 * m.p + rho * u2);
            R meq7 = rrho * (uz * uz - ur * ur);
            R meq8 = rrho * uz * ur;
            mm[0] = (R)0.5 * (udr - rho * ur);
            mm[1] = m1 - s * (m1 - meq1) + h * ((R)2 * rho * ur);
            mm[2] = (R)-3 * r * ((R)3 * m.p + rho * u2) + (R)0.5 * (-udr - rho * ur);
            mm[3] = rrho * uz + (R)0.5 * Fz;
            mm[4] = -mm[3];
            mm[5] = rrho * ur + (R)0.5 * Fr;
            mm[6] = -mm[5];
            mm[7] = m7 - s * (m7 - meq7) + h * ((R)(2.0 / 3.0) * (uz * dzr - ur * drr));
            mm[8] = m8 - s * (m8 - meq8) + h * ((R)(1.0 / 3.0) * (uz * drr + ur * dzr));
            from_moments(mm, gv);
        }
        return;
    }
    {
        R mm[9], meq[9], srcv[9];
        to_moments(fv, mm);
        // r phi is the conserved moment sum f itself: use it, not r*(sum/r),
        // so that rounding cannot bias the phase mass
        R mass = mm[0];
        meq[0] = mass; meq[1] = (R)-2 * mass; meq[2] = mass;
        meq[3] = Jz; meq[4] = -Jz; meq[5] = Jr; meq[6] = -Jr; meq[7] = 0; meq[8] = 0;
        srcv[0] = 0; srcv[1] = 0; srcv[2] = 0;
        srcv[3] = src1; srcv[4] = -src1; srcv[5] = src2; srcv[6] = -src2; srcv[7] = 0; srcv[8] = 0;
        relax(mm, P.sf, meq, srcv);
        from_moments(mm, fv);
        // rest population from the conserved sum: sum f+ = sum f up to one rounding
        fv[0] = mass - ((((fv[1] + fv[2]) + (fv[3] + fv[4])) + ((fv[5] + fv[6]) + (fv[7] + fv[8]))));
    }
    // ---- g (hydrodynamics)
    {
        R mm[9], meq[9], srcv[9], s[9];
        to_moments(gv, mm);
        meq[0] = 0;
        meq[1] = (R)3 * r * ((R)2 * m.p + rho * u2);
        meq[2] = (R)-3 * r * ((R)3 * m.p + rho * u2);
        meq[3] = rrho * uz; meq[4] = -rrho * uz;
        meq[5] = rrho * ur; meq[6] = -rrho * ur;
        meq[7] = rrho * (uz * uz - ur * ur);
        meq[8] = rrho * uz * ur;
        srcv[0] = udr - rho * ur;                  // = r u . grad rho
        srcv[1] = (R)2 * rho * ur;
        srcv[2] = -udr - rho * ur;
        srcv[3] = Fz; srcv[4] = -Fz; srcv[5] = Fr; srcv[6] = -Fr;
        srcv[7] = (R)(2.0 / 3.0) * (uz * dzr - ur * drr);
        srcv[8] = (R)(1.0 / 3.0) * (uz * drr + ur * dzr);
#pragma unroll
        for (int a = 0; a < 9; ++a)
            s[a] = P.sg[a];
        s[1] = P.free_s1 ? P.sg[1] : m.s_nu; s[7] = m.s_nu; s[8] = m.s_nu;
        relax(mm, s, meq, srcv);
        from_moments(mm, gv);
    }
}

// ------------------------------------------------------- tile scheduling --
// Workgroups are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous run of tiles so neighbouring tiles share its L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int nx = 8;
    int q = nb / nx, rem = nb % nx;
    int x = b % nx, l = b / nx;
    return x * q + (x < rem ? x : rem) + l;
}

// Cell h of the 2-wide ring around a TZ x TR tile, as (cz, cr) in the
// (TR+4) x (TZ+4) LDS tile: first the TZ inner cells of the four ring rows
// (two below, two above; with TZ the wavefront size and the workgroup a whole
// number of waves, each wave holds one ring row), then the 16 corner cells,
// then the two left and two right cells of every interior row.
template <int TZ, int TR>
__device__ __forceinline__ void ring_cell(int h, int &cz, int &cr)
{
    if (h < 4 * TZ) {
        int q = h / TZ;
        cr = q < 2 ? q : TR + q;
        cz = 2 + h % TZ;
    } else if (h < 4 * TZ + 16) {
        int hh = h - 4 * TZ, q = hh >> 2, c = hh & 3;
        cr = q < 2 ? q : TR + q;
        cz = c < 2 ? c : TZ + c;
    } else {
        int hh = h - 4 * TZ - 16, c = hh & 3;
        cr = 2 + (hh >> 2);
        cz = c < 2 ? c : TZ + c;
    }
}

// Fill the (TR+4) x (TZ+4) phase-field tile whose interior origin is (k0, j0).
// Cells outside the grid hold the ghost values of Sec. 2.3.  The calling
// thread's own cell (tx, ty) is written by the caller.
template <typename T, typename R, int TZ, int TR>
__device__ __forceinline__ void fill_halo(const Geom &g, const T *__restrict__ f, int k0, int j0,
                                          R (*tile)[TZ + 4])
{
    constexpr int NH = (TZ + 4) * (TR + 4) - TZ * TR;
    for (int h = threadIdx.x; h < NH; h += TZ * TR) {
        int cz, cr;
        ring_cell<TZ, TR>(h, cz, cr);
        int kk = ghost_col(k0 + cz - 2, g.nz, g.zper);
        int jj = ghost_row(j0 + cr - 2, g.nr);
        tile[cr][cz] = phase_at<T, R>(g, f, kk, jj);
    }
}

template <typename R, int TZ>
__device__ __forceinline__ void read_stencil(R (*tile)[TZ + 4], int tx, int ty, Stencil<R> &s)
{
    const int x = tx + 2, y = ty + 2;
    s.c = tile[y][x];
    s.e = tile[y][x + 1]; s.w = tile[y][x - 1]; s.n = tile[y + 1][x]; s.s = tile[y - 1][x];
    s.ee = tile[y][x + 2]; s.ww = tile[y][x - 2]; s.nn = tile[y + 2][x]; s.ss = tile[y - 2][x];
    s.ne = tile[y + 1][x + 1]; s.nw = tile[y + 1][x - 1]; s.se = tile[y - 1][x + 1]; s.sw = tile[y - 1][x - 1];
    s.nne = tile[y + 2][x + 2]; s.nnw = tile[y + 2][x - 2]; s.sse = tile[y - 2][x + 2]; s.ssw = tile[y - 2][x - 2];
}

// One time step of the TZ x TR tile (tz, tr) of a case (tile column, row): every global load (own f and
// g, previous-step values, the ring's f) is issued before the first LDS write,
// so the workgroup waits for memory once; then the barrier, the stencil and
// the collision of the tile's own nodes, and the stores.
// Pulls: population i arriving at node n comes from n - c_iz - c_ir*nz of
// plane i.  Interior and seam tiles read through raw buffers, the plane and
// link shift being the scalar offset (pull9_buf); boundary tiles fold plane,
// link shift and node into one 32-bit byte offset per access on a uniform
// 64-bit base (9 planes of a case stay below 4 GiB), selected by the boundary
// rules (pull_off).
struct Pitch {
    uint32_t plane;     // bytes between population planes
    uint32_t row;       // bytes between rows
};

template <typename T>
__device__ __forceinline__ Pitch pitch_of(const Geom &g)
{
    return Pitch{(uint32_t)(g.plane * (int64_t)sizeof(T)), (uint32_t)(g.nz * (int)sizeof(T))};
}

template <int I, typename T>
__device__ __forceinline__ uint32_t link_offset(const Pitch &p)
{
    return (uint32_t)I * p.plane - (uint32_t)(link_r(I) * (int)p.row) - (uint32_t)(link_z(I) * (int)sizeof(T));
}

// Stores stream past L2 with the non-temporal hint at device scope (cache
// policy bits nt and sc1; measured in FP32: the default policy 7 % slower,
// the hint at the default scope 0.4 % slower), keeping L2 for the f lines
// that neighbouring tiles read again for their phase-field ring (the hint on
// the f loads costs 20-30 %).  Loads keep the default policy (see tile_step).
#ifndef AXI_STREAMING
#define AXI_STREAMING 1
#endif
// Raw buffer view of a group of planes (stride 0, the full 32-bit record
// count, the fourth word as the gfx9 family takes it): an access is the
// node's byte offset (vector) plus a uniform plane and link offset (scalar),
// and the memory instruction adds the two, so an interior tile's loads and
// every store cost no vector address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, -1, 0x00020000);
}

// cache policy of the streamed accesses: the non-temporal bit
constexpr int STREAM_POL = AXI_STREAMING ? (2 | 16) : 0;

template <typename T, int POL>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, POL));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, POL));
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, STREAM_POL);
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, STREAM_POL);
}

// Byte offsets of a node (in-grid column c, element size es) and of its
// column neighbours c - 1 (m) and c + 1 (p), wrapped across the periodic z
// ends: away from the two end columns all three are the node's own offset,
// and the column shift of a link stays in its scalar offset.
struct ColOff {
    uint32_t m, o, p;
};
template <bool WRAP>
__device__ __forceinline__ ColOff col_off(uint32_t off, int c, const Geom &g, uint32_t es)
{
    if constexpr (!WRAP) {
        return ColOff{off, off, off};
    } else {
        const uint32_t span = (uint32_t)g.nz * es;
        return ColOff{off + (c == 0 ? span : 0u), off, off - (c == g.nz - 1 ? span : 0u)};
    }
}

// a column of a tile's ring, wrapped into the grid across the periodic z ends
template <bool WRAP>
__device__ __forceinline__ int wrap_col(int c, int nz)
{
    if constexpr (!WRAP)
        return c;
    else
        return c < 0 ? c + nz : (c >= nz ? c - nz : c);
}

// the vector offset of the source of population I (column k - c_Iz)
template <int I>
__device__ __forceinline__ uint32_t link_voff(const ColOff &co)
{
    constexpr int CZ = link_z(I);
    return CZ > 0 ? co.m : (CZ < 0 ? co.p : co.o);
}

// the nine pulls of a node whose sources are all plain neighbours (columns
// possibly wrapped): every link offset is non-negative (population i reads
// plane i, whose offset exceeds any row or column shift)
template <typename T, typename R, int POL>
__device__ __forceinline__ void pull9_buf(__amdgpu_buffer_rsrc_t r, const Pitch &p, const ColOff &co, R v[9])
{
    v[0] = (R)buf_load<T, POL>(r, link_voff<0>(co), link_offset<0, T>(p));
    v[1] = (R)buf_load<T, POL>(r, link_voff<1>(co), link_offset<1, T>(p));
    v[2] = (R)buf_load<T, POL>(r, link_voff<2>(co), link_offset<2, T>(p));
    v[3] = (R)buf_load<T, POL>(r, link_voff<3>(co), link_offset<3, T>(p));
    v[4] = (R)buf_load<T, POL>(r, link_voff<4>(co), link_offset<4, T>(p));
    v[5] = (R)buf_load<T, POL>(r, link_voff<5>(co), link_offset<5, T>(p));
    v[6] = (R)buf_load<T, POL>(r, link_voff<6>(co), link_offset<6, T>(p));
    v[7] = (R)buf_load<T, POL>(r, link_voff<7>(co), link_offset<7, T>(p));
    v[8] = (R)buf_load<T, POL>(r, link_voff<8>(co), link_offset<8, T>(p));
}

// Byte offset of the source of population I arriving at node (k, j), whose own
// offset is `own` = (j*nz + k)*sizeof(T): the boundary rules of pull_slot
// written as selects on the interior offset, so that a tile touching the
// boundary issues its loads back to back like an interior tile.
template <int I, typename T>
__device__ __forceinline__ uint32_t pull_off(const Geom &g, const Pitch &p, int k, int j, uint32_t own)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    uint32_t off = own + link_offset<I, T>(p);
    bool wall = false;
    if constexpr (CZ != 0) {
        bool out = (CZ > 0) ? (k - CZ < 0) : (k - CZ >= g.nz);
        if (g.zper)
            off = out ? off + (CZ > 0 ? p.row : (uint32_t)0 - p.row) : off;
        else
            wall = out;
    }
    if constexpr (CR < 0)
        wall = wall || (j - CR >= g.nr);
    if constexpr (CR > 0)   // row -1 lies beyond the axis: mirror image on row 0
        off = (j - CR < 0) ? off + (uint32_t)(axis_image(I) - I) * p.plane + p.row : off;
    return wall ? own + (uint32_t)reverse_link(I) * p.plane : off;
}

template <typename T, typename R>
__device__ __forceinline__ void pull9_bc(const char *base, const Geom &g, const Pitch &p, int k, int j, R v[9])
{
    const uint32_t own = (uint32_t)(j * g.nz + k) * (uint32_t)sizeof(T);
    const uint32_t o[9] = {pull_off<0, T>(g, p, k, j, own), pull_off<1, T>(g, p, k, j, own),
                           pull_off<2, T>(g, p, k, j, own), pull_off<3, T>(g, p, k, j, own),
                           pull_off<4, T>(g, p, k, j, own), pull_off<5, T>(g, p, k, j, own),
                           pull_off<6, T>(g, p, k, j, own), pull_off<7, T>(g, p, k, j, own),
                           pull_off<8, T>(g, p, k, j, own)};
#pragma unroll
    for (int i = 0; i < 9; ++i)
        v[i] = (R) * (const T *)(base + o[i]);
}

template <typename T, typename R, int TZ, int TR, int MODE>
__device__ __forceinline__ void tile_step(const Geom &g, const Phys<R> &P, int tz, int tr,
                                          const T *__restrict__ fin, const T *__restrict__ gin,
                                          T *__restrict__ fout, T *__restrict__ gout,
                                          T *__restrict__ aux, R (*tile)[TZ + 4])
{
    constexpr int NT = TZ * TR;
    constexpr int NH = (TZ + 4) * (TR + 4) - NT;
    constexpr int NHI = (NH + NT - 1) / NT;
    int k0 = tz * TZ, j0 = tr * TR;
    static_assert(TZ == 64, "a tile row is one wavefront");
    // the row is wave-uniform: scalar row arithmetic
    int tx = threadIdx.x % TZ, ty = __builtin_amdgcn_readfirstlane(threadIdx.x / TZ);
    int k = k0 + tx, j = j0 + ty;
    // the ring reads populations up to 3 cells beyond the tile: if all of them
    // are inside the grid, no boundary or ghost rule can apply (uniform
    // branch); with periodic z and rows clear of the axis and the r-wall,
    // only columns wrap (plain: the same path, with wrapped column offsets)
    const bool rows_in = (j0 >= 3) && (j0 + TR + 3 <= g.nr);
    const bool interior = rows_in && (k0 >= 3) && (k0 + TZ + 3 <= g.nz);
    const bool plain = interior || (rows_in && g.zper && (g.nz >= TZ + 6));
    bool inside = (k < g.nz) && (j < g.nr);
    int64_t n = (int64_t)j * g.nz + k;

    R fv[9], gv[9];
    R php = 0, uzp = 0, urp = 0;
    R hphi[NHI];
    int hcz[NHI], hcr[NHI];
    int jo = j;
    // rows inside the grid: interior tiles (WRAP false: all three column
    // offsets are the node's own) and tiles at the periodic z ends (WRAP
    // true), each instantiated on its own; a node beyond the last column
    // (ragged tile) evaluates phi at its periodic image and reads its own g
    // and aux there without using them
    auto plain_loads = [&](auto wrap) {
        constexpr bool WRAP = decltype(wrap)::value;
        const int ko = (WRAP && k >= g.nz) ? k - g.nz : k;
        const ColOff co = col_off<WRAP>((uint32_t)(j * g.nz + ko) * (uint32_t)sizeof(T), ko, g, sizeof(T));
        const Pitch pt = pitch_of<T>(g);
        const __amdgpu_buffer_rsrc_t fr = raw_rsrc(fin), gr = raw_rsrc(gin), ar = raw_rsrc(aux);
        // g and aux loads keep the default cache policy as well: the shifted
        // g pulls of a wave share their end lines with the neighbouring
        // tile's, and the non-temporal hint on them measured 1 % slower
        pull9_buf<T, R, 0>(fr, pt, co, fv);
        pull9_buf<T, R, 0>(gr, pt, co, gv);
        php = (R)buf_load<T, 0>(ar, co.o, 0);
        uzp = (R)buf_load<T, 0>(ar, co.o, pt.plane);
        urp = (R)buf_load<T, 0>(ar, co.o, 2 * pt.plane);
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int h = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (h < NH) {
                ring_cell<TZ, TR>(h, hcz[q], hcr[q]);
                int jj = j0 + hcr[q] - 2;
                int kk = wrap_col<WRAP>(k0 + hcz[q] - 2, g.nz);
                R v[9];
                pull9_buf<T, R, 0>(fr, pt, col_off<WRAP>((uint32_t)(jj * g.nz + kk) * (uint32_t)sizeof(T), kk, g,
                                                          sizeof(T)), v);
                hphi[q] = sum9(v) * inv_radius<R>(jj);
            }
        }
    };
    if (interior) {
        plain_loads(std::false_type{});
    } else if (plain) {
        plain_loads(std::true_type{});
    } else {
        // a tile that touches the boundary: the same loads through pull_off;
        // a thread beyond the grid evaluates phi at its ghost cell (Sec. 2.3)
        // and reads its own g and aux at that cell without using them
        const Pitch pt = pitch_of<T>(g);
        const char *fb = (const char *)fin, *gb = (const char *)gin, *ab = (const char *)aux;
        int ko = inside ? k : ghost_col(k, g.nz, g.zper);
        jo = inside ? j : ghost_row(j, g.nr);
        pull9_bc<T, R>(fb, g, pt, ko, jo, fv);
        pull9_bc<T, R>(gb, g, pt, ko, jo, gv);
        const uint32_t offo = (uint32_t)(jo * g.nz + ko) * (uint32_t)sizeof(T);
        php = (R)*(const T *)(ab + offo);
        uzp = (R)*(const T *)(ab + (offo + pt.plane));
        urp = (R)*(const T *)(ab + (offo + 2 * pt.plane));
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int h = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (h < NH) {
                ring_cell<TZ, TR>(h, hcz[q], hcr[q]);
                int kk = ghost_col(k0 + hcz[q] - 2, g.nz, g.zper);
                int jj = ghost_row(j0 + hcr[q] - 2, g.nr);
                R v[9];
                pull9_bc<T, R>(fb, g, pt, kk, jj, v);
                hphi[q] = sum9(v) * inv_radius<R>(jj);
            }
        }
    }
    tile[ty + 2][tx + 2] = sum9(fv) * inv_radius<R>(jo);
#pragma unroll
    for (int q = 0; q < NHI; ++q)
        if (hcz[q] >= 0)
            tile[hcr[q]][hcz[q]] = hphi[q];
    __syncthreads();
    if (inside) {
        Stencil<R> st;
        read_stencil<R, TZ>(tile, tx, ty, st);
        R r = (R)j + (R)0.5, ir = inv_radius<R>(j);
        Macro<R> m;
        macro_state(P, r, ir, st, gv, uzp, urp, m);
        collide_node<MODE>(P, r, ir, m, php, uzp, urp, fv, gv);
        const uint32_t off = (uint32_t)n * (uint32_t)sizeof(T);
        const uint32_t pb = (uint32_t)(g.plane * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t fo = raw_rsrc(fout), go = raw_rsrc(gout), ao = raw_rsrc(aux);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            buf_store((T)fv[i], fo, off, (uint32_t)i * pb);
            buf_store((T)gv[i], go, off, (uint32_t)i * pb);
        }
        buf_store((T)m.phi, ao, off, 0);
        buf_store((T)m.uz, ao, off, pb);
        buf_store((T)m.ur, ao, off, 2 * pb);
    }
}

// Per-case record of a batch, read by every workgroup working on the case.
// Buffers are byte offsets from the pool base, a kernel argument, so that every
// access is known to be a global-memory access.
template <typename R>
struct CaseDesc {
    Geom g;
    Phys<R> P;
    uint64_t pop[2][2];  // [buffer][f or g]
    uint64_t aux;
    int cur0;            // buffer holding the state at the start of the launch sequence
    int pad;
    int64_t t0;          // the case's time when the table was uploaded (gravity ramps)
    Codec C;             // FP16-deviation storage only
};

// One work item of a batched step: tile (tz, tr) of the case in slot `slot`,
// its column and row of tiles decoded on the host (an integer division by a
// run-time divisor costs a kernel some twenty vector instructions).
struct WorkItem {
    int32_t slot;
    int32_t tz, tr;
    int32_t pad;
};

} // namespace axi
