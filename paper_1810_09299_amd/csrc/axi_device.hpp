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
    lap = (R)(8.0 / 9.0) * ((s.e + s.w) + (s.n + s.s)) - a2 * ((s.ee + s.ww) + (s.nn + s.ss)) +
          (R)(2.0 / 9.0) * ((s.ne + s.nw) + (s.se + s.sw)) - d2 * ((s.nne + s.nnw) + (s.sse + s.ssw)) -
          (R)(25.0 / 6.0) * s.c;
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
    m.s_nu = (R)1 / tau_g;
    R s2 = P.sg2;
    R s_p = (m.s_nu + s2 - m.s_nu * s2) / ((R)2 * m.s_nu * s2);

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
template <typename R>
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
        R ig = (R)1 / sqrt(gsq);
        nz = m.dz * ig;
        nr = m.dr * ig;
    }
    R src1 = (Jz - Jz_p) + (R)(1.0 / 3.0) * r * nz * lam;
    R src2 = (Jr - Jr_p) + (R)(1.0 / 3.0) * r * nr * lam;
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
        R uz = m.uz, ur = m.ur, rho = m.rho;
        R u2 = uz * uz + ur * ur;
        R dzr = r * P.drho * m.dz;                 // d_z (r rho)
        R drr = r * P.drho * m.dr + rho;           // d_r (r rho)
        R Fz = r * (m.fsz + m.gzf);
        R Fr = r * m.fsr + m.p - (R)2 * rho * m.nu * ur * ir;
        R rrho = r * rho;
        R mm[9], meq[9], srcv[9], s[9];
        to_moments(gv, mm);
        meq[0] = 0;
        meq[1] = (R)3 * r * ((R)2 * m.p + rho * u2);
        meq[2] = (R)-3 * r * ((R)3 * m.p + rho * u2);
        meq[3] = rrho * uz; meq[4] = -rrho * uz;
        meq[5] = rrho * ur; meq[6] = -rrho * ur;
        meq[7] = rrho * (uz * uz - ur * ur);
        meq[8] = rrho * uz * ur;
        R udr = uz * dzr + ur * drr;               // u . grad(r rho)
        srcv[0] = udr - rho * ur;                  // = r u . grad rho
        srcv[1] = (R)2 * rho * ur;
        srcv[2] = -udr - rho * ur;
        srcv[3] = Fz; srcv[4] = -Fz; srcv[5] = Fr; srcv[6] = -Fr;
        srcv[7] = (R)(2.0 / 3.0) * (uz * dzr - ur * drr);
        srcv[8] = (R)(1.0 / 3.0) * (uz * drr + ur * dzr);
#pragma unroll
        for (int a = 0; a < 9; ++a)
            s[a] = P.sg[a];
        s[1] = m.s_nu; s[7] = m.s_nu; s[8] = m.s_nu;
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
// (TR+4) x (TZ+4) LDS tile: two full rows below, two full rows above, then the
// two left and two right cells of every interior row.
template <int TZ, int TR>
__device__ __forceinline__ void ring_cell(int h, int &cz, int &cr)
{
    constexpr int LZ = TZ + 4, LR = TR + 4;
    if (h < 2 * LZ) {
        cr = h / LZ; cz = h - cr * LZ;
    } else if (h < 4 * LZ) {
        int hh = h - 2 * LZ;
        cr = LR - 2 + hh / LZ; cz = hh % LZ;
    } else {
        int hh = h - 4 * LZ;
        cr = 2 + (hh >> 2);
        int c = hh & 3;
        cz = c < 2 ? c : LZ - 4 + c;
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

// One time step of the TZ x TR tile t of a case: every global load (own f and
// g, previous-step values, the ring's f) is issued before the first LDS write,
// so the workgroup waits for memory once; then the barrier, the stencil and
// the collision of the tile's own nodes, and the stores.
// Pull of the 9 populations arriving at node offset n = j*nz + k when no
// boundary rule can apply: plain neighbour reads, one uniform base pointer per
// population plane and a 32-bit offset per thread.
template <typename T, typename R>
__device__ __forceinline__ void pull9_interior(const Geom &g, const T *__restrict__ src, uint32_t n, R v[9])
{
    const uint32_t nz = (uint32_t)g.nz;
    v[0] = (R)(src + 0 * g.plane)[n];
    v[1] = (R)(src + 1 * g.plane)[n - 1];
    v[2] = (R)(src + 2 * g.plane)[n - nz];
    v[3] = (R)(src + 3 * g.plane)[n + 1];
    v[4] = (R)(src + 4 * g.plane)[n + nz];
    v[5] = (R)(src + 5 * g.plane)[n - nz - 1];
    v[6] = (R)(src + 6 * g.plane)[n - nz + 1];
    v[7] = (R)(src + 7 * g.plane)[n + nz + 1];
    v[8] = (R)(src + 8 * g.plane)[n + nz - 1];
}

template <typename T, typename R, int TZ, int TR>
__device__ __forceinline__ void tile_step(const Geom &g, const Phys<R> &P, int t,
                                          const T *__restrict__ fin, const T *__restrict__ gin,
                                          T *__restrict__ fout, T *__restrict__ gout,
                                          T *__restrict__ aux, R (*tile)[TZ + 4])
{
    constexpr int NT = TZ * TR;
    constexpr int NH = (TZ + 4) * (TR + 4) - NT;
    constexpr int NHI = (NH + NT - 1) / NT;
    int tz = t % g.tiles_z, tr = t / g.tiles_z;
    int k0 = tz * TZ, j0 = tr * TR;
    int tx = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    int k = k0 + tx, j = j0 + ty;
    // the ring reads populations up to 3 cells beyond the tile: if all of them
    // are inside the grid, no boundary or ghost rule can apply (uniform branch)
    bool interior = (j0 >= 3) && (j0 + TR + 3 <= g.nr) && (k0 >= 3) && (k0 + TZ + 3 <= g.nz);
    bool inside = (k < g.nz) && (j < g.nr);
    int64_t n = (int64_t)j * g.nz + k;

    R fv[9], gv[9];
    R php = 0, uzp = 0, urp = 0;
    R hphi[NHI];
    int hcz[NHI], hcr[NHI];
    int jo = j;
    if (interior) {
        uint32_t n32 = (uint32_t)n;
        pull9_interior<T, R>(g, fin, n32, fv);
        pull9_interior<T, R>(g, gin, n32, gv);
        php = (R)aux[n32];
        uzp = (R)(aux + g.plane)[n32];
        urp = (R)(aux + 2 * g.plane)[n32];
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int h = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (h < NH) {
                ring_cell<TZ, TR>(h, hcz[q], hcr[q]);
                int jj = j0 + hcr[q] - 2;
                uint32_t nh = (uint32_t)(jj * g.nz + k0 + hcz[q] - 2);
                R v[9];
                pull9_interior<T, R>(g, fin, nh, v);
                hphi[q] = sum9(v) * inv_radius<R>(jj);
            }
        }
    } else {
        int ko = inside ? k : ghost_col(k, g.nz, g.zper);
        jo = inside ? j : ghost_row(j, g.nr);
        pull9<T, R>(g, fin, ko, jo, fv);
        if (inside) {
            pull9<T, R>(g, gin, k, j, gv);
            php = (R)aux[n];
            uzp = (R)aux[g.plane + n];
            urp = (R)aux[2 * g.plane + n];
        }
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int h = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (h < NH) {
                ring_cell<TZ, TR>(h, hcz[q], hcr[q]);
                int kk = ghost_col(k0 + hcz[q] - 2, g.nz, g.zper);
                int jj = ghost_row(j0 + hcr[q] - 2, g.nr);
                hphi[q] = phase_at<T, R>(g, fin, kk, jj);
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
        collide_node(P, r, ir, m, php, uzp, urp, fv, gv);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            fout[(int64_t)i * g.plane + n] = (T)fv[i];
            gout[(int64_t)i * g.plane + n] = (T)gv[i];
        }
        aux[n] = (T)m.phi;
        aux[g.plane + n] = (T)m.uz;
        aux[2 * g.plane + n] = (T)m.ur;
    }
}

// Per-case record of a batch, read by every workgroup working on the case.
template <typename R>
struct CaseDesc {
    Geom g;
    Phys<R> P;
    void *pop[2][2];     // [buffer][f or g]
    void *aux;
    int cur0;            // buffer holding the state at the start of the launch sequence
    int pad;
};

// One work item of a batched step: tile `tile` of the case in slot `slot`.
struct WorkItem {
    int slot;
    int tile;
};

} // namespace axi
