// FP16-deviation storage of the populations (storage precision 2): the
// device codec and the tile update that uses it.  Arithmetic is FP32.
//
// Stored form of a case:
//   f_0            FP32 plane (the rest population, see "mass" below)
//   f_1..f_8       FP16 planes: h = (f_p - phi_s * b_p(r_s)) / r_s * sf
//   g_0..g_8       FP16 planes: h = (g_p / r_s) * sg
//   phi            two FP32 planes, read from one and written to the other
//   u_z, u_r       FP32 planes, updated in place
// where s is the node that stores the value, r_s its radius, phi_s its phase
// field (the FP32 value stored with it) and b_p(r) = w_p (r + c_pr / 2) the
// post-collision f_p / phi of a node at radius r in a uniform field at rest
// (what the neighbour at r + c_pr receives: the initial state's form).
// Storing the deviation from that bulk value, divided by r, keeps the FP16
// numbers small and independent of the radius; sf and sg are powers of two.
// The shifted-storage idea follows Lehmann et al., Phys. Rev. E 106, 015308
// (2022); the r-weighted reference is specific to the axisymmetric populations.
//
// Mass: a decoded f_p (p >= 1) is rounded to a multiple of the quantum
// q(j) = 2^(floor(log2 r_j) - 21) of the storing node's row j, and f_0 is
// stored as (sum of the node's pulled populations) - (sum of its decoded
// f_1..f_8).  Every sum of a node's populations then adds multiples of the
// smallest quantum of three neighbouring rows whose magnitudes stay below
// 2^24 such quanta, so FP32 adds them exactly: sum_nodes sum_p f is conserved
// exactly from step to step, not only to rounding.
#pragma once

#include "axi_device.hpp"

namespace axi {

typedef _Float16 half_t;

__device__ __forceinline__ float pow2f(int e) { return __int_as_float((127 + e) << 23); }

// floor(log2(j + 1/2)) for a row index j >= 0
__device__ __forceinline__ int row_log2(int j) { return j == 0 ? -1 : 31 - __builtin_clz((unsigned)j); }

// rounded to a multiple of the quantum of row j (exact power-of-two scalings)
__device__ __forceinline__ float quantize_row(float x, int j)
{
    int e = row_log2(j) - 21;
    return __builtin_rintf(x * pow2f(-e)) * pow2f(e);
}

// b_p(r) = w_p (r + c_pr / 2), p >= 1, with p known at compile time ...
template <int P>
__device__ __forceinline__ float bulk_factor(float rs)
{
    constexpr float w = P <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f;
    return w * (rs + 0.5f * (float)link_r(P));
}

// ... or only at run time (the same operations, so the same value)
__device__ __forceinline__ float bulk_factor_rt(int p, float rs)
{
    const float w = p <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f;
    const int c = (p == 2 || p == 5 || p == 6) ? 1 : ((p == 4 || p == 7 || p == 8) ? -1 : 0);
    return w * (rs + 0.5f * (float)c);
}

// f_p (p >= 1) stored at a node of row js (radius rs) with phase field phis,
// fac = b_p(rs): phis * fac + h * rs / sf on the row's grid.  Formed directly
// in units of the row's quantum q (the factors times 1/q are exact
// power-of-two scalings), one fused multiply-add, rounded to an integer.
__device__ __forceinline__ float decode_f(half_t h, float phis, float fac, float rs, int js, const Codec &C)
{
    const int e = row_log2(js) - 21;
    const float qinv = pow2f(-e);
    const float y = __builtin_fmaf((float)h, rs * (C.isf * qinv), phis * (fac * qinv));
    return __builtin_rintf(y) * pow2f(e);
}

__device__ __forceinline__ half_t encode_f(float v, float phin, float fac, float ir, const Codec &C)
{
    return (half_t)((v - phin * fac) * (C.sf * ir));
}

__device__ __forceinline__ float decode_g(half_t h, float rs, const Codec &C) { return (float)h * (rs * C.isg); }

__device__ __forceinline__ half_t encode_g(float v, float ir, const Codec &C) { return (half_t)(v * (C.sg * ir)); }

// Slot that population I arriving at node (k, j) is pulled from, as
// (population p, node (ks, js)): the boundary rules of pull_slot as selects.
template <int I>
__device__ __forceinline__ void pull_source(const Geom &g, int k, int j, int &p, int &ks, int &js)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    ks = k - CZ;
    js = j - CR;
    p = I;
    bool wall = false;
    if constexpr (CZ != 0) {
        bool out = (CZ > 0) ? (ks < 0) : (ks >= g.nz);
        if (g.zper)
            ks = out ? (CZ > 0 ? ks + g.nz : ks - g.nz) : ks;
        else
            wall = out;
    }
    if constexpr (CR < 0)
        wall = wall || (js >= g.nr);
    if constexpr (CR > 0) {
        bool ax = js < 0;
        p = ax ? axis_image(I) : I;
        js = ax ? 0 : js;
    }
    p = wall ? reverse_link(I) : p;
    ks = wall ? k : ks;
    js = wall ? j : js;
}

// Pointers of one case in FP16-deviation storage for one step.
struct HalfState {
    const float *f0in;
    const half_t *fin;    // plane p of f at fin + (p - 1) * plane, p = 1..8
    const half_t *gin;    // plane p of g at gin + p * plane
    float *f0out;
    half_t *fout;
    half_t *gout;
    const float *phin;    // phase field of the stored state
    float *phout;         // phase field written by this step
    float *uz;            // u_z, u_r planes (in place)
    float *ur;
};

template <typename T>
__device__ __forceinline__ T ld_at(const void *base, uint32_t off) { return *(const T *)((const char *)base + off); }
template <typename T>
__device__ __forceinline__ T ld_nt(const void *base, uint32_t off)
{
    return __builtin_nontemporal_load((const T *)((const char *)base + off));
}
template <typename T>
__device__ __forceinline__ void st_nt(void *base, uint32_t off, T v)
{
    __builtin_nontemporal_store(v, (T *)((char *)base + off));
}

// Window position of a source node (ks, js) in the (TR+6) x (TZ+6) tile of
// stored phase fields around the tile at (k0, j0); periodic sources that
// wrapped are moved back next to the tile; clamped so that values no interior
// node uses stay inside the array.
template <int TZ, int TR>
__device__ __forceinline__ void window_pos(const Geom &g, int k0, int j0, int ks, int js, int &wz, int &wr)
{
    int dz = ks - k0 + 3, dr = js - j0 + 3;
    if (g.zper) {
        dz = dz < 0 ? dz + g.nz : dz;
        dz = dz >= TZ + 6 ? dz - g.nz : dz;
    }
    wz = dz < 0 ? 0 : (dz > TZ + 5 ? TZ + 5 : dz);
    wr = dr < 0 ? 0 : (dr > TR + 5 ? TR + 5 : dr);
}

// The f values arriving at a node as stored (f_0 and 8 FP16 words); decoding
// needs the window, so it waits for the barrier.
struct RawF {
    float f0;
    half_t h[8];
};

// ---- tiles that touch the boundary: sources through pull_source
template <int I>
__device__ __forceinline__ half_t raw_bc_one(const Geom &g, const HalfState &S, int k, int j)
{
    int p, ks, js;
    pull_source<I>(g, k, j, p, ks, js);
    return ld_at<half_t>(S.fin, (uint32_t)((p - 1) * g.plane + js * g.nz + ks) * 2u);
}

__device__ __forceinline__ void raw_bc(const Geom &g, const HalfState &S, int k, int j, RawF &rf)
{
    rf.f0 = ld_at<float>(S.f0in, (uint32_t)(j * g.nz + k) * 4u);
    rf.h[0] = raw_bc_one<1>(g, S, k, j);
    rf.h[1] = raw_bc_one<2>(g, S, k, j);
    rf.h[2] = raw_bc_one<3>(g, S, k, j);
    rf.h[3] = raw_bc_one<4>(g, S, k, j);
    rf.h[4] = raw_bc_one<5>(g, S, k, j);
    rf.h[5] = raw_bc_one<6>(g, S, k, j);
    rf.h[6] = raw_bc_one<7>(g, S, k, j);
    rf.h[7] = raw_bc_one<8>(g, S, k, j);
}

template <int I, int TZ, int TR>
__device__ __forceinline__ float decode_bc_one(const Geom &g, const Codec &C, half_t h, int k, int j, int k0, int j0,
                                               float (*win)[TZ + 6])
{
    int p, ks, js, wz, wr;
    pull_source<I>(g, k, j, p, ks, js);
    window_pos<TZ, TR>(g, k0, j0, ks, js, wz, wr);
    const float rs = (float)js + 0.5f;
    return decode_f(h, win[wr][wz], bulk_factor_rt(p, rs), rs, js, C);
}

template <int TZ, int TR>
__device__ __forceinline__ void decode_bc(const Geom &g, const Codec &C, const RawF &rf, int k, int j, int k0, int j0,
                                          float (*win)[TZ + 6], float v[9])
{
    v[0] = rf.f0;
    v[1] = decode_bc_one<1, TZ, TR>(g, C, rf.h[0], k, j, k0, j0, win);
    v[2] = decode_bc_one<2, TZ, TR>(g, C, rf.h[1], k, j, k0, j0, win);
    v[3] = decode_bc_one<3, TZ, TR>(g, C, rf.h[2], k, j, k0, j0, win);
    v[4] = decode_bc_one<4, TZ, TR>(g, C, rf.h[3], k, j, k0, j0, win);
    v[5] = decode_bc_one<5, TZ, TR>(g, C, rf.h[4], k, j, k0, j0, win);
    v[6] = decode_bc_one<6, TZ, TR>(g, C, rf.h[5], k, j, k0, j0, win);
    v[7] = decode_bc_one<7, TZ, TR>(g, C, rf.h[6], k, j, k0, j0, win);
    v[8] = decode_bc_one<8, TZ, TR>(g, C, rf.h[7], k, j, k0, j0, win);
}

template <int I>
__device__ __forceinline__ float pull_g_bc_one(const Geom &g, const HalfState &S, const Codec &C, int k, int j)
{
    int p, ks, js;
    pull_source<I>(g, k, j, p, ks, js);
    half_t h = ld_nt<half_t>(S.gin, (uint32_t)(p * g.plane + js * g.nz + ks) * 2u);
    return decode_g(h, (float)js + 0.5f, C);
}

__device__ __forceinline__ void pull_g_bc(const Geom &g, const HalfState &S, const Codec &C, int k, int j, float v[9])
{
    v[0] = pull_g_bc_one<0>(g, S, C, k, j);
    v[1] = pull_g_bc_one<1>(g, S, C, k, j);
    v[2] = pull_g_bc_one<2>(g, S, C, k, j);
    v[3] = pull_g_bc_one<3>(g, S, C, k, j);
    v[4] = pull_g_bc_one<4>(g, S, C, k, j);
    v[5] = pull_g_bc_one<5>(g, S, C, k, j);
    v[6] = pull_g_bc_one<6>(g, S, C, k, j);
    v[7] = pull_g_bc_one<7>(g, S, C, k, j);
    v[8] = pull_g_bc_one<8>(g, S, C, k, j);
}

// ---- interior tiles: every source is the plain neighbour.  Byte offsets:
// node n's own offset plus a per-link constant (uniform), as in tile_step.
struct HalfPitch {
    uint32_t plane;   // bytes between FP16 planes
    uint32_t row;     // bytes between FP16 rows
};

template <int I>
__device__ __forceinline__ uint32_t half_link(const HalfPitch &p)
{
    return (uint32_t)I * p.plane - (uint32_t)(link_r(I) * (int)p.row) - (uint32_t)(link_z(I) * 2);
}

// f plane p (1..8) at fin + (p - 1) * plane: the offset n*2 + half_link<I> - plane
template <int I>
__device__ __forceinline__ half_t raw_in_one(const HalfState &S, const HalfPitch &hp, uint32_t own2)
{
    return ld_at<half_t>(S.fin, own2 + half_link<I>(hp) - hp.plane);
}

__device__ __forceinline__ void raw_in(const HalfState &S, const HalfPitch &hp, uint32_t own2, RawF &rf)
{
    rf.f0 = ld_at<float>(S.f0in, own2 * 2u);
    rf.h[0] = raw_in_one<1>(S, hp, own2);
    rf.h[1] = raw_in_one<2>(S, hp, own2);
    rf.h[2] = raw_in_one<3>(S, hp, own2);
    rf.h[3] = raw_in_one<4>(S, hp, own2);
    rf.h[4] = raw_in_one<5>(S, hp, own2);
    rf.h[5] = raw_in_one<6>(S, hp, own2);
    rf.h[6] = raw_in_one<7>(S, hp, own2);
    rf.h[7] = raw_in_one<8>(S, hp, own2);
}

template <int I, int TZ>
__device__ __forceinline__ float decode_in_one(const Codec &C, half_t h, float (*win)[TZ + 6], int wz, int wr, int j)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    const int js = j - CR;
    const float rs = (float)js + 0.5f;
    return decode_f(h, win[wr - CR][wz - CZ], bulk_factor<I>(rs), rs, js, C);
}

// (wz, wr): the node's own window position, j its row
template <int TZ>
__device__ __forceinline__ void decode_in(const Codec &C, const RawF &rf, float (*win)[TZ + 6], int wz, int wr, int j,
                                          float v[9])
{
    v[0] = rf.f0;
    v[1] = decode_in_one<1, TZ>(C, rf.h[0], win, wz, wr, j);
    v[2] = decode_in_one<2, TZ>(C, rf.h[1], win, wz, wr, j);
    v[3] = decode_in_one<3, TZ>(C, rf.h[2], win, wz, wr, j);
    v[4] = decode_in_one<4, TZ>(C, rf.h[3], win, wz, wr, j);
    v[5] = decode_in_one<5, TZ>(C, rf.h[4], win, wz, wr, j);
    v[6] = decode_in_one<6, TZ>(C, rf.h[5], win, wz, wr, j);
    v[7] = decode_in_one<7, TZ>(C, rf.h[6], win, wz, wr, j);
    v[8] = decode_in_one<8, TZ>(C, rf.h[7], win, wz, wr, j);
}

template <int I>
__device__ __forceinline__ float pull_g_in_one(const HalfState &S, const HalfPitch &hp, const Codec &C,
                                               uint32_t own2, float r)
{
    return decode_g(ld_nt<half_t>(S.gin, own2 + half_link<I>(hp)), r - (float)link_r(I), C);
}

__device__ __forceinline__ void pull_g_in(const HalfState &S, const HalfPitch &hp, const Codec &C, uint32_t own2,
                                          float r, float v[9])
{
    v[0] = pull_g_in_one<0>(S, hp, C, own2, r);
    v[1] = pull_g_in_one<1>(S, hp, C, own2, r);
    v[2] = pull_g_in_one<2>(S, hp, C, own2, r);
    v[3] = pull_g_in_one<3>(S, hp, C, own2, r);
    v[4] = pull_g_in_one<4>(S, hp, C, own2, r);
    v[5] = pull_g_in_one<5>(S, hp, C, own2, r);
    v[6] = pull_g_in_one<6>(S, hp, C, own2, r);
    v[7] = pull_g_in_one<7>(S, hp, C, own2, r);
    v[8] = pull_g_in_one<8>(S, hp, C, own2, r);
}

// ---- periodic z, rows clear of the axis and the r-wall: every source is the
// plain neighbour except that its column wraps; decoding is the interior one
// (the window holds the wrapped phase fields at the tile's own positions).
// w[d + 1] = column k + d wrapped into [0, nz), k within one period of it.
__device__ __forceinline__ void wrap3(int k, int nz, int w[3])
{
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        int x = k + d;
        w[d + 1] = x < 0 ? x + nz : (x >= nz ? x - nz : x);
    }
}

template <int I>
__device__ __forceinline__ half_t raw_zw_one(const HalfState &S, const Geom &g, int j, const int w[3])
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    return ld_at<half_t>(S.fin, (uint32_t)((I - 1) * g.plane + (j - CR) * g.nz + w[1 - CZ]) * 2u);
}

__device__ __forceinline__ void raw_zw(const HalfState &S, const Geom &g, int k, int j, RawF &rf)
{
    int w[3];
    wrap3(k, g.nz, w);
    rf.f0 = ld_at<float>(S.f0in, (uint32_t)(j * g.nz + w[1]) * 4u);
    rf.h[0] = raw_zw_one<1>(S, g, j, w);
    rf.h[1] = raw_zw_one<2>(S, g, j, w);
    rf.h[2] = raw_zw_one<3>(S, g, j, w);
    rf.h[3] = raw_zw_one<4>(S, g, j, w);
    rf.h[4] = raw_zw_one<5>(S, g, j, w);
    rf.h[5] = raw_zw_one<6>(S, g, j, w);
    rf.h[6] = raw_zw_one<7>(S, g, j, w);
    rf.h[7] = raw_zw_one<8>(S, g, j, w);
}

template <int I>
__device__ __forceinline__ float pull_g_zw_one(const HalfState &S, const Geom &g, const Codec &C, int j,
                                               const int w[3], float r)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    half_t h = ld_nt<half_t>(S.gin, (uint32_t)(I * g.plane + (j - CR) * g.nz + w[1 - CZ]) * 2u);
    return decode_g(h, r - (float)CR, C);
}

__device__ __forceinline__ void pull_g_zw(const HalfState &S, const Geom &g, const Codec &C, int k, int j,
                                          float v[9])
{
    int w[3];
    wrap3(k, g.nz, w);
    const float r = (float)j + 0.5f;
    v[0] = pull_g_zw_one<0>(S, g, C, j, w, r);
    v[1] = pull_g_zw_one<1>(S, g, C, j, w, r);
    v[2] = pull_g_zw_one<2>(S, g, C, j, w, r);
    v[3] = pull_g_zw_one<3>(S, g, C, j, w, r);
    v[4] = pull_g_zw_one<4>(S, g, C, j, w, r);
    v[5] = pull_g_zw_one<5>(S, g, C, j, w, r);
    v[6] = pull_g_zw_one<6>(S, g, C, j, w, r);
    v[7] = pull_g_zw_one<7>(S, g, C, j, w, r);
    v[8] = pull_g_zw_one<8>(S, g, C, j, w, r);
}

// Store of node n (row j): f_1..f_8 encoded against the node's new phase
// field, f_0 so that the decoded populations sum exactly to `mass`.
template <int P>
__device__ __forceinline__ float store_f_one(const HalfState &S, const Codec &C, const HalfPitch &hp, uint32_t own2,
                                             float v, float phi, float r, float ir, int j)
{
    const float fac = bulk_factor<P>(r);
    half_t h = encode_f(v, phi, fac, ir, C);
    st_nt(S.fout, own2 + (uint32_t)(P - 1) * hp.plane, h);
    return decode_f(h, phi, fac, r, j, C);
}

__device__ __forceinline__ void store_node(const HalfState &S, const Codec &C, const HalfPitch &hp, uint32_t own2,
                                           int j, float r, float ir, float mass, float phi, float uz, float ur,
                                           const float fv[9], const float gv[9])
{
    float d1 = store_f_one<1>(S, C, hp, own2, fv[1], phi, r, ir, j);
    float d2 = store_f_one<2>(S, C, hp, own2, fv[2], phi, r, ir, j);
    float d3 = store_f_one<3>(S, C, hp, own2, fv[3], phi, r, ir, j);
    float d4 = store_f_one<4>(S, C, hp, own2, fv[4], phi, r, ir, j);
    float d5 = store_f_one<5>(S, C, hp, own2, fv[5], phi, r, ir, j);
    float d6 = store_f_one<6>(S, C, hp, own2, fv[6], phi, r, ir, j);
    float d7 = store_f_one<7>(S, C, hp, own2, fv[7], phi, r, ir, j);
    float d8 = store_f_one<8>(S, C, hp, own2, fv[8], phi, r, ir, j);
    const uint32_t own4 = own2 * 2u;
    st_nt(S.f0out, own4, mass - (((d1 + d2) + (d3 + d4)) + ((d5 + d6) + (d7 + d8))));
#pragma unroll
    for (int i = 0; i < 9; ++i)
        st_nt(S.gout, own2 + (uint32_t)i * hp.plane, encode_g(gv[i], ir, C));
    st_nt(S.phout, own4, phi);
    st_nt(S.uz, own4, uz);
    st_nt(S.ur, own4, ur);
}

// One step (or, with MOMENTS, the macroscopic prefix written to fld) of the
// TZ x TR tile t of a case in FP16-deviation storage.  Same structure as
// tile_step, plus a first phase that stages the stored phase fields around
// the tile (reach 3: the ring's pulls) in LDS for decoding.
template <int TZ, int TR, int MODE, bool MOMENTS>
__device__ __forceinline__ void tile_step_h(const Geom &g, const Phys<float> &P, const Codec &C, int t,
                                            const HalfState &S, double *__restrict__ fld, float (*tile)[TZ + 4],
                                            float (*win)[TZ + 6])
{
    constexpr int NT = TZ * TR;
    constexpr int NH = (TZ + 4) * (TR + 4) - NT;
    constexpr int NHI = (NH + NT - 1) / NT;
    constexpr int WZ = TZ + 6, WR = TR + 6, NW = WZ * WR;
    constexpr int NWI = (NW + NT - 1) / NT;
    int tz = t % g.tiles_z, tr = t / g.tiles_z;
    int k0 = tz * TZ, j0 = tr * TR;
    static_assert(TZ == 64, "a tile row is one wavefront");
    // the row is wave-uniform: scalar row arithmetic
    int tx = threadIdx.x % TZ, ty = __builtin_amdgcn_readfirstlane(threadIdx.x / TZ);
    int k = k0 + tx, j = j0 + ty;
    // the ring's pulls and the window reach 3 cells beyond the tile: if all of
    // them are inside the grid, no boundary or ghost rule applies (uniform);
    // with periodic z and rows clear of the axis and the r-wall only columns
    // wrap (zwrap: interior decoding, wrapped load addresses)
    const bool rows_in = (j0 >= 3) && (j0 + TR + 3 <= g.nr);
    const bool interior = rows_in && (k0 >= 3) && (k0 + TZ + 3 <= g.nz);
    const bool zwrap = !interior && rows_in && g.zper && (g.nz >= TZ + 6);
    const bool plain = interior || zwrap;
    bool inside = (k < g.nz) && (j < g.nr);
    const HalfPitch hp{(uint32_t)(g.plane * 2), (uint32_t)(g.nz * 2)};

    // stored phase fields around the tile (ghost-mapped outside the grid:
    // wrapped when periodic, else values that no decode reads)
    float wv[NWI];
#pragma unroll
    for (int q = 0; q < NWI; ++q) {
        int w = threadIdx.x + q * NT;
        if (w < NW) {
            int kk = k0 - 3 + w % WZ, jj = j0 - 3 + w / WZ;
            if (!interior) {
                kk = ghost_col(kk, g.nz, g.zper);
                jj = ghost_row(jj, g.nr);
            }
            wv[q] = ld_at<float>(S.phin, (uint32_t)(jj * g.nz + kk) * 4u);
        }
    }

    float gv[9], fv[9];
    float uzp, urp;
    RawF own, ring[NHI];
    int hcz[NHI], hcr[NHI], rk[NHI], rj[NHI];
    const int ko = inside ? k : ghost_col(k, g.nz, g.zper);
    const int jo = inside ? j : ghost_row(j, g.nr);
    const uint32_t own2 = (uint32_t)(jo * g.nz + ko) * 2u;
    if (interior) {
        raw_in(S, hp, own2, own);
        pull_g_in(S, hp, C, own2, (float)jo + 0.5f, gv);
    } else if (zwrap) {
        raw_zw(S, g, k, j, own);
        pull_g_zw(S, g, C, k, j, gv);
    } else {
        raw_bc(g, S, ko, jo, own);
        pull_g_bc(g, S, C, ko, jo, gv);
    }
    uzp = ld_nt<float>(S.uz, own2 * 2u);
    urp = ld_nt<float>(S.ur, own2 * 2u);
#pragma unroll
    for (int q = 0; q < NHI; ++q) {
        int hidx = threadIdx.x + q * NT;
        hcz[q] = -1;
        if (hidx < NH) {
            ring_cell<TZ, TR>(hidx, hcz[q], hcr[q]);
            if (interior) {
                rk[q] = k0 + hcz[q] - 2;
                rj[q] = j0 + hcr[q] - 2;
                raw_in(S, hp, (uint32_t)(rj[q] * g.nz + rk[q]) * 2u, ring[q]);
            } else if (zwrap) {
                rk[q] = k0 + hcz[q] - 2;
                rj[q] = j0 + hcr[q] - 2;
                raw_zw(S, g, rk[q], rj[q], ring[q]);
            } else {
                rk[q] = ghost_col(k0 + hcz[q] - 2, g.nz, g.zper);
                rj[q] = ghost_row(j0 + hcr[q] - 2, g.nr);
                raw_bc(g, S, rk[q], rj[q], ring[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NWI; ++q) {
        int w = threadIdx.x + q * NT;
        if (w < NW) win[w / WZ][w % WZ] = wv[q];
    }
    __syncthreads();
    if (plain)
        decode_in<TZ>(C, own, win, tx + 3, ty + 3, jo, fv);
    else
        decode_bc<TZ, TR>(g, C, own, ko, jo, k0, j0, win, fv);
    tile[ty + 2][tx + 2] = sum9(fv) * inv_radius<float>(jo);
#pragma unroll
    for (int q = 0; q < NHI; ++q)
        if (hcz[q] >= 0) {
            float v[9];
            // waves that hold one ring row decode with a wave-uniform row
            const int hw = (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~(TZ - 1)) + q * NT;
            int jr = rj[q];
            if (hw < 4 * TZ) jr = __builtin_amdgcn_readfirstlane(jr);
            if (plain)
                decode_in<TZ>(C, ring[q], win, hcz[q] + 1, hcr[q] + 1, jr, v);
            else
                decode_bc<TZ, TR>(g, C, ring[q], rk[q], jr, k0, j0, win, v);
            tile[hcr[q]][hcz[q]] = sum9(v) * inv_radius<float>(jr);
        }
    // the stored (previous-step) phase field of the node itself
    const float php = win[ty + 3][tx + 3];
    __syncthreads();
    if (!inside) return;
    Stencil<float> st;
    read_stencil<float, TZ>(tile, tx, ty, st);
    const float r = (float)j + 0.5f, ir = inv_radius<float>(j);
    Macro<float> m;
    macro_state(P, r, ir, st, gv, uzp, urp, m);
    if constexpr (MOMENTS) {
        const int64_t n = (int64_t)j * g.nz + k;
        fld[n] = (double)m.phi;
        fld[g.plane + n] = (double)m.rho;
        fld[2 * g.plane + n] = (double)m.uz;
        fld[3 * g.plane + n] = (double)m.ur;
        fld[4 * g.plane + n] = (double)m.p;
    } else {
        const float mass = sum9(fv);
        collide_node<MODE>(P, r, ir, m, php, uzp, urp, fv, gv);
        store_node(S, C, hp, own2, j, r, ir, mass, m.phi, m.uz, m.ur, fv, gv);
    }
}

} // namespace axi
