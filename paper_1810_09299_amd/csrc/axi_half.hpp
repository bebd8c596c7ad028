// FP16-deviation storage of the populations (storage precision 2): the
// device codec and the tile update that uses it.  Arithmetic is FP32.
//
// Stored form of a case:
//   f_0            FP32 plane (the rest population, see "mass" below)
//   f_1..f_8       FP16 planes: the slot that node d reads as population q
//                  holds h = (f_q - phi_d b_q(r_d)) / r_d * sf
//   g_0..g_8       FP16 planes: h = (g_p / r_s) * sg, rounded stochastically
//                  (unbiased) by the step, with random words hashed from the
//                  node and the step's time, so the same in any tile or batch
//   phi            two FP32 planes, read from one and written to the other
//   u_z, u_r       FP32 planes, updated in place
// where d is the node that will read the slot (the neighbour it streams to;
// at the axis the axis-row node the specular rule hands it to; at a wall the
// node that wrote it, which reads it back reversed), q the population it
// arrives as, r_d the reader's radius, phi_d the reader's phase field of the
// step that wrote the slot (the FP32 value the reader stored in that step), s
// the node that stores a g value, and b_q(r) = w_q (r - c_qr / 2) what a node
// at radius r receives along q in a uniform field at rest (the initial
// state's form).  Storing the deviation from that bulk value, divided by r,
// keeps the FP16 numbers small and independent of the radius; sf and sg are
// powers of two.  Referencing the reader means a node decodes everything it
// pulls with its own previous phase field and row; the writer finds the
// reader's new phase field in its phase-field tile (the neighbour's cell,
// whose ghost cell across the axis is the axis-row reader) or, at a wall, has
// it in hand.  The shifted-storage idea follows Lehmann et al., Phys. Rev. E
// 106, 015308 (2022); the r-weighted, reader-referenced form is specific to
// the axisymmetric populations.
//
// A slot's row (for r_d above and the quantum below) is the row of the
// writer's neighbour along the link, ghost-mapped: the reader's row, except
// for a diagonal slot bounced back at a z wall, where it is the neighbouring
// row.
//
// Mass: a decoded f_q (q >= 1) is rounded to a multiple of the quantum
// q(j) = 2^(floor(log2 r_j) - 21) of its slot's row j, and f_0 is stored as
// (sum of the node's pulled populations) - (sum of the decoded values of the
// eight slots it writes).  Every sum of a node's populations then adds
// multiples of the smallest quantum of three neighbouring rows whose
// magnitudes stay below 2^24 such quanta, so FP32 adds them exactly: sum_nodes
// sum_p f is conserved exactly from step to step, not only to rounding.
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

// b_q(r) = w_q (r - c_qr / 2), q >= 1, for the node at radius r that pulls
// population q: the slot's b_p = w_p (r_s + c_pr / 2) in every case (the
// neighbour r_s = r - c_qr with p = q; a wall or the axis, r_s = r with
// c_pr = -c_qr), the same half-integer times the same weight, so the same
// float.  q known at compile time ...
template <int Q>
__device__ __forceinline__ float bulk_factor(float r)
{
    constexpr float w = Q <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f;
    return w * (r - 0.5f * (float)link_r(Q));
}

// ... or only at run time (the same operations, so the same value)
__device__ __forceinline__ float bulk_factor_rt(int q, float r)
{
    const float w = q <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f;
    const int c = (q == 2 || q == 5 || q == 6) ? 1 : ((q == 4 || q == 7 || q == 8) ? -1 : 0);
    return w * (r - 0.5f * (float)c);
}

// 1.5 * 2^23 quanta of row j: a float of that binade has the row's quantum
// as its unit in the last place, so adding it to a value of magnitude below
// 2^22 quanta rounds the value onto the row's grid (to nearest, ties to
// even) and subtracting it again is exact.  Built from the exponent bits alone.
__device__ __forceinline__ float row_bias(int j)
{
    return __int_as_float(((127 + row_log2(j) + 2) << 23) | 0x00400000);
}

// f_q (q >= 1) pulled by a node of row jd (radius rd) with previous phase
// field phid, fac = b_q(rd): phid * fac + h * rd / sf on the row's grid.
// Two fused multiply-adds in the biased binade of row_bias: the first puts
// phid * fac on the grid, the second adds the stored deviation and rounds onto
// the grid again; then the bias comes off exactly.  |f_q| stays far below the
// 2^22 quanta (2^(floor(log2 rd) + 1) > rd) the bias allows.
__device__ __forceinline__ float decode_f(half_t h, float phid, float fac, float rd, int jd, const Codec &C)
{
    const float cb = row_bias(jd);
    return __builtin_fmaf((float)h, rd * C.isf, __builtin_fmaf(phid, fac, cb)) - cb;
}

// ird: an approximation of 1 / rd is enough (the decode reads h as stored)
__device__ __forceinline__ half_t encode_f(float v, float phid, float fac, float ird, const Codec &C)
{
    return (half_t)(__builtin_fmaf(-phid, fac, v) * (C.sf * ird));
}

// (a fused multiply-add with a zero addend: the product rounded once, as a
// multiply, but one mixed-precision instruction with the conversion)
__device__ __forceinline__ float decode_g(half_t h, float rs, const Codec &C)
{
    return __builtin_fmaf((float)h, rs * C.isg, 0.0f);
}

__device__ __forceinline__ half_t encode_g(float v, float ir, const Codec &C) { return (half_t)(v * (C.sg * ir)); }

// encode_g with stochastic rounding, as the step stores g: v_cvt_sr_f16_f32
// rounds away from the truncated value with probability equal to the
// discarded fraction of an FP16 ulp (the threshold is the random word, its
// high bits deciding), so the stored code is unbiased and a g that changes
// by less than half an ulp per step still changes on average
__device__ __forceinline__ half_t encode_g_sr(float v, float ir, const Codec &C, uint32_t rnd)
{
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    const half2_t z = {(half_t)0.0f, (half_t)0.0f};
    return __builtin_amdgcn_cvt_sr_f16_f32(z, v * (C.sg * ir), rnd, false)[0];
}

// The nine random words of the g roundings of node n in the step keyed by
// key = mix32(t): two chained hashes of n and the key and their exclusive
// or; words 3..8 are the same three rotated by 13 and 26 bits, so that each
// rounding decides on its own high bits.  Any two of the nine are
// independent (the third word is independent of either hash alone), which
// is what the variance of a sum of the rounding errors depends on; a third
// hash measured 0.8 % slower.
struct RoundBits {
    uint32_t h[3];
};
__device__ __forceinline__ RoundBits round_bits(uint32_t n, uint32_t key)
{
    RoundBits b;
    b.h[0] = mix32(n ^ key);
    b.h[1] = mix32(b.h[0] ^ 0x9e3779b9u);
    b.h[2] = b.h[0] ^ b.h[1];
    return b;
}
__device__ __forceinline__ uint32_t round_word(const RoundBits &b, int i)
{
    const int rot = 13 * (i / 3);
    const uint32_t h = b.h[i % 3];
    return rot == 0 ? h : ((h >> rot) | (h << (32 - rot)));
}

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

// Whether the slot that node (k, j) writes for population P is bounced back
// at a wall -- a z wall, the r-wall, or a corner that also touches the axis:
// the inverse of the wall rule of pull_source.  Then the node reads it back
// itself; beyond the axis only, the axis-row node (k + c_Pz, 0) reads it.
template <int P>
__device__ __forceinline__ bool slot_walled(const Geom &g, int k, int j)
{
    constexpr int CZ = link_z(P), CR = link_r(P);
    bool wall = false;
    if constexpr (CZ != 0)
        wall = !g.zper && (k + CZ < 0 || k + CZ >= g.nz);
    if constexpr (CR > 0)
        wall = wall || (j + CR >= g.nr);
    return wall;
}

// Pointers of one case in FP16-deviation storage for one step.
struct HalfState {
    const float *f0in;
    const half_t *fin;    // plane p of f at fin + (p - 1) * plane, p = 1..8
    const half_t *gin;    // plane p of g at gin + p * plane
    float *f0out;
    half_t *fout;
    half_t *gout;
    const float *phin;    // phase field of the stored state (the previous step's)
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

// The f values arriving at a node as stored (f_0 and 8 FP16 words) and the
// node's previous phase field, the reference they are decoded against.
struct RawF {
    float f0;
    half_t h[8];
    float ph;
};

// The phase field of a node for the stencil and the macroscopic state (Eq. 16),
// from what it pulls as stored.  In exact arithmetic the decoded populations
// sum to f_0 + (r_d / sf) sum_q h_q + phid sum_q b_q(r_d) (before the row grid),
// and sum_{q >= 1} b_q(r) = 5r / 9: the moving weights sum to 5/9 and their
// c_qr to zero.  Evaluated in that form -- one multiply-add per stored word
// -- it is within a few quanta (a few 1e-7 of phi) of the sum of the decoded
// values; every node and every ring cell of a neighbouring tile forms it the
// same way, so the phase field of a node does not depend on who computes it.
// The exact sums that the mass needs use the decoded values (decode_node).
__device__ __forceinline__ float phi_of(const Codec &C, const RawF &rf, int j)
{
    const float r = (float)j + 0.5f;
    const float a = r * C.isf;
    float acc = rf.ph * (r * (5.0f / 9.0f));
#pragma unroll
    for (int q = 0; q < 8; ++q)
        acc = __builtin_fmaf((float)rf.h[q], a, acc);
    return (acc + rf.f0) * __builtin_amdgcn_rcpf(r);
}

// every arriving f_q of a node of row j with previous phase field ph
__device__ __forceinline__ void decode_node(const Codec &C, const RawF &rf, int j, float v[9])
{
    const float r = (float)j + 0.5f;
    v[0] = rf.f0;
    v[1] = decode_f(rf.h[0], rf.ph, bulk_factor<1>(r), r, j, C);
    v[2] = decode_f(rf.h[1], rf.ph, bulk_factor<2>(r), r, j, C);
    v[3] = decode_f(rf.h[2], rf.ph, bulk_factor<3>(r), r, j, C);
    v[4] = decode_f(rf.h[3], rf.ph, bulk_factor<4>(r), r, j, C);
    v[5] = decode_f(rf.h[4], rf.ph, bulk_factor<5>(r), r, j, C);
    v[6] = decode_f(rf.h[5], rf.ph, bulk_factor<6>(r), r, j, C);
    v[7] = decode_f(rf.h[6], rf.ph, bulk_factor<7>(r), r, j, C);
    v[8] = decode_f(rf.h[7], rf.ph, bulk_factor<8>(r), r, j, C);
}

// ---- tiles that touch the boundary: sources through pull_source

// row of the slot that population I arriving at (k, j) comes from: j, except
// for a diagonal slot bounced back at a z wall (the neighbour's row, mapped)
template <int I>
__device__ __forceinline__ int slot_row(const Geom &g, int k, int j)
{
    constexpr int CZ = link_z(I), CR = link_r(I);
    if constexpr (CZ == 0 || CR == 0) {
        return j;
    } else {
        const bool zwall = !g.zper && (CZ > 0 ? k - CZ < 0 : k - CZ >= g.nz);
        return zwall ? ghost_row(j - CR, g.nr) : j;
    }
}

template <int I>
__device__ __forceinline__ float decode_bc_one(const Geom &g, const Codec &C, half_t h, float ph, int k, int j, float r)
{
    const int jx = slot_row<I>(g, k, j);
    return decode_f(h, ph, bulk_factor<I>(r), (float)jx + 0.5f, jx, C);
}

template <int I>
__device__ __forceinline__ float phi_bc_one(const Geom &g, const Codec &C, half_t h, int k, int j, float acc)
{
    return __builtin_fmaf((float)h, ((float)slot_row<I>(g, k, j) + 0.5f) * C.isf, acc);
}

// phi_of near the boundary: a diagonal slot bounced back at a z wall carries
// its own row's scale (the same float as phi_of wherever every slot row is j)
__device__ __forceinline__ float phi_of_bc(const Geom &g, const Codec &C, const RawF &rf, int k, int j)
{
    const float r = (float)j + 0.5f;
    float acc = rf.ph * (r * (5.0f / 9.0f));
    acc = phi_bc_one<1>(g, C, rf.h[0], k, j, acc);
    acc = phi_bc_one<2>(g, C, rf.h[1], k, j, acc);
    acc = phi_bc_one<3>(g, C, rf.h[2], k, j, acc);
    acc = phi_bc_one<4>(g, C, rf.h[3], k, j, acc);
    acc = phi_bc_one<5>(g, C, rf.h[4], k, j, acc);
    acc = phi_bc_one<6>(g, C, rf.h[5], k, j, acc);
    acc = phi_bc_one<7>(g, C, rf.h[6], k, j, acc);
    acc = phi_bc_one<8>(g, C, rf.h[7], k, j, acc);
    return (acc + rf.f0) * __builtin_amdgcn_rcpf(r);
}

// every arriving f_q of node (k, j) near the boundary
__device__ __forceinline__ void decode_bc(const Geom &g, const Codec &C, const RawF &rf, int k, int j, float v[9])
{
    const float r = (float)j + 0.5f;
    v[0] = rf.f0;
    v[1] = decode_bc_one<1>(g, C, rf.h[0], rf.ph, k, j, r);
    v[2] = decode_bc_one<2>(g, C, rf.h[1], rf.ph, k, j, r);
    v[3] = decode_bc_one<3>(g, C, rf.h[2], rf.ph, k, j, r);
    v[4] = decode_bc_one<4>(g, C, rf.h[3], rf.ph, k, j, r);
    v[5] = decode_bc_one<5>(g, C, rf.h[4], rf.ph, k, j, r);
    v[6] = decode_bc_one<6>(g, C, rf.h[5], rf.ph, k, j, r);
    v[7] = decode_bc_one<7>(g, C, rf.h[6], rf.ph, k, j, r);
    v[8] = decode_bc_one<8>(g, C, rf.h[7], rf.ph, k, j, r);
}
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
    rf.ph = ld_at<float>(S.phin, (uint32_t)(j * g.nz + k) * 4u);
    rf.h[0] = raw_bc_one<1>(g, S, k, j);
    rf.h[1] = raw_bc_one<2>(g, S, k, j);
    rf.h[2] = raw_bc_one<3>(g, S, k, j);
    rf.h[3] = raw_bc_one<4>(g, S, k, j);
    rf.h[4] = raw_bc_one<5>(g, S, k, j);
    rf.h[5] = raw_bc_one<6>(g, S, k, j);
    rf.h[6] = raw_bc_one<7>(g, S, k, j);
    rf.h[7] = raw_bc_one<8>(g, S, k, j);
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

// ---- tiles whose ring and readers are clear of the axis, the r-wall and the
// z walls (every source is the plain neighbour; with periodic z its column
// may wrap).  The FP16 planes are read and written as buffers: a link's plane
// and its row and column shift are one scalar offset, the node's byte offset
// the vector offset, and the memory instruction adds them, so no access
// costs a vector add.  The column shift of a link lives in the vector offset
// only where the column wraps (ColOff).
struct HalfRsrc {
    __amdgpu_buffer_rsrc_t fin, gin, fout, gout;
    int plane, row;   // bytes between FP16 planes, between FP16 rows
};

// the f input base sits F_SHIFT bytes below the planes, so that every link's
// scalar offset is non-negative (only population 1, from column k - 1 of
// plane 0, reaches below its plane)
constexpr int F_SHIFT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, int below)
{
    // raw buffer (stride 0) of the largest record count: offsets as with a
    // plain pointer; fourth word as the gfx9 family takes it
    return __builtin_amdgcn_make_buffer_rsrc((void *)((const char *)base - below), 0, 0x7fffffff, 0x00020000);
}

__device__ __forceinline__ HalfRsrc half_rsrc(const HalfState &S, const Geom &g)
{
    return HalfRsrc{plane_rsrc(S.fin, F_SHIFT), plane_rsrc(S.gin, 0), plane_rsrc(S.fout, 0),
                    plane_rsrc(S.gout, 0), (int)(g.plane * 2), g.nz * 2};
}

// scalar offset of the source of population I: plane, row and column shift
template <int I>
__device__ __forceinline__ int link_soff(const HalfRsrc &R, int plane_index, int below)
{
    return plane_index * R.plane - link_r(I) * R.row - link_z(I) * 2 + below;
}

__device__ __forceinline__ half_t as_half(unsigned short b) { return __builtin_bit_cast(half_t, b); }
__device__ __forceinline__ unsigned short half_bits(half_t h) { return __builtin_bit_cast(unsigned short, h); }

template <int I>
__device__ __forceinline__ half_t raw_plain_one(const HalfRsrc &R, const ColOff &co)
{
    return as_half(__builtin_amdgcn_raw_buffer_load_b16(R.fin, (int)link_voff<I>(co), link_soff<I>(R, I - 1, F_SHIFT), 0));
}

// a node's f0, previous phi (FP32 planes) and the eight FP16 words it pulls
__device__ __forceinline__ void raw_plain(const HalfRsrc &R, const HalfState &S, const ColOff &co, RawF &rf)
{
    rf.f0 = ld_at<float>(S.f0in, co.o * 2u);
    rf.ph = ld_at<float>(S.phin, co.o * 2u);
    rf.h[0] = raw_plain_one<1>(R, co);
    rf.h[1] = raw_plain_one<2>(R, co);
    rf.h[2] = raw_plain_one<3>(R, co);
    rf.h[3] = raw_plain_one<4>(R, co);
    rf.h[4] = raw_plain_one<5>(R, co);
    rf.h[5] = raw_plain_one<6>(R, co);
    rf.h[6] = raw_plain_one<7>(R, co);
    rf.h[7] = raw_plain_one<8>(R, co);
}

// g pulls: read once, so non-temporal (cache policy bit nt)
template <int I>
__device__ __forceinline__ float pull_g_plain_one(const HalfRsrc &R, const Codec &C, const ColOff &co, float r)
{
    const half_t h = as_half(__builtin_amdgcn_raw_buffer_load_b16(R.gin, (int)link_voff<I>(co), link_soff<I>(R, I, 0), 2));
    return decode_g(h, r - (float)link_r(I), C);
}

__device__ __forceinline__ void pull_g_plain(const HalfRsrc &R, const Codec &C, const ColOff &co, float r, float v[9])
{
    v[0] = pull_g_plain_one<0>(R, C, co, r);
    v[1] = pull_g_plain_one<1>(R, C, co, r);
    v[2] = pull_g_plain_one<2>(R, C, co, r);
    v[3] = pull_g_plain_one<3>(R, C, co, r);
    v[4] = pull_g_plain_one<4>(R, C, co, r);
    v[5] = pull_g_plain_one<5>(R, C, co, r);
    v[6] = pull_g_plain_one<6>(R, C, co, r);
    v[7] = pull_g_plain_one<7>(R, C, co, r);
    v[8] = pull_g_plain_one<8>(R, C, co, r);
}

// Store of node (tx, ty) of the tile: f_1..f_8 encoded against their
// readers' new phase fields -- the tile cell at the link's offset (ghost cells
// included), or the node itself where the slot is bounced back at a wall --
// and rows (the row of the link's neighbour, ghost-mapped: the reader's row,
// except for a diagonal slot bounced back at a z wall, whose row is that of
// its neighbour), f_0 so that the decoded populations sum exactly to `mass`.
// PLAIN: no slot of the tile meets a wall.  The bulk factor is the reader's
// b_q(r_d) in every case: w_P (r + c_Pr / 2), the same half-integer times the
// same weight.
template <int P, bool PLAIN, int TZ>
__device__ __forceinline__ float store_f_one(const Geom &g, const HalfRsrc &R, const Codec &C, uint32_t own2, float v,
                                             float phi, float r, float (*tile)[TZ + 4], int tx, int ty, int k, int j)
{
    constexpr int CZ = link_z(P), CR = link_r(P);
    constexpr float w = P <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f;
    const float fac = w * (r + 0.5f * (float)CR);
    const int jx = ghost_row(j + CR, g.nr);
    float phx = tile[ty + 2 + CR][tx + 2 + CZ];
    if constexpr (!PLAIN)
        phx = slot_walled<P>(g, k, j) ? phi : phx;
    const float rx = (float)jx + 0.5f;
    half_t h = encode_f(v, phx, fac, __builtin_amdgcn_rcpf(rx), C);
    __builtin_amdgcn_raw_buffer_store_b16(half_bits(h), R.fout, (int)own2, (P - 1) * R.plane, 2);
    return decode_f(h, phx, fac, rx, jx, C);
}

// SR: g rounded stochastically, with the random words of node (k, j) in the
// step keyed by key; else to nearest.
template <bool PLAIN, int TZ, bool SR>
__device__ __forceinline__ void store_node(const Geom &g, const HalfState &S, const HalfRsrc &R, const Codec &C,
                                           uint32_t own2, float (*tile)[TZ + 4], int tx, int ty, int k, int j,
                                           float r, float ir, float mass, float phi, float uz, float ur,
                                           const float fv[9], const float gv[9], uint32_t key)
{
    float d1 = store_f_one<1, PLAIN, TZ>(g, R, C, own2, fv[1], phi, r, tile, tx, ty, k, j);
    float d2 = store_f_one<2, PLAIN, TZ>(g, R, C, own2, fv[2], phi, r, tile, tx, ty, k, j);
    float d3 = store_f_one<3, PLAIN, TZ>(g, R, C, own2, fv[3], phi, r, tile, tx, ty, k, j);
    float d4 = store_f_one<4, PLAIN, TZ>(g, R, C, own2, fv[4], phi, r, tile, tx, ty, k, j);
    float d5 = store_f_one<5, PLAIN, TZ>(g, R, C, own2, fv[5], phi, r, tile, tx, ty, k, j);
    float d6 = store_f_one<6, PLAIN, TZ>(g, R, C, own2, fv[6], phi, r, tile, tx, ty, k, j);
    float d7 = store_f_one<7, PLAIN, TZ>(g, R, C, own2, fv[7], phi, r, tile, tx, ty, k, j);
    float d8 = store_f_one<8, PLAIN, TZ>(g, R, C, own2, fv[8], phi, r, tile, tx, ty, k, j);
    const uint32_t own4 = own2 * 2u;
    st_nt(S.f0out, own4, mass - (((d1 + d2) + (d3 + d4)) + ((d5 + d6) + (d7 + d8))));
    if constexpr (SR) {
        const RoundBits rb = round_bits((uint32_t)(j * g.nz + k), key);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            __builtin_amdgcn_raw_buffer_store_b16(half_bits(encode_g_sr(gv[i], ir, C, round_word(rb, i))), R.gout,
                                                  (int)own2, i * R.plane, 2);
    } else {
        (void)key;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            __builtin_amdgcn_raw_buffer_store_b16(half_bits(encode_g(gv[i], ir, C)), R.gout, (int)own2, i * R.plane,
                                                  2);
    }
    st_nt(S.phout, own4, phi);
    st_nt(S.uz, own4, uz);
    st_nt(S.ur, own4, ur);
}

// One step (or, with MOMENTS, the macroscopic prefix written to F) of the
// TZ x TR tile (tz, tr) of a case in FP16-deviation storage.  Same structure as
// tile_step; each node (of the tile and of the ring) decodes what it pulls
// with its own previous phase field, loaded with its populations.
template <int TZ, int TR, int MODE, bool MOMENTS, bool SR = false>
__device__ __forceinline__ void tile_step_h(const Geom &g, const Phys<float> &P, const Codec &C, int tz, int tr,
                                            const HalfState &S, const Fields &F, float (*tile)[TZ + 4],
                                            NodeMoments *mo = nullptr)
{
    constexpr int NT = TZ * TR;
    constexpr int NH = (TZ + 4) * (TR + 4) - NT;
    constexpr int NHI = (NH + NT - 1) / NT;
    int k0 = tz * TZ, j0 = tr * TR;
    static_assert(TZ == 64, "a tile row is one wavefront");
    // the row is wave-uniform: scalar row arithmetic
    int tx = threadIdx.x % TZ, ty = __builtin_amdgcn_readfirstlane(threadIdx.x / TZ);
    int k = k0 + tx, j = j0 + ty;
    // the ring's pulls and its readers reach 3 cells beyond the tile: if all
    // of them are inside the grid, no boundary or ghost rule applies
    // (uniform); with periodic z and rows clear of the axis and the r-wall
    // only columns wrap (zwrap: wrapped load addresses)
    const bool rows_in = (j0 >= 3) && (j0 + TR + 3 <= g.nr);
    const bool interior = rows_in && (k0 >= 3) && (k0 + TZ + 3 <= g.nz);
    const bool zwrap = !interior && rows_in && g.zper && (g.nz >= TZ + 6);
    const bool plain = interior || zwrap;
    bool inside = (k < g.nz) && (j < g.nr);
    const HalfRsrc R = half_rsrc(S, g);

    float gv[9], fv[9];
    float uzp, urp, php;
    // nodes of the tile outside the grid compute their ghost images (no store);
    // the row stays wave-uniform
    const int ko = inside ? k : ghost_col(k, g.nz, g.zper);
    const int jo = ghost_row(j, g.nr);
    const uint32_t own2 = (uint32_t)(jo * g.nz + ko) * 2u;
    if (plain) {
        // every row of the tile and its ring is inside the grid (jo = j)
        RawF own, ring[NHI];
        int hcz[NHI], hcr[NHI], rj[NHI];
        // one path for interior tiles and for tiles at the periodic z ends:
        // an interior tile's nodes and ring never reach column 0 or nz - 1,
        // so its column offsets stay its own (a second instance of the loads
        // without the wrap measured slower: one more register, larger code)
        const ColOff co = col_off<true>(own2, ko, g, 2u);
        raw_plain(R, S, co, own);
        pull_g_plain(R, C, co, (float)j + 0.5f, gv);
        uzp = ld_nt<float>(S.uz, own2 * 2u);
        urp = ld_nt<float>(S.ur, own2 * 2u);
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int hidx = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (hidx < NH) {
                ring_cell<TZ, TR>(hidx, hcz[q], hcr[q]);
                const int rk = wrap_col<true>(k0 + hcz[q] - 2, g.nz);
                rj[q] = j0 + hcr[q] - 2;
                raw_plain(R, S, col_off<true>((uint32_t)(rj[q] * g.nz + rk) * 2u, rk, g, 2u), ring[q]);
            }
        }
        decode_node(C, own, j, fv);
        tile[ty + 2][tx + 2] = phi_of(C, own, j);
#pragma unroll
        for (int q = 0; q < NHI; ++q)
            if (hcz[q] >= 0) {
                // waves that hold one ring row work with a wave-uniform row
                const int hw = (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~(TZ - 1)) + q * NT;
                int jr = rj[q];
                if (hw < 4 * TZ) jr = __builtin_amdgcn_readfirstlane(jr);
                tile[hcr[q]][hcz[q]] = phi_of(C, ring[q], jr);
            }
        php = own.ph;
    } else {
        // boundary rules; ring cells outside the grid are their ghost images
        RawF own, ring[NHI];
        int hcz[NHI], hcr[NHI], rk[NHI], rj[NHI];
        raw_bc(g, S, ko, jo, own);
        pull_g_bc(g, S, C, ko, jo, gv);
        uzp = ld_nt<float>(S.uz, own2 * 2u);
        urp = ld_nt<float>(S.ur, own2 * 2u);
#pragma unroll
        for (int q = 0; q < NHI; ++q) {
            int hidx = threadIdx.x + q * NT;
            hcz[q] = -1;
            if (hidx < NH) {
                ring_cell<TZ, TR>(hidx, hcz[q], hcr[q]);
                rk[q] = ghost_col(k0 + hcz[q] - 2, g.nz, g.zper);
                rj[q] = ghost_row(j0 + hcr[q] - 2, g.nr);
                raw_bc(g, S, rk[q], rj[q], ring[q]);
            }
        }
        decode_bc(g, C, own, ko, jo, fv);
        tile[ty + 2][tx + 2] = phi_of_bc(g, C, own, ko, jo);
#pragma unroll
        for (int q = 0; q < NHI; ++q)
            if (hcz[q] >= 0)
                tile[hcr[q]][hcz[q]] = phi_of_bc(g, C, ring[q], rk[q], rj[q]);
        php = own.ph;
    }
    __syncthreads();
    if constexpr (MOMENTS) mo->valid = inside;
    if (!inside) return;
    Stencil<float> st;
    read_stencil<float, TZ>(tile, tx, ty, st);
    const float r = (float)j + 0.5f, ir = inv_radius<float>(j);
    Macro<float> m;
    macro_state(P, r, ir, st, gv, uzp, urp, m);
    if constexpr (MOMENTS) {
        const int64_t n = (int64_t)j * g.nz + k;
        F.phi[n] = (double)m.phi;
        F.rho[n] = (double)m.rho;
        F.uz[n] = (double)m.uz;
        F.ur[n] = (double)m.ur;
        F.p[n] = (double)m.p;
        // the decoded values sum exactly in FP32 (the per-row grid)
        *mo = NodeMoments{true, j, k, (double)m.phi, (double)m.rho, (double)m.uz, (double)m.ur, (double)m.p,
                          (double)sum9(fv)};
    } else {
        const float mass = sum9(fv);
        collide_node<MODE>(P, r, ir, m, php, uzp, urp, fv, gv);
        if (plain)
            store_node<true, TZ, SR>(g, S, R, C, own2, tile, tx, ty, k, j, r, ir, mass, m.phi, m.uz, m.ur, fv, gv,
                                     P.round_key);
        else
            store_node<false, TZ, SR>(g, S, R, C, own2, tile, tx, ty, k, j, r, ir, mass, m.phi, m.uz, m.ur, fv, gv,
                                      P.round_key);
    }
}

} // namespace axi
