// lbm_axi: C-ABI library for one case of the axisymmetric Allen-Cahn MRT
// lattice Boltzmann method on one MI355X (gfx950).  Declarations and the
// contract of every entry point: include/lbm_axi.h.
//
// Device state of one case (caller-owned block, offsets 256-byte aligned):
//   pop[2][2][9][plane]  ping-pong x {f, g} x populations, storage type T
//   aux[3][plane]        previous-step phi, u_z, u_r (T), updated in place
//   fld[5][plane]        double scratch: moments fields / state transfer
//   red[...]             double scratch for the diagnostics reductions
// plane = nr*nz rounded up to 64 elements, plus 64; SoA, z fastest.
//
// One step = one launch of step_kernel: every workgroup owns a 64 x TR tile,
// pulls the f populations of its tile plus a 2-cell ring (the ring's extra
// reads hit L2), forms phi in LDS, and then finishes its own nodes: stencil,
// pressure, velocity, both collisions, store.  No grid-wide synchronisation.

#include "case_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

using namespace axi;

namespace {

constexpr int RED_BLOCKS = 512; // diagnostics partial blocks
constexpr int RED_THREADS = 256;
constexpr int NPART = 12;       // partial sums per block
constexpr double CS = 0.57735026918962576451;   // lattice sound speed 1/sqrt(3)

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

} // namespace

namespace axi {
// Elements between population planes: 256-byte aligned, plus PLANE_PAD spare
// elements so that planes and buffers are not a power of two apart (on 16
// cases of 256 x 512 pads of 0..1088 elements measured within 2% of each other).
int64_t plane_elems(int nr, int nz)
{
    return (int64_t)round_up((size_t)nr * nz, 64) + PLANE_PAD;
}
} // namespace axi

namespace {

// ------------------------------------------------------------------ kernels

// t = 0: u = 0, p = 0, g = 0 and the phase-field population at the discrete
// fixed point of a uniform phi: f^eq(phi0, u = 0) of Eq. 11 plus the
// non-equilibrium part h that balances the equilibrium's radial flux M phi.
// With s3..s6 = 1/tau_f and tau_f = 3M + 1/2 (Eq. 18), h_i = -tau_f w_i c_ir phi0,
// so f_i = w_i phi0 (r + 3 M c_ir - tau_f c_ir) = w_i phi0 (r - c_ir / 2).
// Values go into the slots the first step pulls from (the pull map is a bijection).
template <typename T>
__global__ void init_kernel(Geom g, const double *__restrict__ phi0, T *__restrict__ f,
                            T *__restrict__ gp, T *__restrict__ aux)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nn = (int64_t)g.nr * g.nz;
    if (n >= nn) return;
    int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
    double ph = phi0[n];
    double r = (double)j + 0.5;
    double mid = ph * r, up = ph * (r - 0.5), down = ph * (r + 0.5);
    const double w0 = 4.0 / 9.0, w1 = 1.0 / 9.0, w5 = 1.0 / 36.0;
    f[pull_slot<0>(g, k, j)] = (T)(w0 * mid);
    f[pull_slot<1>(g, k, j)] = (T)(w1 * mid);
    f[pull_slot<2>(g, k, j)] = (T)(w1 * up);
    f[pull_slot<3>(g, k, j)] = (T)(w1 * mid);
    f[pull_slot<4>(g, k, j)] = (T)(w1 * down);
    f[pull_slot<5>(g, k, j)] = (T)(w5 * up);
    f[pull_slot<6>(g, k, j)] = (T)(w5 * up);
    f[pull_slot<7>(g, k, j)] = (T)(w5 * down);
    f[pull_slot<8>(g, k, j)] = (T)(w5 * down);
    for (int i = 0; i < 9; ++i)
        gp[(int64_t)i * g.plane + n] = (T)0;
    aux[n] = (T)ph;
    aux[g.plane + n] = (T)0;
    aux[2 * g.plane + n] = (T)0;
}

// One time step of every node (see the header comment of this file).
template <typename T, typename R, int TR, int MODE>
__global__ __launch_bounds__(TZ *TR) void step_kernel(Geom g, Phys<R> P, const T *__restrict__ fin,
                                                      const T *__restrict__ gin, T *__restrict__ fout,
                                                      T *__restrict__ gout, T *__restrict__ aux)
{
    __shared__ R tile[TR + 4][TZ + 4];
    int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step<T, R, TZ, TR, MODE>(g, P, t, fin, gin, fout, gout, aux, tile);
}

// Fields at time t (the macroscopic prefix of a step), in double.
template <typename T, typename R, int TR>
__global__ __launch_bounds__(TZ *TR) void moments_kernel(Geom g, Phys<R> P, const T *__restrict__ fin,
                                                         const T *__restrict__ gin,
                                                         const T *__restrict__ aux, double *__restrict__ fld)
{
    __shared__ R tile[TR + 4][TZ + 4];
    int t = xcd_tile(blockIdx.x, gridDim.x);
    int tz = t % g.tiles_z, tr = t / g.tiles_z;
    int k0 = tz * TZ, j0 = tr * TR;
    int tx = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    int k = k0 + tx, j = j0 + ty;
    bool inside = (k < g.nz) && (j < g.nr);
    tile[ty + 2][tx + 2] = phase_at<T, R>(g, fin, ghost_col(k, g.nz, g.zper), ghost_row(j, g.nr));
    fill_halo<T, R, TZ, TR>(g, fin, k0, j0, tile);
    __syncthreads();
    if (!inside) return;
    Stencil<R> st;
    read_stencil<R, TZ>(tile, tx, ty, st);
    R gv[9];
    pull9<T, R>(g, gin, k, j, gv);
    int64_t n = (int64_t)j * g.nz + k;
    R uzp = (R)aux[g.plane + n], urp = (R)aux[2 * g.plane + n];
    R r = (R)j + (R)0.5, ir = inv_radius<R>(j);
    Macro<R> m;
    macro_state(P, r, ir, st, gv, uzp, urp, m);
    fld[n] = (double)m.phi;
    fld[g.plane + n] = (double)m.rho;
    fld[2 * g.plane + n] = (double)m.uz;
    fld[3 * g.plane + n] = (double)m.ur;
    fld[4 * g.plane + n] = (double)m.p;
}

__device__ __forceinline__ int64_t slot_rt(const Geom &g, int i, int k, int j)
{
    switch (i) {
    case 0: return pull_slot<0>(g, k, j);
    case 1: return pull_slot<1>(g, k, j);
    case 2: return pull_slot<2>(g, k, j);
    case 3: return pull_slot<3>(g, k, j);
    case 4: return pull_slot<4>(g, k, j);
    case 5: return pull_slot<5>(g, k, j);
    case 6: return pull_slot<6>(g, k, j);
    case 7: return pull_slot<7>(g, k, j);
    default: return pull_slot<8>(g, k, j);
    }
}

// post-propagation plane i of a population buffer -> double [nr][nz]
template <typename T>
__global__ void gather_plane_kernel(Geom g, int i, const T *__restrict__ buf, double *__restrict__ out)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
    out[n] = (double)buf[slot_rt(g, i, k, j)];
}

// inverse of gather_plane_kernel
template <typename T>
__global__ void scatter_plane_kernel(Geom g, int i, const double *__restrict__ in, T *__restrict__ buf)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
    buf[slot_rt(g, i, k, j)] = (T)in[n];
}

template <typename A, typename B>
__global__ void convert_kernel(int64_t count, const A *__restrict__ in, B *__restrict__ out)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n < count) out[n] = (B)in[n];
}

// ------------------------------------------- FP16-deviation storage kernels

// population i arriving at (k, j) from buffer side B (q: 0 for f, 1 for g)
__device__ void slot_of(const Geom &g, int i, int k, int j, int &p, int &ks, int &js)
{
    switch (i) {
    case 0: pull_source<0>(g, k, j, p, ks, js); break;
    case 1: pull_source<1>(g, k, j, p, ks, js); break;
    case 2: pull_source<2>(g, k, j, p, ks, js); break;
    case 3: pull_source<3>(g, k, j, p, ks, js); break;
    case 4: pull_source<4>(g, k, j, p, ks, js); break;
    case 5: pull_source<5>(g, k, j, p, ks, js); break;
    case 6: pull_source<6>(g, k, j, p, ks, js); break;
    case 7: pull_source<7>(g, k, j, p, ks, js); break;
    default: pull_source<8>(g, k, j, p, ks, js); break;
    }
}

// row of the slot that population i (1..8) arriving at (k, j) comes from
__device__ int row_of(const Geom &g, int i, int k, int j)
{
    switch (i) {
    case 1: return slot_row<1>(g, k, j);
    case 2: return slot_row<2>(g, k, j);
    case 3: return slot_row<3>(g, k, j);
    case 4: return slot_row<4>(g, k, j);
    case 5: return slot_row<5>(g, k, j);
    case 6: return slot_row<6>(g, k, j);
    case 7: return slot_row<7>(g, k, j);
    default: return slot_row<8>(g, k, j);
    }
}

// t = 0 as init_kernel: every f_q (q >= 1) a node pulls is the uniform-field
// value phi0 b_q(r) its slot is referenced to, so every stored deviation is 0;
// f_0 on the row's grid.
__global__ void init_kernel_h(Geom g, Codec C, const double *__restrict__ phi0, HalfBuf B, float *__restrict__ uz,
                              float *__restrict__ ur)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nn = (int64_t)g.nr * g.nz;
    if (n >= nn) return;
    int j = (int)(n / g.nz);
    double ph = phi0[n];
    double r = (double)j + 0.5;
    B.f0[n] = quantize_row((float)(4.0 / 9.0 * (ph * r)), j);
    for (int p = 1; p < 9; ++p)
        B.f[(int64_t)(p - 1) * g.plane + n] = (half_t)0.0f;
    for (int i = 0; i < 9; ++i)
        B.g[(int64_t)i * g.plane + n] = (half_t)0.0f;
    B.phi[n] = (float)ph;
    uz[n] = 0.0f;
    ur[n] = 0.0f;
}

// six waves per SIMD (80 VGPRs) for 64 x 8 and 64 x 16 tiles with the unit-
// rate MRT and SRT forms: three workgroups per CU (the boundary path would
// otherwise take a few more registers); the general forms need more and
// spill under that bound, which costs more than the occupancy
template <int TR, int MODE>
__global__ __launch_bounds__(TZ *TR) __attribute__((amdgpu_waves_per_eu(
    (TR >= 8 && (MODE == COLLIDE_MRT_UNIT || MODE == COLLIDE_SRT)) ? 6 : 1))) void step_kernel_h(Geom g, Phys<float> P, Codec C, HalfState S)
{
    __shared__ float tile[TR + 4][TZ + 4];
    int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step_h<TZ, TR, MODE, false>(g, P, C, t, S, nullptr, tile);
}

template <int TR>
__global__ __launch_bounds__(TZ *TR) void moments_kernel_h(Geom g, Phys<float> P, Codec C, HalfState S,
                                                           double *__restrict__ fld)
{
    __shared__ float tile[TR + 4][TZ + 4];
    int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step_h<TZ, TR, COLLIDE_MRT, true>(g, P, C, t, S, fld, tile);
}

__global__ void gather_plane_h(Geom g, Codec C, HalfBuf B, int i, int q, double *__restrict__ out)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
    int p, ks, js;
    slot_of(g, i, k, j, p, ks, js);
    int64_t s = (int64_t)js * g.nz + ks;
    float rs = (float)js + 0.5f, rd = (float)j + 0.5f;
    float v;
    if (q == 1)
        v = decode_g(B.g[(int64_t)p * g.plane + s], rs, C);
    else if (p == 0)
        v = B.f0[s];
    else {  // referenced to the reader (k, j), population i
        const int jx = row_of(g, i, k, j);
        v = decode_f(B.f[(int64_t)(p - 1) * g.plane + s], B.phi[n], bulk_factor_rt(i, rd), (float)jx + 0.5f, jx, C);
    }
    out[n] = (double)v;
}

// inverse of gather_plane_h (the phase field of side B must be set first)
__global__ void scatter_plane_h(Geom g, Codec C, HalfBuf B, int i, int q, const double *__restrict__ in)
{
    int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)g.nr * g.nz) return;
    int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
    int p, ks, js;
    slot_of(g, i, k, j, p, ks, js);
    int64_t s = (int64_t)js * g.nz + ks;
    float rs = (float)js + 0.5f, rd = (float)j + 0.5f;
    float v = (float)in[n];
    if (q == 1)
        B.g[(int64_t)p * g.plane + s] = encode_g(v, 1.0f / rs, C);
    else if (p == 0)
        B.f0[s] = quantize_row(v, js);
    else
        B.f[(int64_t)(p - 1) * g.plane + s] =
            encode_f(v, B.phi[n], bulk_factor_rt(i, rd), 1.0f / ((float)row_of(g, i, k, j) + 0.5f), C);
}

// sum of the f that node n pulls in FP16-deviation storage (exact in FP32);
// over all nodes it is the sum of every stored value (a pull is a bijection)
__device__ double node_mass_h(const Geom &g, const Codec &C, const HalfBuf &B, int64_t n, int j)
{
    const int k = (int)(n - (int64_t)j * g.nz);
    const float rd = (float)j + 0.5f;
    double s = (double)B.f0[n];
    const float ph = B.phi[n];
    for (int i = 1; i < 9; ++i) {
        int p, ks, js;
        slot_of(g, i, k, j, p, ks, js);
        const int jx = row_of(g, i, k, j);
        s += (double)decode_f(B.f[(int64_t)(p - 1) * g.plane + (int64_t)js * g.nz + ks], ph, bulk_factor_rt(i, rd),
                              (float)jx + 0.5f, jx, C);
    }
    return s;
}

// ----------------------------------------------------------- diagnostics


// block-wide tree reductions (fixed order: deterministic)
__device__ double block_sum(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ double block_max(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}
__device__ double block_min(double v, double *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// pass 1: sums over nodes and over every f slot
template <typename T>
__global__ __launch_bounds__(RED_THREADS) void diag_pass1(Geom g, int gas, const T *__restrict__ f,
                                                          const double *__restrict__ fld,
                                                          double *__restrict__ part, int half, Codec C,
                                                          HalfBuf B)
{
    __shared__ double sh[RED_THREADS];
    int64_t nn = (int64_t)g.nr * g.nz;
    double a[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    a[3] = 0.0;          // max |u|
    a[7] = INFINITY;     // min axis phi
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += stride) {
        int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
        double r = j + 0.5;
        double phi = fld[n], rho = fld[g.plane + n], uz = fld[2 * g.plane + n];
        double ur = fld[3 * g.plane + n], p = fld[4 * g.plane + n];
        double fs = 0.0;
        if (half)
            fs = node_mass_h(g, C, B, n, j);
        else
            for (int i = 0; i < 9; ++i)
                fs += (double)f[(int64_t)i * g.plane + n];
        double psi = gas ? 1.0 - phi : phi;
        a[0] += fs;
        a[1] += r * rho;
        a[2] += r * rho * uz;
        double um = sqrt(uz * uz + ur * ur);
        a[3] = fmax(a[3], um);
        // psi-weighted over the dispersed phase's region psi > 1/100: on a
        // large grid a bulk phase field a little off 0 or 1 would otherwise
        // outweigh the drop; the tanh tail left out is ~W/400 of a cell
        double wt = psi > 0.01 ? r * psi : 0.0;
        a[4] += wt;
        a[5] += wt * k;
        a[6] += wt * uz;
        if (j == 0) a[7] = fmin(a[7], phi);
        bool bad = !(isfinite(phi) && isfinite(uz) && isfinite(ur) && isfinite(p));
        a[8] += bad ? 1.0 : 0.0;
        if (bad) a[3] = INFINITY;
    }
    double out[NPART];
    out[0] = block_sum(a[0], sh);
    out[1] = block_sum(a[1], sh);
    out[2] = block_sum(a[2], sh);
    out[3] = block_max(a[3], sh);
    out[4] = block_sum(a[4], sh);
    out[5] = block_sum(a[5], sh);
    out[6] = block_sum(a[6], sh);
    out[7] = block_min(a[7], sh);
    out[8] = block_sum(a[8], sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 9; ++q)
            part[(int64_t)blockIdx.x * NPART + q] = out[q];
}

__global__ __launch_bounds__(RED_THREADS) void diag_pass2(int nblocks, const double *__restrict__ part,
                                                          DiagDev *__restrict__ d)
{
    __shared__ double sh[RED_THREADS];
    double a[9];
    for (int q = 0; q < 9; ++q) a[q] = (q == 3) ? 0.0 : (q == 7 ? INFINITY : 0.0);
    for (int b = threadIdx.x; b < nblocks; b += RED_THREADS) {
        const double *p = part + (int64_t)b * NPART;
        a[0] += p[0]; a[1] += p[1]; a[2] += p[2]; a[3] = fmax(a[3], p[3]);
        a[4] += p[4]; a[5] += p[5]; a[6] += p[6]; a[7] = fmin(a[7], p[7]); a[8] += p[8];
    }
    double s0 = block_sum(a[0], sh), s1 = block_sum(a[1], sh), s2 = block_sum(a[2], sh);
    double mx = block_max(a[3], sh), s4 = block_sum(a[4], sh), s5 = block_sum(a[5], sh);
    double s6 = block_sum(a[6], sh), mn = block_min(a[7], sh), s8 = block_sum(a[8], sh);
    if (threadIdx.x == 0) {
        d->phase_mass = s0; d->fluid_mass = s1; d->mom_z = s2; d->umax = mx;
        d->spsi = s4;
        d->centroid_z = s4 > 0 ? s5 / s4 : 0.0;
        d->rise_u = s4 > 0 ? s6 / s4 : 0.0;
        d->R_eq = s4 > 0 ? cbrt(1.5 * s4) : 0.0;
        d->min_axis_phi = mn; d->nonfinite = s8;
    }
}

// pass 3: pressure inside and outside the dispersed phase
__global__ __launch_bounds__(RED_THREADS) void diag_pass3(Geom g, double W, const double *__restrict__ fld,
                                                          const DiagDev *__restrict__ d,
                                                          double *__restrict__ part)
{
    __shared__ double sh[RED_THREADS];
    int64_t nn = (int64_t)g.nr * g.nz;
    double zc = d->centroid_z, Rq = d->R_eq;
    double si = 0, ci = 0, so = 0, co = 0;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += stride) {
        int j = (int)(n / g.nz), k = (int)(n - (int64_t)j * g.nz);
        double dz = k - zc, r = j + 0.5;
        double dist = sqrt(dz * dz + r * r);
        double p = fld[4 * g.plane + n];
        if (dist < Rq - 2.0 * W) {
            si += p; ci += 1.0;
        } else if (dist > Rq + 2.0 * W) {
            bool near_wall = (j > g.nr - 4) || (!g.zper && (k < 3 || k > g.nz - 4));
            if (!near_wall) { so += p; co += 1.0; }
        }
    }
    double a = block_sum(si, sh), b = block_sum(ci, sh), c = block_sum(so, sh), e = block_sum(co, sh);
    if (threadIdx.x == 0) {
        double *p = part + (int64_t)blockIdx.x * NPART;
        p[0] = a; p[1] = b; p[2] = c; p[3] = e;
    }
}

__device__ double psi_at(const Geom &g, int gas, const double *fld, int j, int k)
{
    double phi = fld[(int64_t)j * g.nz + k];
    return gas ? 1.0 - phi : phi;
}

__global__ __launch_bounds__(RED_THREADS) void diag_pass4(Geom g, int gas, int nblocks,
                                                          const double *__restrict__ part,
                                                          const double *__restrict__ fld, DiagDev *__restrict__ d)
{
    __shared__ double sh[RED_THREADS];
    double a = 0, b = 0, c = 0, e = 0;
    for (int q = threadIdx.x; q < nblocks; q += RED_THREADS) {
        const double *p = part + (int64_t)q * NPART;
        a += p[0]; b += p[1]; c += p[2]; e += p[3];
    }
    a = block_sum(a, sh); b = block_sum(b, sh); c = block_sum(c, sh); e = block_sum(e, sh);
    if (threadIdx.x != 0) return;
    d->p_in = b > 0 ? a / b : 0.0;
    d->p_out = e > 0 ? c / e : 0.0;
    d->dp = d->p_in - d->p_out;
    // semi-axes: psi = 1/2 crossings around the centroid column
    int kc = (int)floor(d->centroid_z + 0.5);
    kc = kc < 0 ? 0 : (kc >= g.nz ? g.nz - 1 : kc);
    d->semi_z = 0.0;
    d->semi_r = 0.0;
    if (psi_at(g, gas, fld, 0, kc) > 0.5) {
        double zlo = kc, zhi = kc;
        int pos = kc, idx = kc;
        for (int s = 0; s < g.nz; ++s) {
            int mp = pos - 1, mi = mp;
            if (g.zper) mi = (mp % g.nz + g.nz) % g.nz;
            else if (mp < 0) { zlo = pos - 0.5; break; }
            double va = psi_at(g, gas, fld, 0, mi), vb = psi_at(g, gas, fld, 0, idx);
            if (va <= 0.5) { zlo = mp + (0.5 - va) / (vb - va); break; }
            pos = mp; idx = mi; zlo = pos;
        }
        pos = kc; idx = kc;
        for (int s = 0; s < g.nz; ++s) {
            int pp = pos + 1, pi = pp;
            if (g.zper) pi = pp % g.nz;
            else if (pp >= g.nz) { zhi = pos + 0.5; break; }
            double va = psi_at(g, gas, fld, 0, idx), vb = psi_at(g, gas, fld, 0, pi);
            if (vb <= 0.5) { zhi = pos + (va - 0.5) / (va - vb); break; }
            pos = pp; idx = pi; zhi = pos;
        }
        d->semi_z = 0.5 * (zhi - zlo);
        double rc = g.nr;
        for (int j = 0; j + 1 < g.nr; ++j) {
            double va = psi_at(g, gas, fld, j, kc), vb = psi_at(g, gas, fld, j + 1, kc);
            if (vb <= 0.5) { rc = j + 0.5 + (va - 0.5) / (va - vb); break; }
        }
        d->semi_r = rc;
    }
}

} // namespace

// ------------------------------------------------------------------- host



namespace {

struct Layout {
    int64_t plane;
    size_t esize, fbytes, gbytes, off_pop, off_aux, off_fld, off_part, off_diag, total;
};

bool finite(double x) { return std::isfinite(x); }

int validate(const lbm_axi_params *p)
{
    if (!p) return LBM_AXI_EINVAL;
    if (p->nr < 4 || p->nz < 4) return LBM_AXI_EINVAL;
    // the 9 population planes of a buffer stay below 2^32 bytes (32-bit offsets)
    if ((int64_t)p->nr * p->nz > ((int64_t)1 << 25)) return LBM_AXI_EINVAL;
    if (p->z_periodic != 0 && p->z_periodic != 1) return LBM_AXI_EINVAL;
    if (p->precision != LBM_AXI_FP64 && p->precision != LBM_AXI_FP32 && p->precision != LBM_AXI_FP16D)
        return LBM_AXI_EINVAL;
    if (p->dispersed_gas != 0 && p->dispersed_gas != 1) return LBM_AXI_EINVAL;
    if (p->collision != LBM_AXI_MRT && p->collision != LBM_AXI_SRT && p->collision != LBM_AXI_NMRT)
        return LBM_AXI_EINVAL;
    const double vals[] = {p->W, p->mobility, p->sigma, p->rho_l, p->rho_g, p->nu_l, p->nu_g, p->g_z};
    for (double v : vals)
        if (!finite(v)) return LBM_AXI_EINVAL;
    if (!(p->W > 0) || !(p->mobility > 0) || p->sigma < 0) return LBM_AXI_EINVAL;
    if (!(p->rho_l > 0) || !(p->rho_g > 0) || !(p->nu_l > 0) || !(p->nu_g > 0)) return LBM_AXI_EINVAL;
    for (int a = 0; a < 9; ++a) {
        bool fd = (a >= 3 && a <= 6), gd = (a == 1 || a == 7 || a == 8);
        if (!fd && !(finite(p->s_f[a]) && p->s_f[a] >= 0 && p->s_f[a] < 2)) return LBM_AXI_EINVAL;
        if (!gd && !(finite(p->s_g[a]) && p->s_g[a] >= 0 && p->s_g[a] < 2)) return LBM_AXI_EINVAL;
    }
    if (!(p->s_g[2] > 0)) return LBM_AXI_EINVAL;  // s_p of Eq. 33 divides by s_2^g
    return LBM_AXI_OK;
}

Layout layout_of(const lbm_axi_params *p)
{
    Layout L;
    L.plane = plane_elems(p->nr, p->nz);
    const size_t pl = (size_t)L.plane;
    size_t aux_bytes;
    if (p->precision == LBM_AXI_FP16D) {
        // f: the FP32 f_0 plane, then 8 FP16 planes; g: 9 FP16 planes;
        // aux: phase field (two sides), u_z, u_r in FP32
        L.esize = 2;
        L.fbytes = round_up(pl * 4 + 8 * pl * 2, 256);
        L.gbytes = round_up(9 * pl * 2, 256);
        aux_bytes = 4 * pl * 4;
    } else {
        L.esize = p->precision == LBM_AXI_FP64 ? 8 : 4;
        L.fbytes = L.gbytes = 9 * pl * L.esize;
        aux_bytes = 3 * pl * L.esize;
    }
    L.off_pop = 0;
    L.off_aux = round_up(L.off_pop + 2 * (L.fbytes + L.gbytes), 256);
    L.off_fld = round_up(L.off_aux + aux_bytes, 256);
    L.off_part = round_up(L.off_fld + 5 * (size_t)L.plane * 8, 256);
    L.off_diag = round_up(L.off_part + (size_t)RED_BLOCKS * NPART * 8, 256);
    L.total = round_up(L.off_diag + sizeof(DiagDev), 256);
    return L;
}

template <typename R>
Phys<R> make_phys(const lbm_axi_params *p)
{
    Phys<R> P;
    P.rho_l = (R)p->rho_l;
    P.rho_g = (R)p->rho_g;
    P.drho = (R)(p->rho_l - p->rho_g);
    P.nu_g = (R)p->nu_g;
    P.dnu = (R)(p->nu_l - p->nu_g);
    P.mob = (R)p->mobility;
    P.lam4W = (R)(4.0 / p->W);
    P.beta4 = (R)(4.0 * 12.0 * p->sigma / p->W);
    P.kap = (R)(1.5 * p->sigma * p->W);
    P.g_z = (R)p->g_z;
    double s_tau_f = 1.0 / (3.0 * p->mobility + 0.5);        // Eq. 18
    for (int a = 0; a < 9; ++a) {
        P.sf[a] = (R)((a >= 3 && a <= 6) ? s_tau_f : p->s_f[a]);
        P.sg[a] = (R)p->s_g[a];
    }
    P.sg2 = (R)p->s_g[2];
    P.isg2 = (R)(1.0 / p->s_g[2]);
    bool unit = true;
    for (int a = 0; a < 9; ++a) {
        if (!(a >= 3 && a <= 6) && p->s_f[a] != 1.0) unit = false;
        if (!(a == 1 || a == 7 || a == 8) && p->s_g[a] != 1.0) unit = false;
    }
    P.srt = p->collision == LBM_AXI_SRT;
    if (P.srt)
        for (int a = 0; a < 9; ++a)
            P.sf[a] = (R)s_tau_f;
    P.nmrt = p->collision == LBM_AXI_NMRT;
    P.unit_rates = (unit && p->collision == LBM_AXI_MRT) ? 1 : 0;
    P.mode = P.srt ? COLLIDE_SRT : (P.nmrt ? COLLIDE_NMRT : (P.unit_rates ? COLLIDE_MRT_UNIT : COLLIDE_MRT));
    return P;
}

// FP16 scales (powers of two).  f: deviations of f/r from the bulk form stay
// well below 0.1, stored times 2^10.  g: g/r is of the order of the pressure,
// whose scale is the capillary pressure 4 sigma / W at the smallest resolved
// radius or the hydrostatic range rho_l g_z L; it is stored times 2^4 / that
// scale, which leaves 12 binades above it and 18 normal binades below it.
Codec make_codec(const lbm_axi_params *p)
{
    double gref = std::max(4.0 * p->sigma / p->W,
                           std::max(p->rho_l * std::fabs(p->g_z) * (double)std::max(p->nr, p->nz), 1e-6 * p->rho_l));
    int eg = 4 - (int)std::ceil(std::log2(gref));
    Codec C;
    C.sf = std::ldexp(1.0f, 10);
    C.isf = std::ldexp(1.0f, -10);
    C.sg = std::ldexp(1.0f, eg);
    C.isg = std::ldexp(1.0f, -eg);
    return C;
}

#define HIP_OK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return LBM_AXI_EDEVICE; \
    } while (0)

int launch_ok() { return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EDEVICE; }

template <typename T, typename R, int TR>
void launch_step(lbm_axi_case *c, const Phys<R> &P)
{
    const T *fin = (const T *)c->pop[c->cur][0];
    const T *gin = (const T *)c->pop[c->cur][1];
    T *fout = (T *)c->pop[c->cur ^ 1][0];
    T *gout = (T *)c->pop[c->cur ^ 1][1];
    if (P.mode == COLLIDE_MRT_UNIT)
        step_kernel<T, R, TR, COLLIDE_MRT_UNIT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(
            c->geom, P, fin, gin, fout, gout, (T *)c->aux);
    else if (P.mode == COLLIDE_SRT)
        step_kernel<T, R, TR, COLLIDE_SRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(
            c->geom, P, fin, gin, fout, gout, (T *)c->aux);
    else if (P.mode == COLLIDE_NMRT)
        step_kernel<T, R, TR, COLLIDE_NMRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(
            c->geom, P, fin, gin, fout, gout, (T *)c->aux);
    else
        step_kernel<T, R, TR, COLLIDE_MRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(
            c->geom, P, fin, gin, fout, gout, (T *)c->aux);
}

template <typename T, typename R>
void launch_step_tr(lbm_axi_case *c, const Phys<R> &P)
{
    switch (c->tile_r) {
    case 2: launch_step<T, R, 2>(c, P); break;
    case 4: launch_step<T, R, 4>(c, P); break;
    case 16: launch_step<T, R, 16>(c, P); break;
    default: launch_step<T, R, 8>(c, P); break;
    }
}

template <int TR>
void launch_step_h(lbm_axi_case *c)
{
    HalfState S = half_state(c, c->cur);
    if (c->P32.mode == COLLIDE_MRT_UNIT)
        step_kernel_h<TR, COLLIDE_MRT_UNIT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, c->P32, c->codec, S);
    else if (c->P32.mode == COLLIDE_SRT)
        step_kernel_h<TR, COLLIDE_SRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, c->P32, c->codec, S);
    else if (c->P32.mode == COLLIDE_NMRT)
        step_kernel_h<TR, COLLIDE_NMRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, c->P32, c->codec, S);
    else
        step_kernel_h<TR, COLLIDE_MRT><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, c->P32, c->codec, S);
}

void launch_step_h_tr(lbm_axi_case *c)
{
    switch (c->tile_r) {
    case 2: launch_step_h<2>(c); break;
    case 4: launch_step_h<4>(c); break;
    case 16: launch_step_h<16>(c); break;
    default: launch_step_h<8>(c); break;
    }
}

int do_steps(lbm_axi_case *c, int64_t n)
{
    for (int64_t s = 0; s < n; ++s) {
        if (c->prm.precision == LBM_AXI_FP64)
            launch_step_tr<double, double>(c, c->P64);
        else if (c->prm.precision == LBM_AXI_FP16D)
            launch_step_h_tr(c);
        else
            launch_step_tr<float, float>(c, c->P32);
        c->cur ^= 1;
        c->t += 1;
    }
    return launch_ok();
}

constexpr int MOM_TR = 4;

int run_moments(lbm_axi_case *c)
{
    Geom g = geom_for(c, MOM_TR);
    if (c->prm.precision == LBM_AXI_FP64)
        moments_kernel<double, double, MOM_TR><<<g.tiles, TZ * MOM_TR, 0, c->stream>>>(
            g, c->P64, (const double *)c->pop[c->cur][0], (const double *)c->pop[c->cur][1],
            (const double *)c->aux, c->fld);
    else if (c->prm.precision == LBM_AXI_FP16D)
        moments_kernel_h<MOM_TR><<<g.tiles, TZ * MOM_TR, 0, c->stream>>>(g, c->P32, c->codec, half_state(c, c->cur),
                                                                         c->fld);
    else
        moments_kernel<float, float, MOM_TR><<<g.tiles, TZ * MOM_TR, 0, c->stream>>>(
            g, c->P32, (const float *)c->pop[c->cur][0], (const float *)c->pop[c->cur][1],
            (const float *)c->aux, c->fld);
    return launch_ok();
}

int run_diag(lbm_axi_case *c)
{
    Geom g = c->geom;
    int gas = c->prm.dispersed_gas;
    const int half = c->prm.precision == LBM_AXI_FP16D;
    const HalfBuf B = half ? half_buf(c, c->cur) : HalfBuf{};
    if (c->prm.precision == LBM_AXI_FP64)
        diag_pass1<double><<<RED_BLOCKS, RED_THREADS, 0, c->stream>>>(g, gas, (const double *)c->pop[c->cur][0],
                                                                      c->fld, c->part, 0, c->codec, B);
    else
        diag_pass1<float><<<RED_BLOCKS, RED_THREADS, 0, c->stream>>>(g, gas, (const float *)c->pop[c->cur][0],
                                                                     c->fld, c->part, half, c->codec, B);
    diag_pass2<<<1, RED_THREADS, 0, c->stream>>>(RED_BLOCKS, c->part, c->diag);
    diag_pass3<<<RED_BLOCKS, RED_THREADS, 0, c->stream>>>(g, c->prm.W, c->fld, c->diag, c->part);
    diag_pass4<<<1, RED_THREADS, 0, c->stream>>>(g, gas, RED_BLOCKS, c->part, c->fld, c->diag);
    return launch_ok();
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)((n + threads - 1) / threads); }

} // namespace

namespace axi {
HalfBuf half_buf(const lbm_axi_case *c, int b)
{
    const int64_t pl = c->geom.plane;
    HalfBuf B;
    B.f0 = (float *)c->pop[b][0];
    B.f = (half_t *)((char *)c->pop[b][0] + pl * 4);
    B.g = (half_t *)c->pop[b][1];
    // aux planes: phase field of side 0, u_z, u_r, phase field of side 1
    B.phi = (float *)c->aux + (b ? 3 * pl : 0);
    return B;
}

HalfState half_state(const lbm_axi_case *c, int cur)
{
    HalfBuf in = half_buf(c, cur), out = half_buf(c, cur ^ 1);
    HalfState S;
    S.f0in = in.f0;
    S.fin = in.f;
    S.gin = in.g;
    S.phin = in.phi;
    S.f0out = out.f0;
    S.fout = out.f;
    S.gout = out.g;
    S.phout = out.phi;
    S.uz = (float *)c->aux + c->geom.plane;
    S.ur = (float *)c->aux + 2 * c->geom.plane;
    return S;
}

Geom geom_for(const lbm_axi_case *c, int tile_r)
{
    Geom g;
    g.nr = c->prm.nr;
    g.nz = c->prm.nz;
    g.zper = c->prm.z_periodic;
    g.plane = plane_elems(g.nr, g.nz);
    g.tiles_z = (g.nz + TZ - 1) / TZ;
    g.tiles = g.tiles_z * ((g.nr + tile_r - 1) / tile_r);
    return g;
}
} // namespace axi

namespace {
typedef float copy_vec __attribute__((ext_vector_type(4)));

// one 16-byte element per thread, non-temporal both ways: on this part the
// fastest plain copy measured (against grid-stride loops and unrolled forms)
__global__ __launch_bounds__(256) void device_copy_kernel(const copy_vec *__restrict__ src,
                                                          copy_vec *__restrict__ dst, size_t n)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}
} // namespace

extern "C" {

size_t lbm_axi_state_bytes(const lbm_axi_params *params)
{
    if (validate(params) != LBM_AXI_OK) return 0;
    return layout_of(params).total;
}

int lbm_axi_init(const lbm_axi_params *params, void *dev_state, size_t dev_bytes,
                 const double *phi0_host, void *hip_stream, lbm_axi_case **out)
{
    if (!out) return LBM_AXI_EINVAL;
    *out = nullptr;
    int rc = validate(params);
    if (rc) return rc;
    if (!dev_state || !phi0_host || ((uintptr_t)dev_state & 255)) return LBM_AXI_EINVAL;
    Layout L = layout_of(params);
    if (dev_bytes < L.total) return LBM_AXI_ENOMEM;

    lbm_axi_case *c = new (std::nothrow) lbm_axi_case;
    if (!c) return LBM_AXI_ENOMEM;
    c->prm = *params;
    c->stream = (hipStream_t)hip_stream;
    c->base = (char *)dev_state;
    c->bytes = dev_bytes;
    c->t = 0;
    c->cur = 0;
    c->tile_r = 8;
    c->esize = L.esize;
    for (int b = 0; b < 2; ++b)
        for (int q = 0; q < 2; ++q)
            c->pop[b][q] = c->base + L.off_pop + (size_t)b * (L.fbytes + L.gbytes) + (size_t)q * L.fbytes;
    c->aux = c->base + L.off_aux;
    c->fld = (double *)(c->base + L.off_fld);
    c->part = (double *)(c->base + L.off_part);
    c->diag = (DiagDev *)(c->base + L.off_diag);
    c->P64 = make_phys<double>(params);
    c->P32 = make_phys<float>(params);
    c->codec = make_codec(params);
    c->geom = geom_for(c, c->tile_r);

    int64_t nn = (int64_t)params->nr * params->nz;
    if (hipMemcpyAsync(c->fld, phi0_host, nn * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        delete c;
        return LBM_AXI_EDEVICE;
    }
    if (params->precision == LBM_AXI_FP64)
        init_kernel<double><<<blocks_for(nn, 256), 256, 0, c->stream>>>(
            c->geom, c->fld, (double *)c->pop[0][0], (double *)c->pop[0][1], (double *)c->aux);
    else if (params->precision == LBM_AXI_FP16D)
        init_kernel_h<<<blocks_for(nn, 256), 256, 0, c->stream>>>(c->geom, c->codec, c->fld, half_buf(c, 0),
                                                                   (float *)c->aux + c->geom.plane,
                                                                   (float *)c->aux + 2 * c->geom.plane);
    else
        init_kernel<float><<<blocks_for(nn, 256), 256, 0, c->stream>>>(
            c->geom, c->fld, (float *)c->pop[0][0], (float *)c->pop[0][1], (float *)c->aux);
    if (launch_ok() != LBM_AXI_OK || hipStreamSynchronize(c->stream) != hipSuccess) {
        delete c;
        return LBM_AXI_EDEVICE;
    }
    *out = c;
    return LBM_AXI_OK;
}

int lbm_axi_step(lbm_axi_case *c, int64_t nsteps)
{
    if (!c) return LBM_AXI_ESTATE;
    if (nsteps < 0) return LBM_AXI_EINVAL;
    return do_steps(c, nsteps);
}

int lbm_axi_moments(lbm_axi_case *c, double *phi, double *rho, double *uz, double *ur, double *p,
                    lbm_axi_diag *diag)
{
    if (!c) return LBM_AXI_ESTATE;
    int rc = run_moments(c);
    if (rc) return rc;
    rc = run_diag(c);
    if (rc) return rc;
    int64_t nn = (int64_t)c->prm.nr * c->prm.nz;
    int64_t plane = c->geom.plane;
    double *outs[5] = {phi, rho, uz, ur, p};
    for (int q = 0; q < 5; ++q)
        if (outs[q])
            HIP_OK(hipMemcpyAsync(outs[q], c->fld + q * plane, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    DiagDev d;
    HIP_OK(hipMemcpyAsync(&d, c->diag, sizeof(DiagDev), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (diag) {
        diag->t = c->t;
        diag->phase_mass = d.phase_mass;
        diag->fluid_mass = d.fluid_mass;
        diag->mom_z = d.mom_z;
        diag->umax = d.umax;
        diag->p_in = d.p_in;
        diag->p_out = d.p_out;
        diag->dp = d.dp;
        diag->R_eq = d.R_eq;
        diag->semi_z = d.semi_z;
        diag->semi_r = d.semi_r;
        diag->centroid_z = d.centroid_z;
        diag->rise_u = d.rise_u;
        diag->min_axis_phi = d.min_axis_phi;
        diag->nonfinite = (int64_t)d.nonfinite;
    }
    if (d.nonfinite > 0 || !(d.umax <= CS)) return LBM_AXI_EUNSTABLE;
    return LBM_AXI_OK;
}

int lbm_axi_get_state(lbm_axi_case *c, double *f, double *g, double *aux, int64_t *t)
{
    if (!c) return LBM_AXI_ESTATE;
    Geom G = c->geom;
    int64_t nn = (int64_t)G.nr * G.nz;
    unsigned nb = blocks_for(nn, 256);
    const bool half = c->prm.precision == LBM_AXI_FP16D;
    double *outs[2] = {f, g};
    for (int q = 0; q < 2; ++q) {
        if (!outs[q]) continue;
        for (int i = 0; i < 9; ++i) {
            if (half)
                gather_plane_h<<<nb, 256, 0, c->stream>>>(G, c->codec, half_buf(c, c->cur), i, q, c->fld);
            else if (c->prm.precision == LBM_AXI_FP64)
                gather_plane_kernel<double><<<nb, 256, 0, c->stream>>>(G, i, (const double *)c->pop[c->cur][q], c->fld);
            else
                gather_plane_kernel<float><<<nb, 256, 0, c->stream>>>(G, i, (const float *)c->pop[c->cur][q], c->fld);
            if (launch_ok()) return LBM_AXI_EDEVICE;
            HIP_OK(hipMemcpyAsync(outs[q] + i * nn, c->fld, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
        }
    }
    if (aux) {
        for (int q = 0; q < 3; ++q) {
            if (half)
                convert_kernel<float, double><<<nb, 256, 0, c->stream>>>(
                    nn, q == 0 ? half_buf(c, c->cur).phi : (const float *)c->aux + q * G.plane, c->fld);
            else if (c->prm.precision == LBM_AXI_FP64)
                convert_kernel<double, double><<<nb, 256, 0, c->stream>>>(nn, (const double *)c->aux + q * G.plane, c->fld);
            else
                convert_kernel<float, double><<<nb, 256, 0, c->stream>>>(nn, (const float *)c->aux + q * G.plane, c->fld);
            if (launch_ok()) return LBM_AXI_EDEVICE;
            HIP_OK(hipMemcpyAsync(aux + q * nn, c->fld, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIP_OK(hipStreamSynchronize(c->stream));
        }
    }
    if (t) *t = c->t;
    return LBM_AXI_OK;
}

int lbm_axi_set_state(lbm_axi_case *c, const double *f, const double *g, const double *aux, int64_t t)
{
    if (!c) return LBM_AXI_ESTATE;
    if (!f || !g || !aux || t < 0) return LBM_AXI_EINVAL;
    Geom G = c->geom;
    int64_t nn = (int64_t)G.nr * G.nz;
    unsigned nb = blocks_for(nn, 256);
    const bool half = c->prm.precision == LBM_AXI_FP16D;
    if (half) {
        // the stored phase field first: FP16 f values are encoded against it
        for (int q = 0; q < 3; ++q) {
            HIP_OK(hipMemcpyAsync(c->fld, aux + q * nn, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
            convert_kernel<double, float><<<nb, 256, 0, c->stream>>>(
                nn, c->fld, q == 0 ? half_buf(c, c->cur).phi : (float *)c->aux + q * G.plane);
            if (launch_ok()) return LBM_AXI_EDEVICE;
            HIP_OK(hipStreamSynchronize(c->stream));
        }
    }
    const double *ins[2] = {f, g};
    for (int q = 0; q < 2; ++q)
        for (int i = 0; i < 9; ++i) {
            HIP_OK(hipMemcpyAsync(c->fld, ins[q] + i * nn, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
            if (half)
                scatter_plane_h<<<nb, 256, 0, c->stream>>>(G, c->codec, half_buf(c, c->cur), i, q, c->fld);
            else if (c->prm.precision == LBM_AXI_FP64)
                scatter_plane_kernel<double><<<nb, 256, 0, c->stream>>>(G, i, c->fld, (double *)c->pop[c->cur][q]);
            else
                scatter_plane_kernel<float><<<nb, 256, 0, c->stream>>>(G, i, c->fld, (float *)c->pop[c->cur][q]);
            if (launch_ok()) return LBM_AXI_EDEVICE;
            HIP_OK(hipStreamSynchronize(c->stream));
        }
    for (int q = 0; q < 3 && !half; ++q) {
        HIP_OK(hipMemcpyAsync(c->fld, aux + q * nn, nn * sizeof(double), hipMemcpyHostToDevice, c->stream));
        if (c->prm.precision == LBM_AXI_FP64)
            convert_kernel<double, double><<<nb, 256, 0, c->stream>>>(nn, c->fld, (double *)c->aux + q * G.plane);
        else
            convert_kernel<double, float><<<nb, 256, 0, c->stream>>>(nn, c->fld, (float *)c->aux + q * G.plane);
        if (launch_ok()) return LBM_AXI_EDEVICE;
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    c->t = t;
    return LBM_AXI_OK;
}

int lbm_axi_time(const lbm_axi_case *c, int64_t *t)
{
    if (!c || !t) return c ? LBM_AXI_EINVAL : LBM_AXI_ESTATE;
    *t = c->t;
    return LBM_AXI_OK;
}

int lbm_axi_set_tile(lbm_axi_case *c, int32_t tile_r)
{
    if (!c) return LBM_AXI_ESTATE;
    if (tile_r == 0) tile_r = 8;
    if (tile_r != 2 && tile_r != 4 && tile_r != 8 && tile_r != 16) return LBM_AXI_EINVAL;
    c->tile_r = tile_r;
    c->geom = geom_for(c, tile_r);
    return LBM_AXI_OK;
}

int lbm_axi_destroy(lbm_axi_case *c)
{
    delete c;
    return LBM_AXI_OK;
}

int lbm_axi_device_copy(const void *src, void *dst, size_t bytes, void *hip_stream)
{
    if (bytes == 0)
        return LBM_AXI_OK;
    const size_t n = bytes / 16, blocks = (n + 255) / 256;
    if (!src || !dst || bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16 || blocks > (size_t)INT32_MAX)
        return LBM_AXI_EINVAL;
    const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst;
    if (s0 < d0 + bytes && d0 < s0 + bytes)
        return LBM_AXI_EINVAL;
    device_copy_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)hip_stream>>>((const copy_vec *)src, (copy_vec *)dst, n);
    return hipGetLastError() == hipSuccess ? LBM_AXI_OK : LBM_AXI_EDEVICE;
}

const char *lbm_axi_strerror(int code)
{
    switch (code) {
    case LBM_AXI_OK: return "ok";
    case LBM_AXI_EINVAL: return "invalid argument or parameter";
    case LBM_AXI_ENOMEM: return "device block smaller than lbm_axi_state_bytes()";
    case LBM_AXI_EDEVICE: return "HIP runtime error";
    case LBM_AXI_EUNSTABLE: return "non-finite field or |u| above the lattice sound speed";
    case LBM_AXI_EBUSY: return "no free slot or memory";
    case LBM_AXI_ESTATE: return "invalid handle or slot";
    default: return "unknown error";
    }
}

} // extern "C"
