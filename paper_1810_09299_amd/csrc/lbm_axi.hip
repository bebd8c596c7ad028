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
//   diag                 the diagnostics record (lbm_axi_diag) reduced on the device
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
#include <mutex>
#include <new>

using namespace axi;

namespace {

constexpr int DIAG_THREADS = 256;  // workgroup of the diagnostics passes (4 waves)
constexpr int DIAG_BLOCKS = 512;   // at most this many moments-pass partials
constexpr int PRS_BLOCKS = 256;    // at most this many pressure-pass partials
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
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step<T, R, TZ, TR, MODE>(g, P, t % g.tiles_z, t / g.tiles_z, fin, gin, fout, gout, aux, tile);
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

// six waves per SIMD for 64 x 8 and 64 x 16 tiles, as batch_step_kernel_h
template <int TR, int MODE, bool SR>
__global__ __launch_bounds__(TZ *TR) __attribute__((amdgpu_waves_per_eu(
    TR >= 8 ? 6 : 1))) void step_kernel_h(Geom g, Phys<float> P, Codec C, HalfState S)
{
    __shared__ float tile[TR + 4][TZ + 4];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    tile_step_h<TZ, TR, MODE, false, SR>(g, P, C, t % g.tiles_z, t / g.tiles_z, S, Fields{}, tile);
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
//
// The read-back is three launches, the reductions in double:
//   moments_kernel  the fields at time t (the macroscopic prefix of a step),
//                   and on the way the sums over the nodes: phase mass (the f
//                   each node pulls), fluid mass, momentum, max |u|, the
//                   psi-weighted sums, min axis phi and the non-finite count;
//                   at most DIAG_BLOCKS workgroups stride over the tiles, each
//                   leaving one partial
//   diag_pressure   at most PRS_BLOCKS workgroups; each first reduces the
//                   partial psi sums (in the order diag_final reduces them,
//                   so the same centroid and R_eq), then sums the pressure inside and
//                   outside over its nodes and finds its nearest psi = 1/2
//                   crossings around the centroid column (axis row left and
//                   right, the column upwards)
//   diag_final      one workgroup: the remaining reductions and the record
// Within a wave, values are combined by an xor butterfly of lane shuffles;
// the four waves of a workgroup then meet in LDS behind a single barrier.
// The order of every sum is fixed, so the diagnostics are deterministic.
// (Folding the final reduction into the last workgroup of a pass to finish
// measured slower: the device-scope release it needs writes back each XCD's
// L2, fields included, from every workgroup.)
//
// Scratch of one read-back (doubles): DIAG_BLOCKS x NSUM partials, then
// PRS_BLOCKS x NPRS partials; every read-back writes the partials it reads.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

enum { RED_SUM = 0, RED_MAX = 1, RED_MIN = 2 };

// N values per thread reduced over the workgroup (DIAG_THREADS = 4 waves);
// kinds[q] says how value q combines.  Every thread receives the results.
template <int N>
__device__ __forceinline__ void block_reduce(double (&v)[N], const int (&kinds)[N], double (*sh)[N])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < N; ++q)
        v[q] = kinds[q] == RED_SUM ? wave_sum(v[q]) : (kinds[q] == RED_MAX ? wave_max(v[q]) : wave_min(v[q]));
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < N; ++q) sh[wv][q] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const double a = sh[0][q], b = sh[1][q], c = sh[2][q], d = sh[3][q];
        v[q] = kinds[q] == RED_SUM ? (a + b) + (c + d)
                                   : (kinds[q] == RED_MAX ? fmax(fmax(a, b), fmax(c, d)) : fmin(fmin(a, b), fmin(c, d)));
    }
}

// partial sums of the moments pass, per workgroup
enum { S_MASS, S_FLUID, S_MOMZ, S_UMAX, S_PSI, S_PSIZ, S_PSIU, S_MINAX, S_BAD, NSUM };
constexpr int S_KIND[NSUM] = {RED_SUM, RED_SUM, RED_SUM, RED_MAX, RED_SUM, RED_SUM, RED_SUM, RED_MIN, RED_SUM};
// partials of diag_pressure: pressure sums and counts, and the distances of
// the nearest psi <= 1/2 crossings from the centroid column (see diag_record)
enum { P_IN, P_NIN, P_OUT, P_NOUT, P_LEFT, P_RIGHT, P_UP, NPRS };
constexpr int P_KIND[NPRS] = {RED_SUM, RED_SUM, RED_SUM, RED_SUM, RED_MIN, RED_MIN, RED_MIN};
constexpr double NONE = 2147483647.0;     // no crossing

__device__ __forceinline__ void diag_init(double (&a)[NSUM])
{
#pragma unroll
    for (int q = 0; q < NSUM; ++q) a[q] = 0.0;
    a[S_MINAX] = INFINITY;
}

// one node's share of the first reduction
__device__ __forceinline__ void diag_add(double (&a)[NSUM], int gas, int j, int k, double phi, double rho, double uz,
                                         double ur, double p, double mass)
{
    const double r = j + 0.5;
    const double psi = gas ? 1.0 - phi : phi;
    a[S_MASS] += mass;
    a[S_FLUID] += r * rho;
    a[S_MOMZ] += r * rho * uz;
    a[S_UMAX] = fmax(a[S_UMAX], sqrt(uz * uz + ur * ur));
    // psi-weighted over the dispersed phase's region psi > 1/100: on a large
    // grid a bulk phase field a little off 0 or 1 would otherwise outweigh the
    // drop; the tanh tail left out is ~W/400 of a cell
    const double wt = psi > 0.01 ? r * psi : 0.0;
    a[S_PSI] += wt;
    a[S_PSIZ] += wt * k;
    a[S_PSIU] += wt * uz;
    if (j == 0) a[S_MINAX] = fmin(a[S_MINAX], phi);
    const bool bad = !(isfinite(phi) && isfinite(uz) && isfinite(ur) && isfinite(p));
    a[S_BAD] += bad ? 1.0 : 0.0;
    if (bad) a[S_UMAX] = INFINITY;
}

// workgroups of the moments pass: one per tile, at most DIAG_BLOCKS
inline int moments_blocks(const Geom &g) { return std::min(g.tiles, DIAG_BLOCKS); }

// layout of the read-back scratch
struct DiagScratch {
    double *sums;        // [DIAG_BLOCKS][NSUM]
    double *prs;         // [PRS_BLOCKS][NPRS]
};
constexpr size_t DIAG_SCRATCH_DOUBLES = (size_t)DIAG_BLOCKS * NSUM + (size_t)PRS_BLOCKS * NPRS;

__host__ __device__ inline DiagScratch diag_scratch(double *base)
{
    DiagScratch d;
    d.sums = base;
    d.prs = base + (size_t)DIAG_BLOCKS * NSUM;
    return d;
}

// totals of the first reduction over n partials, in partial order; every
// thread receives them
__device__ __forceinline__ void reduce_sums(int n, const double *__restrict__ part, double (&a)[NSUM],
                                            double (*sh)[NSUM])
{
    diag_init(a);
    for (int b = threadIdx.x; b < n; b += DIAG_THREADS) {
        const double *q = part + (int64_t)b * NSUM;
        a[S_MASS] += q[S_MASS];
        a[S_FLUID] += q[S_FLUID];
        a[S_MOMZ] += q[S_MOMZ];
        a[S_UMAX] = fmax(a[S_UMAX], q[S_UMAX]);
        a[S_PSI] += q[S_PSI];
        a[S_PSIZ] += q[S_PSIZ];
        a[S_PSIU] += q[S_PSIU];
        a[S_MINAX] = fmin(a[S_MINAX], q[S_MINAX]);
        a[S_BAD] += q[S_BAD];
    }
    __syncthreads();                     // sh may still be read by an earlier reduction
    block_reduce<NSUM>(a, S_KIND, sh);
}

// the psi sums of reduce_sums alone: the same partials per lane in the same
// order and the same tree, so the same values
__device__ __forceinline__ void reduce_psi(int n, const double *__restrict__ part, double &spsi, double &spsiz,
                                           double (*sh)[2])
{
    double v[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < n; b += DIAG_THREADS) {
        v[0] += part[(int64_t)b * NSUM + S_PSI];
        v[1] += part[(int64_t)b * NSUM + S_PSIZ];
    }
    const int kinds[2] = {RED_SUM, RED_SUM};
    block_reduce<2>(v, kinds, sh);
    spsi = v[0];
    spsiz = v[1];
}

template <typename T, typename R, int TR>
__global__ __launch_bounds__(TZ *TR) void moments_kernel(Geom g, Phys<R> P, const T *__restrict__ fin,
                                                         const T *__restrict__ gin,
                                                         const T *__restrict__ aux, Fields F, int gas,
                                                         double *__restrict__ scratch)
{
    static_assert(TZ * TR == DIAG_THREADS, "the reductions take four waves");
    __shared__ R tile[TR + 4][TZ + 4];
    __shared__ double sh[4][NSUM];
    double a[NSUM];
    diag_init(a);
    const int tx = threadIdx.x % TZ, ty = threadIdx.x / TZ;
    for (int t = blockIdx.x; t < g.tiles; t += gridDim.x) {
        const int tz = t % g.tiles_z, tr = t / g.tiles_z;
        const int k0 = tz * TZ, j0 = tr * TR;
        const int k = k0 + tx, j = j0 + ty;
        const bool inside = (k < g.nz) && (j < g.nr);
        const int jo = ghost_row(j, g.nr), ko = ghost_col(k, g.nz, g.zper);
        R fv[9], gv[9];
        // every load of the tile before its barrier: one wait on memory (g
        // and aux of a node beyond the grid are read at its ghost cell and
        // not used)
        pull9<T, R>(g, fin, ko, jo, fv);
        pull9<T, R>(g, gin, ko, jo, gv);
        const int64_t n = (int64_t)j * g.nz + k, no = (int64_t)jo * g.nz + ko;
        const R uzp = (R)aux[g.plane + no], urp = (R)aux[2 * g.plane + no];
        tile[ty + 2][tx + 2] = sum9(fv) * inv_radius<R>(jo);
        fill_halo<T, R, TZ, TR>(g, fin, k0, j0, tile);
        __syncthreads();
        if (inside) {
            Stencil<R> st;
            read_stencil<R, TZ>(tile, tx, ty, st);
            R r = (R)j + (R)0.5, ir = inv_radius<R>(j);
            Macro<R> m;
            macro_state(P, r, ir, st, gv, uzp, urp, m);
            F.phi[n] = (double)m.phi;
            F.rho[n] = (double)m.rho;
            F.uz[n] = (double)m.uz;
            F.ur[n] = (double)m.ur;
            F.p[n] = (double)m.p;
            double mass = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) mass += (double)fv[i];
            diag_add(a, gas, j, k, (double)m.phi, (double)m.rho, (double)m.uz, (double)m.ur, (double)m.p, mass);
        }
        __syncthreads();    // the LDS tile is refilled for the next tile
    }
    block_reduce<NSUM>(a, S_KIND, sh);
    if (threadIdx.x < NSUM) diag_scratch(scratch).sums[(int64_t)blockIdx.x * NSUM + threadIdx.x] = a[threadIdx.x];
}

template <int TR>
__global__ __launch_bounds__(TZ *TR) void moments_kernel_h(Geom g, Phys<float> P, Codec C, HalfState S, Fields F,
                                                           int gas, double *__restrict__ scratch)
{
    static_assert(TZ * TR == DIAG_THREADS, "the reductions take four waves");
    __shared__ float tile[TR + 4][TZ + 4];
    __shared__ double sh[4][NSUM];
    double a[NSUM];
    diag_init(a);
    for (int t = blockIdx.x; t < g.tiles; t += gridDim.x) {
        NodeMoments mo;
        tile_step_h<TZ, TR, COLLIDE_MRT, true>(g, P, C, t % g.tiles_z, t / g.tiles_z, S, F, tile, &mo);
        if (mo.valid) diag_add(a, gas, mo.j, mo.k, mo.phi, mo.rho, mo.uz, mo.ur, mo.p, mo.mass);
        __syncthreads();    // the LDS tile is refilled for the next tile
    }
    block_reduce<NSUM>(a, S_KIND, sh);
    if (threadIdx.x < NSUM) diag_scratch(scratch).sums[(int64_t)blockIdx.x * NSUM + threadIdx.x] = a[threadIdx.x];
}

__device__ __forceinline__ double psi_at(const Geom &g, int gas, const double *phi, int j, int k)
{
    const double v = phi[(int64_t)j * g.nz + k];
    return gas ? 1.0 - v : v;
}

__device__ __forceinline__ int wrap_col(int k, int nz) { return k < 0 ? k + nz : (k >= nz ? k - nz : k); }

// the column nearest the centroid
__device__ __forceinline__ int centroid_column(const Geom &g, double zc)
{
    const int kc = (int)floor(zc + 0.5);
    return kc < 0 ? 0 : (kc >= g.nz ? g.nz - 1 : kc);
}

// The diagnostics record from the totals, the reduced pressure partials and
// the phase field (the semi-axes).  The axial semi-axis is half the distance
// between the nearest psi = 1/2 crossings left and right of the centroid
// column kc on the axis row (a wall bounds the walk half a cell beyond the
// last column; with periodic z a walk that finds none ends one period away),
// the radial one the crossing up column kc (nr if none), each linearly
// interpolated between the two nodes around it; both 0 when kc's axis node is
// not in the dispersed phase.
__device__ void diag_record(const Geom &g, int gas, const double *tot, const double (&pp)[NPRS],
                            const double *__restrict__ phi, int64_t t, lbm_axi_diag *__restrict__ out)
{
    const double spsi = tot[S_PSI];
    const double zc = spsi > 0 ? tot[S_PSIZ] / spsi : 0.0;
    lbm_axi_diag d;
    d.t = t;
    d.phase_mass = tot[S_MASS];
    d.fluid_mass = tot[S_FLUID];
    d.mom_z = tot[S_MOMZ];
    d.umax = tot[S_UMAX];
    d.centroid_z = zc;
    d.rise_u = spsi > 0 ? tot[S_PSIU] / spsi : 0.0;
    d.R_eq = spsi > 0 ? cbrt(1.5 * spsi) : 0.0;
    d.min_axis_phi = tot[S_MINAX];
    d.nonfinite = (int64_t)tot[S_BAD];
    d.p_in = pp[P_NIN] > 0 ? pp[P_IN] / pp[P_NIN] : 0.0;
    d.p_out = pp[P_NOUT] > 0 ? pp[P_OUT] / pp[P_NOUT] : 0.0;
    d.dp = d.p_in - d.p_out;
    d.semi_z = 0.0;
    d.semi_r = 0.0;
    const int kc = centroid_column(g, zc);
    if (psi_at(g, gas, phi, 0, kc) > 0.5) {
        double zlo, zhi;
        if (pp[P_LEFT] != NONE) {
            const int mp = kc - (int)pp[P_LEFT];
            const double va = psi_at(g, gas, phi, 0, wrap_col(mp, g.nz));
            const double vb = psi_at(g, gas, phi, 0, wrap_col(mp + 1, g.nz));
            zlo = mp + (0.5 - va) / (vb - va);
        } else {
            zlo = g.zper ? (double)(kc - g.nz) : -0.5;
        }
        if (pp[P_RIGHT] != NONE) {
            const int pk = kc + (int)pp[P_RIGHT];
            const double va = psi_at(g, gas, phi, 0, wrap_col(pk - 1, g.nz));
            const double vb = psi_at(g, gas, phi, 0, wrap_col(pk, g.nz));
            zhi = (pk - 1) + (va - 0.5) / (va - vb);
        } else {
            zhi = g.zper ? (double)(kc + g.nz) : g.nz - 0.5;
        }
        d.semi_z = 0.5 * (zhi - zlo);
        if (pp[P_UP] != NONE) {
            const int jr = (int)pp[P_UP];
            const double va = psi_at(g, gas, phi, jr, kc), vb = psi_at(g, gas, phi, jr + 1, kc);
            d.semi_r = jr + 0.5 + (va - 0.5) / (va - vb);
        } else {
            d.semi_r = g.nr;
        }
    }
    *out = d;
}

// pass 2: pressure inside and outside the dispersed phase, and the crossing
// candidates: on the axis row, a node with psi <= 1/2 at distance m left
// (right) of the centroid column kc, counting around the period with periodic
// z (m = 1..nz), only on its own side with walls; up column kc, a node of row
// j >= 1 with psi <= 1/2 stands for the crossing between rows j - 1 and j.
// nsums: the partials of the moments pass.
__global__ __launch_bounds__(DIAG_THREADS) void diag_pressure(Geom g, int gas, double W, Fields F, int nsums,
                                                               double *__restrict__ scratch)
{
    __shared__ double shs[4][2];
    __shared__ double sh[4][NPRS];
    const DiagScratch D = diag_scratch(scratch);
    double spsi, spsiz;
    reduce_psi(nsums, D.sums, spsi, spsiz, shs);
    const double zc = spsi > 0 ? spsiz / spsi : 0.0, Rq = spsi > 0 ? cbrt(1.5 * spsi) : 0.0;
    const int kc = centroid_column(g, zc);
    const int64_t nn = (int64_t)g.nr * g.nz;
    double a[NPRS] = {0, 0, 0, 0, NONE, NONE, NONE};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn; n += stride) {
        // nr*nz <= 2^25: a 32-bit division
        const int j = (int)n / g.nz, k = (int)n - j * g.nz;
        const double dz = k - zc, r = j + 0.5;
        const double dist = sqrt(dz * dz + r * r);
        const double p = F.p[n];
        if (dist < Rq - 2.0 * W) {
            a[P_IN] += p;
            a[P_NIN] += 1.0;
        } else if (dist > Rq + 2.0 * W) {
            const bool near_wall = (j > g.nr - 4) || (!g.zper && (k < 3 || k > g.nz - 4));
            if (!near_wall) {
                a[P_OUT] += p;
                a[P_NOUT] += 1.0;
            }
        }
        if ((j == 0 || k == kc) && psi_at(g, gas, F.phi, j, k) <= 0.5) {
            if (j == 0) {
                int ml = kc - k, mr = k - kc;
                if (g.zper) {
                    ml = ml <= 0 ? ml + g.nz : ml;
                    mr = mr <= 0 ? mr + g.nz : mr;
                }
                if (ml > 0) a[P_LEFT] = fmin(a[P_LEFT], (double)ml);
                if (mr > 0) a[P_RIGHT] = fmin(a[P_RIGHT], (double)mr);
            }
            if (k == kc && j >= 1) a[P_UP] = fmin(a[P_UP], (double)(j - 1));
        }
    }
    block_reduce<NPRS>(a, P_KIND, sh);
    if (threadIdx.x < NPRS) D.prs[(int64_t)blockIdx.x * NPRS + threadIdx.x] = a[threadIdx.x];
}

// pass 3 (one workgroup): the totals of both passes and the record.  The
// totals of the moments pass reduce exactly as in every workgroup of
// diag_pressure, so the centroid is the one it used.
__global__ __launch_bounds__(DIAG_THREADS) void diag_final(Geom g, int gas, int nsums, int nprs,
                                                            const double *__restrict__ scratch,
                                                            const double *__restrict__ phi, int64_t t,
                                                            lbm_axi_diag *__restrict__ out)
{
    __shared__ double shs[4][NSUM];
    __shared__ double sh[4][NPRS];
    const DiagScratch D = diag_scratch((double *)scratch);
    // the pressure partials are read before the first reduction waits
    double pp[NPRS] = {0, 0, 0, 0, NONE, NONE, NONE};
    for (int b = threadIdx.x; b < nprs; b += DIAG_THREADS) {
        const double *w = D.prs + (int64_t)b * NPRS;
        for (int x = 0; x < NPRS; ++x) pp[x] = P_KIND[x] == RED_SUM ? pp[x] + w[x] : fmin(pp[x], w[x]);
    }
    double tot[NSUM];
    reduce_sums(nsums, D.sums, tot, shs);
    block_reduce<NPRS>(pp, P_KIND, sh);
    if (threadIdx.x == 0) diag_record(g, gas, tot, pp, phi, t, out);
}

// Reduction scratch of lbm_axi_moments_noalloc, one copy per device the
// library runs on (held until the process ends).  Its size does not depend on
// the grid: the read-back's passes stride over the nodes with at most
// DIAG_BLOCKS and PRS_BLOCKS workgroups.  Host code never uses this name as an
// address: it takes the device address once per device (noalloc_scratch).
static __device__ __align__(256) double scratch[DIAG_SCRATCH_DOUBLES];

} // namespace

// ------------------------------------------------------------------- host



namespace {

// device addresses of `scratch`, taken once per device with that device current
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_addr[MAX_DEVICES];

int noalloc_scratch(int dev, double **out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return LBM_AXI_EDEVICE;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_AXI_EDEVICE;
        scratch_addr[dev] = ptr;
    }
    *out = (double *)scratch_addr[dev];
    return LBM_AXI_OK;
}

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
    if (p->free_s1 != 0 && p->free_s1 != 1) return LBM_AXI_EINVAL;
    if (p->fp16_rounding != LBM_AXI_ROUND_NEAREST && p->fp16_rounding != LBM_AXI_ROUND_STOCHASTIC)
        return LBM_AXI_EINVAL;
    if (p->fp16_rounding != LBM_AXI_ROUND_NEAREST && p->precision != LBM_AXI_FP16D) return LBM_AXI_EINVAL;
    if (p->free_s1 && p->collision == LBM_AXI_SRT) return LBM_AXI_EINVAL;
    if (p->free_s1 && !(std::isfinite(p->s_g[1]) && p->s_g[1] > 0 && p->s_g[1] < 2)) return LBM_AXI_EINVAL;
    if (!std::isfinite(p->g_ramp) || p->g_ramp < 0) return LBM_AXI_EINVAL;
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
    L.off_diag = round_up(L.off_part + DIAG_SCRATCH_DOUBLES * 8, 256);
    L.total = round_up(L.off_diag + sizeof(lbm_axi_diag), 256);
    return L;
}

template <typename R>
Phys<R> make_phys(const lbm_axi_params *p)
{
    Phys<R> P;
    P.round_key = 0;
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
    P.free_s1 = p->free_s1;
    P.isg1 = (R)(p->free_s1 ? 1.0 / p->s_g[1] : 0.0);
    P.g_full = p->g_z;
    P.g_ramp = p->g_ramp;
    bool unit = !p->free_s1;
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

template <typename R>
Phys<R> phys_at(const Phys<R> &P, int64_t t);

template <int TR, bool SR>
void launch_step_h(lbm_axi_case *c)
{
    HalfState S = half_state(c, c->cur);
    const Phys<float> P = phys_at(c->P32, c->t);
    if (P.mode == COLLIDE_MRT_UNIT)
        step_kernel_h<TR, COLLIDE_MRT_UNIT, SR><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, P, c->codec, S);
    else if (P.mode == COLLIDE_SRT)
        step_kernel_h<TR, COLLIDE_SRT, SR><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, P, c->codec, S);
    else if (P.mode == COLLIDE_NMRT)
        step_kernel_h<TR, COLLIDE_NMRT, SR><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, P, c->codec, S);
    else
        step_kernel_h<TR, COLLIDE_MRT, SR><<<c->geom.tiles, TZ * TR, 0, c->stream>>>(c->geom, P, c->codec, S);
}

template <bool SR>
void launch_step_h_sr(lbm_axi_case *c)
{
    switch (c->tile_r) {
    case 2: launch_step_h<2, SR>(c); break;
    case 4: launch_step_h<4, SR>(c); break;
    case 16: launch_step_h<16, SR>(c); break;
    default: launch_step_h<8, SR>(c); break;
    }
}

void launch_step_h_tr(lbm_axi_case *c)
{
    if (c->prm.fp16_rounding == LBM_AXI_ROUND_STOCHASTIC)
        launch_step_h_sr<true>(c);
    else
        launch_step_h_sr<false>(c);
}

// the case's rates with the acceleration of the step from time t
template <typename R>
Phys<R> phys_at(const Phys<R> &P, int64_t t)
{
    Phys<R> Q = P;
    Q.g_z = (R)ramp_accel(P.g_full, P.g_ramp, t);
    Q.round_key = mix32((uint32_t)t);
    return Q;
}

int do_steps(lbm_axi_case *c, int64_t n)
{
    for (int64_t s = 0; s < n; ++s) {
        if (c->prm.precision == LBM_AXI_FP64)
            launch_step_tr<double, double>(c, phys_at(c->P64, c->t));
        else if (c->prm.precision == LBM_AXI_FP16D)
            launch_step_h_tr(c);
        else
            launch_step_tr<float, float>(c, phys_at(c->P32, c->t));
        c->cur ^= 1;
        c->t += 1;
    }
    return launch_ok();
}

constexpr int MOM_TR = 4;

// the case's double planes of the moments fields
Fields case_fields(const lbm_axi_case *c)
{
    const int64_t pl = c->geom.plane;
    double *f = c->fld;
    return Fields{f, f + pl, f + 2 * pl, f + 3 * pl, f + 4 * pl};
}

// The read-back of a case: fields into F, the diagnostics record into the
// device record `out`; `scratch` holds the reductions' partials
// (DIAG_SCRATCH_DOUBLES doubles; nothing in it needs to start at zero).
int run_readback(lbm_axi_case *c, const Fields &F, double *scratch, lbm_axi_diag *out)
{
    const Geom g = geom_for(c, MOM_TR);
    const int gas = c->prm.dispersed_gas;
    const int nb = moments_blocks(g);
    // the fields at time t: the prefix of the step from t, with its acceleration
    if (c->prm.precision == LBM_AXI_FP64)
        moments_kernel<double, double, MOM_TR><<<nb, TZ * MOM_TR, 0, c->stream>>>(
            g, phys_at(c->P64, c->t), (const double *)c->pop[c->cur][0], (const double *)c->pop[c->cur][1],
            (const double *)c->aux, F, gas, scratch);
    else if (c->prm.precision == LBM_AXI_FP16D)
        moments_kernel_h<MOM_TR><<<nb, TZ * MOM_TR, 0, c->stream>>>(g, phys_at(c->P32, c->t), c->codec,
                                                                    half_state(c, c->cur), F, gas, scratch);
    else
        moments_kernel<float, float, MOM_TR><<<nb, TZ * MOM_TR, 0, c->stream>>>(
            g, phys_at(c->P32, c->t), (const float *)c->pop[c->cur][0], (const float *)c->pop[c->cur][1],
            (const float *)c->aux, F, gas, scratch);
    const int64_t nn = (int64_t)g.nr * g.nz;
    const int np = (int)std::min<int64_t>(PRS_BLOCKS, (nn + DIAG_THREADS - 1) / DIAG_THREADS);
    diag_pressure<<<np, DIAG_THREADS, 0, c->stream>>>(g, gas, c->prm.W, F, nb, scratch);
    diag_final<<<1, DIAG_THREADS, 0, c->stream>>>(g, gas, nb, np, scratch, F.phi, c->t, out);
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

    // the allocation-free read-back's scratch address on this device, taken
    // here with the device current
    int dev = 0;
    double *scratch_ptr = nullptr;
    if (hipGetDevice(&dev) != hipSuccess || noalloc_scratch(dev, &scratch_ptr) != LBM_AXI_OK) return LBM_AXI_EDEVICE;
    lbm_axi_case *c = new (std::nothrow) lbm_axi_case;
    if (!c) return LBM_AXI_ENOMEM;
    c->device = dev;
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
    c->diag = (lbm_axi_diag *)(c->base + L.off_diag);
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
    const Fields F = case_fields(c);
    int rc = run_readback(c, F, c->part, c->diag);
    if (rc) return rc;
    int64_t nn = (int64_t)c->prm.nr * c->prm.nz;
    double *outs[5] = {phi, rho, uz, ur, p};
    const double *planes[5] = {F.phi, F.rho, F.uz, F.ur, F.p};
    for (int q = 0; q < 5; ++q)
        if (outs[q])
            HIP_OK(hipMemcpyAsync(outs[q], planes[q], nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    lbm_axi_diag d;
    HIP_OK(hipMemcpyAsync(&d, c->diag, sizeof(lbm_axi_diag), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    if (diag) *diag = d;
    if (d.nonfinite > 0 || !(d.umax <= CS)) return LBM_AXI_EUNSTABLE;
    return LBM_AXI_OK;
}

int lbm_axi_moments_noalloc(lbm_axi_case *c, double *phi, double *rho, double *uz, double *ur, double *p,
                            lbm_axi_diag *diag)
{
    if (!c) return LBM_AXI_ESTATE;
    if (!phi || !rho || !uz || !ur || !p || !diag) return LBM_AXI_EINVAL;
    if ((int64_t)c->prm.nr * c->prm.nz > ((int64_t)1 << 25)) return LBM_AXI_EINVAL;
    double *sc = nullptr;
    if (noalloc_scratch(c->device, &sc) != LBM_AXI_OK) return LBM_AXI_EDEVICE;
    return run_readback(c, Fields{phi, rho, uz, ur, p}, sc, diag);
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
