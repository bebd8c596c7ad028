/*
 * lbm_axi: MI355X (gfx950) implementation of one time step of the
 * axisymmetric Allen-Cahn MRT lattice Boltzmann model for two-phase flow with
 * large density ratio (Liang, Li, Chen & Xu, arXiv:1810.09299).
 *
 * One step advances two r-weighted D2Q9 populations on the (r, z) half-plane:
 *   f  the phase-field population (Sec. 2.2, Eqs. 9-23): equilibrium of
 *      Eq. 11 carrying the extra radial flux M*phi, source of Eqs. 14-15 and
 *      22-23, phi = sum f / r (Eq. 16);
 *   g  the hydrodynamic population (Sec. 2.3, Eqs. 24-37): equilibrium of
 *      Eqs. 25-26, forcing distribution of Eqs. 27-30, velocity of Eq. 32 and
 *      pressure of Eq. 33;
 * both collided in moment space (Eqs. 19, 21-22, 36-37) with the transform M
 * of Sec. 2.2, the phase field differentiated by the isotropic stencils of
 * Eqs. 39-40, and propagated (Eq. 20) with the axis and wall conditions of
 * Sec. 2.3.
 *
 * Grid conventions: row j (0 <= j < nr) sits at r = j + 1/2, the first lattice
 * line half a cell from the axis (Sec. 2.3); column k (0 <= k < nz) at z = k.
 * The r-wall lies half-way beyond the last row; with z walls, the z walls lie
 * half-way beyond the first and last columns.  Every host field is [nr][nz]
 * with z fastest; host population arrays are [9][nr][nz] in the population
 * order of Eq. 12 with the paper's x axis along z and y along r.
 *
 * Ownership: the caller owns every buffer.  The device state is one block of
 * at least lbm_axi_state_bytes() bytes in device memory; it must stay alive
 * and untouched until lbm_axi_destroy().  The library owns only the opaque
 * handle.  All device work is ordered on the HIP stream given at init; calls
 * that return host data synchronise that stream.  A handle must not be used
 * from two threads at once.
 *
 * Every function returns LBM_AXI_OK (0) or a negative error code; nothing is
 * printed and nothing aborts.
 */
#ifndef LBM_AXI_H
#define LBM_AXI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_AXI_OK 0
#define LBM_AXI_EINVAL (-1)    /* a parameter or argument is out of range          */
#define LBM_AXI_ENOMEM (-2)    /* the device block is smaller than required         */
#define LBM_AXI_EDEVICE (-3)   /* a HIP call failed                                 */
#define LBM_AXI_EUNSTABLE (-4) /* non-finite values or |u| > c_s found by moments   */
#define LBM_AXI_EBUSY (-5)     /* no free slot or memory (batching)                 */
#define LBM_AXI_ESTATE (-6)    /* bad handle or slot                                */

#define LBM_AXI_FP64 0         /* populations, aux and arithmetic in double          */
#define LBM_AXI_FP32 1         /* populations, aux and arithmetic in float           */
/* FP16-deviation storage, float arithmetic: f_1..f_8 stored as FP16 deviations
 * from the uniform-field form w_i phi (r - c_ir/2) of the node that will read
 * them (its stored FP32 phi of the writing step as the reference, divided by
 * r, scaled by a power of two), g as FP16 g/r scaled by a power of two chosen
 * from the case's pressure scale (4 sigma / W, the hydrostatic range), f_0,
 * phi and u in FP32.  Decoded f values are rounded to a per-row power-of-two
 * grid and f_0 closes each node's sum, so the phase mass sum f is conserved
 * exactly from step to step.  100 bytes move per lattice update (FP32: 168,
 * FP64: 336). */
#define LBM_AXI_FP16D 2

/* How a step rounds the g populations it stores in FP16-deviation storage.
 * NEAREST: to nearest, so a g whose value changes by less than half an FP16
 * ulp (2^-12 of itself) per step keeps its stored value, and hydrodynamics
 * slower than that stall.  STOCHASTIC: up or down with the probabilities
 * that make the stored value unbiased (gfx950 v_cvt_sr_f16_f32), the random
 * words hashed from the node and the case's time t, so a case's results are
 * the same in any tile shape, batch or launch configuration; about 4 % more
 * time per step.  The f populations and the mass closure are the same in
 * both. */
#define LBM_AXI_ROUND_NEAREST 0
#define LBM_AXI_ROUND_STOCHASTIC 1

/* Collision (Sec. 2.2-2.3).  MRT: the moment-space relaxation with the rates
 * s_f, s_g below.  SRT: the special case noted at the end of Sec. 2.2, every
 * rate equal -- 1/tau_f (Eq. 18) for f and 1/tau_g(phi) (Eq. 34) for g,
 * including s_2^g in s_p of Eq. 33; s_f and s_g are then ignored.
 * NMRT: the non-orthogonal extension named in Sec. 4 -- the same relaxation
 * with the raw-moment basis (1, c_z, c_r, c_z^2 + c_r^2, c_z^2 - c_r^2,
 * c_z c_r, c_z^2 c_r, c_z c_r^2, c_z^2 c_r^2) in place of M, equilibria and
 * sources being the population forms of Eqs. 11, 15, 25-26 and 29 in those
 * moments.  s_f and s_g keep the orthogonal order; each raw row takes the rate
 * of the moment it stands for (rows in the order above: s[0], s[3], s[5],
 * s[1], s[7], s[8], s[6], s[4], s[2]).  s_p of Eq. 33 becomes
 * (3 tau_g - 1/s_2^g - 1)/2, the coefficient the Chapman-Enskog step of
 * Appendix C gives for this basis. */
#define LBM_AXI_MRT 0
#define LBM_AXI_SRT 1
#define LBM_AXI_NMRT 2

/* free_s1 = 1 is an extension beyond the paper's method: the energy moment e
 * of g relaxes at s_g[1] as given (0 < s_g[1] < 2), in the collision and in
 * s_p of Eq. 33, instead of the 1/tau_g that Sec. 2.3 ties it to.  The tied
 * rate confines the scheme to tau_g in about (0.65, 1.15) (nu between about
 * 0.05 and 0.22), too narrow for viscosity ratios of 10 or more; the free
 * rate is stable well beyond (tau_g 0.53 to 3.5 tested).  Not with SRT. */
typedef struct {
    int32_t nr, nz;            /* rows (r) and columns (z), each >= 4, nr*nz <= 2^25 */
    int32_t z_periodic;        /* 1: periodic in z; 0: no-slip walls at both z ends  */
    int32_t precision;         /* LBM_AXI_FP64, LBM_AXI_FP32 or LBM_AXI_FP16D        */
    int32_t dispersed_gas;     /* diagnostics only: 0 tracks phi, 1 tracks 1 - phi  */
    int32_t collision;         /* LBM_AXI_MRT, LBM_AXI_SRT or LBM_AXI_NMRT           */
    int32_t free_s1;           /* 0: the paper's s_1^g = 1/tau_g (Eq. 34); 1: an extension, below */
    int32_t fp16_rounding;     /* LBM_AXI_FP16D only: LBM_AXI_ROUND_NEAREST (0) or
                                  LBM_AXI_ROUND_STOCHASTIC (1), below; 0 otherwise   */
    double W;                  /* interface width (Eq. 2), > 0                       */
    double mobility;           /* M of Eq. 1, > 0; sets tau_f by Eq. 18              */
    double sigma;              /* surface tension, >= 0 (k, beta of Eq. 4)           */
    double rho_l, rho_g;       /* bulk densities (Eq. 17), > 0                       */
    double nu_l, nu_g;         /* kinematic viscosities (Eq. 35), > 0; tau_g by Eq. 34 */
    double g_z;                /* axial acceleration: G = ((rho - rho_l) g_z, 0)     */
    double g_ramp;             /* >= 0: g_z is reached linearly over the first g_ramp
                                  steps -- the step from time t uses g_z (t+1)/g_ramp
                                  while t + 1 < g_ramp; 0: from the first step     */
    double s_f[9];             /* f rates (Eq. 13); s_f[3..6] are replaced by 1/tau_f; MRT, NMRT */
    double s_g[9];             /* g rates (Eq. 28); s_g[7,8] (and s_g[1] unless free_s1) are
                                  replaced by 1/tau_g(phi); MRT, NMRT */
} lbm_axi_params;

/* Diagnostics of the fields at time t, reduced in double on the device.
 * psi is the dispersed phase: phi, or 1 - phi when dispersed_gas is set, and
 * sum_D a sum over the nodes with psi > 1/100 (the drop or bubble and its
 * interface; a bulk phase field slightly off 0 or 1 is left out).
 *   phase_mass  sum of all f (= sum r phi), conserved by the method
 *   fluid_mass  sum r rho;  mom_z = sum r rho u_z;  umax = max |u|
 *   centroid_z  sum_D r psi z / sum_D r psi;  rise_u = sum_D r psi u_z / sum_D r psi
 *   R_eq        (1.5 sum_D r psi)^(1/3), the radius of a sphere of that volume
 *   p_in, p_out mean p over nodes closer than R_eq - 2W to (centroid_z, 0), and
 *               over nodes farther than R_eq + 2W at least 3 cells from every
 *               wall;  dp = p_in - p_out
 *   semi_z      half the distance between the psi = 1/2 crossings of the axis
 *               row around the centroid column;  semi_r the psi = 1/2 crossing
 *               up the centroid column (0 if psi <= 1/2 there)
 *   min_axis_phi  min phi along the axis row;  nonfinite  nodes with a
 *               non-finite phi, u or p */
typedef struct {
    int64_t t;
    double phase_mass, fluid_mass, mom_z, umax;
    double p_in, p_out, dp, R_eq, semi_z, semi_r, centroid_z, rise_u, min_axis_phi;
    int64_t nonfinite;
} lbm_axi_diag;

typedef struct lbm_axi_case lbm_axi_case;

/* Bytes of device memory one case needs (0 if the parameters are invalid). */
size_t lbm_axi_state_bytes(const lbm_axi_params *params);

/* Checks the parameters, derives the rates (Eqs. 18, 34) and sets the state to
 * t = 0 (the paper gives no initial populations): u = 0, p = 0, g = 0 (its
 * equilibrium), and f = f^eq(phi0, u = 0) of Eq. 11 plus the non-equilibrium
 * part that makes a uniform phase field an exact fixed point of one step, which
 * works out to f_i = w_i phi0 (r - c_ir / 2).  phi0_host: [nr][nz] doubles,
 * read before return.  dev_state: device pointer, 256-byte aligned, dev_bytes
 * >= lbm_axi_state_bytes().  hip_stream: a hipStream_t (NULL = the null
 * stream).  On success *out receives the handle. */
int lbm_axi_init(const lbm_axi_params *params, void *dev_state, size_t dev_bytes,
                 const double *phi0_host, void *hip_stream, lbm_axi_case **out);

/* Enqueues nsteps >= 0 time steps (Eqs. 9-40, Sec. 2.2-2.3) on the case's
 * stream and returns without waiting.  One kernel launch per step. */
int lbm_axi_step(lbm_axi_case *c, int64_t nsteps);

/* Fields at the current time t (phi of Eq. 16, rho of Eq. 17, u of Eq. 32, p of
 * Eq. 33 -- the first part of the next step, without advancing the state) into
 * caller-owned host arrays [nr][nz] (each may be NULL), and the diagnostics
 * into *diag (may be NULL).  Synchronises the stream.  Returns
 * LBM_AXI_EUNSTABLE, after filling every output, if a field is non-finite or
 * |u| exceeds the lattice sound speed 1/sqrt(3). */
int lbm_axi_moments(lbm_axi_case *c, double *phi, double *rho, double *uz, double *ur,
                    double *p, lbm_axi_diag *diag);

/* For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc: lbm_axi_moments with every
 * output in caller-owned device memory and no host transfer.  phi, rho, uz,
 * ur, p: device arrays of nr*nz doubles ([nr][nz], z fastest); diag: a device
 * lbm_axi_diag.  All required.  Enqueued on the case's stream; returns
 * without waiting and calls no allocating routine.  The reduction partials
 * live in a fixed array of the library in device memory (51 KB per device,
 * held until the process ends), whose size does not depend on the grid:
 * every grid the library accepts (nr*nz <= 2^25) fits, and LBM_AXI_EINVAL is
 * returned beyond.  Each call writes every partial it reads, so nothing has to
 * start at zero; but all calls on one device share that array, so calls that
 * may overlap on one device (other streams, other threads) race -- order them
 * on one stream.  The caller checks diag->nonfinite and diag->umax itself
 * (LBM_AXI_EUNSTABLE needs the record on the host).  LBM_AXI_ESTATE for a NULL
 * case, LBM_AXI_EINVAL for a NULL output, LBM_AXI_EDEVICE if a launch fails. */
int lbm_axi_moments_noalloc(lbm_axi_case *c, double *phi, double *rho, double *uz, double *ur, double *p,
                            lbm_axi_diag *diag);

/* Copies out the state at time t: post-propagation populations f, g
 * ([9][nr][nz] doubles each) and the previous-step (phi, u_z, u_r) that the
 * next step needs for d_t (Eq. 38) and Eq. 33 ([3][nr][nz]).  Any pointer may
 * be NULL.  Synchronises the stream.  Used for checkpoints and checks. */
int lbm_axi_get_state(lbm_axi_case *c, double *f, double *g, double *aux, int64_t *t);

/* Replaces the state by the given one (same layout as lbm_axi_get_state; all
 * three arrays required), rounding to the case's precision.  Synchronises. */
int lbm_axi_set_state(lbm_axi_case *c, const double *f, const double *g, const double *aux,
                      int64_t t);

/* Current time step of the case. */
int lbm_axi_time(const lbm_axi_case *c, int64_t *t);

/* Selects the step kernel's tile (tile_r rows by 64 columns; tile_r in
 * {2, 4, 8, 16}); the results do not depend on it.  0 picks the default. */
int lbm_axi_set_tile(lbm_axi_case *c, int32_t tile_r);

/* Frees the handle (not the caller's device block).  NULL is accepted. */
int lbm_axi_destroy(lbm_axi_case *c);

/* ------------------------------------------------------------------ batches
 * Many independent cases -- any grid sizes, parameters and step counts, one
 * precision -- advanced together: every time step is one kernel launch over
 * all running cases (the same per-node arithmetic as a case run alone, so
 * their populations are bit-identical).  Runs of steps over an unchanged set
 * of running cases are captured once in a hipGraph and replayed.
 *
 * Memory: the caller hands over one device pool (256-byte aligned).  Its
 * first lbm_axi_batch_reserved_bytes() bytes hold the case table, the work
 * list and each case's time (advanced on the device, the key of stochastic
 * g rounding); the rest is split first-fit into per-case blocks of
 * lbm_axi_state_bytes() each, so admission is decided by HBM footprint.  The
 * pool must outlive the batch.  All work is ordered on one stream: the given
 * hipStream_t, or, if NULL, a stream the batch creates and destroys. */
typedef struct lbm_axi_batch lbm_axi_batch;

/* Bytes at the head of the pool used for bookkeeping (0 if invalid). */
size_t lbm_axi_batch_reserved_bytes(int32_t max_cases, int32_t precision);

int lbm_axi_batch_create(void *dev_pool, size_t pool_bytes, int32_t max_cases, int32_t precision,
                         void *hip_stream, lbm_axi_batch **out);

/* Initialises a case as lbm_axi_init does (params->precision must be the
 * batch's) in a free slot and pool block, to run for nsteps steps; *slot
 * receives its index.  The case is initialised on a second stream of the
 * batch, which this call synchronises; steps already enqueued for the running
 * cases go on meanwhile.  The block of a released case is reused only once the
 * work that last touched it has completed: if only such blocks would fit, the
 * call waits for the oldest of them (earlier work only, never the steps
 * enqueued after it).  LBM_AXI_EBUSY when no slot or no block is free, or when
 * the step's work list (at most 2^20 tiles of all running cases together)
 * would overflow; LBM_AXI_ENOMEM when the case is larger than the whole pool
 * after its head. */
int lbm_axi_batch_admit(lbm_axi_batch *b, const lbm_axi_params *params, const double *phi0_host,
                        int64_t nsteps, int32_t *slot);

/* Advances every running case by min(chunk_steps, its remaining steps):
 * one launch per step; cases that reach their step count stop there.
 * Asynchronous: a change in the set of running cases re-uploads the case
 * table and work list through a pinned staging buffer, ordered on the stream
 * after the steps already enqueued.  A run of chunk_steps steps over an
 * unchanged set replays a hipGraph (captured on first use, one per run length
 * and buffer phase); shorter runs are launched directly. */
int lbm_axi_batch_run(lbm_axi_batch *b, int32_t chunk_steps);

/* Does the host-side work lbm_axi_batch_run(b, chunk_steps) would do before
 * its first launch -- rebuilding the work list if the running set changed,
 * capturing the hipGraph of chunk_steps steps for both buffer phases if every
 * running case has that many steps left -- without launching anything, so a
 * later run starts at once.  Asynchronous. */
int lbm_axi_batch_prepare(lbm_axi_batch *b, int32_t chunk_steps);

/* Slots that have completed their steps and are not yet released: up to cap
 * of them into done_slots, their count into *n_done. */
int lbm_axi_batch_poll(lbm_axi_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done);

/* lbm_axi_moments / lbm_axi_get_state of the case in a slot.  A case that has
 * completed its steps is read on the batch's second stream after its last
 * step (the steps of the running cases go on); a running case is read on the
 * step stream, which that synchronises. */
int lbm_axi_batch_moments(lbm_axi_batch *b, int32_t slot, double *phi, double *rho, double *uz,
                          double *ur, double *p, lbm_axi_diag *diag);
int lbm_axi_batch_get_state(lbm_axi_batch *b, int32_t slot, double *f, double *g, double *aux,
                            int64_t *t);

/* Frees a slot (running or not).  Its pool block becomes reusable once the
 * work that last touched it has completed. */
int lbm_axi_batch_release(lbm_axi_batch *b, int32_t slot);

/* Launch configuration (results do not depend on it): tile_r rows per tile in
 * {2, 4, 8, 16} (0: 8); persistent 0 = one workgroup per tile, 1 = a
 * resident grid striding over the tiles; schedule in 0..3: bit 0 set = largest
 * case first, else cases in slot order; bands in {8, 16, 32} (0: 16) =
 * contiguous runs of tiles each case is cut into, all eight XCDs working on
 * the same case at once: band x + 8m going to XCD x (schedule bit 1 clear) or
 * bands x*bands/8 .. (x+1)*bands/8 - 1 going to XCD x (bit 1 set, neighbouring
 * bands sharing an L2).  LBM_AXI_EBUSY if the running cases' work list would
 * overflow with that tile height. */
int lbm_axi_batch_set_config(lbm_axi_batch *b, int32_t tile_r, int32_t persistent, int32_t schedule,
                             int32_t bands);

/* Occupancy of the batch: slots in use, running cases, free pool bytes, and
 * the number of step launches so far.  Any pointer may be NULL. */
int lbm_axi_batch_info(const lbm_axi_batch *b, int32_t *n_used, int32_t *n_running, size_t *free_bytes,
                       int64_t *launches);

/* Waits for all work of the batch (both of its streams). */
int lbm_axi_batch_sync(lbm_axi_batch *b);

/* Releases every slot and frees the handle (not the pool).  NULL is accepted. */
int lbm_axi_batch_destroy(lbm_axi_batch *b);

/* Static description of an error code. */
const char *lbm_axi_strerror(int code);

/* Measurement helper, not part of the method: a plain device-to-device copy
 * of `bytes` from src to dst (device pointers, 16-byte aligned, bytes a
 * multiple of 16, the ranges not overlapping), one 16-byte element per
 * thread with non-temporal loads and stores, launched asynchronously on
 * hip_stream (NULL: the null stream).  It is the stream-copy ceiling that
 * the step kernels' achieved HBM bandwidth is set against beside the
 * published peak.  LBM_AXI_EINVAL for a misaligned pointer or size, or a
 * size beyond 2^31 workgroups of 256 elements; LBM_AXI_EDEVICE if the
 * launch fails.  bytes = 0 launches nothing. */
int lbm_axi_device_copy(const void *src, void *dst, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
