// lbm_axi batches: many independent cases of different sizes and step counts
// advanced together, one fused launch per time step for all of them.
//
// Memory: the caller hands over one device pool.  Its head holds the case
// table (CaseDesc per slot) and the work list; the rest is carved first-fit
// into per-case blocks (the same layout as a single case), so admission is
// decided by HBM footprint.
//
// A step of the batch is one launch of batch_step_kernel over the work list
// (one per collision form present, see COLLIDE_*):
// item w = (slot, tile) runs the same tile body as the single-case kernel, so
// every case's populations are bit-identical to running it alone.  Runs of
// steps with an unchanged set of running cases replay a captured hipGraph.
// The host keeps each case's step count and ping-pong parity; a case stops
// exactly at its requested number of steps.
//
// Nothing here drains the stream while cases run: the case table and work
// list go up through pinned staging buffers, a case is initialised and read
// back on a second stream (ordered by events against the steps), and the
// pool block of a released case is reused only once the work that last
// touched it has completed.

#include "case_internal.hpp"

#include <algorithm>
#include <type_traits>
#include <cstring>
#include <map>
#include <new>
#include <vector>

using namespace axi;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_WORK = 1 << 20;       // work items of one launch
constexpr int NMODE = 4;                // collision forms (COLLIDE_*)
// launch classes: the collision form, plus NMODE for FP16-deviation cases
// whose g is rounded stochastically; each class runs in a kernel of its own
constexpr int NCLASS = 2 * NMODE;

inline size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// mode 0: one workgroup per work item; mode 1: persistent grid striding over
// the work list.  parity: the batch's buffer phase at this step; a case's
// current buffer is its descriptor's cur0 xor the phase.  step: steps since
// the case table was uploaded, for the acceleration of cases whose gravity
// is still ramping up (their descriptors hold their time at the upload).
template <typename R>
__device__ __forceinline__ Phys<R> phys_of(const CaseDesc<R> &d, int step)
{
    Phys<R> P = d.P;
    if (P.g_ramp > 0.0) P.g_z = (R)ramp_accel(P.g_full, P.g_ramp, d.t0 + step);
    return P;
}

template <typename T, typename R, int TR, int MODE>
__global__ __launch_bounds__(TZ *TR) void batch_step_kernel(char *__restrict__ pool,
                                                            const CaseDesc<R> *__restrict__ descs,
                                                            const WorkItem *__restrict__ work, int nwork,
                                                            int parity, int persistent, int step)
{
    __shared__ R tile[TR + 4][TZ + 4];
    // Work items in list order (the host interleaves each case's XCD bands
    // into the list): handing each XCD a contiguous share of the list instead
    // had the XCDs stream from 8 distant cases at once and measured about 20%
    // slower on 16 cases of 256 x 512.
    const int stride = persistent ? (int)gridDim.x : nwork;
    for (int w = blockIdx.x; w < nwork; w += stride) {
        WorkItem it = work[w];
        if (it.slot < 0) continue;      // padding of a short band (uniform)
        const CaseDesc<R> &d = descs[it.slot];
        int cur = d.cur0 ^ parity;
        tile_step<T, R, TZ, TR, MODE>(d.g, phys_of(d, step), it.tz, it.tr, (const T *)(pool + d.pop[cur][0]),
                                      (const T *)(pool + d.pop[cur][1]), (T *)(pool + d.pop[cur ^ 1][0]),
                                      (T *)(pool + d.pop[cur ^ 1][1]), (T *)(pool + d.aux), tile);
        __syncthreads();
    }
}

// The same loop over work items for FP16-deviation storage.  Buffer b of a
// case: f_0 plane then 8 FP16 f planes at pop[b][0], 9 FP16 g planes at
// pop[b][1]; aux planes: phase field of side 0, u_z, u_r, phase field of side 1.
// six waves per SIMD (three workgroups per CU) for 64 x 8 and 64 x 16 tiles:
// the unit-rate MRT and SRT forms fit in 70 VGPRs; the general MRT and the
// non-orthogonal form need 82-84 and spill two VGPRs under the bound, which
// still runs 18 % faster than four waves per SIMD (non-orthogonal form);
// eight waves per SIMD (64 VGPRs) spills in the boundary path and measured
// slower
template <int TR, int MODE, bool SR>
__global__ __launch_bounds__(TZ *TR) __attribute__((amdgpu_waves_per_eu(
    TR >= 8 ? 6 : 1))) void batch_step_kernel_h(char *__restrict__ pool,
                                                              const CaseDesc<float> *__restrict__ descs,
                                                              const WorkItem *__restrict__ work, int nwork,
                                                              int parity, int persistent, int step,
                                                              int64_t *__restrict__ times)
{
    __shared__ float tile[TR + 4][TZ + 4];
    const int stride = persistent ? (int)gridDim.x : nwork;
    for (int w = blockIdx.x; w < nwork; w += stride) {
        WorkItem it = work[w];
        if (it.slot < 0) continue;      // padding of a short band (uniform)
        const CaseDesc<float> &d = descs[it.slot];
        const int cur = d.cur0 ^ parity;
        Phys<float> P = phys_of(d, step);
        if constexpr (SR) {
            // the case's time (the key of its g roundings), kept on the device
            // so that graph replays see it advance: times[2 slot + p] is the
            // time at the start of a launch of phase p; this launch reads its
            // phase's entry and one thread of the case's first tile writes
            // the other phase's, which the next launch reads
            const int64_t tn = times[2 * it.slot + parity];
            if (it.tz == 0 && it.tr == 0 && threadIdx.x == 0) times[2 * it.slot + (parity ^ 1)] = tn + 1;
            P.round_key = mix32((uint32_t)tn);
        }
        const size_t pb4 = (size_t)d.g.plane * 4;
        char *aux = pool + d.aux;
        HalfState S;
        S.f0in = (const float *)(pool + d.pop[cur][0]);
        S.fin = (const half_t *)(pool + d.pop[cur][0] + pb4);
        S.gin = (const half_t *)(pool + d.pop[cur][1]);
        S.f0out = (float *)(pool + d.pop[cur ^ 1][0]);
        S.fout = (half_t *)(pool + d.pop[cur ^ 1][0] + pb4);
        S.gout = (half_t *)(pool + d.pop[cur ^ 1][1]);
        S.phin = (const float *)(aux + (cur ? 3 * pb4 : 0));
        S.phout = (float *)(aux + (cur ? 0 : 3 * pb4));
        S.uz = (float *)(aux + pb4);
        S.ur = (float *)(aux + 2 * pb4);
        tile_step_h<TZ, TR, MODE, false, SR>(d.g, P, d.C, it.tz, it.tr, S, Fields{}, tile);
        __syncthreads();
    }
}

struct Block {
    size_t off, size;
};

// A released block and the event after the last work that touched it.
struct Held {
    Block blk;
    hipEvent_t ev;
};

// Graphs replaced while launches of them may still be queued: destroyed once
// `ev`, recorded after those launches, has completed.
struct Retired {
    std::vector<hipGraphExec_t> execs;
    hipEvent_t ev;
};

// Pinned host buffer an asynchronous upload reads from; refilled only once
// the copy recorded by `ev` has run.
struct Stage {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

constexpr int DEFAULT_BANDS = 16;

} // namespace

struct lbm_axi_batch {
    char *pool;
    size_t pool_bytes;
    int max_cases;
    int precision;
    hipStream_t stream;                 // the steps
    hipStream_t side;                   // initialisation and read-back of cases not running
    bool own_stream;
    int tile_r;
    int persistent;
    int schedule;                       // bit 0: largest case first (else admission order); bit 1: contiguous bands per XCD
    int bands;                          // contiguous tile bands per case (multiple of 8)
    int cu_count;
    int phase;                          // buffer phase of the next step (flips every step)
    int64_t since_upload;               // steps launched since the case table was uploaded
    bool table_ramp;                    // the uploaded table has a case still ramping its gravity
    // device areas in the pool head
    void *d_descs;
    WorkItem *d_work;
    int64_t *d_times;                   // [max_cases][2]: FP16 cases' time per buffer phase
    size_t heap_off;
    std::vector<Block> free_list;       // free heap ranges, sorted by offset
    std::vector<Held> held;             // released blocks whose last work may still run
    std::vector<hipEvent_t> spare_events;
    Stage stage[2];
    int stage_next;
    // slots
    std::vector<lbm_axi_case *> cases;
    std::vector<Block> blocks;
    std::vector<int64_t> remaining;
    std::vector<char> used;
    std::vector<hipEvent_t> done_ev;    // recorded after a case's last step
    // current launch configuration
    std::vector<WorkItem> work;         // grouped by collision form
    int mode_start[NCLASS + 1];         // items of class q: [mode_start[q], mode_start[q + 1])
    std::vector<int> running;           // slots in the work list
    bool dirty;                         // work list / descriptors must be rebuilt
    std::map<int, hipGraphExec_t> graphs;   // by 2 * run length + starting phase
    std::vector<Retired> retired;
    int64_t launches;
};

namespace {

hipEvent_t take_event(lbm_axi_batch *b)
{
    if (!b->spare_events.empty()) {
        hipEvent_t e = b->spare_events.back();
        b->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

// destroy retired graphs whose launches have completed (all of them if wait)
void reap_graphs(lbm_axi_batch *b, bool wait)
{
    for (size_t q = 0; q < b->retired.size();) {
        Retired &r = b->retired[q];
        if (wait) (void)hipEventSynchronize(r.ev);
        if (hipEventQuery(r.ev) == hipSuccess) {
            for (hipGraphExec_t e : r.execs)
                (void)hipGraphExecDestroy(e);
            b->spare_events.push_back(r.ev);
            b->retired.erase(b->retired.begin() + q);
        } else {
            ++q;
        }
    }
}

// the current graphs stop being used; launches of them may still be queued
int drop_graphs(lbm_axi_batch *b)
{
    reap_graphs(b, false);
    if (b->graphs.empty()) return LBM_AXI_OK;
    Retired r;
    r.ev = take_event(b);
    if (!r.ev || hipEventRecord(r.ev, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    for (auto &kv : b->graphs)
        r.execs.push_back(kv.second);
    b->graphs.clear();
    b->retired.push_back(std::move(r));
    return LBM_AXI_OK;
}

bool heap_alloc(lbm_axi_batch *b, size_t bytes, Block &out)
{
    bytes = up(bytes, ALIGN);
    for (size_t q = 0; q < b->free_list.size(); ++q) {
        Block &f = b->free_list[q];
        if (f.size >= bytes) {
            out.off = f.off;
            out.size = bytes;
            f.off += bytes;
            f.size -= bytes;
            if (f.size == 0) b->free_list.erase(b->free_list.begin() + q);
            return true;
        }
    }
    return false;
}

void heap_free(lbm_axi_batch *b, Block blk)
{
    auto it = std::lower_bound(b->free_list.begin(), b->free_list.end(), blk,
                               [](const Block &a, const Block &c) { return a.off < c.off; });
    it = b->free_list.insert(it, blk);
    // coalesce with the neighbours
    size_t q = it - b->free_list.begin();
    if (q + 1 < b->free_list.size() && b->free_list[q].off + b->free_list[q].size == b->free_list[q + 1].off) {
        b->free_list[q].size += b->free_list[q + 1].size;
        b->free_list.erase(b->free_list.begin() + q + 1);
    }
    if (q > 0 && b->free_list[q - 1].off + b->free_list[q - 1].size == b->free_list[q].off) {
        b->free_list[q - 1].size += b->free_list[q].size;
        b->free_list.erase(b->free_list.begin() + q);
    }
}

// Released blocks whose last work has completed go back to the free list;
// with wait_oldest, first wait for the oldest one still held.
void reclaim(lbm_axi_batch *b, bool wait_oldest)
{
    if (wait_oldest && !b->held.empty()) (void)hipEventSynchronize(b->held.front().ev);
    for (size_t q = 0; q < b->held.size();) {
        if (hipEventQuery(b->held[q].ev) == hipSuccess) {
            heap_free(b, b->held[q].blk);
            b->spare_events.push_back(b->held[q].ev);
            b->held.erase(b->held.begin() + q);
        } else {
            ++q;
        }
    }
}

// A pinned staging buffer of at least `bytes`, free for refilling.
Stage *stage_acquire(lbm_axi_batch *b, size_t bytes)
{
    Stage &s = b->stage[b->stage_next];
    b->stage_next ^= 1;
    if (s.pending) {
        if (hipEventSynchronize(s.ev) != hipSuccess) return nullptr;
        s.pending = false;
    }
    if (!s.ev && hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) return nullptr;
    if (s.cap < bytes) {
        if (s.host) (void)hipHostFree(s.host);
        s.host = nullptr;
        s.cap = 0;
        size_t cap = std::max<size_t>(bytes, 64 << 10);
        if (hipHostMalloc(&s.host, cap, hipHostMallocDefault) != hipSuccess) return nullptr;
        s.cap = cap;
    }
    return &s;
}

size_t desc_size(int precision)
{
    return precision == LBM_AXI_FP64 ? sizeof(CaseDesc<double>) : sizeof(CaseDesc<float>);
}

// the kernel a case's tiles run in: its collision form, and for FP16-deviation
// storage with stochastic g rounding the form plus NMODE
int launch_class(const lbm_axi_case *c)
{
    return c->P64.mode + (c->prm.fp16_rounding == LBM_AXI_ROUND_STOCHASTIC ? NMODE : 0);
}

bool valid_precision(int precision)
{
    return precision == LBM_AXI_FP64 || precision == LBM_AXI_FP32 || precision == LBM_AXI_FP16D;
}

template <typename R>
CaseDesc<R> make_desc(const lbm_axi_batch *b, const lbm_axi_case *c, const Phys<R> &P, int tile_r)
{
    CaseDesc<R> d;
    d.g = geom_for(c, tile_r);
    d.P = P;
    for (int q = 0; q < 2; ++q)
        for (int s = 0; s < 2; ++s)
            d.pop[q][s] = (uint64_t)((char *)c->pop[q][s] - b->pool);
    d.aux = (uint64_t)((char *)c->aux - b->pool);
    d.cur0 = c->cur ^ b->phase;
    d.pad = 0;
    d.t0 = c->t;
    d.C = c->codec;
    return d;
}

// Work items of one case: its tiles (row-major) cut into `bands` contiguous
// bands, each XCD's bands in turn, interleaved so that list position w
// belongs to XCD w % 8 (workgroup w runs there, and so does item w + k*grid
// of a persistent grid whose size is a multiple of 8).  All XCDs then work on
// the same case at the same time.  Band order: strided, band x + 8m on XCD x,
// or contiguous, bands x*per .. x*per + per - 1 on XCD x (per = bands / 8), so
// that neighbouring bands -- whose rows the ring and the shifted pulls re-read
// -- share an XCD's L2 except at every per-th band.  Short XCD runs are padded
// with empty items (slot -1).  slot < 0 only counts.
int case_items(int slot, int tiles, int tiles_z, int bands, bool contiguous, std::vector<WorkItem> *out)
{
    const int q = tiles / bands, rem = tiles % bands, per = bands / 8;
    int rounds = 0;
    for (int x = 0; x < 8; ++x) {
        int len = 0;
        for (int m = 0; m < per; ++m) len += q + ((contiguous ? x * per + m : x + 8 * m) < rem ? 1 : 0);
        rounds = std::max(rounds, len);
    }
    if (!out) return 8 * rounds;
    std::vector<int> pos(8, 0), band(8, 0);   // per XCD: position within its current band, band index m
    for (int l = 0; l < rounds; ++l)
        for (int x = 0; x < 8; ++x) {
            // advance XCD x past finished bands
            while (band[x] < per) {
                const int bnd = contiguous ? x * per + band[x] : x + 8 * band[x];
                const int blen = q + (bnd < rem ? 1 : 0);
                if (pos[x] < blen) break;
                ++band[x];
                pos[x] = 0;
            }
            if (band[x] >= per) {
                out->push_back(WorkItem{-1, 0, 0, 0});
                continue;
            }
            const int bnd = contiguous ? x * per + band[x] : x + 8 * band[x];
            const int start = bnd * q + std::min(bnd, rem);
            const int t = start + pos[x];
            out->push_back(WorkItem{slot, t % tiles_z, t / tiles_z, 0});
            ++pos[x];
        }
    return 8 * rounds;
}

// work items the running cases plus `extra` tiles' case would need
int64_t items_needed(const lbm_axi_batch *b, int tile_r, int bands, bool contiguous, const lbm_axi_case *extra)
{
    int64_t n = 0;
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s] && b->remaining[s] > 0)
            n += case_items(-1, geom_for(b->cases[s], tile_r).tiles, 1, bands, contiguous, nullptr);
    if (extra) n += case_items(-1, geom_for(extra, tile_r).tiles, 1, bands, contiguous, nullptr);
    return n;
}

// whether the step from time t of a case still has less than its full gravity
bool ramping_at(const lbm_axi_case *c, int64_t t)
{
    return c->prm.g_ramp > 0.0 && (double)(t + 1) < c->prm.g_ramp;
}

// rebuild the descriptor table and work list for the running cases; the
// upload is ordered on the stream after every step already enqueued
int rebuild(lbm_axi_batch *b)
{
    if (drop_graphs(b)) return LBM_AXI_EDEVICE;
    b->running.clear();
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s] && b->remaining[s] > 0)
            b->running.push_back(s);
    std::vector<int> order = b->running;
    if (b->schedule & 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
            return (int64_t)b->cases[a]->prm.nr * b->cases[a]->prm.nz >
                   (int64_t)b->cases[c]->prm.nr * b->cases[c]->prm.nz;
        });
    // cases grouped by launch class: each class runs in a kernel of its own
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return launch_class(b->cases[a]) < launch_class(b->cases[c]); });
    b->work.clear();
    for (int q = 0; q <= NCLASS; ++q) b->mode_start[q] = 0;
    for (int s : order) {
        const Geom gs = geom_for(b->cases[s], b->tile_r);
        case_items(s, gs.tiles, gs.tiles_z, b->bands, (b->schedule & 2) != 0, &b->work);
        // items of classes <= this case's class end here (classes are sorted)
        for (int q = launch_class(b->cases[s]) + 1; q <= NCLASS; ++q) b->mode_start[q] = (int)b->work.size();
    }
    if ((int64_t)b->work.size() > MAX_WORK) return LBM_AXI_EBUSY;   // admission keeps this from happening
    // descriptors of every used slot, the cases' times, then the work list, in
    // one staging buffer
    const size_t ds = desc_size(b->precision);
    const size_t dbytes = ds * b->max_cases, tbytes = 2 * sizeof(int64_t) * b->max_cases;
    const size_t wbytes = b->work.size() * sizeof(WorkItem);
    Stage *st = stage_acquire(b, dbytes + tbytes + wbytes);
    if (!st) return LBM_AXI_EDEVICE;
    char *host = (char *)st->host;
    memset(host, 0, dbytes + tbytes);
    int64_t *times = (int64_t *)(host + dbytes);
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s]) times[2 * s] = times[2 * s + 1] = b->cases[s]->t;
    for (int s = 0; s < b->max_cases; ++s) {
        if (!b->used[s]) continue;
        if (b->precision == LBM_AXI_FP64) {
            CaseDesc<double> d = make_desc(b, b->cases[s], b->cases[s]->P64, b->tile_r);
            memcpy(host + s * ds, &d, ds);
        } else {
            CaseDesc<float> d = make_desc(b, b->cases[s], b->cases[s]->P32, b->tile_r);
            memcpy(host + s * ds, &d, ds);
        }
    }
    if (wbytes) memcpy(host + dbytes + tbytes, b->work.data(), wbytes);
    if (hipMemcpyAsync(b->d_descs, host, dbytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_AXI_EDEVICE;
    if (hipMemcpyAsync(b->d_times, host + dbytes, tbytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_AXI_EDEVICE;
    if (wbytes &&
        hipMemcpyAsync(b->d_work, host + dbytes + tbytes, wbytes, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_AXI_EDEVICE;
    if (hipEventRecord(st->ev, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    st->pending = true;
    b->dirty = false;
    b->since_upload = 0;
    b->table_ramp = false;
    for (int q : b->running)
        if (ramping_at(b->cases[q], b->cases[q]->t)) b->table_ramp = true;
    return LBM_AXI_OK;
}

template <typename T, typename R, int TR, int MODE, bool SR = false>
void launch_part(lbm_axi_batch *b, int parity, int step, int first, int nwork)
{
    if (nwork <= 0) return;
    int grid = nwork;
    if (b->persistent) {
        int per_cu = sizeof(T) == 8 ? 4 : (sizeof(T) == 2 ? 6 : 8);   // resident waves per SIMD
        int waves = TZ * TR / 64;
        int wg_per_cu = std::max(1, per_cu * 4 / waves);
        grid = std::min(nwork, b->cu_count * wg_per_cu);
        grid = (grid + 7) / 8 * 8;      // keeps item w on XCD w % 8
    }
    if constexpr (std::is_same<T, half_t>::value)
        batch_step_kernel_h<TR, MODE, SR><<<grid, TZ * TR, 0, b->stream>>>(
            b->pool, (const CaseDesc<float> *)b->d_descs, b->d_work + first, nwork, parity, b->persistent, step,
            b->d_times);
    else
        batch_step_kernel<T, R, TR, MODE><<<grid, TZ * TR, 0, b->stream>>>(
            b->pool, (const CaseDesc<R> *)b->d_descs, b->d_work + first, nwork, parity, b->persistent, step);
}

template <typename T, typename R, int TR>
void launch_tr(lbm_axi_batch *b, int parity, int step)
{
    const int *ms = b->mode_start;
    const int nw = (int)b->work.size();
    launch_part<T, R, TR, COLLIDE_MRT>(b, parity, step, ms[0], ms[1] - ms[0]);
    launch_part<T, R, TR, COLLIDE_MRT_UNIT>(b, parity, step, ms[1], ms[2] - ms[1]);
    launch_part<T, R, TR, COLLIDE_SRT>(b, parity, step, ms[2], ms[3] - ms[2]);
    launch_part<T, R, TR, COLLIDE_NMRT>(b, parity, step, ms[3], ms[4] - ms[3]);
    // FP16-deviation cases with stochastic g rounding (no other precision has them)
    if constexpr (std::is_same<T, half_t>::value) {
        launch_part<T, R, TR, COLLIDE_MRT, true>(b, parity, step, ms[4], ms[5] - ms[4]);
        launch_part<T, R, TR, COLLIDE_MRT_UNIT, true>(b, parity, step, ms[5], ms[6] - ms[5]);
        launch_part<T, R, TR, COLLIDE_SRT, true>(b, parity, step, ms[6], ms[7] - ms[6]);
        launch_part<T, R, TR, COLLIDE_NMRT, true>(b, parity, step, ms[7], nw - ms[7]);
    }
}

template <typename T, typename R>
void launch_one(lbm_axi_batch *b, int parity, int step)
{
    switch (b->tile_r) {
    case 2: launch_tr<T, R, 2>(b, parity, step); break;
    case 4: launch_tr<T, R, 4>(b, parity, step); break;
    case 16: launch_tr<T, R, 16>(b, parity, step); break;
    default: launch_tr<T, R, 8>(b, parity, step); break;
    }
}

// n steps starting at buffer phase `phase`, the first `first` steps after the
// table upload
void launch_steps(lbm_axi_batch *b, int n, int phase, int64_t first)
{
    for (int s = 0; s < n; ++s) {
        const int parity = (phase ^ s) & 1;
        const int step = (int)std::min<int64_t>(first + s, INT32_MAX);
        if (b->precision == LBM_AXI_FP64)
            launch_one<double, double>(b, parity, step);
        else if (b->precision == LBM_AXI_FP16D)
            launch_one<half_t, float>(b, parity, step);
        else
            launch_one<float, float>(b, parity, step);
    }
}

// the graph of n steps from the current phase, captured if not yet seen
int graph_for(lbm_axi_batch *b, int n, int phase, hipGraphExec_t *out)
{
    const int key = 2 * n + phase;
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t graph;
        if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return LBM_AXI_EDEVICE;
        launch_steps(b, n, phase, 0);   // no case of the table ramps: the step count is unused
        if (hipStreamEndCapture(b->stream, &graph) != hipSuccess) return LBM_AXI_EDEVICE;
        hipGraphExec_t exec;
        if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return LBM_AXI_EDEVICE;
        }
        (void)hipGraphDestroy(graph);
        it = b->graphs.emplace(key, exec).first;
    }
    *out = it->second;
    return LBM_AXI_OK;
}

// n steps of the running cases (graph replay when use_graph and no case of
// the uploaded table is still ramping its gravity)
int run_span(lbm_axi_batch *b, int n, bool use_graph)
{
    if (n <= 0 || b->work.empty()) return LBM_AXI_OK;
    if (use_graph && !b->table_ramp) {
        hipGraphExec_t exec;
        int rc = graph_for(b, n, b->phase, &exec);
        if (rc) return rc;
        if (hipGraphLaunch(exec, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    } else {
        launch_steps(b, n, b->phase, b->since_upload);
        if (hipGetLastError() != hipSuccess) return LBM_AXI_EDEVICE;
    }
    b->launches += n;
    b->since_upload += n;
    // host bookkeeping: time, remaining steps, buffer of every running case
    const int flip = n & 1;
    b->phase ^= flip;
    bool still_ramping = false;
    for (int s : b->running) {
        lbm_axi_case *c = b->cases[s];
        c->t += n;
        c->cur ^= flip;
        b->remaining[s] -= n;
        still_ramping = still_ramping || ramping_at(c, c->t);
        if (b->remaining[s] == 0) {
            // the set of running cases changes; the case's last step is marked
            // so that reading it back and reusing its block wait for it only
            b->dirty = true;
            hipEvent_t e = b->done_ev[s] ? b->done_ev[s] : take_event(b);
            if (!e || hipEventRecord(e, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
            b->done_ev[s] = e;
        }
    }
    // once every ramp is complete, a fresh table lets the graphs take over
    if (b->table_ramp && !still_ramping) b->dirty = true;
    return LBM_AXI_OK;
}

int check_slot(const lbm_axi_batch *b, int slot)
{
    if (!b) return LBM_AXI_ESTATE;
    if (slot < 0 || slot >= b->max_cases || !b->used[slot]) return LBM_AXI_ESTATE;
    return LBM_AXI_OK;
}

// A case that is not running is read on the side stream after its last step,
// so that the steps of the others go on meanwhile; a running case is read on
// the step stream.
template <typename F>
int with_case_stream(lbm_axi_batch *b, int slot, F &&fn)
{
    lbm_axi_case *c = b->cases[slot];
    if (b->remaining[slot] > 0) return fn(c);
    if (b->done_ev[slot] && hipStreamWaitEvent(b->side, b->done_ev[slot], 0) != hipSuccess) return LBM_AXI_EDEVICE;
    hipStream_t keep = c->stream;
    c->stream = b->side;
    int rc = fn(c);
    c->stream = keep;
    return rc;
}

bool valid_bands(int bands) { return bands == 8 || bands == 16 || bands == 32; }

} // namespace

extern "C" {

size_t lbm_axi_batch_reserved_bytes(int32_t max_cases, int32_t precision)
{
    if (max_cases <= 0 || !valid_precision(precision)) return 0;
    return up(desc_size(precision) * max_cases, ALIGN) + up(sizeof(WorkItem) * (size_t)MAX_WORK, ALIGN) +
           up(2 * sizeof(int64_t) * (size_t)max_cases, ALIGN);
}

int lbm_axi_batch_create(void *dev_pool, size_t pool_bytes, int32_t max_cases, int32_t precision,
                         void *hip_stream, lbm_axi_batch **out)
{
    if (!out) return LBM_AXI_EINVAL;
    *out = nullptr;
    size_t head = lbm_axi_batch_reserved_bytes(max_cases, precision);
    if (!dev_pool || head == 0 || ((uintptr_t)dev_pool & (ALIGN - 1))) return LBM_AXI_EINVAL;
    if (pool_bytes < head) return LBM_AXI_ENOMEM;
    lbm_axi_batch *b = new (std::nothrow) lbm_axi_batch;
    if (!b) return LBM_AXI_ENOMEM;
    b->pool = (char *)dev_pool;
    b->pool_bytes = pool_bytes;
    b->max_cases = max_cases;
    b->precision = precision;
    b->own_stream = false;
    b->stream = (hipStream_t)hip_stream;
    if (!b->stream) {
        // graph capture needs a stream other than the null stream
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return LBM_AXI_EDEVICE;
        }
        b->own_stream = true;
    }
    // default priority, like the step stream
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return LBM_AXI_EDEVICE;
    }
    b->tile_r = 8;
    b->persistent = 0;
    b->schedule = 1;
    b->bands = DEFAULT_BANDS;
    b->phase = 0;
    b->since_upload = 0;
    b->table_ramp = false;
    b->stage_next = 0;
    int dev = 0;
    b->cu_count = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    b->d_descs = b->pool;
    b->d_work = (WorkItem *)(b->pool + up(desc_size(precision) * max_cases, ALIGN));
    b->d_times = (int64_t *)((char *)b->d_work + up(sizeof(WorkItem) * (size_t)MAX_WORK, ALIGN));
    b->heap_off = head;
    b->free_list.push_back(Block{head, pool_bytes - head});
    b->cases.assign(max_cases, nullptr);
    b->blocks.assign(max_cases, Block{0, 0});
    b->remaining.assign(max_cases, 0);
    b->used.assign(max_cases, 0);
    b->done_ev.assign(max_cases, nullptr);
    b->dirty = true;
    for (int q = 0; q <= NCLASS; ++q) b->mode_start[q] = 0;
    b->launches = 0;
    *out = b;
    return LBM_AXI_OK;
}

int lbm_axi_batch_admit(lbm_axi_batch *b, const lbm_axi_params *params, const double *phi0_host,
                        int64_t nsteps, int32_t *slot)
{
    if (!b) return LBM_AXI_ESTATE;
    if (!params || !phi0_host || !slot || nsteps < 0) return LBM_AXI_EINVAL;
    if (params->precision != b->precision) return LBM_AXI_EINVAL;
    size_t bytes = lbm_axi_state_bytes(params);
    if (bytes == 0) return LBM_AXI_EINVAL;
    if (up(bytes, ALIGN) > b->pool_bytes - b->heap_off) return LBM_AXI_ENOMEM;   // never fits
    int s = -1;
    for (int q = 0; q < b->max_cases; ++q)
        if (!b->used[q]) { s = q; break; }
    if (s < 0) return LBM_AXI_EBUSY;
    // the work list of one launch stays within its reserved area
    {
        lbm_axi_case probe;
        probe.prm = *params;
        if (items_needed(b, b->tile_r, b->bands, (b->schedule & 2) != 0, nsteps > 0 ? &probe : nullptr) > MAX_WORK)
            return LBM_AXI_EBUSY;
    }
    Block blk;
    reclaim(b, false);
    while (!heap_alloc(b, bytes, blk)) {
        if (b->held.empty()) return LBM_AXI_EBUSY;
        reclaim(b, true);      // waits for earlier work only: later steps stay queued
    }
    // initialised on the side stream (which it synchronises): the steps of the
    // running cases already enqueued go on meanwhile
    lbm_axi_case *c = nullptr;
    int rc = lbm_axi_init(params, b->pool + blk.off, blk.size, phi0_host, b->side, &c);
    if (rc) {
        heap_free(b, blk);
        return rc;
    }
    c->stream = b->stream;
    b->cases[s] = c;
    b->blocks[s] = blk;
    b->remaining[s] = nsteps;
    b->used[s] = 1;
    b->dirty = true;
    *slot = s;
    return LBM_AXI_OK;
}

int lbm_axi_batch_run(lbm_axi_batch *b, int32_t chunk_steps)
{
    if (!b) return LBM_AXI_ESTATE;
    if (chunk_steps < 0) return LBM_AXI_EINVAL;
    int64_t left = chunk_steps;
    while (left > 0) {
        if (b->dirty) {
            int rc = rebuild(b);
            if (rc) return rc;
        }
        if (b->running.empty()) break;
        int64_t m = left;
        for (int s : b->running)
            m = std::min(m, b->remaining[s]);
        // replay a graph for full chunks; shorter tails are launched directly
        int rc = run_span(b, (int)m, m == chunk_steps);
        if (rc) return rc;
        left -= m;
    }
    return LBM_AXI_OK;
}

int lbm_axi_batch_prepare(lbm_axi_batch *b, int32_t chunk_steps)
{
    if (!b) return LBM_AXI_ESTATE;
    if (chunk_steps < 0) return LBM_AXI_EINVAL;
    if (b->dirty) {
        int rc = rebuild(b);
        if (rc) return rc;
    }
    if (b->running.empty() || chunk_steps == 0 || b->table_ramp) return LBM_AXI_OK;
    for (int s : b->running)
        if (b->remaining[s] < chunk_steps) return LBM_AXI_OK;   // such a run is launched directly
    for (int ph = 0; ph < 2; ++ph) {
        hipGraphExec_t exec;
        int rc = graph_for(b, chunk_steps, ph, &exec);
        if (rc) return rc;
    }
    return LBM_AXI_OK;
}

int lbm_axi_batch_poll(lbm_axi_batch *b, int32_t *done_slots, int32_t cap, int32_t *n_done)
{
    if (!b) return LBM_AXI_ESTATE;
    if (!n_done || cap < 0 || (cap > 0 && !done_slots)) return LBM_AXI_EINVAL;
    int n = 0;
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s] && b->remaining[s] == 0) {
            if (n < cap) done_slots[n] = s;
            ++n;
        }
    *n_done = n;
    return LBM_AXI_OK;
}

int lbm_axi_batch_moments(lbm_axi_batch *b, int32_t slot, double *phi, double *rho, double *uz, double *ur,
                          double *p, lbm_axi_diag *diag)
{
    int rc = check_slot(b, slot);
    if (rc) return rc;
    return with_case_stream(b, slot, [&](lbm_axi_case *c) { return lbm_axi_moments(c, phi, rho, uz, ur, p, diag); });
}

int lbm_axi_batch_get_state(lbm_axi_batch *b, int32_t slot, double *f, double *g, double *aux, int64_t *t)
{
    int rc = check_slot(b, slot);
    if (rc) return rc;
    return with_case_stream(b, slot, [&](lbm_axi_case *c) { return lbm_axi_get_state(c, f, g, aux, t); });
}

int lbm_axi_batch_release(lbm_axi_batch *b, int32_t slot)
{
    int rc = check_slot(b, slot);
    if (rc) return rc;
    // the block is reused once the last work on it has run: the case's last
    // step if it finished (its read-backs synchronised the side stream), else
    // everything enqueued on the step stream so far
    hipEvent_t e = b->done_ev[slot];
    b->done_ev[slot] = nullptr;
    if (b->remaining[slot] > 0 || !e) {
        if (!e) e = take_event(b);
        if (!e || hipEventRecord(e, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    }
    if (hipStreamSynchronize(b->side) != hipSuccess) return LBM_AXI_EDEVICE;
    lbm_axi_destroy(b->cases[slot]);
    b->held.push_back(Held{b->blocks[slot], e});
    b->cases[slot] = nullptr;
    b->used[slot] = 0;
    b->remaining[slot] = 0;
    b->dirty = true;
    return LBM_AXI_OK;
}

int lbm_axi_batch_set_config(lbm_axi_batch *b, int32_t tile_r, int32_t persistent, int32_t schedule,
                             int32_t bands)
{
    if (!b) return LBM_AXI_ESTATE;
    if (tile_r == 0) tile_r = 8;
    if (bands == 0) bands = DEFAULT_BANDS;
    if (tile_r != 2 && tile_r != 4 && tile_r != 8 && tile_r != 16) return LBM_AXI_EINVAL;
    if ((persistent != 0 && persistent != 1) || schedule < 0 || schedule > 3 || !valid_bands(bands))
        return LBM_AXI_EINVAL;
    if (items_needed(b, tile_r, bands, (schedule & 2) != 0, nullptr) > MAX_WORK) return LBM_AXI_EBUSY;
    b->tile_r = tile_r;
    b->persistent = persistent;
    b->schedule = schedule;
    b->bands = bands;
    b->dirty = true;
    return LBM_AXI_OK;
}

int lbm_axi_batch_info(const lbm_axi_batch *b, int32_t *n_used, int32_t *n_running, size_t *free_bytes,
                       int64_t *launches)
{
    if (!b) return LBM_AXI_ESTATE;
    int u = 0, r = 0;
    size_t fb = 0;
    for (int s = 0; s < b->max_cases; ++s) {
        u += b->used[s] ? 1 : 0;
        r += (b->used[s] && b->remaining[s] > 0) ? 1 : 0;
    }
    for (const Block &f : b->free_list)
        fb += f.size;
    for (const Held &h : b->held)
        fb += h.blk.size;
    if (n_used) *n_used = u;
    if (n_running) *n_running = r;
    if (free_bytes) *free_bytes = fb;
    if (launches) *launches = b->launches;
    return LBM_AXI_OK;
}

int lbm_axi_batch_sync(lbm_axi_batch *b)
{
    if (!b) return LBM_AXI_ESTATE;
    if (hipStreamSynchronize(b->stream) != hipSuccess || hipStreamSynchronize(b->side) != hipSuccess)
        return LBM_AXI_EDEVICE;
    return LBM_AXI_OK;
}

int lbm_axi_batch_destroy(lbm_axi_batch *b)
{
    if (!b) return LBM_AXI_OK;
    (void)hipStreamSynchronize(b->stream);
    (void)hipStreamSynchronize(b->side);
    for (auto &kv : b->graphs)
        (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    reap_graphs(b, true);
    for (int s = 0; s < b->max_cases; ++s) {
        if (b->used[s]) lbm_axi_destroy(b->cases[s]);
        if (b->done_ev[s]) (void)hipEventDestroy(b->done_ev[s]);
    }
    for (const Held &h : b->held)
        (void)hipEventDestroy(h.ev);
    for (hipEvent_t e : b->spare_events)
        (void)hipEventDestroy(e);
    for (Stage &st : b->stage) {
        if (st.host) (void)hipHostFree(st.host);
        if (st.ev) (void)hipEventDestroy(st.ev);
    }
    (void)hipStreamDestroy(b->side);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM_AXI_OK;
}

} // extern "C"
