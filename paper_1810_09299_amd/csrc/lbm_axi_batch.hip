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

inline size_t up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// mode 0: one workgroup per work item; mode 1: persistent grid striding over
// the work list
template <typename T, typename R, int TR, int MODE>
__global__ __launch_bounds__(TZ *TR) void batch_step_kernel(char *__restrict__ pool,
                                                            const CaseDesc<R> *__restrict__ descs,
                                                            const WorkItem *__restrict__ work, int nwork,
                                                            int parity, int persistent)
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
        tile_step<T, R, TZ, TR, MODE>(d.g, d.P, it.tile, (const T *)(pool + d.pop[cur][0]),
                                      (const T *)(pool + d.pop[cur][1]), (T *)(pool + d.pop[cur ^ 1][0]),
                                      (T *)(pool + d.pop[cur ^ 1][1]), (T *)(pool + d.aux), tile);
        __syncthreads();
    }
}

// The same loop over work items for FP16-deviation storage.  Buffer b of a
// case: f_0 plane then 8 FP16 f planes at pop[b][0], 9 FP16 g planes at
// pop[b][1]; aux planes: phase field of side 0, u_z, u_r, phase field of side 1.
// six waves per SIMD (80 VGPRs) for 64 x 8 and 64 x 16 tiles with the unit-
// rate MRT and SRT forms: three workgroups per CU (the boundary path would
// otherwise take a few more registers); the general forms need more and
// spill under that bound, which costs more than the occupancy
template <int TR, int MODE>
__global__ __launch_bounds__(TZ *TR) __attribute__((amdgpu_waves_per_eu(
    (TR >= 8 && (MODE == COLLIDE_MRT_UNIT || MODE == COLLIDE_SRT)) ? 6 : 1))) void batch_step_kernel_h(char *__restrict__ pool,
                                                              const CaseDesc<float> *__restrict__ descs,
                                                              const WorkItem *__restrict__ work, int nwork,
                                                              int parity, int persistent)
{
    __shared__ float tile[TR + 4][TZ + 4];
    const int stride = persistent ? (int)gridDim.x : nwork;
    for (int w = blockIdx.x; w < nwork; w += stride) {
        WorkItem it = work[w];
        if (it.slot < 0) continue;      // padding of a short band (uniform)
        const CaseDesc<float> &d = descs[it.slot];
        const int cur = d.cur0 ^ parity;
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
        tile_step_h<TZ, TR, MODE, false>(d.g, d.P, d.C, it.tile, S, nullptr, tile);
        __syncthreads();
    }
}

struct Block {
    size_t off, size;
};

} // namespace

struct lbm_axi_batch {
    char *pool;
    size_t pool_bytes;
    int max_cases;
    int precision;
    hipStream_t stream;
    bool own_stream;
    int tile_r;
    int persistent;
    int schedule;                       // 0 admission order, 1 largest case first
    int cu_count;
    // device areas in the pool head
    void *d_descs;
    WorkItem *d_work;
    size_t heap_off;
    std::vector<Block> free_list;       // free heap ranges, sorted by offset
    // slots
    std::vector<lbm_axi_case *> cases;
    std::vector<Block> blocks;
    std::vector<int64_t> remaining;
    std::vector<char> used;
    // current launch configuration
    std::vector<WorkItem> work;         // grouped by collision form
    int mode_start[NMODE + 1];          // items of form q: [mode_start[q], mode_start[q + 1])
    std::vector<int> running;           // slots in the work list
    bool dirty;                         // work list / descriptors must be rebuilt
    std::map<int, hipGraphExec_t> graphs;   // by run length, for the current work list
    int64_t launches;
};

namespace {

void drop_graphs(lbm_axi_batch *b)
{
    for (auto &kv : b->graphs)
        (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
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

size_t desc_size(int precision)
{
    return precision == LBM_AXI_FP64 ? sizeof(CaseDesc<double>) : sizeof(CaseDesc<float>);
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
    d.cur0 = c->cur;
    d.pad = 0;
    d.C = c->codec;
    return d;
}

// rebuild the descriptor table and work list for the running cases
int rebuild(lbm_axi_batch *b)
{
    drop_graphs(b);
    b->running.clear();
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s] && b->remaining[s] > 0)
            b->running.push_back(s);
    std::vector<int> order = b->running;
    if (b->schedule == 1)
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
            return (int64_t)b->cases[a]->prm.nr * b->cases[a]->prm.nz >
                   (int64_t)b->cases[c]->prm.nr * b->cases[c]->prm.nz;
        });
    // cases grouped by collision form: each form runs in a kernel of its own
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->cases[a]->P64.mode < b->cases[c]->P64.mode; });
    b->work.clear();
    for (int q = 0; q <= NMODE; ++q) b->mode_start[q] = 0;
    // Workgroup b runs on XCD b % 8 and takes item b (b + k*grid when
    // persistent, grid a multiple of 8), so list position w belongs to XCD
    // w % 8.  Each case's tiles (row-major) are cut into 16 contiguous bands;
    // XCD x takes bands x and x + 8 in turn, interleaved into its positions:
    // all XCDs work on the same case at the same time, and most tile
    // neighbours -- whose rows the ring and the shifted pulls re-read -- sit
    // in the same XCD's L2.  Short band pairs are padded with empty items
    // (slot -1) to keep the alignment.
    constexpr int NBAND = 16;
    for (int s : order) {
        Geom g = geom_for(b->cases[s], b->tile_r);
        int q = g.tiles / NBAND, rem = g.tiles % NBAND;
        int len[8] = {0}, rounds = 0;
        for (int x = 0; x < 8; ++x) {
            len[x] = (q + (x < rem ? 1 : 0)) + (q + (x + 8 < rem ? 1 : 0));
            rounds = std::max(rounds, len[x]);
        }
        for (int l = 0; l < rounds; ++l)
            for (int x = 0; x < 8; ++x) {
                if (l >= len[x]) {
                    b->work.push_back(WorkItem{-1, 0});
                    continue;
                }
                // position l of XCD x: band x first, then band x + 8
                const int first = q + (x < rem ? 1 : 0);
                const int band = l < first ? x : x + 8, k = l < first ? l : l - first;
                const int start = band * q + std::min(band, rem);
                b->work.push_back(WorkItem{s, start + k});
            }
        // items of forms <= this case's form end here (forms are sorted)
        for (int q = b->cases[s]->P64.mode + 1; q <= NMODE; ++q) b->mode_start[q] = (int)b->work.size();
    }
    if ((int64_t)b->work.size() > MAX_WORK) return LBM_AXI_EBUSY;
    // descriptors of every used slot
    size_t ds = desc_size(b->precision);
    std::vector<char> host(ds * b->max_cases, 0);
    for (int s = 0; s < b->max_cases; ++s) {
        if (!b->used[s]) continue;
        if (b->precision == LBM_AXI_FP64) {
            CaseDesc<double> d = make_desc(b, b->cases[s], b->cases[s]->P64, b->tile_r);
            memcpy(host.data() + s * ds, &d, ds);
        } else {
            CaseDesc<float> d = make_desc(b, b->cases[s], b->cases[s]->P32, b->tile_r);
            memcpy(host.data() + s * ds, &d, ds);
        }
    }
    if (hipMemcpyAsync(b->d_descs, host.data(), host.size(), hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return LBM_AXI_EDEVICE;
    if (!b->work.empty() &&
        hipMemcpyAsync(b->d_work, b->work.data(), b->work.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                       b->stream) != hipSuccess)
        return LBM_AXI_EDEVICE;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    b->dirty = false;
    return LBM_AXI_OK;
}

template <typename T, typename R, int TR, int MODE>
void launch_part(lbm_axi_batch *b, int parity, int first, int nwork)
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
        batch_step_kernel_h<TR, MODE><<<grid, TZ * TR, 0, b->stream>>>(
            b->pool, (const CaseDesc<float> *)b->d_descs, b->d_work + first, nwork, parity, b->persistent);
    else
        batch_step_kernel<T, R, TR, MODE><<<grid, TZ * TR, 0, b->stream>>>(
            b->pool, (const CaseDesc<R> *)b->d_descs, b->d_work + first, nwork, parity, b->persistent);
}

template <typename T, typename R, int TR>
void launch_tr(lbm_axi_batch *b, int parity)
{
    const int *ms = b->mode_start;
    const int nw = (int)b->work.size();
    launch_part<T, R, TR, COLLIDE_MRT>(b, parity, ms[0], ms[1] - ms[0]);
    launch_part<T, R, TR, COLLIDE_MRT_UNIT>(b, parity, ms[1], ms[2] - ms[1]);
    launch_part<T, R, TR, COLLIDE_SRT>(b, parity, ms[2], ms[3] - ms[2]);
    launch_part<T, R, TR, COLLIDE_NMRT>(b, parity, ms[3], nw - ms[3]);
}

template <typename T, typename R>
void launch_one(lbm_axi_batch *b, int parity)
{
    switch (b->tile_r) {
    case 2: launch_tr<T, R, 2>(b, parity); break;
    case 4: launch_tr<T, R, 4>(b, parity); break;
    case 16: launch_tr<T, R, 16>(b, parity); break;
    default: launch_tr<T, R, 8>(b, parity); break;
    }
}

void launch_steps(lbm_axi_batch *b, int n)
{
    for (int s = 0; s < n; ++s) {
        if (b->precision == LBM_AXI_FP64)
            launch_one<double, double>(b, s & 1);
        else if (b->precision == LBM_AXI_FP16D)
            launch_one<half_t, float>(b, s & 1);
        else
            launch_one<float, float>(b, s & 1);
    }
}

// n steps of the running cases (graph replay when the length was seen before)
int run_span(lbm_axi_batch *b, int n, bool use_graph)
{
    if (n <= 0 || b->work.empty()) return LBM_AXI_OK;
    if (use_graph && b->stream != nullptr) {
        auto it = b->graphs.find(n);
        if (it == b->graphs.end()) {
            hipGraph_t graph;
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return LBM_AXI_EDEVICE;
            launch_steps(b, n);
            if (hipStreamEndCapture(b->stream, &graph) != hipSuccess) return LBM_AXI_EDEVICE;
            hipGraphExec_t exec;
            if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return LBM_AXI_EDEVICE;
            }
            (void)hipGraphDestroy(graph);
            it = b->graphs.emplace(n, exec).first;
        }
        if (hipGraphLaunch(it->second, b->stream) != hipSuccess) return LBM_AXI_EDEVICE;
    } else {
        launch_steps(b, n);
        if (hipGetLastError() != hipSuccess) return LBM_AXI_EDEVICE;
    }
    b->launches += n;
    // host bookkeeping: time, remaining steps, parity of every running case
    bool flip = (n & 1) != 0;
    for (int s : b->running) {
        lbm_axi_case *c = b->cases[s];
        c->t += n;
        if (flip) c->cur ^= 1;
        b->remaining[s] -= n;
    }
    if (flip) b->dirty = true;     // descriptors carry the parity
    for (int s : b->running)
        if (b->remaining[s] == 0) b->dirty = true;
    return LBM_AXI_OK;
}

int check_slot(const lbm_axi_batch *b, int slot)
{
    if (!b) return LBM_AXI_ESTATE;
    if (slot < 0 || slot >= b->max_cases || !b->used[slot]) return LBM_AXI_ESTATE;
    return LBM_AXI_OK;
}

} // namespace

extern "C" {

size_t lbm_axi_batch_reserved_bytes(int32_t max_cases, int32_t precision)
{
    if (max_cases <= 0 || !valid_precision(precision)) return 0;
    return up(desc_size(precision) * max_cases, ALIGN) + up(sizeof(WorkItem) * (size_t)MAX_WORK, ALIGN);
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
    b->tile_r = 8;
    b->persistent = 0;
    b->schedule = 1;
    int dev = 0;
    b->cu_count = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    b->d_descs = b->pool;
    b->d_work = (WorkItem *)(b->pool + up(desc_size(precision) * max_cases, ALIGN));
    b->heap_off = head;
    b->free_list.push_back(Block{head, pool_bytes - head});
    b->cases.assign(max_cases, nullptr);
    b->blocks.assign(max_cases, Block{0, 0});
    b->remaining.assign(max_cases, 0);
    b->used.assign(max_cases, 0);
    b->dirty = true;
    for (int q = 0; q <= NMODE; ++q) b->mode_start[q] = 0;
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
    int s = -1;
    for (int q = 0; q < b->max_cases; ++q)
        if (!b->used[q]) { s = q; break; }
    if (s < 0) return LBM_AXI_EBUSY;
    Block blk;
    if (!heap_alloc(b, bytes, blk)) return LBM_AXI_EBUSY;
    lbm_axi_case *c = nullptr;
    int rc = lbm_axi_init(params, b->pool + blk.off, blk.size, phi0_host, b->stream, &c);
    if (rc) {
        heap_free(b, blk);
        return rc;
    }
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
    return lbm_axi_moments(b->cases[slot], phi, rho, uz, ur, p, diag);
}

int lbm_axi_batch_get_state(lbm_axi_batch *b, int32_t slot, double *f, double *g, double *aux, int64_t *t)
{
    int rc = check_slot(b, slot);
    if (rc) return rc;
    return lbm_axi_get_state(b->cases[slot], f, g, aux, t);
}

int lbm_axi_batch_release(lbm_axi_batch *b, int32_t slot)
{
    int rc = check_slot(b, slot);
    if (rc) return rc;
    // later work on this memory is ordered after earlier work by the stream
    lbm_axi_destroy(b->cases[slot]);
    heap_free(b, b->blocks[slot]);
    b->cases[slot] = nullptr;
    b->used[slot] = 0;
    b->remaining[slot] = 0;
    b->dirty = true;
    return LBM_AXI_OK;
}

int lbm_axi_batch_set_config(lbm_axi_batch *b, int32_t tile_r, int32_t persistent, int32_t schedule)
{
    if (!b) return LBM_AXI_ESTATE;
    if (tile_r == 0) tile_r = 8;
    if (tile_r != 2 && tile_r != 4 && tile_r != 8 && tile_r != 16) return LBM_AXI_EINVAL;
    if ((persistent != 0 && persistent != 1) || (schedule != 0 && schedule != 1)) return LBM_AXI_EINVAL;
    b->tile_r = tile_r;
    b->persistent = persistent;
    b->schedule = schedule;
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
    if (n_used) *n_used = u;
    if (n_running) *n_running = r;
    if (free_bytes) *free_bytes = fb;
    if (launches) *launches = b->launches;
    return LBM_AXI_OK;
}

int lbm_axi_batch_sync(lbm_axi_batch *b)
{
    if (!b) return LBM_AXI_ESTATE;
    return hipStreamSynchronize(b->stream) == hipSuccess ? LBM_AXI_OK : LBM_AXI_EDEVICE;
}

int lbm_axi_batch_destroy(lbm_axi_batch *b)
{
    if (!b) return LBM_AXI_OK;
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (int s = 0; s < b->max_cases; ++s)
        if (b->used[s]) lbm_axi_destroy(b->cases[s]);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM_AXI_OK;
}

} // extern "C"
