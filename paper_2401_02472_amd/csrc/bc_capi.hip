// Host runtime and C ABI (include/bc.h): graph residency, workspace pool, the
// per-source level loop, and argument checking.
//
// The paper's generated host code copies the graph to the device once and
// returns only the modified property (Section "Backend Optimizations",
// host-device transfer analysis); here too the CSR stays resident in a
// bc_graph_t and only BC (plus debug state on request) comes back.
#include <algorithm>
#include <climits>
#include <cmath>
#include <atomic>
#include <cstring>
#include <mutex>
#include <thread>
#include <new>
#include <vector>

#include "bc.h"
#include "bc_internal.h"

using namespace bcx;

namespace {

constexpr size_t kAlign = 256;
constexpr int kLevelGrid = 2048;  // workgroups per level kernel (8192 wavefronts)
constexpr int kCtrlInts = 4;      // see PlainDev::ctrl

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bc_status from_hip(hipError_t e) {
    if (e == hipSuccess) return BC_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return BC_ERR_OUT_OF_MEMORY;
    return BC_ERR_DEVICE;
}

#define BC_TRY_HIP(expr)                          \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return from_hip(_e); \
    } while (0)

// HIP event pairs bracketing kernel launches of one run (measurement only).
struct LaunchTimer {
    std::vector<hipEvent_t> ev;  // 2 per launch
    std::vector<int> cls;
    size_t used = 0;
    bool on = false;
    hipError_t begin(int c, hipStream_t s) {
        if (!on) return hipSuccess;
        if (2 * used + 2 > ev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                // timing only: no system-scope fence (no cache write-back and
                // invalidation around the timed kernels)
                hipError_t r = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
                if (r != hipSuccess) return r;
                ev.push_back(e);
            }
            cls.push_back(0);
        }
        cls[used] = c;
        return hipEventRecord(ev[2 * used], s);
    }
    hipError_t end(hipStream_t s) {
        if (!on) return hipSuccess;
        hipError_t r = hipEventRecord(ev[2 * used + 1], s);
        ++used;
        return r;
    }
    void destroy() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        ev.clear();
        cls.clear();
    }
};

struct PlainWS {
    LaunchTimer timer;
    unsigned long long *d_stats = nullptr;  // 12 counters (see PlainDev::stats)
    void *block = nullptr;
    size_t bytes = 0;
    PlainDev dev{};
    int32_t *h_ctrl = nullptr;  // pinned mirror of dev.ctrl
    int32_t *d_trunc = nullptr; // per-source truncation flags of a run
    size_t trunc_cap = 0;
    hipEvent_t done = nullptr;  // recorded after the last work that used this workspace
    bool busy = false;
};

// Batched workspace: lane-major sigma / c rows for 64 sources, masks, and a
// level array that grows when a batch runs deeper than it holds.
struct BatchWS {
    LaunchTimer timer;
    unsigned long long *d_stats = nullptr;  // 12 counters (see BatchDev::stats)
    void *block = nullptr;     // vis, sigma, coef, ctrl, bc
    size_t bytes = 0;
    uint64_t *F = nullptr;     // [lcap][n], then the extended-range tables
    double *xs = nullptr;
    unsigned long long *xmax = nullptr;
    int32_t *xe = nullptr;
    int32_t lcap = 0;
    int32_t *d_src = nullptr;  // internal source ids of the run
    size_t src_cap = 0;
    int32_t *h_ctrl = nullptr; // pinned mirror of ctrl
    hipEvent_t done = nullptr;
    bool busy = false;
    BatchDev dev{};
};

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
        if (prev_ != dev) (void)hipSetDevice(dev);
        dev_ = dev;
    }
    ~DeviceGuard() {
        if (prev_ >= 0 && prev_ != dev_) (void)hipSetDevice(prev_);
    }

  private:
    int prev_ = -1, dev_ = -1;
};

}  // namespace

struct bc_graph_s {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *d_row_ptr = nullptr;   // CSR in the internal (degree-descending) order
    int32_t *d_col_idx = nullptr;
    int32_t *d_perm = nullptr;      // caller id -> internal id
    int32_t *d_iperm = nullptr;     // internal id -> caller id
    std::vector<int32_t> h_perm;    // same, on the host (source mapping)
    int32_t b3_end = 0, b2_end = 0, b1_end = 0;  // bucket id ranges
    // batched-path work items (vertices of degree > 64 in kChunk-arc chunks)
    int32_t big_end = 0, multi_end = 0;
    uint32_t items = 0;
    int2 *d_item_info = nullptr;
    uint32_t *d_item_first = nullptr;
    // directed graphs: the reversed CSR (arcs into each vertex, internal order)
    // and its chunk items, for the forward pass; for undirected graphs these
    // point at the arrays above
    bool directed = false;
    uint32_t items_in = 0;
    int32_t *d_row_ptr_in = nullptr;
    int32_t *d_col_idx_in = nullptr;
    int2 *d_item_info_in = nullptr;
    uint32_t *d_item_first_in = nullptr;
    uint64_t total_chunks3 = 0;
    // single-source shortest paths: arc weights (internal arc order; NULL =
    // every arc weighs 1) and a workspace used by one call at a time
    int32_t *d_weight = nullptr;
    std::mutex sssp_mu;
    struct Sssp {
        int32_t *dist = nullptr, *stamp = nullptr, *flags = nullptr;
        int32_t *h_flags = nullptr;               // pinned mirror of one flag block
        unsigned long long *d_stats = nullptr;    // 12 counters ([9..11] used)
    } sssp;
    // PageRank workspace (one call at a time)
    std::mutex pr_mu;
    struct Pr {
        void *block = nullptr;        // ranks, shares, partials, slots
        double *diff = nullptr;       // [cap]
        int32_t cap = 0;
        double *h_diff = nullptr;     // pinned, 8 entries
    } prw;  // chunk slots needed by bucket-3 vertices of one source
    size_t device_bytes = 0;
    std::mutex mu;
    std::vector<PlainWS *> plain_pool;
    std::vector<BatchWS *> batch_pool;
    std::atomic<int32_t> depth_hint{16};  // levels launched per source without polling
    std::atomic<int32_t> batch_depth_hint{16};  // levels of the last batched run
    // settings for BC_MODE_AUTO and zero option fields (bc_autotune stores its
    // choice here)
    std::atomic<int32_t> tuned_width{kWave};
    std::atomic<int32_t> tuned_sparse_div{kDefaultSparseDiv};
    std::atomic<int32_t> tuned_min_batched{16};
    // set once a path count did not fit the batched path's uint32 sigma rows:
    // later batches start with double rows
    std::atomic<bool> sigma_wide{false};
    // set once a path count overflowed double: later batches keep level-scaled
    // counts (extended range, host-driven loop only)
    std::atomic<bool> sigma_ext{false};
    // internal streams for batches run at once (created on first use)
    std::mutex stream_mu;
    std::vector<hipStream_t> streams;
    // workspaces of the device-resident level loop (one per batch of a launch)
    std::mutex fused_mu;
    struct Fused {
        void *block = nullptr;
        size_t bytes = 0;
        int32_t cap = 0, lcap = 0;
        BatchDev *d_devs = nullptr;
        int32_t *h_ctrl = nullptr;  // pinned [cap][kCtlInts]
        int32_t *d_ctrl = nullptr;  // [cap][kCtlInts]
        double *d_bc = nullptr;     // [cap][n] per-batch BC (internal order)
        double *d_total = nullptr;  // [n] running BC total of a run (not in the pool)
        int32_t *d_lanes = nullptr;
        size_t lanes_cap = 0;
        int2 *d_batches = nullptr;
        unsigned long long *d_stats = nullptr;  // 12 work counters (as BatchDev::stats)
        std::vector<BatchDev> h_devs;
    } fused;
    // hop distances (internal order, -1 unreached) from two landmarks: the
    // highest-degree vertex and the vertex farthest from it; batches are formed
    // from sources sorted by them
    std::mutex land_mu;
    bool land_ready = false;
    std::vector<int32_t> land1, land2;
    std::atomic<int32_t> profiling{0};
    std::mutex prof_mu;
    bc_profile prof{};
};

namespace {

void fused_release(bc_graph_s *g);

size_t plain_ws_bytes(const bc_graph_s *g) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    size_t b = 0;
    b += align_up(((n + 15) / 16) * sizeof(uint32_t));        // lev3
    b += align_up(((n + 15) / 16) * 16);                      // nextmap
    b += 2 * align_up(n * sizeof(double));                    // sigma, coef
    b += 5 * align_up(n * sizeof(int32_t));                   // 4 queues + chunk slots
    b += align_up(std::max<uint64_t>(g->total_chunks3, 1) * sizeof(double));  // partial
    b += align_up((n + 2) * sizeof(LevelRec));                // lvl
    b += align_up(kCtrlInts * sizeof(int32_t));               // ctrl
    b += align_up(n * sizeof(double));                        // bc (internal order)
    b += align_up(12 * sizeof(unsigned long long));           // work counters
    return b;
}

bc_status plain_ws_create(bc_graph_s *g, PlainWS **out) {
    PlainWS *ws = new (std::nothrow) PlainWS();
    if (!ws) return BC_ERR_OUT_OF_MEMORY;
    ws->bytes = plain_ws_bytes(g);
    hipError_t e = hipMalloc(&ws->block, ws->bytes);
    if (e != hipSuccess) {
        delete ws;
        return from_hip(e);
    }
    e = hipHostMalloc((void **)&ws->h_ctrl, kCtrlInts * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipFree(ws->block);
        if (ws->h_ctrl) (void)hipHostFree(ws->h_ctrl);
        delete ws;
        return from_hip(e);
    }
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    char *p = (char *)ws->block;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align_up(bytes);
        return (void *)r;
    };
    PlainDev &d = ws->dev;
    d.n = g->n;
    d.row_ptr = g->d_row_ptr;
    d.col_idx = g->d_col_idx;
    d.lev3 = (uint32_t *)take(((n + 15) / 16) * sizeof(uint32_t));
    d.nextmap = (uint8_t *)take(((n + 15) / 16) * 16);
    d.sigma = (double *)take(n * sizeof(double));
    d.coef = (double *)take(n * sizeof(double));
    for (int b = 0; b < kBuckets; ++b) d.q[b] = (int32_t *)take(n * sizeof(int32_t));
    d.q3c = (int32_t *)take(n * sizeof(int32_t));
    d.partial = (double *)take(std::max<uint64_t>(g->total_chunks3, 1) * sizeof(double));
    d.lvl = (LevelRec *)take((n + 2) * sizeof(LevelRec));
    d.ctrl = (int32_t *)take(kCtrlInts * sizeof(int32_t));
    d.bc = (double *)take(n * sizeof(double));
    ws->d_stats = (unsigned long long *)take(12 * sizeof(unsigned long long));
    d.stats = nullptr;
    d.b3_end = g->b3_end;
    d.b2_end = g->b2_end;
    d.b1_end = g->b1_end;
    *out = ws;
    return BC_OK;
}

void plain_ws_destroy(PlainWS *ws) {
    if (!ws) return;
    if (ws->done) {
        (void)hipEventSynchronize(ws->done);
        (void)hipEventDestroy(ws->done);
    }
    ws->timer.destroy();
    if (ws->d_trunc) (void)hipFree(ws->d_trunc);
    if (ws->block) (void)hipFree(ws->block);
    if (ws->h_ctrl) (void)hipHostFree(ws->h_ctrl);
    delete ws;
}

// Take an idle workspace (the caller's stream then waits for its previous
// user's work), or make a new one.
bc_status plain_acquire(bc_graph_s *g, hipStream_t stream, PlainWS **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (PlainWS *ws : g->plain_pool) {
            if (!ws->busy) {
                ws->busy = true;
                *out = ws;
                BC_TRY_HIP(hipStreamWaitEvent(stream, ws->done, 0));
                return BC_OK;
            }
        }
    }
    PlainWS *ws = nullptr;
    bc_status st = plain_ws_create(g, &ws);
    if (st != BC_OK) return st;
    ws->busy = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->plain_pool.push_back(ws);
    *out = ws;
    return BC_OK;
}

void plain_release(bc_graph_s *g, PlainWS *ws, hipStream_t stream) {
    (void)hipEventRecord(ws->done, stream);
    std::lock_guard<std::mutex> lk(g->mu);
    ws->busy = false;
}

struct SourceState {
    int32_t *dist = nullptr;   // device, optional export
    double *sigma = nullptr;   // device, optional export
    double *delta = nullptr;   // device, optional export
};

// Add a finished run's event-timed launches and device work counters to the
// graph's measurement totals (the run's stream has been synchronised).
void accumulate_profile(bc_graph_s *g, LaunchTimer &timer, const unsigned long long *d_stats) {
    bc_profile add{};
    for (size_t i = 0; i < timer.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, timer.ev[2 * i], timer.ev[2 * i + 1]) == hipSuccess)
            add.ms[timer.cls[i]] += ms;
        add.launches[timer.cls[i]] += 1;
    }
    unsigned long long cnt[12];
    if (hipMemcpy(cnt, d_stats, sizeof(cnt), hipMemcpyDeviceToHost) == hipSuccess) {
        add.owners[BC_PROF_FORWARD] = (int64_t)cnt[0];
        add.arcs[BC_PROF_FORWARD] = (int64_t)cnt[1];
        add.hits[BC_PROF_FORWARD] = (int64_t)cnt[2];
        add.owners[BC_PROF_COMPACT] = (int64_t)cnt[3];
        add.owners[BC_PROF_REVERSE] = (int64_t)cnt[6];
        add.arcs[BC_PROF_REVERSE] = (int64_t)cnt[7];
        add.hits[BC_PROF_REVERSE] = (int64_t)cnt[8];
        add.owners[BC_PROF_SSSP] = (int64_t)cnt[9];
        add.arcs[BC_PROF_SSSP] = (int64_t)cnt[10];
        add.hits[BC_PROF_SSSP] = (int64_t)cnt[11];
    }
    std::lock_guard<std::mutex> lk(g->prof_mu);
    for (int c = 0; c < BC_PROF_CLASSES; ++c) {
        g->prof.launches[c] += add.launches[c];
        g->prof.ms[c] += add.ms[c];
        g->prof.owners[c] += add.owners[c];
        g->prof.arcs[c] += add.arcs[c];
        g->prof.hits[c] += add.hits[c];
    }
    g->prof.runs += 1;
}

// Forward pass of one source with the host polling the deepest discovered
// level after each chunk of launched levels (used for state exports and for
// sources that outgrew the speculative level count).
bc_status plain_forward_polled(bc_graph_s *g, PlainWS *ws, int32_t s, int32_t chunk0,
                               hipStream_t stream, int32_t *deepest_out) {
    const PlainDev &d = ws->dev;
    BC_TRY_HIP(plain_init_source(d, s, stream));
    int32_t L0 = 0;
    int32_t K = std::max(1, chunk0);
    for (;;) {
        const int32_t Lend = (int32_t)std::min<int64_t>((int64_t)L0 + K, g->n);
        for (int32_t L = L0; L < Lend; ++L) {
            BC_TRY_HIP(ws->timer.begin(BC_PROF_FORWARD, stream));
            BC_TRY_HIP(plain_forward_level(d, L, kLevelGrid, stream));
            BC_TRY_HIP(ws->timer.end(stream));
            BC_TRY_HIP(ws->timer.begin(BC_PROF_COMPACT, stream));
            BC_TRY_HIP(plain_compact(d, L, -1, nullptr, stream));
            BC_TRY_HIP(ws->timer.end(stream));
        }
        BC_TRY_HIP(hipMemcpyAsync(ws->h_ctrl, d.ctrl, kCtrlInts * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, stream));
        BC_TRY_HIP(hipStreamSynchronize(stream));
        const int32_t deepest = ws->h_ctrl[0];
        if (deepest < Lend || Lend >= g->n) {
            *deepest_out = deepest;
            return BC_OK;
        }
        L0 = Lend;
        K = std::min(K * 2, 1024);
    }
}

// Reverse pass of one source, levels hi..1 (hi = deepest level when known,
// else the deepest launched level with `known` false).
hipError_t plain_reverse(PlainWS *ws, int32_t hi, bool known, double *dout, hipStream_t stream) {
    const PlainDev &d = ws->dev;
    for (int32_t L = hi; L >= 1; --L) {
        const int deepest = known ? (L == hi ? 1 : 0) : -1;
        hipError_t e = ws->timer.begin(BC_PROF_REVERSE, stream);
        if (e == hipSuccess) e = plain_backward_level(d, L, deepest, kLevelGrid, dout, stream);
        if (e == hipSuccess) e = ws->timer.end(stream);
        if (e == hipSuccess && !(known && L == hi)) {
            e = ws->timer.begin(BC_PROF_FINISH, stream);
            if (e == hipSuccess) e = plain_finish_reverse(d, L, dout, stream);
            if (e == hipSuccess) e = ws->timer.end(stream);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One source without waiting for the device: K forward steps and K-1 reverse
// steps are enqueued; steps past the deepest level find empty queues and exit.
// If the source has more than K levels, the compaction of level K-1 marks it
// truncated, its reverse steps do nothing, and *trunc_flag is set so that the
// host runs it again.
hipError_t plain_source_speculative(PlainWS *ws, int32_t s, int32_t K, int32_t *trunc_flag,
                                    hipStream_t stream) {
    const PlainDev &d = ws->dev;
    hipError_t e = plain_init_source(d, s, stream);
    for (int32_t L = 0; e == hipSuccess && L < K; ++L) {
        e = ws->timer.begin(BC_PROF_FORWARD, stream);
        if (e == hipSuccess) e = plain_forward_level(d, L, kLevelGrid, stream);
        if (e == hipSuccess) e = ws->timer.end(stream);
        if (e == hipSuccess) e = ws->timer.begin(BC_PROF_COMPACT, stream);
        if (e == hipSuccess) e = plain_compact(d, L, K - 1, trunc_flag, stream);
        if (e == hipSuccess) e = ws->timer.end(stream);
    }
    if (e == hipSuccess) e = plain_reverse(ws, K - 1, false, nullptr, stream);
    return e;
}

// Export buffers of one source in internal order (device temporaries).
struct ExportTmp {
    int32_t *dist = nullptr;
    double *sigma = nullptr;
    double *delta = nullptr;
};

bc_status plain_run(bc_graph_s *g, const int32_t *sources, int32_t k, double *bc_out,
                    const bc_options *opt, hipStream_t stream, const SourceState *exp,
                    const ExportTmp *tmp) {
    PlainWS *ws = nullptr;
    bc_status st = plain_acquire(g, stream, &ws);
    if (st != BC_OK) return st;
    const bool prof = g->profiling.load() != 0;
    ws->dev.stats = prof ? ws->d_stats : nullptr;
    ws->timer.on = prof;
    ws->timer.used = 0;
    const PlainDev &d = ws->dev;
    bc_status result = BC_OK;
    auto fail = [&](bc_status s2) {
        plain_release(g, ws, stream);
        return s2;
    };
    const int32_t user_chunk = opt ? opt->level_chunk : 0;
    const bool polled = exp != nullptr || user_chunk > 0;
    if (!polled && (size_t)k > ws->trunc_cap) {
        if (ws->d_trunc) (void)hipFree(ws->d_trunc);
        ws->d_trunc = nullptr;
        ws->trunc_cap = 0;
        hipError_t ea = hipMalloc(&ws->d_trunc, (size_t)k * sizeof(int32_t));
        if (ea != hipSuccess) return fail(from_hip(ea));
        ws->trunc_cap = (size_t)k;
    }
    hipError_t e = hipMemsetAsync(d.bc, 0, (size_t)g->n * sizeof(double), stream);
    if (e == hipSuccess) e = plain_reset_run(d, stream);
    if (e == hipSuccess && prof)
        e = hipMemsetAsync(ws->d_stats, 0, 12 * sizeof(unsigned long long), stream);
    if (e == hipSuccess && !polled && k > 0)
        e = hipMemsetAsync(ws->d_trunc, 0, (size_t)k * sizeof(int32_t), stream);
    if (e != hipSuccess) return fail(from_hip(e));

    std::vector<int32_t> redo;  // sources run in polled mode
    if (polled) {
        for (int32_t i = 0; i < k; ++i) redo.push_back(i);
    } else {
        const int32_t K = (int32_t)std::min<int64_t>(std::max(2, g->depth_hint.load()), g->n);
        const int32_t period = std::max(1, g->profiling.load());
        for (int32_t i = 0; i < k && e == hipSuccess; ++i) {
            // measurement covers every period-th source only
            const bool sample = prof && (i % period) == 0;
            ws->timer.on = sample;
            ws->dev.stats = sample ? ws->d_stats : nullptr;
            e = plain_source_speculative(ws, g->h_perm[(size_t)sources[i]], K, ws->d_trunc + i,
                                         stream);
        }
        ws->timer.on = prof;
        ws->dev.stats = prof ? ws->d_stats : nullptr;
        if (e != hipSuccess) return fail(from_hip(e));
        if (k > 0) {
            std::vector<int32_t> trunc((size_t)k);
            e = hipMemcpyAsync(trunc.data(), ws->d_trunc, (size_t)k * sizeof(int32_t),
                               hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail(from_hip(e));
            for (int32_t i = 0; i < k; ++i)
                if (trunc[(size_t)i]) redo.push_back(i);
        }
    }
    for (int32_t i : redo) {
        const int32_t s_int = g->h_perm[(size_t)sources[i]];
        const int32_t chunk = user_chunk > 0 ? user_chunk : std::max(2, g->depth_hint.load());
        int32_t deepest = 0;
        st = plain_forward_polled(g, ws, s_int, chunk, stream, &deepest);
        if (st != BC_OK) return fail(st);
        if (deepest + 2 > g->depth_hint.load()) g->depth_hint.store(deepest + 2);
        if (exp) {
            e = plain_export_fill(g->n, tmp->dist, tmp->sigma, tmp->delta, stream);
            if (e != hipSuccess) return fail(from_hip(e));
        }
        e = plain_reverse(ws, deepest, true, exp ? tmp->delta : nullptr, stream);
        if (e != hipSuccess) return fail(from_hip(e));
        if (exp) {
            e = plain_export_levels(d, deepest, tmp->dist, tmp->sigma, stream);
            if (e == hipSuccess && exp[i].dist) e = gather_i32(g->n, g->d_perm, tmp->dist, exp[i].dist, stream);
            if (e == hipSuccess && exp[i].sigma) e = gather_f64(g->n, g->d_perm, tmp->sigma, exp[i].sigma, stream);
            if (e == hipSuccess && exp[i].delta) e = gather_f64(g->n, g->d_perm, tmp->delta, exp[i].delta, stream);
            if (e != hipSuccess) return fail(from_hip(e));
        }
    }
    e = gather_f64(g->n, g->d_perm, d.bc, bc_out, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws->h_ctrl, d.ctrl, kCtrlInts * sizeof(int32_t), hipMemcpyDeviceToHost,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(from_hip(e));
    if (ws->h_ctrl[1] != 0) result = BC_ERR_RANGE;
    {
        // next run: launch two levels more than the deepest seen
        const int32_t seen = ws->h_ctrl[3] + 2;
        if (!polled && seen != g->depth_hint.load()) g->depth_hint.store(std::max(seen, 2));
    }
    if (prof) accumulate_profile(g, ws->timer, ws->d_stats);
    plain_release(g, ws, stream);
    return result;
}

// Device temporaries for the single-source export (internal order).
struct ExportAlloc {
    ExportTmp t;
    hipError_t alloc(size_t n) {
        hipError_t e = hipMalloc(&t.dist, n * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&t.sigma, n * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&t.delta, n * sizeof(double));
        return e;
    }
    ~ExportAlloc() {
        if (t.dist) (void)hipFree(t.dist);
        if (t.sigma) (void)hipFree(t.sigma);
        if (t.delta) (void)hipFree(t.delta);
    }
};

constexpr int kBatchCtrlInts = kCtlInts;

size_t batch_ws_bytes(const bc_graph_s *g) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    size_t b = 0;
    b += align_up(n * sizeof(uint64_t));                 // vis
    b += 2 * align_up(n * kWave * sizeof(double));       // sigma, coef rows
    b += align_up(kBatchCtrlInts * sizeof(int32_t));     // ctrl
    b += align_up(n * sizeof(double));                   // bc
    b += align_up((size_t)std::max(g->multi_end, 1) * sizeof(uint64_t));  // reach
    b += align_up((size_t)std::max(g->multi_end, 1) * kWave * sizeof(double));  // hub sums
    b += align_up((size_t)std::max<uint32_t>(g->items, 1) * kWave * sizeof(double));  // partial
    b += align_up(12 * sizeof(unsigned long long));     // work counters
    b += align_up(n * sizeof(int32_t));                  // candidate list
    // item list of the sparse step (the forward pass's items)
    b += align_up((size_t)std::max<uint32_t>(g->items_in, 1) * sizeof(int32_t));
    b += align_up((size_t)kFrontSets * kFrontWaves * 2 * sizeof(unsigned long long));
    b += align_up(((n + 15) / 16) * 16);                 // candidate marks
    return b;
}

// F[lcap][n] and the extended-range tables xs, xmax, xe ([lcap][64] each).
size_t batch_level_bytes(const bc_graph_s *g, int32_t lcap) {
    return (size_t)lcap * ((size_t)std::max<int32_t>(g->n, 1) * sizeof(uint64_t) +
                           kWave * (sizeof(double) + sizeof(unsigned long long) + sizeof(int32_t)));
}

void batch_ws_destroy(BatchWS *ws) {
    if (!ws) return;
    if (ws->done) {
        (void)hipEventSynchronize(ws->done);
        (void)hipEventDestroy(ws->done);
    }
    ws->timer.destroy();
    if (ws->F) (void)hipFree(ws->F);
    if (ws->d_src) (void)hipFree(ws->d_src);
    if (ws->block) (void)hipFree(ws->block);
    if (ws->h_ctrl) (void)hipHostFree(ws->h_ctrl);
    delete ws;
}

bc_status batch_ws_create(bc_graph_s *g, BatchWS **out) {
    BatchWS *ws = new (std::nothrow) BatchWS();
    if (!ws) return BC_ERR_OUT_OF_MEMORY;
    ws->bytes = batch_ws_bytes(g);
    hipError_t e = hipMalloc(&ws->block, ws->bytes);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&ws->h_ctrl, kBatchCtrlInts * sizeof(int32_t),
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ws->done, hipEventDisableTiming);
    if (e != hipSuccess) {
        batch_ws_destroy(ws);
        return from_hip(e);
    }
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    char *p = (char *)ws->block;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align_up(bytes);
        return (void *)r;
    };
    BatchDev &d = ws->dev;
    d.n = g->n;
    d.row_ptr = g->d_row_ptr;
    d.col_idx = g->d_col_idx;
    d.vis = (uint64_t *)take(n * sizeof(uint64_t));
    d.sigma = (double *)take(n * kWave * sizeof(double));
    d.sigma32 = reinterpret_cast<uint32_t *>(d.sigma);
    d.narrow = 1;
    d.coef = (double *)take(n * kWave * sizeof(double));
    d.ctrl = (int32_t *)take(kBatchCtrlInts * sizeof(int32_t));
    d.bc = (double *)take(n * sizeof(double));
    d.reach = (uint64_t *)take((size_t)std::max(g->multi_end, 1) * sizeof(uint64_t));
    d.hubsig = (double *)take((size_t)std::max(g->multi_end, 1) * kWave * sizeof(double));
    d.partial = (double *)take((size_t)std::max<uint32_t>(g->items, 1) * kWave * sizeof(double));
    d.big_end = g->big_end;
    d.multi_end = g->multi_end;
    d.items = g->items;
    d.item_info = g->d_item_info;
    d.item_first = g->d_item_first;
    d.items_in = g->items_in;
    d.row_ptr_in = g->d_row_ptr_in;
    d.col_idx_in = g->d_col_idx_in;
    d.item_info_in = g->d_item_info_in;
    d.item_first_in = g->d_item_first_in;
    ws->d_stats = (unsigned long long *)take(12 * sizeof(unsigned long long));
    d.stats = nullptr;
    d.clist = (int32_t *)take(n * sizeof(int32_t));
    d.ilist = (int32_t *)take((size_t)std::max<uint32_t>(g->items_in, 1) * sizeof(int32_t));
    d.cand = (uint8_t *)take(((n + 15) / 16) * 16);
    d.front = (unsigned long long *)take((size_t)kFrontSets * kFrontWaves * 2 *
                                         sizeof(unsigned long long));
    d.nnz = g->nnz;
    d.sparse_arcs = g->nnz / kDefaultSparseDiv;
    d.F = nullptr;
    d.lcap = 0;
    *out = ws;
    return BC_OK;
}

bc_status batch_grow_levels(bc_graph_s *g, BatchWS *ws, int32_t lcap) {
    if (lcap <= ws->lcap) return BC_OK;
    if (ws->F) (void)hipFree(ws->F);
    ws->F = nullptr;
    ws->lcap = 0;
    BC_TRY_HIP(hipMalloc(&ws->F, batch_level_bytes(g, lcap)));
    ws->lcap = lcap;
    ws->dev.F = ws->F;
    ws->dev.lcap = lcap;
    ws->xs = (double *)(ws->F + (size_t)lcap * (size_t)std::max<int32_t>(g->n, 1));
    ws->xmax = (unsigned long long *)(ws->xs + (size_t)lcap * kWave);
    ws->xe = (int32_t *)(ws->xmax + (size_t)lcap * kWave);
    return BC_OK;
}

bc_status batch_acquire(bc_graph_s *g, hipStream_t stream, BatchWS **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (BatchWS *ws : g->batch_pool) {
            if (!ws->busy) {
                ws->busy = true;
                *out = ws;
                BC_TRY_HIP(hipStreamWaitEvent(stream, ws->done, 0));
                return BC_OK;
            }
        }
    }
    BatchWS *ws = nullptr;
    bc_status st = batch_ws_create(g, &ws);
    if (st != BC_OK) return st;
    ws->busy = true;
    std::lock_guard<std::mutex> lk(g->mu);
    g->batch_pool.push_back(ws);
    *out = ws;
    return BC_OK;
}

void batch_release(bc_graph_s *g, BatchWS *ws, hipStream_t stream) {
    (void)hipEventRecord(ws->done, stream);
    std::lock_guard<std::mutex> lk(g->mu);
    ws->busy = false;
}

// Hop distances from internal vertex s (internal order) with the plain path.
bc_status bfs_levels(bc_graph_s *g, int32_t s, std::vector<int32_t> &out) {
    PlainWS *ws = nullptr;
    bc_status st = plain_acquire(g, nullptr, &ws);
    if (st != BC_OK) return st;
    ws->timer.on = false;
    ws->dev.stats = nullptr;
    int32_t *d_dist = nullptr;
    hipError_t e = hipMalloc(&d_dist, (size_t)g->n * sizeof(int32_t));
    int32_t deepest = 0;
    if (e == hipSuccess) e = plain_reset_run(ws->dev, nullptr);
    if (e == hipSuccess) st = plain_forward_polled(g, ws, s, 16, nullptr, &deepest);
    else st = from_hip(e);
    if (st == BC_OK) {
        e = plain_export_fill(g->n, d_dist, nullptr, nullptr, nullptr);
        if (e == hipSuccess) e = plain_export_levels(ws->dev, deepest, d_dist, nullptr, nullptr);
        out.resize((size_t)g->n);
        if (e == hipSuccess)
            e = hipMemcpy(out.data(), d_dist, (size_t)g->n * sizeof(int32_t), hipMemcpyDeviceToHost);
        st = from_hip(e);
    }
    if (d_dist) (void)hipFree(d_dist);
    plain_release(g, ws, nullptr);
    return st;
}

bc_status ensure_landmarks(bc_graph_s *g) {
    std::lock_guard<std::mutex> lk(g->land_mu);
    if (g->land_ready) return BC_OK;
    if (g->n == 0) {
        g->land_ready = true;
        return BC_OK;
    }
    bc_status st = bfs_levels(g, 0, g->land1);
    if (st != BC_OK) return st;
    int32_t far = 0;
    for (int32_t v = 0; v < g->n; ++v)
        if (g->land1[(size_t)v] > g->land1[(size_t)far]) far = v;
    st = bfs_levels(g, far, g->land2);
    if (st != BC_OK) return st;
    g->land_ready = true;
    return BC_OK;
}

// One batch of a batched run: lanes [first, first + nlanes) of the run's
// (internal-id) source list; with nseg > 0, its lanes feed nseg request
// outputs described from seg_first on in the run's segment tables.
struct BatchPlan {
    int32_t first, nlanes;
    int32_t seg_first, nseg;
};

// Execute a batch plan.  s_int: internal source ids in lane order.  With
// nseg == 0 everywhere, BC accumulates in the workspace and is gathered into
// bc_out (caller order); otherwise each segment's output (caller order,
// zeroed by the caller) receives its lanes' dependencies.  export_row maps a
// lane of the run to the dist / sigma export row (or NULL: no export).
bc_status run_batch_plan(bc_graph_s *g, const std::vector<int32_t> &s_int,
                         const std::vector<BatchPlan> &plan,
                         const std::vector<int32_t> &seg_start,  // per segment table: nseg+1
                         const std::vector<double *> &seg_out, double *bc_out,
                         hipStream_t stream, const int32_t *export_row, int32_t *dist,
                         double *sigma, int32_t sparse_div) {
    BatchWS *ws = nullptr;
    bc_status st = batch_acquire(g, stream, &ws);
    if (st != BC_OK) return st;
    auto fail = [&](bc_status s2) {
        batch_release(g, ws, stream);
        return s2;
    };
    const int32_t n = g->n;
    const int32_t k = (int32_t)s_int.size();
    const bool prof = g->profiling.load() != 0;
    ws->dev.stats = prof ? ws->d_stats : nullptr;
    ws->timer.on = prof;
    ws->timer.used = 0;
    // frontier arcs below which a level takes the sparse step (0: never)
    ws->dev.sparse_arcs = sparse_div < 0 ? 0 : g->nnz / std::max(sparse_div, 1);
    if (prof) {
        hipError_t ez = hipMemsetAsync(ws->d_stats, 0, 12 * sizeof(unsigned long long), stream);
        if (ez != hipSuccess) return fail(from_hip(ez));
    }
    st = batch_grow_levels(g, ws, std::max(ws->lcap, g->batch_depth_hint.load() + 8));
    if (st != BC_OK) return fail(st);
    // device copies of the lane sources and the segment tables
    const size_t seg_ints = seg_start.size(), seg_ptrs = seg_out.size();
    const size_t need = (size_t)k * sizeof(int32_t) + seg_ints * sizeof(int32_t) +
                        seg_ptrs * sizeof(double *) + 64;
    if (need > ws->src_cap) {
        if (ws->d_src) (void)hipFree(ws->d_src);
        ws->d_src = nullptr;
        ws->src_cap = 0;
        hipError_t ea = hipMalloc(&ws->d_src, need);
        if (ea != hipSuccess) return fail(from_hip(ea));
        ws->src_cap = need;
    }
    int32_t *d_lanes = ws->d_src;
    int32_t *d_seg_start = d_lanes + k;
    double **d_seg_out =
        (double **)(((uintptr_t)(d_seg_start + seg_ints) + 15) & ~(uintptr_t)15);
    int32_t *x_dist = nullptr;
    double *x_sigma = nullptr;
    struct Tmp {
        int32_t *&a;
        double *&b;
        ~Tmp() {
            if (a) (void)hipFree(a);
            if (b) (void)hipFree(b);
        }
    } tmp_guard{x_dist, x_sigma};
    hipError_t e = hipSuccess;
    if (dist) e = hipMalloc(&x_dist, (size_t)kWave * (size_t)n * sizeof(int32_t));
    if (e == hipSuccess && sigma) e = hipMalloc(&x_sigma, (size_t)kWave * (size_t)n * sizeof(double));
    if (e == hipSuccess && k > 0)
        e = hipMemcpyAsync(d_lanes, s_int.data(), (size_t)k * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && seg_ints)
        e = hipMemcpyAsync(d_seg_start, seg_start.data(), seg_ints * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && seg_ptrs)
        e = hipMemcpyAsync(d_seg_out, seg_out.data(), seg_ptrs * sizeof(double *),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && bc_out)
        e = hipMemsetAsync(ws->dev.bc, 0, (size_t)n * sizeof(double), stream);
    if (e == hipSuccess)  // the batches' kernels only ever set the range flag
        e = hipMemsetAsync(ws->dev.ctrl + kCtlRange, 0, sizeof(int32_t), stream);
    if (e != hipSuccess) return fail(from_hip(e));
    int32_t range = 0, run_depth = 0;
    // measurement covers the launches of every stride-th level only (all of
    // them with stride 1): events around every launch slow deep graphs' short
    // level steps
    const int32_t stride = std::max(1, g->profiling.load());
    auto measure = [&](int32_t L) {
        const bool m = prof && L % stride == 0;
        ws->timer.on = m;
        ws->dev.stats = m ? ws->d_stats : nullptr;
    };
    for (size_t bi = 0; bi < plan.size();) {
        const BatchPlan &bp = plan[bi];
        const int32_t nl = bp.nlanes;
        const uint64_t full = nl >= 64 ? ~0ull : ((1ull << nl) - 1ull);
        BatchDev &d = ws->dev;
        d.nseg = bp.nseg;
        d.seg_start = bp.nseg ? d_seg_start + bp.seg_first : nullptr;
        d.seg_out = bp.nseg ? d_seg_out + (bp.seg_first - (int32_t)bi) : nullptr;
        d.iperm = g->d_iperm;
        const bool ext = g->sigma_ext.load();
        d.narrow = (ext || g->sigma_wide.load()) ? 0 : 1;
        d.xs = ext ? ws->xs : nullptr;
        d.xmax = ext ? ws->xmax : nullptr;
        d.xe = ext ? ws->xe : nullptr;
        e = batch_start(d, d_lanes + bp.first, nl, stream);
        if (e != hipSuccess) return fail(from_hip(e));
        int32_t deepest = 0;
        bool restart = false;
        int32_t L0 = 0;
        for (;;) {
            const int32_t K = std::max(2, g->batch_depth_hint.load() + 2);
            const int32_t Lend = std::min(L0 + K, ws->lcap - 1);
            for (int32_t L = L0; L < Lend && e == hipSuccess; ++L) {
                measure(L);
                e = ws->timer.begin(BC_PROF_FORWARD, stream);
                if (e == hipSuccess) e = batch_forward(d, L, full, stream);
                if (e == hipSuccess) e = ws->timer.end(stream);
                if (e == hipSuccess) e = ws->timer.begin(BC_PROF_COMPACT, stream);
                if (e == hipSuccess) e = batch_forward_done(d, L, full, stream);
                if (e == hipSuccess) e = ws->timer.end(stream);
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(ws->h_ctrl, d.ctrl, kBatchCtrlInts * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, stream);
            if (e == hipSuccess) e = hipStreamSynchronize(stream);
            if (e != hipSuccess) return fail(from_hip(e));
            deepest = ws->h_ctrl[0];
            if (ws->h_ctrl[kCtlNarrow]) {  // a path count needs double rows: run again
                g->sigma_wide.store(true);
                restart = true;
                break;
            }
            if (ws->h_ctrl[kCtlRange] && !ext) {  // beyond double: run again level-scaled
                g->sigma_wide.store(true);
                g->sigma_ext.store(true);
                e = hipMemsetAsync(d.ctrl + kCtlRange, 0, sizeof(int32_t), stream);
                if (e != hipSuccess) return fail(from_hip(e));
                restart = true;
                break;
            }
            if (ws->h_ctrl[2]) {  // level array full: grow it and run the batch again
                st = batch_grow_levels(g, ws, ws->lcap * 2);
                if (st != BC_OK) return fail(st);
                restart = true;
                break;
            }
            if (deepest < Lend || Lend >= n) break;
            L0 = Lend;
        }
        if (restart) continue;
        for (int32_t L = deepest; L >= 1 && e == hipSuccess; --L) {
            measure(L);
            if (L != deepest) {
                e = ws->timer.begin(BC_PROF_REVERSE, stream);
                if (e == hipSuccess) e = batch_reverse(d, L, stream);
                if (e == hipSuccess) e = ws->timer.end(stream);
            }
            if (e == hipSuccess) e = ws->timer.begin(BC_PROF_FINISH, stream);
            if (e == hipSuccess) e = batch_finalize(d, L, L == deepest, stream);
            if (e == hipSuccess) e = ws->timer.end(stream);
        }
        if (e == hipSuccess && export_row && (dist || sigma)) {
            e = batch_export(d, deepest, nl, x_dist, x_sigma, stream);
            for (int32_t s2 = 0; s2 < nl && e == hipSuccess; ++s2) {
                const size_t row = (size_t)export_row[bp.first + s2] * (size_t)n;
                if (dist) e = gather_i32(n, g->d_perm, x_dist + (size_t)s2 * n, dist + row, stream);
                if (e == hipSuccess && sigma)
                    e = gather_f64(n, g->d_perm, x_sigma + (size_t)s2 * n, sigma + row, stream);
            }
        }
        if (e != hipSuccess) return fail(from_hip(e));
        range |= ws->h_ctrl[1];
        run_depth = std::max(run_depth, deepest);
        ++bi;
    }
    ws->dev.nseg = 0;
    if (bc_out) e = gather_f64(n, g->d_perm, ws->dev.bc, bc_out, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws->h_ctrl, ws->dev.ctrl, kBatchCtrlInts * sizeof(int32_t),
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(from_hip(e));
    range |= ws->h_ctrl[1];
    if (k > 0) g->batch_depth_hint.store(run_depth);
    if (prof) accumulate_profile(g, ws->timer, ws->d_stats);
    batch_release(g, ws, stream);
    return range ? BC_ERR_RANGE : BC_OK;
}

// BC over the sources with up to `width` sources per batch.  With dist /
// sigma (device, caller order, [k][n]), the per-source state is exported too.
// ---- device-resident level loop ----------------------------------------------

// Bytes of one batch's workspace in the fused pool (vis, sigma / coef rows,
// split-vertex rows, partial rows, the level array).
size_t fused_batch_bytes(const bc_graph_s *g, int32_t lcap) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    const size_t multi = (size_t)std::max(g->multi_end, 1);
    const size_t items = (size_t)std::max<uint32_t>(g->items, 1);
    return align_up(n * sizeof(uint64_t)) + 2 * align_up(n * kWave * sizeof(double)) +
           align_up(multi * sizeof(uint64_t)) + align_up(multi * kWave * sizeof(double)) +
           align_up(items * kWave * sizeof(double)) +
           align_up((size_t)lcap * n * sizeof(uint64_t));
}

// The batch workspaces of the pool (not the run's lane and segment tables).
void fused_release_pool(bc_graph_s *g) {
    auto &f = g->fused;
    if (f.block) (void)hipFree(f.block);
    if (f.d_devs) (void)hipFree(f.d_devs);
    if (f.h_ctrl) (void)hipHostFree(f.h_ctrl);
    if (f.d_batches) (void)hipFree(f.d_batches);
    f.block = nullptr;
    f.d_devs = nullptr;
    f.h_ctrl = nullptr;
    f.d_batches = nullptr;
    f.d_ctrl = nullptr;
    f.d_bc = nullptr;
    f.bytes = 0;
    f.cap = f.lcap = 0;
    f.h_devs.clear();
}

void fused_release(bc_graph_s *g) {
    fused_release_pool(g);
    auto &f = g->fused;
    if (f.d_lanes) (void)hipFree(f.d_lanes);
    if (f.d_total) (void)hipFree(f.d_total);
    if (f.d_stats) (void)hipFree(f.d_stats);
    f.d_lanes = nullptr;
    f.d_total = nullptr;
    f.d_stats = nullptr;
    f.lanes_cap = 0;
}

// Batches per launch that fit the pool budget with `lcap` levels each.
constexpr size_t kFusedBudget = (size_t)4 << 30;
int32_t fused_cap(const bc_graph_s *g, int32_t nbatches, int32_t lcap) {
    const size_t per = fused_batch_bytes(g, lcap);
    return (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)std::max(nbatches, 1),
                                                         kFusedBudget / per));
}

// Pool for `cap` batches with `lcap` levels each (caller holds fused_mu); an
// existing pool at least that large is kept.
bc_status fused_reserve(bc_graph_s *g, int32_t cap, int32_t lcap) {
    auto &f = g->fused;
    if (f.block && f.cap >= cap && f.lcap >= lcap) return BC_OK;
    fused_release_pool(g);
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    const size_t per = fused_batch_bytes(g, lcap);
    const size_t head = align_up((size_t)cap * kCtlInts * sizeof(int32_t)) +
                        align_up((size_t)cap * n * sizeof(double));
    f.bytes = head + (size_t)cap * per;
    hipError_t e = hipMalloc(&f.block, f.bytes);
    if (e == hipSuccess) e = hipMalloc(&f.d_devs, (size_t)cap * sizeof(BatchDev));
    if (e == hipSuccess) e = hipMalloc(&f.d_batches, (size_t)cap * sizeof(int2));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&f.h_ctrl, (size_t)cap * kCtlInts * sizeof(int32_t),
                          hipHostMallocDefault);
    if (e != hipSuccess) {
        fused_release(g);
        return from_hip(e);
    }
    f.cap = cap;
    f.lcap = lcap;
    char *p = (char *)f.block;
    auto take = [&](size_t bytes) {
        char *r = p;
        p += align_up(bytes);
        return (void *)r;
    };
    f.d_ctrl = (int32_t *)take((size_t)cap * kCtlInts * sizeof(int32_t));
    f.d_bc = (double *)take((size_t)cap * n * sizeof(double));
    f.h_devs.assign((size_t)cap, BatchDev{});
    for (int32_t b = 0; b < cap; ++b) {
        BatchDev &d = f.h_devs[(size_t)b];
        d.n = g->n;
        d.row_ptr = g->d_row_ptr;
        d.col_idx = g->d_col_idx;
        d.big_end = g->big_end;
        d.multi_end = g->multi_end;
        d.items = g->items;
        d.item_info = g->d_item_info;
        d.item_first = g->d_item_first;
        d.items_in = g->items_in;
        d.row_ptr_in = g->d_row_ptr_in;
        d.col_idx_in = g->d_col_idx_in;
        d.item_info_in = g->d_item_info_in;
        d.item_first_in = g->d_item_first_in;
        d.iperm = g->d_iperm;
        d.nnz = g->nnz;
        d.lcap = lcap;
        d.ctrl = f.d_ctrl + (size_t)b * kCtlInts;
        d.bc = f.d_bc + (size_t)b * n;
        d.vis = (uint64_t *)take(n * sizeof(uint64_t));
        d.sigma = (double *)take(n * kWave * sizeof(double));
        d.sigma32 = reinterpret_cast<uint32_t *>(d.sigma);
        d.coef = (double *)take(n * kWave * sizeof(double));
        d.reach = (uint64_t *)take((size_t)std::max(g->multi_end, 1) * sizeof(uint64_t));
        d.hubsig = (double *)take((size_t)std::max(g->multi_end, 1) * kWave * sizeof(double));
        d.partial = (double *)take((size_t)std::max<uint32_t>(g->items, 1) * kWave * sizeof(double));
        d.F = (uint64_t *)take((size_t)lcap * n * sizeof(uint64_t));
    }
    return BC_OK;
}

// The whole batch plan with the device-resident level loop: up to `cap`
// batches per launch (one workgroup each).  Without segments, BC (caller
// order) = the batches' BC added in batch order; with segments, each batch
// adds its lanes' dependencies to its requests' outputs (requests of at most
// 64 sources only, so no two batches of a launch share an output).
bc_status fused_run(bc_graph_s *g, const std::vector<int32_t> &s_int,
                    const std::vector<BatchPlan> &plan, const std::vector<int32_t> &seg_start,
                    const std::vector<double *> &seg_out, double *bc_out, hipStream_t stream,
                    const int32_t *export_row, int32_t *dist, double *sigma) {
    std::lock_guard<std::mutex> lk(g->fused_mu);
    const int32_t nb = (int32_t)plan.size();
    const size_t n = (size_t)g->n;
    auto &f = g->fused;
    const bool prof = g->profiling.load() != 0;
    const int32_t lcap = std::max(16, g->batch_depth_hint.load() + 8);
    bc_status st = fused_reserve(g, fused_cap(g, nb, lcap), lcap);
    if (st != BC_OK) return st;
    // the running BC total outlives pool regrowth
    if (bc_out && !f.d_total) BC_TRY_HIP(hipMalloc(&f.d_total, std::max<size_t>(n, 1) * sizeof(double)));
    // lanes and segment tables on the device
    const size_t k = s_int.size();
    const size_t seg_ints = seg_start.size(), seg_ptrs = seg_out.size();
    const size_t need = k * sizeof(int32_t) + seg_ints * sizeof(int32_t) +
                        seg_ptrs * sizeof(double *) + 64;
    if (need > f.lanes_cap) {
        if (f.d_lanes) (void)hipFree(f.d_lanes);
        f.d_lanes = nullptr;
        f.lanes_cap = 0;
        BC_TRY_HIP(hipMalloc(&f.d_lanes, need));
        f.lanes_cap = need;
    }
    int32_t *d_seg_start = f.d_lanes + k;
    double **d_seg_out = (double **)(((uintptr_t)(d_seg_start + seg_ints) + 15) & ~(uintptr_t)15);
    hipError_t e = hipSuccess;
    if (k) e = hipMemcpyAsync(f.d_lanes, s_int.data(), k * sizeof(int32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && seg_ints)
        e = hipMemcpyAsync(d_seg_start, seg_start.data(), seg_ints * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && seg_ptrs)
        e = hipMemcpyAsync(d_seg_out, seg_out.data(), seg_ptrs * sizeof(double *),
                           hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return from_hip(e);
    int32_t *x_dist = nullptr;
    double *x_sigma = nullptr;
    struct Tmp {
        int32_t *&a;
        double *&b;
        ~Tmp() {
            if (a) (void)hipFree(a);
            if (b) (void)hipFree(b);
        }
    } tmp_guard{x_dist, x_sigma};
    if (dist) BC_TRY_HIP(hipMalloc(&x_dist, (size_t)kWave * n * sizeof(int32_t)));
    if (sigma) BC_TRY_HIP(hipMalloc(&x_sigma, (size_t)kWave * n * sizeof(double)));
    LaunchTimer timer;
    timer.on = prof;
    if (prof) {
        if (!f.d_stats) BC_TRY_HIP(hipMalloc(&f.d_stats, 12 * sizeof(unsigned long long)));
        BC_TRY_HIP(hipMemsetAsync(f.d_stats, 0, 12 * sizeof(unsigned long long), stream));
    }
    bool range = false;
    int32_t run_depth = 0;
    std::vector<int2> bt;
    for (int32_t b0 = 0; b0 < nb;) {
        const int32_t m = std::min(f.cap, nb - b0);
        bt.resize((size_t)std::max(m, 1));
        const bool narrow = !g->sigma_wide.load();
        for (int32_t i = 0; i < m; ++i) {
            const BatchPlan &bp = plan[(size_t)(b0 + i)];
            BatchDev &d = f.h_devs[(size_t)i];
            d.narrow = narrow ? 1 : 0;
            d.stats = prof ? f.d_stats : nullptr;
            d.nseg = bp.nseg;
            d.seg_start = bp.nseg ? d_seg_start + bp.seg_first : nullptr;
            d.seg_out = bp.nseg ? d_seg_out + (bp.seg_first - (b0 + i)) : nullptr;
            bt[(size_t)i] = make_int2(bp.first, bp.nlanes);
        }
        e = hipMemcpyAsync(f.d_devs, f.h_devs.data(), (size_t)m * sizeof(BatchDev),
                           hipMemcpyHostToDevice, stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f.d_batches, bt.data(), (size_t)m * sizeof(int2),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = timer.begin(BC_PROF_FUSED, stream);
        if (e == hipSuccess) e = batch_fused(f.d_devs, m, narrow, f.d_lanes, f.d_batches, stream);
        if (e == hipSuccess) e = timer.end(stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(f.h_ctrl, f.d_ctrl, (size_t)m * kCtlInts * sizeof(int32_t),
                               hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) break;
        bool trunc = false, wide = false, over = false;
        for (int32_t i = 0; i < m; ++i) {
            const int32_t *c = f.h_ctrl + (size_t)i * kCtlInts;
            trunc |= c[kCtlTrunc] != 0;
            wide |= c[kCtlNarrow] != 0;
            over |= c[kCtlRange] != 0;
        }
        if (wide) {  // a path count needs double rows: run these batches again
            g->sigma_wide.store(true);
            continue;
        }
        if (over) {  // beyond double: the caller runs the call again level-scaled
            g->sigma_ext.store(true);
            timer.destroy();
            return BC_ERR_RANGE;
        }
        if (trunc) {  // a batch ran deeper than the level array: grow it, run again
            const int32_t l2 = f.lcap * 2;
            fused_release_pool(g);  // the longer arrays may hold fewer batches
            st = fused_reserve(g, fused_cap(g, nb - b0, l2), l2);
            if (st != BC_OK) return st;
            continue;
        }
        for (int32_t i = 0; i < m; ++i) {
            const int32_t *c = f.h_ctrl + (size_t)i * kCtlInts;
            range |= c[kCtlRange] != 0;
            run_depth = std::max(run_depth, c[kCtlDeepest]);
        }
        if (export_row && (dist || sigma)) {
            for (int32_t i = 0; i < m && e == hipSuccess; ++i) {
                const BatchPlan &bp = plan[(size_t)(b0 + i)];
                const BatchDev &d = f.h_devs[(size_t)i];
                e = batch_export(d, f.h_ctrl[(size_t)i * kCtlInts + kCtlDeepest], bp.nlanes, x_dist,
                                 x_sigma, stream);
                for (int32_t s2 = 0; s2 < bp.nlanes && e == hipSuccess; ++s2) {
                    const size_t row = (size_t)export_row[bp.first + s2] * n;
                    if (dist) e = gather_i32(g->n, g->d_perm, x_dist + (size_t)s2 * n, dist + row, stream);
                    if (e == hipSuccess && sigma)
                        e = gather_f64(g->n, g->d_perm, x_sigma + (size_t)s2 * n, sigma + row, stream);
                }
            }
        }
        if (e == hipSuccess && bc_out) e = sum_parts(g->n, f.d_bc, m, f.d_total, stream, b0 > 0);
        if (e != hipSuccess) break;
        b0 += m;
    }
    if (e == hipSuccess && bc_out) {
        if (nb == 0) e = hipMemsetAsync(bc_out, 0, n * sizeof(double), stream);
        else e = gather_f64(g->n, g->d_perm, f.d_total, bc_out, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
        timer.destroy();
        return from_hip(e);
    }
    if (nb > 0) g->batch_depth_hint.store(run_depth);
    if (prof) accumulate_profile(g, timer, f.d_stats);
    timer.destroy();
    return range ? BC_ERR_RANGE : BC_OK;
}

// The device-resident loop runs a batch on one compute unit (up to 256
// batches at once); the host-driven loop runs a batch across the device.
// Measured on MI355X (R-MAT graphs of 53K to 7.6M arcs): one batch takes about
// 2 ms + 50 ns per arc on the device loop and, amortised over the host loop's
// concurrent parts, 0.8 ms + 0.15 ns per arc on the host loop.  AUTO picks
// the loop with the lower estimate for the call's batch count.
bool use_fused(const bc_graph_s *g, int32_t level_loop, int32_t nbatches) {
    if (g->sigma_ext.load()) return false;  // extended range: host loop only
    if (level_loop == BC_LOOP_DEVICE) return true;
    if (level_loop == BC_LOOP_HOST) return false;
    const double arcs = (double)g->nnz;
    const double device = 2e-3 + 50e-9 * arcs;
    const double host = 0.8e-3 + 0.15e-9 * arcs;
    const double rounds = std::ceil((double)nbatches / 256.0);
    return (double)nbatches * host > rounds * device;
}

// Batches run at once for `concurrency` (0: by workspace size; the choice
// depends only on the graph and the batch count, so results are identical
// from run to run).  Parts overlap one another's small kernels and host
// polls; beyond the process's 4 hardware queues they gain nothing, and the
// large graphs' level kernels already fill the device.
int32_t parts_of(const bc_graph_s *g, int32_t concurrency, int32_t nbatches) {
    int32_t p = concurrency;
    if (p <= 0) {
        const size_t ws = batch_ws_bytes(g) + batch_level_bytes(g, 16);
        p = ws <= ((size_t)1 << 30) ? 4 : (ws <= ((size_t)16 << 30) ? 2 : 1);
    }
    return std::max(1, std::min(p, nbatches));
}

bc_status get_streams(bc_graph_s *g, int32_t p, std::vector<hipStream_t> &out) {
    std::lock_guard<std::mutex> lk(g->stream_mu);
    while ((int32_t)g->streams.size() < p) {
        hipStream_t st = nullptr;
        BC_TRY_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        g->streams.push_back(st);
    }
    out.assign(g->streams.begin(), g->streams.begin() + p);
    return BC_OK;
}

bc_status batched_run(bc_graph_s *g, const int32_t *sources, int32_t k, double *bc_out,
                      int32_t width, int32_t sparse_div, int32_t concurrency,
                      int32_t level_loop, hipStream_t stream, int32_t *dist, double *sigma) {
    // Batch composition: sources sorted by their distances to the two
    // landmarks, so that the 64 sources of a batch lie close together and see
    // most vertices at the same level (their frontier masks share lanes, the
    // row gathers are dense).  BC is a sum over sources, so any grouping gives
    // the same result up to rounding; the order depends only on the inputs.
    std::vector<int32_t> order((size_t)k);
    for (int32_t i = 0; i < k; ++i) order[(size_t)i] = i;
    if (k > width && !g->directed) {  // the landmarks' BFS runs undirected
        bc_status st = ensure_landmarks(g);
        if (st != BC_OK) return st;
        const uint32_t far = 0x7fffffff;
        auto key = [&](int32_t i) {
            const int32_t v = g->h_perm[(size_t)sources[i]];
            const int32_t a = g->land1[(size_t)v], b = g->land2[(size_t)v];
            return std::make_pair(a < 0 ? far : (uint32_t)a, b < 0 ? far : (uint32_t)b);
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t x, int32_t y) { return key(x) < key(y); });
    }
    std::vector<int32_t> s_int((size_t)k);
    for (int32_t i = 0; i < k; ++i) s_int[(size_t)i] = g->h_perm[(size_t)sources[order[(size_t)i]]];
    std::vector<BatchPlan> plan;
    for (int32_t b0 = 0; b0 < k; b0 += width) plan.push_back({b0, std::min(width, k - b0), 0, 0});
    if (use_fused(g, level_loop, (int32_t)plan.size())) {
        // a count beyond double's range sends the call to the host loop
        const bc_status st =
            fused_run(g, s_int, plan, {}, {}, bc_out, stream, order.data(), dist, sigma);
        if (st != BC_ERR_RANGE || !g->sigma_ext.load()) return st;
    }
    const int32_t P = parts_of(g, concurrency, (int32_t)plan.size());
    if (P <= 1)
        return run_batch_plan(g, s_int, plan, {}, {}, bc_out, stream, order.data(), dist, sigma,
                              sparse_div);
    // P parts of consecutive batches, each on its own stream and workspace,
    // ordered after the caller's earlier work; BC = the parts' sum in part
    // order, on the caller's stream
    std::vector<hipStream_t> streams;
    bc_status st = get_streams(g, P, streams);
    if (st != BC_OK) return st;
    const size_t n = (size_t)g->n;
    double *parts = nullptr;
    hipEvent_t ev_start = nullptr;
    std::vector<hipEvent_t> ev_done((size_t)P, nullptr);
    auto cleanup = [&]() {
        if (parts) (void)hipFree(parts);
        if (ev_start) (void)hipEventDestroy(ev_start);
        for (hipEvent_t ev : ev_done)
            if (ev) (void)hipEventDestroy(ev);
    };
    hipError_t e = hipMalloc(&parts, (size_t)P * n * sizeof(double));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_start, hipEventDisableTiming);
    for (int32_t i = 0; i < P && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&ev_done[(size_t)i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev_start, stream);
    for (int32_t i = 0; i < P && e == hipSuccess; ++i) e = hipStreamWaitEvent(streams[i], ev_start, 0);
    if (e != hipSuccess) {
        cleanup();
        return from_hip(e);
    }
    const int32_t nb = (int32_t)plan.size();
    std::vector<bc_status> status((size_t)P, BC_OK);
    std::vector<std::thread> workers;
    for (int32_t i = 0; i < P; ++i) {
        workers.emplace_back([&, i]() {
            DeviceGuard dg(g->device);
            const int32_t b0 = (int32_t)((int64_t)nb * i / P), b1 = (int32_t)((int64_t)nb * (i + 1) / P);
            std::vector<BatchPlan> sub(plan.begin() + b0, plan.begin() + b1);
            status[(size_t)i] = run_batch_plan(g, s_int, sub, {}, {}, parts + (size_t)i * n,
                                               streams[(size_t)i], order.data(), dist, sigma,
                                               sparse_div);
            if (hipEventRecord(ev_done[(size_t)i], streams[(size_t)i]) != hipSuccess &&
                status[(size_t)i] == BC_OK)
                status[(size_t)i] = BC_ERR_DEVICE;
        });
    }
    for (std::thread &t : workers) t.join();
    bc_status result = BC_OK;
    for (bc_status s2 : status) {
        if (s2 != BC_OK && s2 != BC_ERR_RANGE) {
            result = s2;
            break;
        }
        if (s2 == BC_ERR_RANGE) result = BC_ERR_RANGE;
    }
    for (int32_t i = 0; i < P && e == hipSuccess; ++i) e = hipStreamWaitEvent(stream, ev_done[i], 0);
    if (e == hipSuccess && (result == BC_OK || result == BC_ERR_RANGE))
        e = sum_parts(g->n, parts, P, bc_out, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    cleanup();
    if (e != hipSuccess) return from_hip(e);
    return result;
}

// Several requests in one run.  A request of at most 64 sources never
// straddles two batches; a larger one fills whole batches from a batch start
// and its remainder starts a batch.  Every request's result is then made of
// the same lanes in the same order whatever else shares its batches.
bc_status multi_run(bc_graph_s *g, const int32_t *sources, const int32_t *req_start,
                    int32_t nreq, double *const *outs, hipStream_t stream) {
    const int32_t k = req_start[nreq];
    std::vector<int32_t> s_int((size_t)k);
    for (int32_t i = 0; i < k; ++i) s_int[(size_t)i] = g->h_perm[(size_t)sources[i]];
    std::vector<BatchPlan> plan;
    std::vector<int32_t> seg_start;
    std::vector<double *> seg_out;
    // segments of the batch being filled
    std::vector<std::pair<int32_t, int32_t>> cur;  // (request, lanes)
    int32_t cur_first = 0, pos = 0;
    auto close = [&]() {
        if (pos == 0) return;
        BatchPlan bp{cur_first, pos, (int32_t)seg_start.size(), (int32_t)cur.size()};
        // seg_out entries of batch b are stored at seg_first - b (one fewer
        // entry than seg_start per batch): keep both tables aligned by index
        int32_t a = 0;
        for (auto &sg : cur) {
            seg_start.push_back(a);
            a += sg.second;
        }
        seg_start.push_back(a);
        for (auto &sg : cur) seg_out.push_back(outs[sg.first]);
        plan.push_back(bp);
        cur.clear();
        cur_first += pos;
        pos = 0;
    };
    for (int32_t r = 0; r < nreq; ++r) {
        int32_t m = req_start[r + 1] - req_start[r];
        if (m == 0) continue;
        if (pos > 0 && (m > kWave || pos + m > kWave)) close();
        while (m > 0) {
            const int32_t t = std::min(kWave - pos, m);
            cur.push_back({r, t});
            pos += t;
            m -= t;
            if (pos == kWave) close();
        }
    }
    close();
    for (int32_t r = 0; r < nreq; ++r) {
        hipError_t e = hipMemsetAsync(outs[r], 0, (size_t)g->n * sizeof(double), stream);
        if (e != hipSuccess) return from_hip(e);
    }
    // the device-resident loop runs a launch's batches at once: only when no
    // request spans two batches (no two workgroups add to one output)
    bool spans = false;
    for (int32_t r = 0; r < nreq; ++r) spans |= req_start[r + 1] - req_start[r] > kWave;
    if (!spans && use_fused(g, BC_LOOP_AUTO, (int32_t)plan.size())) {
        const bc_status st = fused_run(g, s_int, plan, seg_start, seg_out, nullptr, stream,
                                       nullptr, nullptr, nullptr);
        if (st != BC_ERR_RANGE || !g->sigma_ext.load()) return st;
        // beyond double's range: outputs cleared and the call run again level-scaled
        for (int32_t r = 0; r < nreq; ++r) {
            hipError_t e = hipMemsetAsync(outs[r], 0, (size_t)g->n * sizeof(double), stream);
            if (e != hipSuccess) return from_hip(e);
        }
    }
    return run_batch_plan(g, s_int, plan, seg_start, seg_out, nullptr, stream, nullptr, nullptr,
                          nullptr, g->tuned_sparse_div.load());
}

// Mode selection: BC_MODE_AUTO picks the batched path from the graph's
// crossover source count on (16 until bc_autotune measures it).
// A plain run whose counts overflowed double: the graph switches to the
// batched path's extended range for this and every later call.
void plain_overflowed(bc_graph_s *g) {
    g->sigma_wide.store(true);
    g->sigma_ext.store(true);
}

bool use_batched(const bc_graph_s *g, const bc_options *opt, int32_t k) {
    // only the batched path has the extended range and directed graphs
    if (g->sigma_ext.load() || g->directed) return true;
    const int32_t mode = opt ? opt->mode : BC_MODE_AUTO;
    if (mode == BC_MODE_BATCHED) return true;
    if (mode == BC_MODE_PLAIN) return false;
    return k >= g->tuned_min_batched.load();
}

int32_t batch_width_of(const bc_graph_s *g, const bc_options *opt) {
    return (opt && opt->batch_width > 0) ? opt->batch_width : g->tuned_width.load();
}

int32_t sparse_div_of(const bc_graph_s *g, const bc_options *opt) {
    return (opt && opt->sparse_div != 0) ? opt->sparse_div : g->tuned_sparse_div.load();
}

bc_status check_options(const bc_options *opt) {
    if (!opt) return BC_OK;
    if (opt->mode < BC_MODE_AUTO || opt->mode > BC_MODE_BATCHED) return BC_ERR_INVALID_ARG;
    if (opt->batch_width < 0 || opt->batch_width > 64) return BC_ERR_INVALID_ARG;
    if (opt->level_chunk < 0 || opt->level_chunk > 1024) return BC_ERR_INVALID_ARG;
    if (opt->sparse_div < -1 || opt->sparse_div > (1 << 20)) return BC_ERR_INVALID_ARG;
    if (opt->concurrency < 0 || opt->concurrency > kMaxParts) return BC_ERR_INVALID_ARG;
    if (opt->level_loop < BC_LOOP_AUTO || opt->level_loop > BC_LOOP_DEVICE)
        return BC_ERR_INVALID_ARG;
    for (int i = 0; i < 2; ++i)
        if (opt->reserved[i] != 0) return BC_ERR_INVALID_ARG;
    return BC_OK;
}

bc_status check_sources(const bc_graph_s *g, const int32_t *sources, int32_t k) {
    if (k < 0) return BC_ERR_INVALID_ARG;
    if (k > 0 && !sources) return BC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < k; ++i)
        if (sources[i] < 0 || sources[i] >= g->n) return BC_ERR_INVALID_ARG;
    return BC_OK;
}

// Structural checks of a host CSR; with `symmetric`, also that the arc
// multiset equals its transpose.
bc_status validate_csr(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                       bool symmetric) {
    if (row_ptr[0] != 0) return BC_ERR_INVALID_GRAPH;
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) return BC_ERR_INVALID_GRAPH;
    const int64_t nnz = row_ptr[n];
    for (int64_t e = 0; e < nnz; ++e)
        if (col_idx[e] < 0 || col_idx[e] >= n) return BC_ERR_INVALID_GRAPH;
    if (!symmetric) return BC_OK;
    // transpose by counting sort; rows of the transpose come out ascending
    std::vector<int64_t> toff((size_t)n + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) toff[(size_t)col_idx[e] + 1]++;
    for (int32_t v = 0; v < n; ++v) toff[(size_t)v + 1] += toff[(size_t)v];
    for (int32_t v = 0; v < n; ++v)
        if (toff[(size_t)v + 1] - toff[(size_t)v] != (int64_t)row_ptr[v + 1] - row_ptr[v])
            return BC_ERR_INVALID_GRAPH;
    std::vector<int32_t> tcol((size_t)nnz);
    std::vector<int64_t> cur(toff.begin(), toff.end() - 1);
    for (int32_t u = 0; u < n; ++u)
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) tcol[(size_t)cur[col_idx[e]]++] = u;
    std::vector<int32_t> row;
    for (int32_t v = 0; v < n; ++v) {
        row.assign(col_idx + row_ptr[v], col_idx + row_ptr[v + 1]);
        std::sort(row.begin(), row.end());
        if (!std::equal(row.begin(), row.end(), tcol.begin() + toff[(size_t)v]))
            return BC_ERR_INVALID_GRAPH;
    }
    return BC_OK;
}

// The graph's device arrays (the reversed CSR and its items only when they
// are arrays of their own, i.e. for a directed graph).
void free_graph_arrays(bc_graph_s *g) {
    if (g->directed) {
        if (g->d_row_ptr_in) (void)hipFree(g->d_row_ptr_in);
        if (g->d_col_idx_in) (void)hipFree(g->d_col_idx_in);
        if (g->d_item_info_in) (void)hipFree(g->d_item_info_in);
        if (g->d_item_first_in) (void)hipFree(g->d_item_first_in);
    }
    g->d_row_ptr_in = g->d_col_idx_in = nullptr;
    g->d_item_info_in = nullptr;
    g->d_item_first_in = nullptr;
    if (g->d_row_ptr) (void)hipFree(g->d_row_ptr);
    if (g->d_col_idx) (void)hipFree(g->d_col_idx);
    if (g->d_perm) (void)hipFree(g->d_perm);
    if (g->d_iperm) (void)hipFree(g->d_iperm);
    if (g->d_item_info) (void)hipFree(g->d_item_info);
    if (g->d_item_first) (void)hipFree(g->d_item_first);
    if (g->d_weight) (void)hipFree(g->d_weight);
    auto &w = g->sssp;
    if (w.dist) (void)hipFree(w.dist);
    if (w.stamp) (void)hipFree(w.stamp);
    if (w.flags) (void)hipFree(w.flags);
    if (w.h_flags) (void)hipHostFree(w.h_flags);
    if (w.d_stats) (void)hipFree(w.d_stats);
    w = bc_graph_s::Sssp{};
    auto &pw = g->prw;
    if (pw.block) (void)hipFree(pw.block);
    if (pw.diff) (void)hipFree(pw.diff);
    if (pw.h_diff) (void)hipHostFree(pw.h_diff);
    pw = bc_graph_s::Pr{};
    g->d_weight = nullptr;
    g->d_row_ptr = g->d_col_idx = g->d_perm = g->d_iperm = nullptr;
    g->d_item_info = nullptr;
    g->d_item_first = nullptr;
}

}  // namespace

extern "C" {

const char *bc_status_str(bc_status s) {
    switch (s) {
        case BC_OK: return "ok";
        case BC_ERR_INVALID_ARG: return "invalid argument";
        case BC_ERR_INVALID_GRAPH: return "invalid graph";
        case BC_ERR_OUT_OF_MEMORY: return "out of device memory";
        case BC_ERR_RANGE: return "shortest-path counts out of the representable range";
        case BC_ERR_DEVICE: return "HIP runtime error";
        case BC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

bc_status bc_create_graph(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          uint32_t flags, void *stream, bc_graph_t *out) {
    if (!out || n < 0 || !row_ptr) return BC_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)(BC_GRAPH_TRUST_SYMMETRIC | BC_GRAPH_INPUT_ON_DEVICE |
                            BC_GRAPH_DIRECTED))
        return BC_ERR_INVALID_ARG;
    const bool on_device = (flags & BC_GRAPH_INPUT_ON_DEVICE) != 0;
    const bool directed = (flags & BC_GRAPH_DIRECTED) != 0;
    const bool check_sym = !(flags & (BC_GRAPH_TRUST_SYMMETRIC | BC_GRAPH_DIRECTED));
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> h_rp, h_ci;
    const int32_t *rp_host = row_ptr;
    const int32_t *ci_host = col_idx;
    if (on_device) {
        h_rp.resize((size_t)n + 1);
        BC_TRY_HIP(hipMemcpy(h_rp.data(), row_ptr, ((size_t)n + 1) * sizeof(int32_t),
                             hipMemcpyDeviceToHost));
        rp_host = h_rp.data();
        if (rp_host[0] != 0) return BC_ERR_INVALID_GRAPH;
        for (int32_t v = 0; v < n; ++v)
            if (rp_host[v + 1] < rp_host[v]) return BC_ERR_INVALID_GRAPH;
        // the neighbour ids are checked on the host too: the relabelling
        // kernel indexes with them
        if (rp_host[n] > 0 && !col_idx) return BC_ERR_INVALID_ARG;
        h_ci.resize((size_t)rp_host[n]);
        if (rp_host[n] > 0)
            BC_TRY_HIP(hipMemcpy(h_ci.data(), col_idx, (size_t)rp_host[n] * sizeof(int32_t),
                                 hipMemcpyDeviceToHost));
        ci_host = h_ci.data();
        bc_status vs = validate_csr(n, rp_host, ci_host, check_sym);
        if (vs != BC_OK) return vs;
    } else {
        if (n > 0 && row_ptr[n] > 0 && !col_idx) return BC_ERR_INVALID_ARG;
        bc_status vs = validate_csr(n, row_ptr, col_idx, check_sym);
        if (vs != BC_OK) return vs;
    }
    const int64_t nnz = rp_host[n];
    if (nnz > 0 && !col_idx) return BC_ERR_INVALID_ARG;

    // directed: the arcs into each vertex (caller ids), by counting sort
    std::vector<int32_t> in_rp, in_ci;
    if (directed) {
        in_rp.assign((size_t)n + 1, 0);
        for (int64_t e = 0; e < nnz; ++e) in_rp[(size_t)ci_host[e] + 1]++;
        for (int32_t v = 0; v < n; ++v) in_rp[(size_t)v + 1] += in_rp[(size_t)v];
        in_ci.resize((size_t)std::max<int64_t>(nnz, 1));
        std::vector<int32_t> cur(in_rp.begin(), in_rp.end() - 1);
        for (int32_t u = 0; u < n; ++u)
            for (int32_t e = rp_host[u]; e < rp_host[u + 1]; ++e)
                in_ci[(size_t)cur[(size_t)ci_host[e]]++] = u;
    }
    auto out_deg = [&](int32_t o) { return rp_host[o + 1] - rp_host[o]; };
    auto in_deg = [&](int32_t o) { return directed ? in_rp[(size_t)o + 1] - in_rp[(size_t)o]
                                                   : out_deg(o); };
    // the order key: the degree, or for a directed graph the larger of the two
    auto key_deg = [&](int32_t o) { return std::max(out_deg(o), in_deg(o)); };

    int device = 0;
    BC_TRY_HIP(hipGetDevice(&device));
    bc_graph_s *g = new (std::nothrow) bc_graph_s();
    if (!g) return BC_ERR_OUT_OF_MEMORY;
    g->device = device;
    g->n = n;
    g->nnz = nnz;
    g->directed = directed;

    // Internal order: key degree descending, ties by caller id (counting sort).
    int32_t maxdeg = 0;
    for (int32_t v = 0; v < n; ++v) maxdeg = std::max(maxdeg, key_deg(v));
    std::vector<int64_t> start((size_t)maxdeg + 2, 0);
    for (int32_t v = 0; v < n; ++v) start[(size_t)(maxdeg - key_deg(v)) + 1]++;
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    std::vector<int32_t> iperm((size_t)std::max(n, 1));
    g->h_perm.assign((size_t)std::max(n, 1), 0);
    for (int32_t v = 0; v < n; ++v) {
        const int32_t slot = (int32_t)start[(size_t)(maxdeg - key_deg(v))]++;
        iperm[(size_t)slot] = v;
        g->h_perm[(size_t)v] = slot;
    }
    std::vector<int32_t> new_rp((size_t)n + 1, 0), new_rp_in;
    if (directed) new_rp_in.assign((size_t)n + 1, 0);
    for (int32_t u = 0; u < n; ++u) {
        const int32_t o = iperm[(size_t)u];
        const int32_t dgr = out_deg(o);
        new_rp[(size_t)u + 1] = new_rp[(size_t)u] + dgr;
        if (directed) new_rp_in[(size_t)u + 1] = new_rp_in[(size_t)u] + in_deg(o);
        // one-source path buckets (id ranges; undirected graphs only run there,
        // where the order makes them exact)
        const int b = degree_bucket(dgr);
        if (b == 3) g->b3_end = u + 1;
        if (b >= 2) g->b2_end = u + 1;
        if (b >= 1) g->b1_end = u + 1;
    }
    uint64_t chunks = 0;
    for (int32_t u = 0; u < g->b3_end; ++u) chunks += chunks_of(out_deg(iperm[(size_t)u]));
    g->total_chunks3 = chunks;
    // batched work items: internal ids are key-degree-descending, so the
    // vertices of key degree > 64 (> kChunk) are a prefix; each of them has at
    // least one item per direction
    std::vector<int2> item_info, item_info_in;
    std::vector<uint32_t> item_first, item_first_in;
    for (int32_t u = 0; u < n; ++u) {
        const int32_t o = iperm[(size_t)u];
        if (key_deg(o) <= kB1MaxDeg) break;
        g->big_end = u + 1;
        if (key_deg(o) > kChunk) g->multi_end = u + 1;
        item_first.push_back((uint32_t)item_info.size());
        for (int32_t j = 0; j == 0 || j * kChunk < out_deg(o); ++j)
            item_info.push_back(make_int2(u, j));
        if (directed) {
            item_first_in.push_back((uint32_t)item_info_in.size());
            for (int32_t j = 0; j == 0 || j * kChunk < in_deg(o); ++j)
                item_info_in.push_back(make_int2(u, j));
        }
    }
    item_first.push_back((uint32_t)item_info.size());
    if (directed) item_first_in.push_back((uint32_t)item_info_in.size());
    g->items = (uint32_t)item_info.size();
    g->items_in = directed ? (uint32_t)item_info_in.size() : g->items;

    const size_t rp_bytes = ((size_t)n + 1) * sizeof(int32_t);
    const size_t ci_bytes = std::max<size_t>((size_t)nnz, 1) * sizeof(int32_t);
    const size_t pm_bytes = (size_t)std::max(n, 1) * sizeof(int32_t);
    int32_t *t_rp = nullptr, *t_ci = nullptr, *t_rp_in = nullptr, *t_ci_in = nullptr;
    hipError_t e = hipMalloc(&g->d_row_ptr, rp_bytes);
    if (e == hipSuccess) e = hipMalloc(&g->d_col_idx, ci_bytes);
    if (e == hipSuccess) e = hipMalloc(&g->d_perm, pm_bytes);
    if (e == hipSuccess) e = hipMalloc(&g->d_iperm, pm_bytes);
    if (e == hipSuccess && !on_device) e = hipMalloc(&t_rp, rp_bytes);
    if (e == hipSuccess && !on_device) e = hipMalloc(&t_ci, ci_bytes);
    if (directed) {
        if (e == hipSuccess) e = hipMalloc(&g->d_row_ptr_in, rp_bytes);
        if (e == hipSuccess) e = hipMalloc(&g->d_col_idx_in, ci_bytes);
        if (e == hipSuccess) e = hipMalloc(&t_rp_in, rp_bytes);
        if (e == hipSuccess) e = hipMalloc(&t_ci_in, ci_bytes);
    }
    const int32_t *old_rp = on_device ? row_ptr : t_rp;
    const int32_t *old_ci = on_device ? col_idx : t_ci;
    if (e == hipSuccess && !on_device)
        e = hipMemcpyAsync(t_rp, row_ptr, rp_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !on_device && nnz > 0)
        e = hipMemcpyAsync(t_ci, col_idx, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_row_ptr, new_rp.data(), rp_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_perm, g->h_perm.data(), pm_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->d_iperm, iperm.data(), pm_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = relabel_csr(n, nnz, old_rp, old_ci, g->d_row_ptr, g->d_perm, g->d_iperm, g->d_col_idx,
                        st);
    if (directed) {
        if (e == hipSuccess)
            e = hipMemcpyAsync(t_rp_in, in_rp.data(), rp_bytes, hipMemcpyHostToDevice, st);
        if (e == hipSuccess && nnz > 0)
            e = hipMemcpyAsync(t_ci_in, in_ci.data(), (size_t)nnz * sizeof(int32_t),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->d_row_ptr_in, new_rp_in.data(), rp_bytes, hipMemcpyHostToDevice,
                               st);
        if (e == hipSuccess)
            e = relabel_csr(n, nnz, t_rp_in, t_ci_in, g->d_row_ptr_in, g->d_perm, g->d_iperm,
                            g->d_col_idx_in, st);
    }
    auto upload_items = [&](const std::vector<int2> &info, const std::vector<uint32_t> &first,
                            int2 **d_info, uint32_t **d_first) {
        if (e == hipSuccess)
            e = hipMalloc(d_info, std::max<size_t>(info.size(), 1) * sizeof(int2));
        if (e == hipSuccess) e = hipMalloc(d_first, first.size() * sizeof(uint32_t));
        if (e == hipSuccess && !info.empty())
            e = hipMemcpyAsync(*d_info, info.data(), info.size() * sizeof(int2),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(*d_first, first.data(), first.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, st);
    };
    upload_items(item_info, item_first, &g->d_item_info, &g->d_item_first);
    if (directed) upload_items(item_info_in, item_first_in, &g->d_item_info_in, &g->d_item_first_in);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (t_rp) (void)hipFree(t_rp);
    if (t_ci) (void)hipFree(t_ci);
    if (t_rp_in) (void)hipFree(t_rp_in);
    if (t_ci_in) (void)hipFree(t_ci_in);
    if (!directed) {  // the forward pass reads the same arrays
        g->d_row_ptr_in = g->d_row_ptr;
        g->d_col_idx_in = g->d_col_idx;
        g->d_item_info_in = g->d_item_info;
        g->d_item_first_in = g->d_item_first;
    }
    if (e != hipSuccess) {
        free_graph_arrays(g);
        delete g;
        return from_hip(e);
    }
    g->device_bytes = (directed ? 2 : 1) * (rp_bytes + ci_bytes) + 2 * pm_bytes;
    *out = g;
    return BC_OK;
}

bc_status bc_destroy_graph(bc_graph_t g) {
    if (!g) return BC_OK;
    DeviceGuard dg(g->device);
    for (PlainWS *ws : g->plain_pool) plain_ws_destroy(ws);
    g->plain_pool.clear();
    for (hipStream_t st : g->streams) (void)hipStreamDestroy(st);
    g->streams.clear();
    fused_release(g);
    for (BatchWS *ws : g->batch_pool) batch_ws_destroy(ws);
    g->batch_pool.clear();
    free_graph_arrays(g);
    delete g;
    return BC_OK;
}

bc_status bc_graph_info(bc_graph_t g, int32_t *n, int64_t *nnz, size_t *device_bytes) {
    if (!g) return BC_ERR_INVALID_ARG;
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (device_bytes) *device_bytes = g->device_bytes;
    return BC_OK;
}

bc_status bc_run_async(bc_graph_t g, const int32_t *sources, int32_t k, double *bc_out_dev,
                       const bc_options *opt, void *stream) {
    if (!g || (!bc_out_dev && g->n > 0)) return BC_ERR_INVALID_ARG;
    bc_status st = check_options(opt);
    if (st != BC_OK) return st;
    st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    if (g->n == 0) return BC_OK;
    DeviceGuard dg(g->device);
    if (!use_batched(g, opt, k)) {
        st = plain_run(g, sources, k, bc_out_dev, opt, (hipStream_t)stream, nullptr, nullptr);
        if (st != BC_ERR_RANGE) return st;
        plain_overflowed(g);
    }
    return batched_run(g, sources, k, bc_out_dev, batch_width_of(g, opt), sparse_div_of(g, opt),
                       opt ? opt->concurrency : 0, opt ? opt->level_loop : 0,
                       (hipStream_t)stream, nullptr, nullptr);
}

bc_status bc_run(bc_graph_t g, const int32_t *sources, int32_t k, double *bc_out) {
    if (!g || (!bc_out && g->n > 0)) return BC_ERR_INVALID_ARG;
    bc_status st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    if (g->n == 0) return BC_OK;
    DeviceGuard dg(g->device);
    double *d_bc = nullptr;
    BC_TRY_HIP(hipMalloc(&d_bc, (size_t)g->n * sizeof(double)));
    st = BC_ERR_RANGE;
    if (!use_batched(g, nullptr, k)) {
        st = plain_run(g, sources, k, d_bc, nullptr, nullptr, nullptr, nullptr);
        if (st == BC_ERR_RANGE) plain_overflowed(g);
    }
    if (st == BC_ERR_RANGE)
        st = batched_run(g, sources, k, d_bc, batch_width_of(g, nullptr), sparse_div_of(g, nullptr),
                         0, 0, nullptr, nullptr, nullptr);
    if (st == BC_OK || st == BC_ERR_RANGE) {
        hipError_t e = hipMemcpy(bc_out, d_bc, (size_t)g->n * sizeof(double),
                                 hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = from_hip(e);
    }
    (void)hipFree(d_bc);
    return st;
}

bc_status bc_run_detail(bc_graph_t g, const int32_t *sources, int32_t k, const bc_options *opt,
                        double *bc_out, int32_t *dist, double *sigma) {
    if (!g || (!bc_out && g->n > 0)) return BC_ERR_INVALID_ARG;
    bc_status st = check_options(opt);
    if (st != BC_OK) return st;
    st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    if (g->n == 0) return BC_OK;
    DeviceGuard dg(g->device);
    const size_t n = (size_t)g->n;
    double *d_bc = nullptr;
    int32_t *d_dist = nullptr;
    double *d_sigma = nullptr;
    hipError_t e = hipMalloc(&d_bc, n * sizeof(double));
    if (e == hipSuccess && dist) e = hipMalloc(&d_dist, std::max<size_t>(1, (size_t)k) * n * sizeof(int32_t));
    if (e == hipSuccess && sigma) e = hipMalloc(&d_sigma, std::max<size_t>(1, (size_t)k) * n * sizeof(double));
    if (e != hipSuccess) {
        (void)hipFree(d_bc);
        (void)hipFree(d_dist);
        (void)hipFree(d_sigma);
        return from_hip(e);
    }
    std::vector<SourceState> exp((size_t)std::max(k, 1));
    for (int32_t i = 0; i < k; ++i) {
        exp[i].dist = d_dist ? d_dist + (size_t)i * n : nullptr;
        exp[i].sigma = d_sigma ? d_sigma + (size_t)i * n : nullptr;
    }
    const bool batched = !opt || opt->mode != BC_MODE_PLAIN || g->sigma_ext.load() || g->directed;
    ExportAlloc tmp;
    if (!batched && (dist || sigma) && (e = tmp.alloc(n)) != hipSuccess) {
        (void)hipFree(d_bc);
        (void)hipFree(d_dist);
        (void)hipFree(d_sigma);
        return from_hip(e);
    }
    st = BC_ERR_RANGE;
    if (!batched) {
        st = plain_run(g, sources, k, d_bc, opt, nullptr, (dist || sigma) ? exp.data() : nullptr,
                       &tmp.t);
        if (st == BC_ERR_RANGE) plain_overflowed(g);
    }
    if (st == BC_ERR_RANGE)
        st = batched_run(g, sources, k, d_bc, batch_width_of(g, opt), sparse_div_of(g, opt),
                         opt ? opt->concurrency : 0, opt ? opt->level_loop : 0, nullptr, d_dist,
                         d_sigma);
    if (st == BC_OK || st == BC_ERR_RANGE) {
        e = hipMemcpy(bc_out, d_bc, n * sizeof(double), hipMemcpyDeviceToHost);
        if (e == hipSuccess && dist)
            e = hipMemcpy(dist, d_dist, (size_t)k * n * sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess && sigma)
            e = hipMemcpy(sigma, d_sigma, (size_t)k * n * sizeof(double), hipMemcpyDeviceToHost);
        if (e != hipSuccess) st = from_hip(e);
    }
    (void)hipFree(d_bc);
    (void)hipFree(d_dist);
    (void)hipFree(d_sigma);
    return st;
}

bc_status bc_run_multi(bc_graph_t g, const int32_t *sources, const int32_t *req_start,
                       int32_t nreq, double *const *bc_outs, void *stream) {
    if (!g || nreq < 0 || (nreq > 0 && (!req_start || !bc_outs))) return BC_ERR_INVALID_ARG;
    if (nreq == 0) return BC_OK;
    if (req_start[0] != 0) return BC_ERR_INVALID_ARG;
    for (int32_t r = 0; r < nreq; ++r) {
        if (req_start[r + 1] < req_start[r]) return BC_ERR_INVALID_ARG;
        if (!bc_outs[r] && g->n > 0) return BC_ERR_INVALID_ARG;
    }
    bc_status st = check_sources(g, sources, req_start[nreq]);
    if (st != BC_OK) return st;
    if (g->n == 0) return BC_OK;
    DeviceGuard dg(g->device);
    return multi_run(g, sources, req_start, nreq, bc_outs, (hipStream_t)stream);
}

bc_status bc_single_source(bc_graph_t g, int32_t s, int32_t *dist, double *sigma,
                           double *delta) {
    if (!g || ((!dist || !sigma) && g->n > 0)) return BC_ERR_INVALID_ARG;
    if (s < 0 || s >= g->n) return BC_ERR_INVALID_ARG;
    if (g->directed) return BC_ERR_UNSUPPORTED;  // the one-source path is undirected
    DeviceGuard dg(g->device);
    const size_t n = (size_t)g->n;
    double *d_bc = nullptr, *d_sigma = nullptr, *d_delta = nullptr;
    int32_t *d_dist = nullptr;
    hipError_t e = hipMalloc(&d_bc, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_dist, n * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&d_sigma, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&d_delta, n * sizeof(double));
    bc_status st = from_hip(e);
    if (st == BC_OK) {
        SourceState exp;
        exp.dist = d_dist;
        exp.sigma = d_sigma;
        exp.delta = d_delta;
        ExportAlloc tmp;
        e = tmp.alloc(n);
        st = e != hipSuccess ? from_hip(e)
                             : plain_run(g, &s, 1, d_bc, nullptr, nullptr, &exp, &tmp.t);
        if (st == BC_OK || st == BC_ERR_RANGE) {
            e = hipMemcpy(dist, d_dist, n * sizeof(int32_t), hipMemcpyDeviceToHost);
            if (e == hipSuccess) e = hipMemcpy(sigma, d_sigma, n * sizeof(double), hipMemcpyDeviceToHost);
            if (e == hipSuccess && delta)
                e = hipMemcpy(delta, d_delta, n * sizeof(double), hipMemcpyDeviceToHost);
            if (e != hipSuccess) st = from_hip(e);
        }
    }
    (void)hipFree(d_bc);
    (void)hipFree(d_dist);
    (void)hipFree(d_sigma);
    (void)hipFree(d_delta);
    return st;
}

bc_status bc_set_weights(bc_graph_t g, const int32_t *weight) {
    if (!g || (!weight && g->nnz > 0)) return BC_ERR_INVALID_ARG;
    int32_t maxw = 0;
    for (int64_t e = 0; e < g->nnz; ++e) {
        if (weight[e] < 0) return BC_ERR_INVALID_ARG;
        maxw = std::max(maxw, weight[e]);
    }
    // every distance must fit int32 (and stay below the "unreached" value)
    if ((int64_t)maxw * std::max<int64_t>(g->n - 1, 0) >= (int64_t)INT32_MAX) return BC_ERR_RANGE;
    if (g->n == 0 || g->nnz == 0) return BC_OK;
    DeviceGuard dg(g->device);
    std::lock_guard<std::mutex> lk(g->sssp_mu);
    // the caller's row offsets, from the internal ones and the permutation
    const size_t n = (size_t)g->n;
    std::vector<int32_t> new_rp(n + 1), old_rp(n + 1, 0);
    BC_TRY_HIP(hipMemcpy(new_rp.data(), g->d_row_ptr, (n + 1) * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
    for (size_t o = 0; o < n; ++o) {
        const int32_t u = g->h_perm[o];
        old_rp[o + 1] = old_rp[o] + (new_rp[(size_t)u + 1] - new_rp[(size_t)u]);
    }
    int32_t *t_rp = nullptr, *t_w = nullptr, *w_new = nullptr;
    hipError_t e = hipMalloc(&t_rp, (n + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&t_w, (size_t)g->nnz * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&w_new, (size_t)g->nnz * sizeof(int32_t));
    if (e == hipSuccess)
        e = hipMemcpy(t_rp, old_rp.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(t_w, weight, (size_t)g->nnz * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = permute_arc_values(g->n, g->nnz, t_rp, t_w, g->d_row_ptr, g->d_iperm, w_new, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (t_rp) (void)hipFree(t_rp);
    if (t_w) (void)hipFree(t_w);
    if (e != hipSuccess) {
        if (w_new) (void)hipFree(w_new);
        return from_hip(e);
    }
    if (g->d_weight) (void)hipFree(g->d_weight);
    g->d_weight = w_new;
    return BC_OK;
}

bc_status bc_sssp(bc_graph_t g, int32_t source, int32_t *dist_dev, void *stream_) {
    if (!g || source < 0 || source >= g->n || !dist_dev) return BC_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    std::lock_guard<std::mutex> lk(g->sssp_mu);
    const hipStream_t stream = (hipStream_t)stream_;
    auto &w = g->sssp;
    constexpr int32_t K = 8;  // passes queued per host poll
    if (!w.dist) {
        hipError_t e = hipMalloc(&w.dist, (size_t)g->n * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&w.stamp, (size_t)g->n * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&w.flags, 2 * K * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&w.d_stats, 12 * sizeof(unsigned long long));
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&w.h_flags, K * sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (w.dist) (void)hipFree(w.dist);
            if (w.stamp) (void)hipFree(w.stamp);
            if (w.flags) (void)hipFree(w.flags);
            if (w.d_stats) (void)hipFree(w.d_stats);
            w = bc_graph_s::Sssp{};
            return from_hip(e);
        }
    }
    const int32_t stride = std::max(1, g->profiling.load());
    const bool prof = g->profiling.load() != 0;
    LaunchTimer timer;
    SsspDev d{};
    d.n = g->n;
    d.big_end = g->big_end;
    d.items = g->items;
    d.row_ptr = g->d_row_ptr;
    d.col_idx = g->d_col_idx;
    d.weight = g->d_weight;
    d.item_info = g->d_item_info;
    d.dist = w.dist;
    d.stamp = w.stamp;
    hipError_t e = hipSuccess;
    if (prof) e = hipMemsetAsync(w.d_stats, 0, 12 * sizeof(unsigned long long), stream);
    if (e == hipSuccess) e = sssp_init(g->n, w.dist, w.stamp, g->h_perm[(size_t)source], stream);
    // flag of pass p (1, 2, ...) in block ((p-1)/K) & 1; a block is cleared
    // before its chunk of passes is queued
    auto slot = [&](int32_t p) { return w.flags + (((p - 1) / K) & 1) * K + (p - 1) % K; };
    bool done = false;
    for (int32_t p0 = 1; e == hipSuccess && !done; p0 += K) {
        if (p0 > g->n + K) {  // more passes than a shortest path has arcs: cannot happen
            e = hipErrorUnknown;
            break;
        }
        e = hipMemsetAsync(slot(p0), 0, K * sizeof(int32_t), stream);
        for (int32_t p = p0; p < p0 + K && e == hipSuccess; ++p) {
            const bool m = prof && (p - 1) % stride == 0;
            timer.on = m;
            d.stats = m ? w.d_stats + 9 : nullptr;
            e = timer.begin(BC_PROF_SSSP, stream);
            if (e == hipSuccess) e = sssp_pass(d, p, p == 1 ? nullptr : slot(p - 1), slot(p), stream);
            if (e == hipSuccess) e = timer.end(stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(w.h_flags, slot(p0), K * sizeof(int32_t), hipMemcpyDeviceToHost,
                               stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        for (int32_t q = 0; q < K && e == hipSuccess; ++q) done |= w.h_flags[q] == 0;
    }
    if (e == hipSuccess) e = sssp_export(g->n, g->d_perm, w.dist, dist_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && prof) accumulate_profile(g, timer, w.d_stats);
    timer.destroy();
    return from_hip(e);
}

bc_status bc_pagerank(bc_graph_t g, double damping, double tol, int32_t max_iter, double *pr_dev,
                      int32_t *iterations, void *stream_) {
    if (!g || !pr_dev || max_iter < 1 || !(damping >= 0.0 && damping <= 1.0) || !(tol >= 0.0))
        return BC_ERR_INVALID_ARG;
    if (iterations) *iterations = 0;
    if (g->n == 0) {
        if (iterations) *iterations = 1;
        return BC_OK;
    }
    DeviceGuard dg(g->device);
    std::lock_guard<std::mutex> lk(g->pr_mu);
    const hipStream_t stream = (hipStream_t)stream_;
    auto &w = g->prw;
    const size_t n = (size_t)g->n;
    const size_t items = std::max<uint32_t>(g->items_in, 1);
    constexpr int32_t K = 8;  // iterations queued per host poll
    if (!w.block) {
        const size_t bytes = 4 * align_up(n * sizeof(double)) + align_up(items * sizeof(double)) +
                             align_up(2 * (size_t)kFrontWaves * sizeof(double));
        hipError_t e = hipMalloc(&w.block, bytes);
        if (e == hipSuccess)
            e = hipHostMalloc((void **)&w.h_diff, K * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            if (w.block) (void)hipFree(w.block);
            w = bc_graph_s::Pr{};
            return from_hip(e);
        }
    }
    if (w.cap < max_iter) {
        if (w.diff) (void)hipFree(w.diff);
        w.diff = nullptr;
        w.cap = 0;
        BC_TRY_HIP(hipMalloc(&w.diff, (size_t)max_iter * sizeof(double)));
        w.cap = max_iter;
    }
    PrDev d{};
    d.n = g->n;
    d.big_end = g->big_end;
    d.multi_end = g->multi_end;
    d.items_in = g->items_in;
    d.row_ptr = g->d_row_ptr;
    d.row_ptr_in = g->d_row_ptr_in;
    d.col_idx_in = g->d_col_idx_in;
    d.item_info_in = g->d_item_info_in;
    d.item_first_in = g->d_item_first_in;
    char *p = (char *)w.block;
    auto take = [&](size_t b) {
        char *r = p;
        p += align_up(b);
        return (double *)r;
    };
    d.pr[0] = take(n * sizeof(double));
    d.pr[1] = take(n * sizeof(double));
    d.contrib[0] = take(n * sizeof(double));
    d.contrib[1] = take(n * sizeof(double));
    d.partial = take(items * sizeof(double));
    d.slots = take(2 * (size_t)kFrontWaves * sizeof(double));
    d.diff = w.diff;
    d.damping = damping;
    d.base = (1.0 - damping) / (double)g->n;
    d.tol = tol;
    const bool prof = g->profiling.load() != 0;
    const int32_t stride = std::max(1, g->profiling.load());
    LaunchTimer timer;
    hipError_t e = pagerank_init(d, max_iter, stream);
    int32_t done = max_iter;  // iterations run
    for (int32_t i0 = 0; e == hipSuccess && i0 < max_iter; i0 += K) {
        const int32_t i1 = std::min(max_iter, i0 + K);
        for (int32_t i = i0; i < i1 && e == hipSuccess; ++i) {
            timer.on = prof && i % stride == 0;
            e = timer.begin(BC_PROF_PAGERANK, stream);
            if (e == hipSuccess) e = pagerank_pull(d, i, stream);
            if (e == hipSuccess) e = timer.end(stream);
            if (e == hipSuccess) e = pagerank_finish(d, i, stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(w.h_diff, w.diff + i0, (size_t)(i1 - i0) * sizeof(double),
                               hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        bool stop = false;
        for (int32_t i = i0; i < i1 && e == hipSuccess && !stop; ++i) {
            const double x = w.h_diff[i - i0];
            if (x >= 0.0 && x <= tol) {
                done = i + 1;
                stop = true;
            }
        }
        if (stop) break;
    }
    if (e == hipSuccess) e = gather_f64(g->n, g->d_perm, d.pr[done & 1], pr_dev, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e == hipSuccess && prof) {
        // timing only: no work counters for PageRank (its bytes follow from the graph)
        bc_profile add{};
        for (size_t i = 0; i < timer.used; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, timer.ev[2 * i], timer.ev[2 * i + 1]) == hipSuccess)
                add.ms[timer.cls[i]] += ms;
            add.launches[timer.cls[i]] += 1;
        }
        std::lock_guard<std::mutex> lk2(g->prof_mu);
        g->prof.launches[BC_PROF_PAGERANK] += add.launches[BC_PROF_PAGERANK];
        g->prof.ms[BC_PROF_PAGERANK] += add.ms[BC_PROF_PAGERANK];
        g->prof.runs += 1;
    }
    timer.destroy();
    if (e != hipSuccess) return from_hip(e);
    if (iterations) *iterations = done;
    return BC_OK;
}

bc_status bc_workspace_bytes(bc_graph_t g, int32_t k, const bc_options *opt, size_t *bytes) {
    if (!g || !bytes || k < 0) return BC_ERR_INVALID_ARG;
    bc_status st = check_options(opt);
    if (st != BC_OK) return st;
    if (!use_batched(g, opt, k)) {
        *bytes = plain_ws_bytes(g);
        return BC_OK;
    }
    const int32_t width = batch_width_of(g, opt);
    const int32_t nb = (k + width - 1) / width;
    const int32_t lcap = std::max(16, g->batch_depth_hint.load() + 8);
    if (use_fused(g, opt ? opt->level_loop : 0, nb)) {
        // the device-loop pool: per-batch workspaces, BC arrays and control words
        const int32_t cap = fused_cap(g, nb, lcap);
        const size_t n = (size_t)std::max<int32_t>(g->n, 1);
        *bytes = (size_t)cap * (fused_batch_bytes(g, lcap) + n * sizeof(double) +
                                kCtlInts * sizeof(int32_t)) + n * sizeof(double);
    } else {
        // one workspace per concurrent part
        const int32_t parts = parts_of(g, opt ? opt->concurrency : 0, nb);
        *bytes = (size_t)parts * (batch_ws_bytes(g) + batch_level_bytes(g, lcap));
    }
    return BC_OK;
}

bc_status bc_profile_enable(bc_graph_t g, int32_t on) {
    if (!g || on < 0) return BC_ERR_INVALID_ARG;
    g->profiling.store(on);
    return BC_OK;
}

bc_status bc_profile_read(bc_graph_t g, bc_profile *out, int32_t reset) {
    if (!g || !out) return BC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g->prof_mu);
    *out = g->prof;
    if (reset) g->prof = bc_profile{};
    return BC_OK;
}

bc_status bc_trim_workspaces(bc_graph_t g) {
    if (!g) return BC_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    std::vector<PlainWS *> idle;
    std::vector<BatchWS *> idle_b;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        std::vector<PlainWS *> keep;
        for (PlainWS *ws : g->plain_pool) (ws->busy ? keep : idle).push_back(ws);
        g->plain_pool.swap(keep);
        std::vector<BatchWS *> keep_b;
        for (BatchWS *ws : g->batch_pool) (ws->busy ? keep_b : idle_b).push_back(ws);
        g->batch_pool.swap(keep_b);
    }
    for (PlainWS *ws : idle) plain_ws_destroy(ws);
    for (BatchWS *ws : idle_b) batch_ws_destroy(ws);
    return BC_OK;
}

bc_status bc_autotune(bc_graph_t g, const int32_t *sources, int32_t k, void *stream_,
                      bc_tuning *out) {
    if (!g || k < 1) return BC_ERR_INVALID_ARG;
    bc_status st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    const int32_t m = std::min(k, kWave);
    bc_tuning t{};
    t.batch_width = g->tuned_width.load();
    t.sparse_div = g->tuned_sparse_div.load();
    t.min_batched = g->tuned_min_batched.load();
    t.sample = m;
    if (g->n == 0) {
        if (out) *out = t;
        return BC_OK;
    }
    DeviceGuard dg(g->device);
    const hipStream_t stream = (hipStream_t)stream_;
    double *d_bc = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc(&d_bc, (size_t)g->n * sizeof(double));
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    auto cleanup = [&]() {
        if (d_bc) (void)hipFree(d_bc);
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        if (ev[1]) (void)hipEventDestroy(ev[1]);
    };
    if (e != hipSuccess) {
        cleanup();
        return from_hip(e);
    }
    // best of two runs (the first also sets up workspaces, landmarks and the
    // depth hints)
    auto timed = [&](auto &&run, double &ms) -> bc_status {
        ms = 1e30;
        for (int rep = 0; rep < 2; ++rep) {
            hipError_t e2 = hipEventRecord(ev[0], stream);
            if (e2 != hipSuccess) return from_hip(e2);
            bc_status s2 = run();
            if (s2 != BC_OK && s2 != BC_ERR_RANGE) return s2;
            e2 = hipEventRecord(ev[1], stream);
            if (e2 == hipSuccess) e2 = hipEventSynchronize(ev[1]);
            float f = 0.f;
            if (e2 == hipSuccess) e2 = hipEventElapsedTime(&f, ev[0], ev[1]);
            if (e2 != hipSuccess) return from_hip(e2);
            ms = std::min(ms, (double)f);
        }
        return BC_OK;
    };
    auto batched = [&](int32_t width, int32_t div, double &ms) {
        return timed([&]() { return batched_run(g, sources, m, d_bc, width, div, 1, BC_LOOP_AUTO,
                                                stream, nullptr, nullptr); }, ms);
    };
    // sparse-step threshold at width 64 (the default first), then width 32
    // with the best threshold; a setting replaces the current choice only when
    // it is more than 2 % faster (on one sample batch, near-equal settings
    // swap places from run to run)
    constexpr double kTuneMargin = 0.98;
    const int32_t divs[] = {kDefaultSparseDiv, -1, 16, 256};
    double best_ms = 1e30;
    int32_t best_div = kDefaultSparseDiv, best_width = kWave;
    for (int32_t div : divs) {
        double ms = 0;
        st = batched(kWave, div, ms);
        if (st != BC_OK) break;
        if (div == kDefaultSparseDiv || ms < best_ms * kTuneMargin) {
            best_ms = ms;
            best_div = div;
        }
    }
    if (st == BC_OK && m > 32) {
        double ms = 0;
        st = batched(32, best_div, ms);
        if (st == BC_OK && ms < best_ms * kTuneMargin) {
            best_ms = ms;
            best_width = 32;
        }
    }
    // one-source-at-a-time path on up to 4 sources
    // (none for a directed graph, which always takes the batched path)
    double plain_ms = 1e30;
    const int32_t p = std::min(m, 4);
    if (st == BC_OK && !g->directed)
        st = timed([&]() { return plain_run(g, sources, p, d_bc, nullptr, stream, nullptr,
                                            nullptr); }, plain_ms);
    cleanup();
    if (st != BC_OK) return st;
    const double per_source = std::max(plain_ms / p, 1e-6);
    // the batched path wins for a single batch once k * per_source exceeds
    // the batch time; beyond 64 sources it wins when it won at 64
    const double ratio = std::ceil(best_ms / per_source);
    const int32_t min_batched = ratio > (double)kWave ? INT32_MAX
                                                      : std::max<int32_t>(2, (int32_t)ratio);
    g->tuned_width.store(best_width);
    g->tuned_sparse_div.store(best_div);
    g->tuned_min_batched.store(min_batched);
    t.batch_width = best_width;
    t.sparse_div = best_div;
    t.min_batched = min_batched;
    t.plain_ms_per_source = per_source;
    t.batch_ms = best_ms;
    if (out) *out = t;
    return BC_OK;
}

}  // extern "C"
