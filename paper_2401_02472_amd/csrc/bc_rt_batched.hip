// Host side of the batched path: batch workspaces, batch composition
// (landmark order), the host-driven level loop, the device-resident loop's
// workspace pool, concurrent parts and multi-request batching.
#include "bc_runtime.h"

namespace bcx {

// Chunk items with a partial row: both passes' items (the forward pass runs
// over the arcs into each vertex, the reverse pass over the arcs out of it).
size_t partial_rows(const bc_graph_s::BcItems &t) {
    return (size_t)std::max<uint32_t>(std::max(t.items, t.items_in), 1);
}

size_t partial_rows(const bc_graph_s *g) { return partial_rows(g->bci); }

// The batched path's work items of a workspace: tables t.
void set_items(const bc_graph_s::BcItems &t, BatchDev &d) {
    d.big_end = t.big_end;
    d.multi_end = t.multi_end;
    d.chunk = t.chunk;
    d.items = t.items;
    d.item_info = t.info;
    d.item_first = t.first;
    d.items_in = t.items_in;
    d.item_info_in = t.info_in;
    d.item_first_in = t.first_in;
}

// ... the graph's current tables (the host-driven loop's).
void set_items(const bc_graph_s *g, BatchDev &d) { set_items(g->bci, d); }

// Rows of the graph's counts: double once a count passed 32 bits (or the
// extended range is on), uint32 before.
bool sigma_rows_wide(const bc_graph_s *g) { return g->sigma_wide.load() || g->sigma_ext.load(); }

size_t batch_ws_bytes_rows(const bc_graph_s *g, int32_t H, bool wide) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    const size_t lanes = (size_t)H * kWave;
    size_t b = 0;
    b += align_up(n * H * sizeof(uint64_t));             // vis
    b += align_up(n * lanes * (wide ? sizeof(double) : sizeof(uint32_t)));  // sigma rows
    b += align_up(n * lanes * sizeof(double));           // coef rows
    b += align_up(kBatchCtrlInts * sizeof(int32_t));     // ctrl
    b += align_up(n * H * sizeof(double));               // bc, one array per half
    b += align_up((size_t)std::max(g->bci.multi_end, 1) * H * sizeof(uint64_t));  // reach
    b += align_up(partial_rows(g) * lanes * sizeof(double));  // chunk partial rows
    b += align_up(kStatWords * sizeof(unsigned long long));     // work counters
    b += align_up(n * sizeof(int32_t));                  // candidate list
    // item list of the sparse step (the forward pass's items)
    b += align_up((size_t)std::max<uint32_t>(g->bci.items_in, 1) * sizeof(int32_t));
    b += align_up((size_t)kFrontSets * kFrontWaves * 2 * sizeof(unsigned long long));
    b += align_up(((n + 15) / 16) * 16);                 // candidate marks
    return b;
}

size_t batch_ws_bytes(const bc_graph_s *g, int32_t H) {
    return batch_ws_bytes_rows(g, H, sigma_rows_wide(g));
}

// F[lcap][n][H] and the extended-range tables xs, xmax, xe ([lcap][H][64] each).
size_t batch_level_bytes(const bc_graph_s *g, int32_t lcap, int32_t H) {
    return (size_t)lcap * H *
           ((size_t)std::max<int32_t>(g->n, 1) * sizeof(uint64_t) +
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
    if (ws->wide_sigma) (void)hipFree(ws->wide_sigma);
    if (ws->block) (void)hipFree(ws->block);
    if (ws->h_ctrl) (void)hipHostFree(ws->h_ctrl);
    delete ws;
}

bc_status batch_ws_create(bc_graph_s *g, int32_t H, BatchWS **out) {
    BatchWS *ws = new (std::nothrow) BatchWS();
    if (!ws) return BC_ERR_OUT_OF_MEMORY;
    ws->H = H;
    ws->gen = g->bci_gen.load();
    ws->wide = sigma_rows_wide(g);  // read once: the layout below follows it
    ws->bytes = batch_ws_bytes_rows(g, H, ws->wide);
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
    const size_t lanes = (size_t)H * kWave;
    d.n = g->n;
    d.H = H;
    d.row_ptr = g->d_row_ptr;
    d.col_idx = g->d_col_idx;
    d.vis = (uint64_t *)take(n * H * sizeof(uint64_t));
    d.sigma = (double *)take(n * lanes * (ws->wide ? sizeof(double) : sizeof(uint32_t)));
    d.sigma32 = reinterpret_cast<uint32_t *>(d.sigma);
    d.narrow = 1;
    d.coef = (double *)take(n * lanes * sizeof(double));
    d.ctrl = (int32_t *)take(kBatchCtrlInts * sizeof(int32_t));
    d.bc = (double *)take(n * H * sizeof(double));
    d.reach = (uint64_t *)take((size_t)std::max(g->bci.multi_end, 1) * H * sizeof(uint64_t));
    d.partial = (double *)take(partial_rows(g) * lanes * sizeof(double));
    set_items(g, d);
    d.row_ptr_in = g->d_row_ptr_in;
    d.col_idx_in = g->d_col_idx_in;
    ws->d_stats = (unsigned long long *)take(kStatWords * sizeof(unsigned long long));
    d.stats = nullptr;
    d.clist = (int32_t *)take(n * sizeof(int32_t));
    d.ilist = (int32_t *)take((size_t)std::max<uint32_t>(g->bci.items_in, 1) * sizeof(int32_t));
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

// Double-sized sigma rows for a workspace built with uint32 ones (its own
// region stays unused).
bc_status batch_widen(bc_graph_s *g, BatchWS *ws) {
    if (ws->wide) return BC_OK;
    const size_t bytes = (size_t)std::max<int32_t>(g->n, 1) * ws->H * kWave * sizeof(double);
    BC_TRY_HIP(hipMalloc(&ws->wide_sigma, bytes));
    ws->wide = true;
    ws->bytes += bytes;
    ws->dev.sigma = (double *)ws->wide_sigma;
    ws->dev.sigma32 = reinterpret_cast<uint32_t *>(ws->wide_sigma);
    return BC_OK;
}

bc_status batch_grow_levels(bc_graph_s *g, BatchWS *ws, int32_t lcap) {
    if (lcap <= ws->lcap) return BC_OK;
    if (ws->F) (void)hipFree(ws->F);
    ws->F = nullptr;
    ws->lcap = 0;
    const int32_t H = ws->H;
    BC_TRY_HIP(hipMalloc(&ws->F, batch_level_bytes(g, lcap, H)));
    ws->lcap = lcap;
    ws->dev.F = ws->F;
    ws->dev.lcap = lcap;
    ws->xs = (double *)(ws->F + (size_t)lcap * H * (size_t)std::max<int32_t>(g->n, 1));
    ws->xmax = (unsigned long long *)(ws->xs + (size_t)lcap * H * kWave);
    ws->xe = (int32_t *)(ws->xmax + (size_t)lcap * H * kWave);
    return BC_OK;
}

bc_status batch_acquire(bc_graph_s *g, int32_t H, hipStream_t stream, BatchWS **out) {
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (BatchWS *ws : g->batch_pool) {
            if (!ws->busy && ws->H == H && ws->gen == g->bci_gen.load()) {
                ws->busy = true;
                *out = ws;
                BC_TRY_HIP(hipStreamWaitEvent(stream, ws->done, 0));
                return BC_OK;
            }
        }
    }
    BatchWS *ws = nullptr;
    bc_status st = batch_ws_create(g, H, &ws);
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

constexpr size_t kMaxChunkGraphs = 16;

ChunkGraphs::~ChunkGraphs() {
    for (Entry &e : entries)
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (cap) (void)hipStreamDestroy(cap);
}

hipError_t ChunkGraphs::replay(const BatchDev &d, int32_t dir, int32_t K, int32_t nlanes,
                               hipStream_t stream) {
    Entry *hit = nullptr;
    for (Entry &en : entries)
        if (en.dir == dir && en.K == K && en.nlanes == nlanes &&
            std::memcmp(&en.d, &d, sizeof(BatchDev)) == 0) {
            hit = &en;
            break;
        }
    if (!hit) {
        if (!cap) {
            const hipError_t ec = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
            if (ec != hipSuccess) return ec;
        }
        // kernel launches only (no memset nodes): K relative steps, then the
        // base moved by K levels
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        for (int32_t i = 0; i < K && e == hipSuccess; ++i) {
            const int32_t L = kRelLevel + i;
            if (dir > 0) {
                e = batch_forward(d, L, nlanes, cap);
                if (e == hipSuccess) e = batch_forward_done(d, L, cap);
            } else {
                e = batch_reverse(d, L, cap);
                if (e == hipSuccess) e = batch_finalize_rel(d, L, cap);
            }
        }
        if (e == hipSuccess) e = batch_level_advance(d, dir * K, cap);
        hipGraph_t graph = nullptr;
        const hipError_t ee = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = ee;
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return e;
        if (entries.size() >= kMaxChunkGraphs) {
            // every earlier launch of the workspace's graphs is ordered before
            // this stream's current work (the workspace is acquired on it)
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                (void)hipGraphExecDestroy(exec);
                return e;
            }
            (void)hipGraphExecDestroy(entries.front().exec);
            entries.erase(entries.begin());
        }
        Entry en;
        en.dir = dir;
        en.K = K;
        en.nlanes = nlanes;
        en.d = d;
        en.exec = exec;
        entries.push_back(en);
        hit = &entries.back();
    }
    return hipGraphLaunch(hit->exec, stream);
}

// One batch: clear and seed, the forward levels in chunks with one host poll
// per chunk, then the reverse levels.  A path count that needs double rows
// (or the extended range) switches the graph to them and asks for a rerun; a
// level array too short for the batch asks for a longer one.  With cg, each
// chunk of levels is one replayed graph instead of its launches.
hipError_t drive_batch(bc_graph_s *g, BatchDev &d, const ExtTables &ext, const int32_t *lanes_dev,
                       int32_t nl, int32_t *h_ctrl, hipStream_t stream, LaunchTimer &timer,
                       unsigned long long *d_stats, int32_t stride, BatchOutcome &how,
                       int32_t &deepest, ChunkGraphs *cg, bool wide_ok) {
    const int32_t n = g->n;
    const bool prof = d_stats != nullptr;
    auto measure = [&](int32_t L) {
        const bool m = prof && L % stride == 0;
        timer.on = m;
        d.stats = m ? d_stats : nullptr;
    };
    const bool use_ext = g->sigma_ext.load();
    const bool wide = use_ext || g->sigma_wide.load();
    how = BatchOutcome::Done;
    deepest = 0;
    if (wide && !wide_ok) {  // uint32-sized rows cannot take double counts
        how = BatchOutcome::NeedWide;
        return hipSuccess;
    }
    d.narrow = wide ? 0 : 1;
    d.xs = use_ext ? ext.xs : nullptr;
    d.xmax = use_ext ? ext.xmax : nullptr;
    d.xe = use_ext ? ext.xe : nullptr;
    hipError_t e = batch_start(d, lanes_dev, nl, stream);
    if (e != hipSuccess) return e;
    int32_t L0 = 0;
    for (;;) {
        const int32_t K = std::max(2, g->batch_depth_hint.load() + 2);
        const int32_t Lend = std::min(L0 + K, d.lcap - 1);
        // (a replayed chunk runs levels L0 .. L0+K-1; those past the level
        // array's end return at once, as the host loop would not launch them)
        if (cg) e = cg->replay(d, 1, K, nl, stream);
        for (int32_t L = L0; !cg && L < Lend && e == hipSuccess; ++L) {
            measure(L);
            e = timer.begin(BC_PROF_FORWARD, stream);
            if (e == hipSuccess) e = batch_forward(d, L, nl, stream);
            if (e == hipSuccess) e = timer.end(stream);
            if (e == hipSuccess) e = timer.begin(BC_PROF_COMPACT, stream);
            if (e == hipSuccess) e = batch_forward_done(d, L, stream);
            if (e == hipSuccess) e = timer.end(stream);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(h_ctrl, d.ctrl, kBatchCtrlInts * sizeof(int32_t),
                               hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
        deepest = h_ctrl[kCtlDeepest];
        if (h_ctrl[kCtlNarrow]) {  // a path count needs double rows: run again
            g->sigma_wide.store(true);
            how = BatchOutcome::Rerun;
            return hipSuccess;
        }
        if (h_ctrl[kCtlRange] && !use_ext) {  // beyond double: run again level-scaled
            g->sigma_wide.store(true);
            g->sigma_ext.store(true);
            how = BatchOutcome::Rerun;
            return hipMemsetAsync(d.ctrl + kCtlRange, 0, sizeof(int32_t), stream);
        }
        if (h_ctrl[kCtlTrunc]) {
            how = BatchOutcome::Grow;
            return hipSuccess;
        }
        if (deepest < Lend || Lend >= n) break;
        L0 = Lend;
    }
    if (cg) {
        // chunks of K levels from the deepest one down (levels below 1 return
        // at once); the first chunk's base is the deepest level
        const int32_t K = std::max(2, g->batch_depth_hint.load() + 2);
        if (deepest >= 1) e = batch_level_from_deepest(d, stream);
        for (int32_t done = 0; done < deepest && e == hipSuccess; done += K)
            e = cg->replay(d, -1, K, 0, stream);
        return e;
    }
    for (int32_t L = deepest; L >= 1 && e == hipSuccess; --L) {
        measure(L);
        if (L != deepest) {
            e = timer.begin(BC_PROF_REVERSE, stream);
            if (e == hipSuccess) e = batch_reverse(d, L, stream);
            if (e == hipSuccess) e = timer.end(stream);
        }
        if (e == hipSuccess) e = timer.begin(BC_PROF_FINISH, stream);
        if (e == hipSuccess) e = batch_finalize(d, L, L == deepest, stream);
        if (e == hipSuccess) e = timer.end(stream);
    }
    return e;
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
                         double *sigma, int32_t sparse_div, bool graphs) {
    // two lane words per vertex when a batch has more than 64 sources (never
    // with request segments: their lanes are summed within one 64-lane word)
    int32_t H = 1;
    for (const BatchPlan &bp : plan) H = std::max(H, bp.nlanes > kWave ? 2 : 1);
    BatchWS *ws = nullptr;
    bc_status st = batch_acquire(g, H, stream, &ws);
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
    // frontier arcs below which a level takes the sparse step (0: never); the
    // halves of a two-word batch count their frontiers separately
    ws->dev.sparse_arcs = sparse_div < 0 ? 0 : H * (g->nnz / std::max(sparse_div, 1));
    if (prof) {
        hipError_t ez = hipMemsetAsync(ws->d_stats, 0, kStatWords * sizeof(unsigned long long), stream);
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
    if (dist) e = hipMalloc(&x_dist, (size_t)H * kWave * (size_t)n * sizeof(int32_t));
    if (e == hipSuccess && sigma)
        e = hipMalloc(&x_sigma, (size_t)H * kWave * (size_t)n * sizeof(double));
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
        e = hipMemsetAsync(ws->dev.bc, 0, (size_t)H * n * sizeof(double), stream);
    if (e == hipSuccess)  // the batches' kernels only ever set the range flag
        e = hipMemsetAsync(ws->dev.ctrl + kCtlRange, 0, sizeof(int32_t), stream);
    if (e != hipSuccess) return fail(from_hip(e));
    int32_t range = 0, run_depth = 0;
    int64_t level_steps = 0;  // forward and reverse, over the batches
    // measurement covers the launches of every stride-th level only (all of
    // them with stride 1): events around every launch slow deep graphs' short
    // level steps
    const int32_t stride = std::max(1, g->profiling.load());
    for (size_t bi = 0; bi < plan.size();) {
        const BatchPlan &bp = plan[bi];
        const int32_t nl = bp.nlanes;
        BatchDev &d = ws->dev;
        d.nseg = bp.nseg;
        d.seg_start = bp.nseg ? d_seg_start + bp.seg_first : nullptr;
        d.seg_out = bp.nseg ? d_seg_out + (bp.seg_first - (int32_t)bi) : nullptr;
        d.iperm = g->d_iperm;
        BatchOutcome how = BatchOutcome::Done;
        int32_t deepest = 0;
        const ExtTables ext{ws->xs, ws->xmax, ws->xe};
        // (measured runs launch every step: the events go around each launch)
        e = drive_batch(g, d, ext, d_lanes + bp.first, nl, ws->h_ctrl, stream, ws->timer,
                        prof ? ws->d_stats : nullptr, stride, how, deepest,
                        graphs && !prof ? &ws->graphs : nullptr, ws->wide);
        if (e != hipSuccess) return fail(from_hip(e));
        if (how == BatchOutcome::NeedWide) {  // double rows from now on
            st = batch_widen(g, ws);
            if (st != BC_OK) return fail(st);
            continue;
        }
        if (how == BatchOutcome::Rerun) continue;
        if (how == BatchOutcome::Grow) {  // level array full: grow it, run the batch again
            st = batch_grow_levels(g, ws, ws->lcap * 2);
            if (st != BC_OK) return fail(st);
            continue;
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
        level_steps += 2 * (int64_t)deepest + 1;
        ++bi;
    }
    ws->dev.nseg = 0;
    // the halves' BC arrays added (half 0 + half 1, in place)
    if (bc_out && H > 1) e = sum_parts(n, ws->dev.bc, H, ws->dev.bc, stream);
    if (e == hipSuccess && bc_out) e = gather_f64(n, g->d_perm, ws->dev.bc, bc_out, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws->h_ctrl, ws->dev.ctrl, kBatchCtrlInts * sizeof(int32_t),
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(from_hip(e));
    range |= ws->h_ctrl[1];
    if (k > 0) g->batch_depth_hint.store(run_depth);
    if (prof) accumulate_profile(g, ws->timer, ws->d_stats, level_steps);
    batch_release(g, ws, stream);
    return range ? BC_ERR_RANGE : BC_OK;
}

// ---- device-resident level loop ----------------------------------------------

// Bytes of one batch's workspace in the fused pool (vis, sigma / coef rows,
// split-vertex rows, partial rows, the level array).
size_t fused_batch_bytes(const bc_graph_s *g, int32_t lcap) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    const bc_graph_s::BcItems t = base_items(g);
    const size_t multi = (size_t)std::max(t.multi_end, 1);
    return align_up(n * sizeof(uint64_t)) + 2 * align_up(n * kWave * sizeof(double)) +
           align_up(multi * sizeof(uint64_t)) + align_up(partial_rows(t) * kWave * sizeof(double)) +
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
    const bc_graph_s::BcItems items = base_items(g);
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
        d.H = 1;
        d.row_ptr = g->d_row_ptr;
        d.col_idx = g->d_col_idx;
        set_items(items, d);
        d.row_ptr_in = g->d_row_ptr_in;
        d.col_idx_in = g->d_col_idx_in;
        d.iperm = g->d_iperm;
        d.nnz = g->nnz;
        d.lcap = lcap;
        d.ctrl = f.d_ctrl + (size_t)b * kCtlInts;
        d.bc = f.d_bc + (size_t)b * n;
        d.vis = (uint64_t *)take(n * sizeof(uint64_t));
        d.sigma = (double *)take(n * kWave * sizeof(double));
        d.sigma32 = reinterpret_cast<uint32_t *>(d.sigma);
        d.coef = (double *)take(n * kWave * sizeof(double));
        d.reach = (uint64_t *)take((size_t)std::max(items.multi_end, 1) * sizeof(uint64_t));
        d.partial = (double *)take(partial_rows(items) * kWave * sizeof(double));
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
        if (!f.d_stats) BC_TRY_HIP(hipMalloc(&f.d_stats, kStatWords * sizeof(unsigned long long)));
        BC_TRY_HIP(hipMemsetAsync(f.d_stats, 0, kStatWords * sizeof(unsigned long long), stream));
    }
    bool range = false;
    int32_t run_depth = 0;
    int64_t level_steps = 0;  // forward and reverse, over the batches
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
            level_steps += 2 * (int64_t)c[kCtlDeepest] + 1;
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
    if (prof) accumulate_profile(g, timer, f.d_stats, level_steps);
    timer.destroy();
    return range ? BC_ERR_RANGE : BC_OK;
}

bc_status make_plan(bc_graph_s *g, const int32_t *sources, int32_t k, int32_t width,
                    std::vector<int32_t> &order, std::vector<int32_t> &s_int,
                    std::vector<BatchPlan> &plan);

// Several graphs' batches in one device-resident launch (one per row width):
// each graph's plan is batched_run's at width 64 and each batch runs on its
// graph's pool, so every graph's BC is bit-identical to its own device-loop
// run.  A graph that cannot join (extended range, more batches than its pool
// holds at once) or whose batches call for a rerun (wider rows, a longer
// level array, counts past double's range) runs on its own afterwards, as
// bc_run_async with the device-resident loop would run it.
bc_status run_graphs(bc_graph_s *const *gs, int32_t ng, const int32_t *const *sources,
                     const int32_t *ks, double *const *outs, int32_t level_loop,
                     int32_t *loops, hipStream_t stream) {
    // BC_LOOP_AUTO: the graphs that join are the prefix, by one batch's
    // estimated device-loop time, that minimises the launch (its slowest
    // batch, times the rounds of 256 batches: the batches run side by side,
    // one workgroup each) plus the host-loop estimates of the graphs left out
    // (the cost model of use_fused)
    std::vector<char> join((size_t)ng, level_loop == BC_LOOP_HOST ? 0 : 1);
    if (level_loop == BC_LOOP_AUTO) {
        std::vector<int32_t> idx;
        for (int32_t i = 0; i < ng; ++i)
            if (gs[i]->n > 0 && ks[i] > 0) idx.push_back(i);
        auto dev_t = [&](int32_t i) { return 2e-3 + 50e-9 * (double)gs[i]->nnz; };
        auto host_t = [&](int32_t i) {
            return std::ceil((double)ks[i] / kWave) * (0.8e-3 + 0.15e-9 * (double)gs[i]->nnz);
        };
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int32_t a, int32_t b) { return dev_t(a) < dev_t(b); });
        double rest = 0.0;
        for (int32_t i : idx) rest += host_t(i);
        double best = rest;  // nothing joins
        size_t best_j = 0;
        double batches = 0.0;
        for (size_t j = 0; j < idx.size(); ++j) {
            rest -= host_t(idx[j]);
            batches += std::ceil((double)ks[idx[j]] / kWave);
            const double t = dev_t(idx[j]) * std::ceil(batches / 256.0) + rest;
            if (t < best) {
                best = t;
                best_j = j + 1;
            }
        }
        std::fill(join.begin(), join.end(), 0);
        for (size_t j = 0; j < best_j; ++j) join[(size_t)idx[j]] = 1;
    }
    struct Part {
        int32_t i = 0;                  // graph index
        std::vector<int32_t> order, s_int;
        std::vector<BatchPlan> plan;
        int32_t lane0 = 0;              // first lane in the combined lane array
        bool narrow = true;             // row width, read once for the call
        bool alone = false;
    };
    std::vector<Part> parts;
    std::vector<int32_t> alone;
    bc_status st = BC_OK;
    for (int32_t i = 0; i < ng && st == BC_OK; ++i) {
        bc_graph_s *g = gs[i];
        if (g->n == 0) continue;
        const int32_t lcap = std::max(16, g->batch_depth_hint.load() + 8);
        const int32_t nb = (ks[i] + kWave - 1) / kWave;
        if (!join[(size_t)i] || ks[i] == 0 || g->sigma_ext.load() || fused_cap(g, nb, lcap) < nb) {
            alone.push_back(i);
            continue;
        }
        Part p;
        p.i = i;
        st = make_plan(g, sources[i], ks[i], kWave, p.order, p.s_int, p.plan);
        parts.push_back(std::move(p));
    }
    if (st != BC_OK) return st;
    // every pool of the launch held, locked in address order
    std::vector<bc_graph_s *> locked;
    for (const Part &p : parts) locked.push_back(gs[p.i]);
    std::sort(locked.begin(), locked.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (bc_graph_s *g : locked) locks.emplace_back(g->fused_mu);
    int32_t lanes = 0, batches = 0;
    for (Part &p : parts) {
        bc_graph_s *g = gs[p.i];
        const int32_t lcap = std::max(16, g->batch_depth_hint.load() + 8);
        st = fused_reserve(g, (int32_t)p.plan.size(), lcap);
        if (st == BC_OK && !g->fused.d_total)
            st = from_hip(hipMalloc(&g->fused.d_total, (size_t)g->n * sizeof(double)));
        if (st != BC_OK) return st;
        p.lane0 = lanes;
        p.narrow = !g->sigma_wide.load();
        lanes += (int32_t)p.s_int.size();
        batches += (int32_t)p.plan.size();
    }
    int32_t *d_lanes = nullptr;
    BatchDev *d_devs = nullptr;
    int2 *d_bt = nullptr;
    struct Tmp {
        int32_t *&a;
        BatchDev *&b;
        int2 *&c;
        ~Tmp() {
            if (a) (void)hipFree(a);
            if (b) (void)hipFree(b);
            if (c) (void)hipFree(c);
        }
    } tmp_guard{d_lanes, d_devs, d_bt};
    hipError_t e = hipSuccess;
    if (batches > 0) {
        e = hipMalloc(&d_lanes, (size_t)std::max(lanes, 1) * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&d_devs, (size_t)batches * sizeof(BatchDev));
        if (e == hipSuccess) e = hipMalloc(&d_bt, (size_t)batches * sizeof(int2));
    }
    // host tables: lanes, batch views and (first lane, lane count) per batch,
    // the narrow-row graphs' batches first
    std::vector<int32_t> h_lanes((size_t)std::max(lanes, 1));
    std::vector<BatchDev> h_devs;
    std::vector<int2> h_bt;
    int32_t n_narrow = 0;
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
        for (Part &p : parts) {
            bc_graph_s *g = gs[p.i];
            const bool narrow = p.narrow;
            if (narrow != (pass == 0)) continue;
            auto &f = g->fused;
            std::copy(p.s_int.begin(), p.s_int.end(), h_lanes.begin() + p.lane0);
            for (size_t b = 0; b < p.plan.size(); ++b) {
                BatchDev d = f.h_devs[b];
                d.narrow = narrow ? 1 : 0;
                d.stats = nullptr;
                d.nseg = 0;
                d.seg_start = nullptr;
                d.seg_out = nullptr;
                h_devs.push_back(d);
                h_bt.push_back(make_int2(p.lane0 + p.plan[b].first, p.plan[b].nlanes));
            }
            if (pass == 0) n_narrow += (int32_t)p.plan.size();
        }
    }
    if (h_devs.size() != (size_t)batches || h_bt.size() != (size_t)batches) return BC_ERR_DEVICE;
    if (e == hipSuccess && batches > 0)
        e = hipMemcpyAsync(d_lanes, h_lanes.data(), (size_t)lanes * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && batches > 0)
        e = hipMemcpyAsync(d_devs, h_devs.data(), (size_t)batches * sizeof(BatchDev),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess && batches > 0)
        e = hipMemcpyAsync(d_bt, h_bt.data(), (size_t)batches * sizeof(int2),
                           hipMemcpyHostToDevice, stream);
    // the launches: narrow rows, then double rows
    if (e == hipSuccess && n_narrow > 0)
        e = batch_fused(d_devs, n_narrow, true, d_lanes, d_bt, stream);
    if (e == hipSuccess && batches > n_narrow)
        e = batch_fused(d_devs + n_narrow, batches - n_narrow, false, d_lanes, d_bt + n_narrow,
                        stream);
    for (Part &p : parts) {
        if (e != hipSuccess) break;
        auto &f = gs[p.i]->fused;
        e = hipMemcpyAsync(f.h_ctrl, f.d_ctrl, p.plan.size() * kCtlInts * sizeof(int32_t),
                           hipMemcpyDeviceToHost, stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return from_hip(e);
    bool range = false;
    for (Part &p : parts) {
        bc_graph_s *g = gs[p.i];
        auto &f = g->fused;
        const int32_t nb = (int32_t)p.plan.size();
        bool redo = false, over = false;
        int32_t depth = 0;
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t *c = f.h_ctrl + (size_t)b * kCtlInts;
            if (c[kCtlNarrow]) {  // a path count needs double rows
                g->sigma_wide.store(true);
                redo = true;
            }
            if (c[kCtlTrunc]) redo = true;  // a batch ran deeper than the level array
            over |= c[kCtlRange] != 0;
            depth = std::max(depth, c[kCtlDeepest]);
        }
        if (over) g->sigma_ext.store(true);  // beyond double: level-scaled, host loop
        if (redo || over) {
            p.alone = true;
            continue;
        }
        g->batch_depth_hint.store(depth);
        e = sum_parts(g->n, f.d_bc, nb, f.d_total, stream, false);
        if (e == hipSuccess) e = gather_f64(g->n, g->d_perm, f.d_total, outs[p.i], stream);
        if (e != hipSuccess) return from_hip(e);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return from_hip(e);
    locks.clear();
    for (const Part &p : parts)
        if (p.alone) alone.push_back(p.i);
    std::sort(alone.begin(), alone.end());
    for (int32_t i = 0; loops && i < ng; ++i) loops[i] = BC_LOOP_DEVICE;
    for (int32_t i : alone) {
        bc_graph_s *g = gs[i];
        // as the graph would run alone with the loop it was given (a graph
        // left out of the launch: the host loop)
        const int32_t loop = join[(size_t)i] ? BC_LOOP_DEVICE : BC_LOOP_HOST;
        if (loops) loops[i] = use_fused(g, loop, (ks[i] + kWave - 1) / kWave, kWave)
                                  ? BC_LOOP_DEVICE : BC_LOOP_HOST;
        const bc_status s2 = batched_run(g, sources[i], ks[i], outs[i], kWave,
                                         g->tuned_sparse_div.load(), 0, loop, stream,
                                         nullptr, nullptr);
        if (s2 == BC_ERR_RANGE) range = true;
        else if (s2 != BC_OK) return s2;
    }
    return range ? BC_ERR_RANGE : BC_OK;
}

// The device-resident loop runs a batch on one compute unit (up to 256
// batches at once); the host-driven loop runs a batch across the device.
// Measured on MI355X (R-MAT graphs of 53K to 7.6M arcs): one batch takes about
// 2 ms + 50 ns per arc on the device loop and, amortised over the host loop's
// concurrent parts, 0.8 ms + 0.15 ns per arc on the host loop.  AUTO picks
// the loop with the lower estimate for the call's batch count.
bool use_fused(const bc_graph_s *g, int32_t level_loop, int32_t nbatches, int32_t width) {
    if (g->sigma_ext.load()) return false;  // extended range: host loop only
    if (width > kWave) return false;        // one lane word per vertex only
    if (level_loop == BC_LOOP_DEVICE) return true;
    if (level_loop == BC_LOOP_HOST || level_loop == BC_LOOP_GRAPH) return false;
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
int32_t parts_of(const bc_graph_s *g, int32_t concurrency, int32_t nbatches, int32_t H) {
    int32_t p = concurrency;
    if (p <= 0) {
        const size_t ws = batch_ws_bytes(g, H) + batch_level_bytes(g, 16, H);
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

// Batch composition: sources sorted by their distances to the two landmarks,
// so that the sources of a batch lie close together and see most vertices at
// the same level (their frontier masks share lanes, the row gathers are
// dense).  BC is a sum over sources, so any grouping gives the same result up
// to rounding; the order depends only on the inputs.  order[i] = caller index
// of lane i of the run, s_int = its internal source ids, plan = batches of
// `width` lanes.
bc_status make_plan(bc_graph_s *g, const int32_t *sources, int32_t k, int32_t width,
                    std::vector<int32_t> &order, std::vector<int32_t> &s_int,
                    std::vector<BatchPlan> &plan) {
    order.assign((size_t)k, 0);
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
    s_int.assign((size_t)k, 0);
    for (int32_t i = 0; i < k; ++i) s_int[(size_t)i] = g->h_perm[(size_t)sources[order[(size_t)i]]];
    plan.clear();
    for (int32_t b0 = 0; b0 < k; b0 += width) plan.push_back({b0, std::min(width, k - b0), 0, 0});
    return BC_OK;
}

bc_status batched_run(bc_graph_s *g, const int32_t *sources, int32_t k, double *bc_out,
                      int32_t width, int32_t sparse_div, int32_t concurrency,
                      int32_t level_loop, hipStream_t stream, int32_t *dist, double *sigma) {
    std::vector<int32_t> order, s_int;
    std::vector<BatchPlan> plan;
    {
        const bc_status st0 = make_plan(g, sources, k, width, order, s_int, plan);
        if (st0 != BC_OK) return st0;
    }
    if (use_fused(g, level_loop, (int32_t)plan.size(), width)) {
        // a count beyond double's range sends the call to the host loop
        const bc_status st =
            fused_run(g, s_int, plan, {}, {}, bc_out, stream, order.data(), dist, sigma);
        if (st != BC_ERR_RANGE || !g->sigma_ext.load()) return st;
    }
    const int32_t P = parts_of(g, concurrency, (int32_t)plan.size(), width > kWave ? 2 : 1);
    if (P <= 1)
        return run_batch_plan(g, s_int, plan, {}, {}, bc_out, stream, order.data(), dist, sigma,
                              sparse_div, level_loop == BC_LOOP_GRAPH);
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
                                               sparse_div, level_loop == BC_LOOP_GRAPH);
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
    if (!spans && use_fused(g, BC_LOOP_AUTO, (int32_t)plan.size(), kWave)) {
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
                          nullptr, g->tuned_sparse_div.load(), false);
}

// Mode selection: BC_MODE_AUTO picks the batched path from the graph's

}  // namespace bcx
