// Host loop of the one-source-at-a-time path: its workspace pool, the
// speculative per-source level launches, polled forward passes, and the
// measurement totals shared by every path.
#include "bc_runtime.h"

namespace bcx {

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
    b += align_up(kStatWords * sizeof(unsigned long long));           // work counters
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
    ws->d_stats = (unsigned long long *)take(kStatWords * sizeof(unsigned long long));
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

// Add a finished run's event-timed launches and device work counters to the
// graph's measurement totals (the run's stream has been synchronised).
void accumulate_profile(bc_graph_s *g, LaunchTimer &timer, const unsigned long long *d_stats,
                        int64_t levels) {
    bc_profile add{};
    for (size_t i = 0; i < timer.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, timer.ev[2 * i], timer.ev[2 * i + 1]) == hipSuccess)
            add.ms[timer.cls[i]] += ms;
        add.launches[timer.cls[i]] += 1;
    }
    unsigned long long cnt[kStatWords];
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
        add.vertices[BC_PROF_FORWARD] = (int64_t)cnt[12];
        add.vertices[BC_PROF_REVERSE] = (int64_t)cnt[13];
    }
    std::lock_guard<std::mutex> lk(g->prof_mu);
    for (int c = 0; c < BC_PROF_CLASSES; ++c) {
        g->prof.launches[c] += add.launches[c];
        g->prof.ms[c] += add.ms[c];
        g->prof.owners[c] += add.owners[c];
        g->prof.arcs[c] += add.arcs[c];
        g->prof.hits[c] += add.hits[c];
        g->prof.vertices[c] += add.vertices[c];
    }
    g->prof.levels += levels;
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
        e = hipMemsetAsync(ws->d_stats, 0, kStatWords * sizeof(unsigned long long), stream);
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
    if (prof) {
        // level steps: every source run (truncated ones again when re-run)
        // takes depth + 1 forward and depth reverse steps
        const int64_t runs = (polled ? 0 : k) + (int64_t)redo.size();
        const int64_t depths = (int64_t)ws->h_ctrl[4] + ws->h_ctrl[0];
        accumulate_profile(g, ws->timer, ws->d_stats, 2 * depths + runs);
    }
    plain_release(g, ws, stream);
    return result;
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

}  // namespace bcx
