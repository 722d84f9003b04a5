// Host loops of the paper's two other propagation algorithms on the resident
// graph: single-source shortest paths (fixed-point passes) and PageRank (pull
// iterations).
#include "bc_runtime.h"

using namespace bcx;

extern "C" {

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
        if (e == hipSuccess) e = hipMalloc(&w.d_stats, kStatWords * sizeof(unsigned long long));
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
    if (prof) e = hipMemsetAsync(w.d_stats, 0, kStatWords * sizeof(unsigned long long), stream);
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

}  // extern "C"
