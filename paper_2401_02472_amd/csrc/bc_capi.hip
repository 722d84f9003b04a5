// C ABI (include/bc.h): argument checks, mode policy and the BC entry
// points.  Graph creation lives in bc_rt_graph.hip, the run loops in
// bc_rt_plain.hip and bc_rt_batched.hip, the autotuner in bc_tune.hip, SSSP
// and PageRank in bc_rt_algos.hip.
#include "bc_runtime.h"

using namespace bcx;

namespace bcx {

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

int32_t batch_width_of(const bc_graph_s *g, const bc_options *opt, int32_t k) {
    if (opt && opt->batch_width > 0) return opt->batch_width;
    const int32_t w = g->tuned_width.load();
    // a tuned width above 64 was timed on a sample that runs on the host
    // loop; where 64-wide batches of the whole run take the device-resident
    // loop (one lane word per vertex), those are the faster choice
    const int32_t loop = opt ? opt->level_loop : BC_LOOP_AUTO;
    if (w > kWave && k > 0 && use_fused(g, loop, (k + kWave - 1) / kWave, kWave)) return kWave;
    return w;
}

int32_t sparse_div_of(const bc_graph_s *g, const bc_options *opt) {
    return (opt && opt->sparse_div != 0) ? opt->sparse_div : g->tuned_sparse_div.load();
}

bc_status check_options(const bc_options *opt) {
    if (!opt) return BC_OK;
    if (opt->mode < BC_MODE_AUTO || opt->mode > BC_MODE_BATCHED) return BC_ERR_INVALID_ARG;
    if (opt->batch_width < 0 || opt->batch_width > 2 * kWave) return BC_ERR_INVALID_ARG;
    if (opt->level_chunk < 0 || opt->level_chunk > 1024) return BC_ERR_INVALID_ARG;
    if (opt->sparse_div < -1 || opt->sparse_div > (1 << 20)) return BC_ERR_INVALID_ARG;
    if (opt->concurrency < 0 || opt->concurrency > kMaxParts) return BC_ERR_INVALID_ARG;
    if (opt->level_loop < BC_LOOP_AUTO || opt->level_loop > BC_LOOP_GRAPH)
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

}  // namespace bcx

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
        case BC_ERR_TOO_LARGE: return "the run does not fit the fixed device array of the allocation-free call";
    }
    return "unknown status";
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
    return batched_run(g, sources, k, bc_out_dev, batch_width_of(g, opt, k), sparse_div_of(g, opt),
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
        st = batched_run(g, sources, k, d_bc, batch_width_of(g, nullptr, k), sparse_div_of(g, nullptr),
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
        st = batched_run(g, sources, k, d_bc, batch_width_of(g, opt, k), sparse_div_of(g, opt),
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

bc_status bc_run_graphs(const bc_graph_t *graphs, int32_t ngraphs, const int32_t *const *sources,
                        const int32_t *ks, double *const *bc_outs_dev, int32_t level_loop,
                        int32_t *loops, void *stream) {
    if (ngraphs < 0 || (ngraphs > 0 && (!graphs || !sources || !ks || !bc_outs_dev)))
        return BC_ERR_INVALID_ARG;
    if (level_loop != BC_LOOP_AUTO && level_loop != BC_LOOP_HOST && level_loop != BC_LOOP_DEVICE)
        return BC_ERR_INVALID_ARG;
    for (int32_t i = 0; i < ngraphs; ++i) {
        bc_graph_s *g = graphs[i];
        if (!g || ks[i] < 0 || (!bc_outs_dev[i] && g->n > 0)) return BC_ERR_INVALID_ARG;
        if (g->device != graphs[0]->device) return BC_ERR_INVALID_ARG;
        for (int32_t j = 0; j < i; ++j)
            if (graphs[j] == g) return BC_ERR_INVALID_ARG;  // each graph once
        const bc_status st = check_sources(g, sources[i], ks[i]);
        if (st != BC_OK) return st;
    }
    if (ngraphs == 0) return BC_OK;
    DeviceGuard dg(graphs[0]->device);
    return run_graphs(graphs, ngraphs, sources, ks, bc_outs_dev, level_loop, loops,
                      (hipStream_t)stream);
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

bc_status bc_workspace_bytes(bc_graph_t g, int32_t k, const bc_options *opt, size_t *bytes) {
    if (!g || !bytes || k < 0) return BC_ERR_INVALID_ARG;
    bc_status st = check_options(opt);
    if (st != BC_OK) return st;
    if (!use_batched(g, opt, k)) {
        *bytes = plain_ws_bytes(g);
        return BC_OK;
    }
    const int32_t width = batch_width_of(g, opt, k);
    const int32_t nb = (k + width - 1) / width;
    const int32_t H = width > kWave ? 2 : 1;
    const int32_t lcap = std::max(16, g->batch_depth_hint.load() + 8);
    if (use_fused(g, opt ? opt->level_loop : 0, nb, width)) {
        // the device-loop pool: per-batch workspaces, BC arrays and control words
        const int32_t cap = fused_cap(g, nb, lcap);
        const size_t n = (size_t)std::max<int32_t>(g->n, 1);
        *bytes = (size_t)cap * (fused_batch_bytes(g, lcap) + n * sizeof(double) +
                                kCtlInts * sizeof(int32_t)) + n * sizeof(double);
    } else {
        // one workspace per concurrent part
        const int32_t parts = parts_of(g, opt ? opt->concurrency : 0, nb, H);
        *bytes = (size_t)parts * (batch_ws_bytes(g, H) + batch_level_bytes(g, lcap, H));
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

bc_status bc_workspace_held(bc_graph_t g, size_t *bytes) {
    if (!g || !bytes) return BC_ERR_INVALID_ARG;
    size_t b = 0;
    {
        std::lock_guard<std::mutex> lk(g->mu);
        for (const PlainWS *ws : g->plain_pool) b += ws->bytes + ws->trunc_cap * sizeof(int32_t);
        for (const BatchWS *ws : g->batch_pool)
            b += ws->bytes + (ws->lcap ? batch_level_bytes(g, ws->lcap, ws->H) : 0) + ws->src_cap;
    }
    {
        std::lock_guard<std::mutex> lk(g->fused_mu);
        const auto &f = g->fused;
        if (f.block)
            b += f.bytes + (size_t)f.cap * (sizeof(BatchDev) + sizeof(int2));
        if (f.d_total) b += (size_t)std::max<int32_t>(g->n, 1) * sizeof(double);
        b += f.lanes_cap;
    }
    *bytes = b;
    return BC_OK;
}

bc_status bc_trim_workspaces(bc_graph_t g) {
    if (!g) return BC_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    {
        // the device-loop pool, unless a run holds it
        std::unique_lock<std::mutex> lk(g->fused_mu, std::try_to_lock);
        if (lk.owns_lock()) fused_release(g);
    }
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

#ifdef BC_CHECK_EXEC
// Check builds only (not part of include/bc.h): cross-lane helper calls made
// with part of a wave inactive, over every kernel file, since the last call.
unsigned int bc_debug_exec_partial(void) {
    return exec_partial_batched() + exec_partial_plain() + exec_partial_sssp() +
           exec_partial_pagerank();
}
#endif

}  // extern "C"
