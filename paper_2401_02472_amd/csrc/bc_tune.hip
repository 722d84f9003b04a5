// The autotuner behind BC_MODE_AUTO.
#include "bc_runtime.h"

using namespace bcx;

extern "C" {

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
