// The autotuner behind BC_MODE_AUTO, and its cache of choices by graph shape.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "bc_runtime.h"

namespace bcx {
namespace {

// Shape of a graph for the tuning cache: n, arc count, direction, and the
// vertex counts of its degree classes in 64ths of n (graphs drawn from one
// generator at one size share it).
struct ShapeKey {
    int64_t n = 0, nnz = 0;
    int32_t directed = 0;
    int32_t cls[33] = {};
    bool operator==(const ShapeKey &o) const {
        if (n != o.n || nnz != o.nnz || directed != o.directed) return false;
        for (int c = 0; c < 33; ++c)
            if (cls[c] != o.cls[c]) return false;
        return true;
    }
};

struct Choice {
    int32_t width, sparse_div, min_batched, cut, chunk;
    double plain_ms, batch_ms;
};

ShapeKey shape_of(const bc_graph_s *g) {
    ShapeKey k;
    k.n = g->n;
    k.nnz = g->nnz;
    k.directed = g->directed ? 1 : 0;
    const double n = (double)std::max<int32_t>(g->n, 1);
    for (int c = 0; c < 33; ++c) k.cls[c] = (int32_t)std::lround(64.0 * (double)g->deg_class[c] / n);
    return k;
}

std::mutex cache_mu;
std::vector<std::pair<ShapeKey, Choice>> cache;  // this process's choices

const char *cache_file() {
    const char *f = std::getenv("BC_MI355X_TUNE_CACHE");
    return (f && *f) ? f : nullptr;
}

// One line per shape: "bc-tune 1 n nnz directed cls[0..32] width sparse_div
// min_batched cut chunk plain_ms batch_ms".
bool parse_line(const std::string &line, ShapeKey &k, Choice &c) {
    const char *p = line.c_str();
    char *end = nullptr;
    if (line.compare(0, 10, "bc-tune 1 ") != 0) return false;
    p += 10;
    auto num = [&](int64_t &out) {
        out = std::strtoll(p, &end, 10);
        if (end == p) return false;
        p = end;
        return true;
    };
    int64_t x = 0;
    if (!num(k.n) || !num(k.nnz) || !num(x)) return false;
    k.directed = (int32_t)x;
    for (int i = 0; i < 33; ++i) {
        if (!num(x)) return false;
        k.cls[i] = (int32_t)x;
    }
    int64_t w = 0, dv = 0, mb = 0, cut = 0, ch = 0;
    if (!num(w) || !num(dv) || !num(mb) || !num(cut) || !num(ch)) return false;
    c.width = (int32_t)w;
    c.sparse_div = (int32_t)dv;
    c.min_batched = (int32_t)mb;
    c.cut = (int32_t)cut;
    c.chunk = (int32_t)ch;
    c.plain_ms = std::strtod(p, &end);
    if (end == p) return false;
    p = end;
    c.batch_ms = std::strtod(p, &end);
    if (end == p) return false;
    const bool ok_width = c.width >= 1 && c.width <= 2 * kWave;
    const bool ok_div = c.sparse_div == -1 || (c.sparse_div >= 1 && c.sparse_div <= (1 << 20));
    const bool ok_items = c.cut >= 1 && c.chunk >= kWave && c.chunk % kWave == 0 &&
                          c.chunk <= 4096 && c.chunk >= c.cut;
    return ok_width && ok_div && ok_items && c.min_batched >= 1;
}

// A cached choice for the shape: this process's, else the cache file's.
bool lookup(const ShapeKey &key, Choice &out) {
    std::lock_guard<std::mutex> lk(cache_mu);
    for (const auto &e : cache)
        if (e.first == key) {
            out = e.second;
            return true;
        }
    const char *path = cache_file();
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        ShapeKey k;
        Choice c;
        if (parse_line(buf, k, c) && k == key) {  // the last line for a shape wins
            out = c;
            found = true;
        }
    }
    std::fclose(f);
    if (found) cache.push_back({key, out});
    return found;
}

void remember(const ShapeKey &key, const Choice &c) {
    std::lock_guard<std::mutex> lk(cache_mu);
    bool replaced = false;
    for (auto &e : cache)
        if (e.first == key) {
            e.second = c;
            replaced = true;
        }
    if (!replaced) cache.push_back({key, c});
    const char *path = cache_file();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "bc-tune 1 %lld %lld %d", (long long)key.n, (long long)key.nnz, key.directed);
    for (int i = 0; i < 33; ++i) std::fprintf(f, " %d", key.cls[i]);
    std::fprintf(f, " %d %d %d %d %d %.17g %.17g\n", c.width, c.sparse_div, c.min_batched, c.cut,
                 c.chunk, c.plain_ms, c.batch_ms);
    std::fclose(f);
}

bc_status apply(bc_graph_s *g, const Choice &c) {
    bc_status st = set_bc_items(g, c.cut, c.chunk);
    if (st != BC_OK) return st;
    g->tuned_width.store(c.width);
    g->tuned_sparse_div.store(c.sparse_div);
    g->tuned_min_batched.store(c.min_batched);
    return BC_OK;
}

}  // namespace
}  // namespace bcx

using namespace bcx;

extern "C" {

bc_status bc_autotune(bc_graph_t g, const int32_t *sources, int32_t k, void *stream_,
                      bc_tuning *out) {
    if (!g || k < 1) return BC_ERR_INVALID_ARG;
    bc_status st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    const int32_t m = std::min(k, 2 * kWave);   // the sample
    const int32_t m64 = std::min(m, kWave);     // its first batch of 64
    bc_tuning t{};
    t.batch_width = g->tuned_width.load();
    t.sparse_div = g->tuned_sparse_div.load();
    t.min_batched = g->tuned_min_batched.load();
    t.sample = m;
    t.group_cut = g->bci.cut;
    t.chunk = g->bci.chunk;
    if (g->n == 0) {
        if (out) *out = t;
        return BC_OK;
    }
    const ShapeKey key = shape_of(g);
    Choice known{};
    DeviceGuard dg(g->device);
    if (lookup(key, known)) {
        st = apply(g, known);
        if (st != BC_OK) return st;
        t.batch_width = known.width;
        t.sparse_div = known.sparse_div;
        t.min_batched = known.min_batched;
        t.sample = 0;
        t.plain_ms_per_source = known.plain_ms;
        t.batch_ms = known.batch_ms;
        t.group_cut = known.cut;
        t.chunk = known.chunk;
        t.cached = 1;
        if (out) *out = t;
        return BC_OK;
    }
    const hipStream_t stream = (hipStream_t)stream_;
    const int32_t prev_cut = g->bci.cut, prev_chunk = g->bci.chunk;
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
    auto batched = [&](int32_t count, int32_t width, int32_t div, double &ms) {
        return timed([&]() { return batched_run(g, sources, count, d_bc, width, div, 1,
                                                BC_LOOP_AUTO, stream, nullptr, nullptr); }, ms);
    };
    // sparse-step threshold at width 64 on one batch (the default first);
    // then the widths on the whole sample with the best threshold.  A setting
    // replaces the current choice only when it is more than 2 % faster (on
    // one sample batch, near-equal settings swap places from run to run).
    constexpr double kTuneMargin = 0.98;
    const int32_t divs[] = {kDefaultSparseDiv, -1, 16, 256};
    double div_ms = 1e30;
    int32_t best_div = kDefaultSparseDiv;
    for (int32_t div : divs) {
        double ms = 0;
        st = batched(m64, kWave, div, ms);
        if (st != BC_OK) break;
        if (div == kDefaultSparseDiv || ms < div_ms * kTuneMargin) {
            div_ms = ms;
            best_div = div;
        }
    }
    // degree thresholds of the work items: the cut above which a vertex is
    // split into chunk items (the rest go 64 to a group item), then the
    // chunk size, each on the same batch
    // (the graph's current thresholds were timed above; small graphs start
    // from the finer ones)
    int32_t best_cut = prev_cut, best_chunk = prev_chunk;
    auto items_ms = [&](int32_t cut, int32_t chunk, double &ms) {
        bc_status s2 = set_bc_items(g, cut, chunk);
        if (s2 == BC_OK) s2 = batched(m64, kWave, best_div, ms);
        return s2;
    };
    for (int32_t cut : {4, 8, 16, 32, 64, 128}) {
        if (st != BC_OK) break;
        if (cut == prev_cut || cut > best_chunk) continue;
        double ms = 0;
        st = items_ms(cut, best_chunk, ms);
        if (st == BC_OK && ms < div_ms * kTuneMargin) {
            div_ms = ms;
            best_cut = cut;
        }
    }
    for (int32_t chunk : {64, 128, 256, 512, 1024}) {
        if (st != BC_OK) break;
        if (chunk == prev_chunk || chunk < best_cut) continue;
        double ms = 0;
        st = items_ms(best_cut, chunk, ms);
        if (st == BC_OK && ms < div_ms * kTuneMargin) {
            div_ms = ms;
            best_chunk = chunk;
        }
    }
    if (st == BC_OK) st = set_bc_items(g, best_cut, best_chunk);
    double best_ms = div_ms;
    int32_t best_width = kWave;
    if (st == BC_OK && m > kWave) st = batched(m, kWave, best_div, best_ms);
    for (int32_t width : {32, 2 * kWave}) {
        if (st != BC_OK || m <= std::min(width, kWave)) continue;
        double ms = 0;
        st = batched(m, width, best_div, ms);
        if (st == BC_OK && ms < best_ms * kTuneMargin) {
            best_ms = ms;
            best_width = width;
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
    if (st != BC_OK) {
        (void)set_bc_items(g, prev_cut, prev_chunk);  // the graph's settings as they were
        return st;
    }
    const double per_source = std::max(plain_ms / p, 1e-6);
    // one batch of the chosen width (the sample ran ceil(m / width) of them);
    // the batched path wins for a single batch once k * per_source exceeds
    // the batch time, and beyond one batch when it won for one
    const double batches = std::ceil((double)m / best_width);
    const double ratio = std::ceil(best_ms / batches / per_source);
    const int32_t min_batched = ratio > (double)best_width ? INT32_MAX
                                                           : std::max<int32_t>(2, (int32_t)ratio);
    const Choice c{best_width, best_div, min_batched, best_cut, best_chunk, per_source, best_ms};
    st = apply(g, c);
    if (st != BC_OK) return st;
    remember(key, c);
    t.batch_width = best_width;
    t.sparse_div = best_div;
    t.min_batched = min_batched;
    t.plain_ms_per_source = per_source;
    t.batch_ms = best_ms;
    t.group_cut = best_cut;
    t.chunk = best_chunk;
    if (out) *out = t;
    return BC_OK;
}

bc_status bc_set_work_items(bc_graph_t g, int32_t group_cut, int32_t chunk) {
    if (!g) return BC_ERR_INVALID_ARG;
    DeviceGuard dg(g->device);
    return set_bc_items(g, group_cut, chunk);
}

}  // extern "C"
