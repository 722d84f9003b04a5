// Graph residency: CSR validation, the one-time copy to the device, the
// degree-descending relabelling and the batched path's work-item tables.
//
// The paper's generated host code copies the graph to the device once and
// returns only the modified property (Section "Backend Optimizations",
// host-device transfer analysis); here too the CSR stays resident in a
// bc_graph_t and only BC (plus debug state on request) comes back.
#include "bc_runtime.h"

using namespace bcx;

namespace bcx {

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
// The BC tables back to the default ones (freeing owned arrays).
bc_graph_s::BcItems base_items(const bc_graph_s *g) {
    bc_graph_s::BcItems t{};
    t.big_end = g->big_end;
    t.multi_end = g->multi_end;
    t.items = g->items;
    t.items_in = g->items_in;
    t.info = g->d_item_info;
    t.first = g->d_item_first;
    t.info_in = g->d_item_info_in;
    t.first_in = g->d_item_first_in;
    return t;
}

void reset_bc_items(bc_graph_s *g) {
    auto &t = g->bci;
    if (t.owned) {
        (void)hipFree(t.info);
        (void)hipFree(t.first);
        if (t.info_in != t.info) (void)hipFree(t.info_in);
        if (t.first_in != t.first) (void)hipFree(t.first_in);
    }
    t = base_items(g);
}

void free_graph_arrays(bc_graph_s *g) {
    if (g->bci.owned) reset_bc_items(g);
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

bc_status set_bc_items(bc_graph_s *g, int32_t cut, int32_t chunk) {
    const int32_t n = g->n;
    if (cut < 1 || chunk < kWave || chunk % kWave != 0 || chunk > 4096 || chunk < cut)
        return BC_ERR_INVALID_ARG;
    if (cut == g->bci.cut && chunk == g->bci.chunk) return BC_OK;
    // idle pooled workspaces go (their partial rows follow the items); the
    // device-loop pool too
    (void)bc_trim_workspaces(g);
    if (cut == kB1MaxDeg && chunk == kChunk) {
        reset_bc_items(g);
        g->bci_gen.fetch_add(1);
        return BC_OK;
    }
    // degrees in the internal order (out-arcs; in-arcs of a directed graph)
    std::vector<int32_t> rp((size_t)n + 1), rp_in;
    BC_TRY_HIP(hipMemcpy(rp.data(), g->d_row_ptr, rp.size() * sizeof(int32_t),
                         hipMemcpyDeviceToHost));
    if (g->directed) {
        rp_in.resize((size_t)n + 1);
        BC_TRY_HIP(hipMemcpy(rp_in.data(), g->d_row_ptr_in, rp_in.size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost));
    }
    auto out_deg = [&](int32_t u) { return rp[(size_t)u + 1] - rp[(size_t)u]; };
    auto in_deg = [&](int32_t u) {
        return g->directed ? rp_in[(size_t)u + 1] - rp_in[(size_t)u] : out_deg(u);
    };
    auto key_deg = [&](int32_t u) { return std::max(out_deg(u), in_deg(u)); };
    bc_graph_s::BcItems t;
    t.cut = cut;
    t.chunk = chunk;
    std::vector<int2> info, info_in;
    std::vector<uint32_t> first, first_in;
    // internal ids are key-degree-descending: the vertices above the cut are
    // a prefix, each with at least one item per direction
    for (int32_t u = 0; u < n; ++u) {
        if (key_deg(u) <= cut) break;
        t.big_end = u + 1;
        if (key_deg(u) > chunk) t.multi_end = u + 1;
        first.push_back((uint32_t)info.size());
        for (int32_t j = 0; j == 0 || (int64_t)j * chunk < out_deg(u); ++j)
            info.push_back(make_int2(u, j));
        if (g->directed) {
            first_in.push_back((uint32_t)info_in.size());
            for (int32_t j = 0; j == 0 || (int64_t)j * chunk < in_deg(u); ++j)
                info_in.push_back(make_int2(u, j));
        }
    }
    first.push_back((uint32_t)info.size());
    if (g->directed) first_in.push_back((uint32_t)info_in.size());
    t.items = (uint32_t)info.size();
    t.items_in = g->directed ? (uint32_t)info_in.size() : t.items;
    hipError_t e = hipSuccess;
    auto upload = [&](const std::vector<int2> &in_info, const std::vector<uint32_t> &in_first,
                      int2 **d_info, uint32_t **d_first) {
        if (e == hipSuccess) e = hipMalloc(d_info, std::max<size_t>(in_info.size(), 1) * sizeof(int2));
        if (e == hipSuccess) e = hipMalloc(d_first, in_first.size() * sizeof(uint32_t));
        if (e == hipSuccess && !in_info.empty())
            e = hipMemcpy(*d_info, in_info.data(), in_info.size() * sizeof(int2),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(*d_first, in_first.data(), in_first.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice);
    };
    upload(info, first, &t.info, &t.first);
    if (g->directed) {
        upload(info_in, first_in, &t.info_in, &t.first_in);
    } else {
        t.info_in = t.info;
        t.first_in = t.first;
    }
    t.owned = true;
    if (e != hipSuccess) {
        if (t.info) (void)hipFree(t.info);
        if (t.first) (void)hipFree(t.first);
        if (g->directed && t.info_in) (void)hipFree(t.info_in);
        if (g->directed && t.first_in) (void)hipFree(t.first_in);
        return from_hip(e);
    }
    reset_bc_items(g);  // frees the previous owned tables
    g->bci = t;
    g->bci_gen.fetch_add(1);
    return BC_OK;
}

}  // namespace bcx

extern "C" {

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
    for (int32_t v = 0; v < n; ++v) {
        const int32_t kd = key_deg(v);
        maxdeg = std::max(maxdeg, kd);
        int c = 0;
        while (c < 32 && ((int64_t)1 << c) <= kd) ++c;
        g->deg_class[c]++;
    }
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
    reset_bc_items(g);
    // a graph of few 64-vertex groups takes finer host-loop work items
    if (n > 0 && (n + kWave - 1) / kWave < kFineGroups) {
        const bc_status st = set_bc_items(g, kFineCut, kFineChunk);
        if (st != BC_OK) {
            free_graph_arrays(g);
            delete g;
            return st;
        }
    }
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

}  // extern "C"
