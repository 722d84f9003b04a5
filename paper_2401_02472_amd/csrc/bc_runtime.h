// Host runtime shared by the library's C-ABI translation units: the graph
// handle, the workspace pools, launch timing, and the entry points of the
// plain and batched run loops.  Not part of the public ABI (include/bc.h is).
#pragma once

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "bc.h"
#include "bc_internal.h"

namespace bcx {

constexpr size_t kAlign = 256;
constexpr int kLevelGrid = 2048;  // workgroups per level kernel (8192 wavefronts)
constexpr int kCtrlInts = 5;      // see PlainDev::ctrl

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

inline bc_status from_hip(hipError_t e) {
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
    unsigned long long *d_stats = nullptr;  // kStatWords counters
    void *block = nullptr;
    size_t bytes = 0;
    PlainDev dev{};
    int32_t *h_ctrl = nullptr;  // pinned mirror of dev.ctrl
    int32_t *d_trunc = nullptr; // per-source truncation flags of a run
    size_t trunc_cap = 0;
    hipEvent_t done = nullptr;  // recorded after the last work that used this workspace
    bool busy = false;
};

// Chunks of level steps captured as HIP graphs for replay (BC_LOOP_GRAPH):
// K forward steps (or K reverse steps) with relative levels, then the move of
// the chunk's base level.  A captured graph holds its kernels' arguments, so
// each is kept with the workspace view and lane count it was captured for.
struct ChunkGraphs {
    struct Entry {
        int32_t dir = 0, K = 0, nlanes = 0;
        BatchDev d{};
        hipGraphExec_t exec = nullptr;
    };
    hipStream_t cap = nullptr;   // capture stream (nothing runs on it)
    std::vector<Entry> entries;  // most recently captured last
    ~ChunkGraphs();
    // Launch the chunk on `stream`, capturing it first if needed.
    hipError_t replay(const BatchDev &d, int32_t dir, int32_t K, int32_t nlanes,
                      hipStream_t stream);
};

// Batched workspace: lane-major sigma / c rows for 64 sources (128 with two
// lane words per vertex), masks, and a level array that grows when a batch
// runs deeper than it holds.
struct BatchWS {
    int32_t H = 1;             // lane words per vertex (1: 64 sources, 2: 128)
    LaunchTimer timer;
    unsigned long long *d_stats = nullptr;  // kStatWords counters
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
    int32_t gen = 0;           // the graph's work-item tables it was built for
    // sigma rows sized for doubles (else for uint32: a graph whose counts fit
    // 32 bits); widened by a separate allocation when the graph needs it
    bool wide = true;
    void *wide_sigma = nullptr;
    BatchDev dev{};
    ChunkGraphs graphs;        // replayed level chunks (BC_LOOP_GRAPH)
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

struct SourceState {
    int32_t *dist = nullptr;   // device, optional export
    double *sigma = nullptr;   // device, optional export
    double *delta = nullptr;   // device, optional export
};

// Export buffers of one source in internal order (device temporaries).
struct ExportTmp {
    int32_t *dist = nullptr;
    double *sigma = nullptr;
    double *delta = nullptr;
};

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

}  // namespace bcx

// The graph handle (opaque in bc.h).
struct bc_graph_s {
    using PlainWS = bcx::PlainWS;
    using BatchWS = bcx::BatchWS;
    using BatchDev = bcx::BatchDev;

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
    // The batched BC path's work items: vertices of degree above `cut` (a
    // prefix of the internal order) in chunks of `chunk` arcs, the ones above
    // `chunk` spanning several items.  They start as the tables above (cut 64,
    // chunk 512), which SSSP, PageRank and the device-resident loop keep; a
    // small graph then takes finer ones (kFineCut, kFineChunk), and
    // bc_autotune or bc_set_work_items may rebuild them with other thresholds
    // (owned: separate device arrays).
    struct BcItems {
        int32_t cut = 64, chunk = 512;
        int32_t big_end = 0, multi_end = 0;
        uint32_t items = 0, items_in = 0;
        int2 *info = nullptr, *info_in = nullptr;
        uint32_t *first = nullptr, *first_in = nullptr;
        bool owned = false;
    } bci;
    // bumped whenever the tables change: pooled workspaces built for other
    // tables (their partial rows and item pointers) are not reused
    std::atomic<int32_t> bci_gen{0};
    // single-source shortest paths: arc weights (internal arc order; NULL =
    // every arc weighs 1) and a workspace used by one call at a time
    int32_t *d_weight = nullptr;
    std::mutex sssp_mu;
    struct Sssp {
        int32_t *dist = nullptr, *stamp = nullptr, *flags = nullptr;
        int32_t *h_flags = nullptr;               // pinned mirror of one flag block
        unsigned long long *d_stats = nullptr;    // kStatWords counters ([9..11] used)
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
    std::atomic<int32_t> tuned_width{bcx::kWave};
    std::atomic<int32_t> tuned_sparse_div{bcx::kDefaultSparseDiv};
    std::atomic<int32_t> tuned_min_batched{16};
    // vertex counts per degree class (0: degree 0, c >= 1: degree in
    // [2^(c-1), 2^c)), the shape key of the autotuner's cache
    int64_t deg_class[33] = {};
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
        unsigned long long *d_stats = nullptr;  // kStatWords work counters
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

namespace bcx {

// ---- plain runtime (bc_rt_plain.hip) ----
size_t plain_ws_bytes(const bc_graph_s *g);
void plain_ws_destroy(PlainWS *ws);
bc_status plain_acquire(bc_graph_s *g, hipStream_t stream, PlainWS **out);
void plain_release(bc_graph_s *g, PlainWS *ws, hipStream_t stream);
// `levels`: level steps the run took (forward and reverse, over its sources
// or batches).
void accumulate_profile(bc_graph_s *g, LaunchTimer &timer, const unsigned long long *d_stats,
                        int64_t levels = 0);
bc_status plain_run(bc_graph_s *g, const int32_t *sources, int32_t k, double *bc_out,
                    const bc_options *opt, hipStream_t stream, const SourceState *exp,
                    const ExportTmp *tmp);
bc_status bfs_levels(bc_graph_s *g, int32_t s, std::vector<int32_t> &out);

// ---- batched runtime (bc_rt_batched.hip) ----
size_t partial_rows(const bc_graph_s::BcItems &t);
size_t partial_rows(const bc_graph_s *g);  // of the graph's current tables
void set_items(const bc_graph_s::BcItems &t, BatchDev &d);
void set_items(const bc_graph_s *g, BatchDev &d);
size_t batch_ws_bytes(const bc_graph_s *g, int32_t H);
size_t batch_level_bytes(const bc_graph_s *g, int32_t lcap, int32_t H);
void batch_ws_destroy(BatchWS *ws);
size_t fused_batch_bytes(const bc_graph_s *g, int32_t lcap);
int32_t fused_cap(const bc_graph_s *g, int32_t nbatches, int32_t lcap);
void fused_release(bc_graph_s *g);
bool use_fused(const bc_graph_s *g, int32_t level_loop, int32_t nbatches, int32_t width);
int32_t parts_of(const bc_graph_s *g, int32_t concurrency, int32_t nbatches, int32_t H);
bc_status batched_run(bc_graph_s *g, const int32_t *sources, int32_t k, double *bc_out,
                      int32_t width, int32_t sparse_div, int32_t concurrency,
                      int32_t level_loop, hipStream_t stream, int32_t *dist, double *sigma);
bc_status multi_run(bc_graph_s *g, const int32_t *sources, const int32_t *req_start,
                    int32_t nreq, double *const *outs, hipStream_t stream);
bc_status run_graphs(bc_graph_s *const *gs, int32_t ng, const int32_t *const *sources,
                     const int32_t *ks, double *const *outs, int32_t level_loop,
                     int32_t *loops, hipStream_t stream);
// Extended-range tables of a batch workspace ([lcap][64] each).
struct ExtTables {
    double *xs;
    unsigned long long *xmax;
    int32_t *xe;
};
// Rerun: run the batch again (the graph's rows became wider); Grow: with a
// longer level array; NeedWide: the graph takes double rows and the
// workspace's sigma rows are uint32-sized: widen them, then run the batch.
enum class BatchOutcome { Done, Rerun, Grow, NeedWide };
// cg: replay the level chunks as captured graphs (NULL: launch every step).
// wide_ok: d's sigma rows hold doubles (else uint32 only: a graph that takes
// double rows gets NeedWide before anything is launched).
hipError_t drive_batch(bc_graph_s *g, BatchDev &d, const ExtTables &ext, const int32_t *lanes_dev,
                       int32_t nl, int32_t *h_ctrl, hipStream_t stream, LaunchTimer &timer,
                       unsigned long long *d_stats, int32_t stride, BatchOutcome &how,
                       int32_t &deepest, ChunkGraphs *cg, bool wide_ok);

// ---- graph residency (bc_rt_graph.hip) ----
void free_graph_arrays(bc_graph_s *g);
// Rebuild the batched BC path's work items with degree cut `cut` (vertices of
// higher degree become chunk items) and `chunk` arcs per item; frees every
// pooled batched workspace (their partial rows follow the item count).  No run
// on g may be in flight.
bc_status set_bc_items(bc_graph_s *g, int32_t cut, int32_t chunk);
// The tables built at creation (cut 64, chunk 512): the device-resident loop
// always runs on them (its 16 waves per batch gain nothing from finer items).
bc_graph_s::BcItems base_items(const bc_graph_s *g);

// ---- policy and argument checks (bc_capi.hip) ----
void plain_overflowed(bc_graph_s *g);
bool use_batched(const bc_graph_s *g, const bc_options *opt, int32_t k);
int32_t batch_width_of(const bc_graph_s *g, const bc_options *opt, int32_t k);
int32_t sparse_div_of(const bc_graph_s *g, const bc_options *opt);
bc_status check_options(const bc_options *opt);
bc_status check_sources(const bc_graph_s *g, const int32_t *sources, int32_t k);

}  // namespace bcx
