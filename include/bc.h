/*
 * bc.h -- C ABI of the MI355X (gfx950) Brandes betweenness-centrality library.
 *
 * The operation is the paper's ComputeBC (Section "Background", the BC
 * specification listing): given an unweighted graph, a set of sources and a
 * BC array, BC is zeroed (the attachNodeProperty(BC = 0) statement) and then,
 * for every source, a forward breadth-first pass accumulates shortest-path
 * counts sigma (iterateInBFS) and a reverse pass over the BFS levels, skipping
 * the source, accumulates dependencies delta and adds them to BC
 * (iterateInReverse).  The paper calls this Brandes' algorithm; the result is
 *
 *     BC_S(v) = sum over s in S, s != v, of sum over t != s, t != v of
 *               sigma_st(v) / sigma_st
 *
 * over ordered pairs (no factor 1/2, no normalisation).  S is a multiset: a
 * repeated source counts once per occurrence.  sigma, delta and BC are IEEE
 * double (the listing declares float; double is used because float loses
 * integer exactness of sigma at 2^24 and overflows on deep graphs).  Levels are
 * hop counts, -1 meaning "not reached" (the sentinel of the paper's generated
 * BFS kernel, Section "Code Generation", BFS traversal).
 *
 * Extended range.  Path counts can pass double's range on deep graphs (a
 * 600x600 lattice reaches C(1198, 599) ~ 2^1194).  When a run finds a count
 * beyond DBL_MAX it runs again with level-scaled counts: each level's counts
 * per source are kept times a power of two chosen from the level's largest
 * count, which the reverse pass undoes exactly; the graph then stays in this
 * mode (batched kernels, host-driven level loop) for every later call,
 * whatever the options ask.  Scaling by powers of two is exact, so results
 * keep double's rounding.  BC_ERR_RANGE remains for graphs whose counts span
 * more than about 2^1000 within one level.
 *
 * Graphs are undirected by default: a symmetric CSR (every arc u->v has a
 * matching v->u) with int32 offsets row_ptr[n+1] and int32 neighbours
 * col_idx[row_ptr[n]], the storage the paper uses on host and device (Section
 * "Code Generation", graph representation).  Parallel arcs count as distinct
 * paths; self-loops are accepted and have no effect.  With BC_GRAPH_DIRECTED
 * the CSR lists out-arcs and need not be symmetric: the BFS follows arcs
 * forward, sigma sums over the arcs into v from the previous level (the
 * library keeps the reversed CSR for this, the paper's reverse CSR of Section
 * "Code Generation") and dependencies over the arcs out of v to the next
 * level; BC is then over the ordered pairs (s, t) with t reachable from s.
 * Directed graphs run on the batched path whatever the options ask.
 *
 * Conventions for every call:
 *   - Every call returns a bc_status; no C++ exception crosses this boundary.
 *   - Pointers marked "host" are ordinary host memory; pointers marked
 *     "device" are device memory of the current HIP device (e.g. a torch
 *     tensor's data_ptr()).  Inputs are borrowed for the duration of the call
 *     (asynchronous calls: until the stream reaches the end of the call's
 *     work).  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   - A bc_graph_t is immutable after creation and may be used by several
 *     threads and streams at once; each run takes a private workspace from a
 *     pool owned by the graph.  bc_destroy_graph must not race with runs.
 */
#ifndef BC_MI355X_BC_H
#define BC_MI355X_BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bc_graph_s *bc_graph_t;

typedef enum {
    BC_OK = 0,
    BC_ERR_INVALID_ARG = 1,   /* NULL pointer, k < 0, source out of [0, n), bad option */
    BC_ERR_INVALID_GRAPH = 2, /* row_ptr[0] != 0, row_ptr decreasing, col_idx out of range,
                                 or an arc without its reverse (unless trusted symmetric) */
    BC_ERR_OUT_OF_MEMORY = 3, /* device allocation failed */
    BC_ERR_RANGE = 4,         /* shortest-path counts beyond even the extended range (see
                                 above); outputs are written but meaningless */
    BC_ERR_DEVICE = 5,        /* a HIP runtime call failed */
    BC_ERR_UNSUPPORTED = 6,   /* requested feature not available */
    BC_ERR_TOO_LARGE = 7      /* the run does not fit the fixed device array of
                                 bc_run_async_noalloc (graph too large or too deep) */
} bc_status;

/* bc_create_graph flags */
enum {
    BC_GRAPH_TRUST_SYMMETRIC = 1u << 0, /* skip the host-side symmetry check */
    BC_GRAPH_INPUT_ON_DEVICE = 1u << 1, /* row_ptr / col_idx are device pointers (they are
                                           copied to the host for the same checks) */
    BC_GRAPH_DIRECTED = 1u << 2         /* out-arc CSR of a directed graph (no symmetry) */
};

/* Execution modes (bc_options.mode). */
enum {
    BC_MODE_AUTO = 0,    /* library picks */
    BC_MODE_PLAIN = 1,   /* one source at a time, the paper's source loop */
    BC_MODE_BATCHED = 2  /* several sources share each level step (bitmask frontiers) */
};

typedef struct bc_options {
    int32_t mode;        /* BC_MODE_*                                                   */
    int32_t batch_width; /* batched mode: sources per batch, 1..128 (0 = the graph's
                            setting: bc_autotune's choice, else 64); above 64 a batch
                            keeps two 64-bit lane words per vertex (host-driven loop;
                            bc_run_multi always batches 64)                             */
    int32_t level_chunk; /* plain mode: forward levels launched per host poll, 1..1024
                            (0 = 8)                                                     */
    int32_t sparse_div;  /* batched mode: a forward level whose frontier has fewer than
                            nnz / sparse_div arcs expands from the frontier (visits only
                            the frontier's neighbours) instead of scanning every
                            unvisited vertex; 1..2^20, -1 = never, 0 = the graph's
                            setting (bc_autotune's choice, else 64)                      */
    int32_t concurrency; /* batched mode: batches run at once, each with its own
                            workspace and stream, 1..8 (0 = by workspace size: 4 up to
                            1 GB, 2 up to 16 GB, else 1); BC is the sum of the parts in
                            a fixed order, identical from run to run for one setting   */
    int32_t level_loop;  /* batched mode: BC_LOOP_* (who drives the level loop)           */
    int32_t reserved[2]; /* must be zero                                                 */
} bc_options;

/* bc_options.level_loop.  HOST: the host launches every level step as
 * grid-wide kernels and polls the depth.  DEVICE: one workgroup runs a whole
 * batch (every level, with workgroup barriers) and all batches of the call go
 * in one launch: for small graphs, where launch and polling costs dominate,
 * or many batches.  AUTO picks the loop with the lower estimated time for the
 * call's batch count (a batch on one compute unit against a batch across the
 * device; e.g. DEVICE from about 6 batches at 53K arcs, 27 at 425K, 87 at
 * 1.8M).  A graph in extended range always takes HOST (or GRAPH).  GRAPH:
 * the HOST loop with each chunk of level steps (the levels between two depth
 * polls, forward and reverse) captured once per workspace as a HIP graph and
 * replayed for every batch (the kernels read the chunk's base level from the
 * device), so a chunk costs one launch on the host; results are bit-identical
 * to HOST.  Runs measured with bc_profile_enable launch every step. */
enum {
    BC_LOOP_AUTO = 0,
    BC_LOOP_HOST = 1,
    BC_LOOP_DEVICE = 2,
    BC_LOOP_GRAPH = 3
};

/*
 * Copy an undirected CSR graph to the device and prepare it for runs.
 *   n        vertex count, n >= 0
 *   row_ptr  [n+1] offsets (host, or device with BC_GRAPH_INPUT_ON_DEVICE);
 *            row_ptr[0] = 0, non-decreasing, row_ptr[n] = arc count
 *   col_idx  [row_ptr[n]] neighbour ids in [0, n) (same memory kind as row_ptr)
 *   flags    BC_GRAPH_* bits
 *   stream   stream for the copies (the call waits for them before returning)
 *   out      receives the handle; untouched on error
 * The caller may free row_ptr / col_idx after the call returns.
 * Errors: BC_ERR_INVALID_ARG (NULL out, n < 0, NULL arrays with n > 0),
 * BC_ERR_INVALID_GRAPH, BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.
 */
bc_status bc_create_graph(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                          uint32_t flags, void *stream, bc_graph_t *out);

/* Release the graph, its device copy and every pooled workspace.  NULL is accepted. */
bc_status bc_destroy_graph(bc_graph_t g);

/* n, arc count and device bytes held by the graph (without workspaces).
 * Any output pointer may be NULL. */
bc_status bc_graph_info(bc_graph_t g, int32_t *n, int64_t *nnz, size_t *device_bytes);

/*
 * BC over a source multiset; blocking, host in / host out.
 *   sources  [k] host, each in [0, n); k >= 0 (k = 0 gives all zeros)
 *   bc_out   [n] host, overwritten with BC_S
 * Same as bc_run_async with default options on the default stream followed by
 * a copy to the host.  Errors: BC_ERR_INVALID_ARG (nothing written),
 * BC_ERR_RANGE (written, meaningless), BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.
 */
bc_status bc_run(bc_graph_t g, const int32_t *sources, int32_t k, double *bc_out);

/*
 * BC over a source multiset into device memory, ordered on `stream`.
 *   sources     [k] host (read before the call returns)
 *   bc_out_dev  [n] device, overwritten with BC_S when the stream reaches the
 *               end of the call's work
 *   opt         NULL = defaults
 * Not asynchronous in practice: the level loop is driven from the host, which
 * waits on `stream` (hipStreamSynchronize) after every chunk of forward levels
 * of every batch (one-source path: after every chunk of opt->level_chunk
 * levels) to read the BFS depth, and again at the end of the call; the call
 * returns when all of its work has finished (with concurrent parts, on the
 * library's internal streams too).  BC_ERR_RANGE is therefore always known by
 * the time the call returns.
 */
bc_status bc_run_async(bc_graph_t g, const int32_t *sources, int32_t k, double *bc_out_dev,
                       const bc_options *opt, void *stream);

/*
 * bc_run_async for callers that cannot allocate device memory (code under
 * HIP graph capture elsewhere in the process, tight serving loops, harnesses
 * that forbid hipMalloc): the same batched kernels with the host-driven level
 * loop, one batch at a time, every device buffer of the run carved out of one
 * fixed array of BC_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device from its first use of this call until the process ends.  The call
 * makes no device (or host) allocation; inputs and outputs are the caller's.
 *   sources     [k] host (read before the call returns)
 *   bc_out_dev  [n] device, overwritten with BC_S
 * Batches are the sources in the order given, batch_width at a time (the
 * graph's setting, as for bc_run_async with NULL options), so results agree
 * with bc_run_async up to the rounding of a different grouping of sources.
 * The workspace needs about 1,050 bytes per vertex plus 8 bytes per vertex and
 * level, plus 512 bytes per chunk item of the graph's work items (64 MiB hold
 * graphs of about 55,000 vertices of low degree at 16 levels).  The call
 * waits on `stream` like bc_run_async and has finished its work on return.
 * Calls that overlap on one device share the array and race: the caller
 * serialises them.  Errors: as bc_run_async; BC_ERR_TOO_LARGE, before any
 * device work, when the graph's workspace with two levels does not fit, or
 * after the forward pass when a batch is deeper than the array's level count
 * (bc_out_dev is then not written).
 */
#define BC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bc_status bc_run_async_noalloc(bc_graph_t g, const int32_t *sources, int32_t k,
                               double *bc_out_dev, void *stream);

/*
 * Several BC queries on one graph in one call, sharing batches (the serving
 * path's continuous batching).
 *   sources    [k] host: the requests' sources back to back, k = req_start[nreq]
 *   req_start  [nreq+1] host: request r owns sources[req_start[r] .. req_start[r+1])
 *   nreq       number of requests, >= 0
 *   bc_outs    [nreq] host array of device pointers, each to n doubles, overwritten
 *              with that request's BC (caller vertex order) by the end of the
 *              call's work on `stream`
 * Sources of different requests share the 64-source batches.  A request of at
 * most 64 sources never straddles two batches, and a larger one always splits
 * at the same positions, so each request's result is bit-identical to the one
 * it gets alone.  Waits on `stream` like bc_run_async.  Errors: as
 * bc_run_async; BC_ERR_INVALID_ARG also for a decreasing req_start or a NULL
 * output.
 */
bc_status bc_run_multi(bc_graph_t g, const int32_t *sources, const int32_t *req_start,
                       int32_t nreq, double *const *bc_outs, void *stream);

/*
 * BC of several graphs in one call (Section "Background", ComputeBC, on each
 * graph): graph i from its ks[i] sources into bc_outs_dev[i].  The 64-source
 * batches of the graphs that join go in one device-resident launch, one
 * workgroup per batch (two launches when some graphs keep double rows), so
 * many small graphs of uneven size share a launch; the others run after it on
 * the host-driven loop.  level_loop: BC_LOOP_DEVICE, every graph joins;
 * BC_LOOP_HOST, none does; BC_LOOP_AUTO, the graphs with the shortest batches
 * join, as many as minimise the estimated time of the launch (its slowest
 * batch) plus the host-loop runs of the rest (the cost model of
 * BC_LOOP_AUTO).  Each graph's result is bit-identical to bc_run_async on that
 * graph with BC_MODE_BATCHED, batch_width 64 and the loop reported in
 * loops[i]; a graph that joins but cannot stay (extended range, more batches
 * than its device-loop pool holds at once) or whose batches call for a rerun
 * (double rows, a longer level array) runs on its own afterwards, as such a
 * call would.
 *   graphs       [ngraphs] host array of distinct graphs on one device
 *   sources      [ngraphs] host array of host arrays: sources[i] holds ks[i]
 *                sources of graph i (NULL allowed where ks[i] == 0)
 *   ks           [ngraphs] host, ks[i] >= 0
 *   bc_outs_dev  [ngraphs] host array of device pointers, bc_outs_dev[i] to n_i
 *                doubles, overwritten with BC (caller vertex order)
 *   level_loop   BC_LOOP_AUTO, BC_LOOP_HOST or BC_LOOP_DEVICE
 *   loops        NULL or [ngraphs] host: BC_LOOP_DEVICE or BC_LOOP_HOST per graph
 * Uses each graph's device-loop pool (as bc_run_async with BC_LOOP_DEVICE) and
 * allocates the launch's tables (device memory); waits on `stream`.  Errors:
 * BC_ERR_INVALID_ARG (a NULL array or output, a graph given twice, graphs on
 * different devices, a source out of range, another level_loop), then as
 * bc_run_async.
 */
bc_status bc_run_graphs(const bc_graph_t *graphs, int32_t ngraphs, const int32_t *const *sources,
                        const int32_t *ks, double *const *bc_outs_dev, int32_t level_loop,
                        int32_t *loops, void *stream);

/*
 * One source, full per-vertex state (host outputs), for parity checks, from
 * the one-source-at-a-time path in double (no extended range: counts beyond
 * DBL_MAX give BC_ERR_RANGE, with dist still exact).  Undirected graphs only:
 * BC_ERR_UNSUPPORTED for a graph created with BC_GRAPH_DIRECTED.
 *   dist   [n] host: hop distance from s, -1 if unreachable
 *   sigma  [n] host: number of shortest s-v paths (0 if unreachable)
 *   delta  [n] host or NULL: dependency of s on v (0 for s and unreachable v)
 * Errors as bc_run.
 */
bc_status bc_single_source(bc_graph_t g, int32_t s, int32_t *dist, double *sigma,
                           double *delta);

/*
 * Batched-path detail for parity checks: BC as bc_run, plus, when not NULL,
 * per-source dist [k][n] (int32, host) and sigma [k][n] (double, host), as
 * produced by the batched kernels (opt->mode must be BC_MODE_BATCHED or
 * BC_MODE_PLAIN; NULL opt = batched).  In extended range sigma is the count
 * rounded to double: +infinity where it passes DBL_MAX.
 */
bc_status bc_run_detail(bc_graph_t g, const int32_t *sources, int32_t k, const bc_options *opt,
                        double *bc_out, int32_t *dist, double *sigma);

/* Device bytes one run with k sources and the given options would take for its
 * workspaces (for admission control): one per concurrent part, or the
 * device-resident loop's per-batch pool, at the graph's current level-array
 * estimate (a deeper graph grows it) and row width: while the graph's path
 * counts have fitted 32 bits, host-loop workspaces hold uint32 sigma rows, and
 * the run in which a count first passes 32 bits adds double rows (512 bytes
 * per vertex and 64 sources) to each part's workspace.  opt may be NULL. */
bc_status bc_workspace_bytes(bc_graph_t g, int32_t k, const bc_options *opt, size_t *bytes);

/* Free pooled workspaces that are idle (the one-source and batched pools'
 * idle entries, and the device-resident loop's pool when no run holds it).
 * Safe while other runs are in flight. */
bc_status bc_trim_workspaces(bc_graph_t g);

/* Device bytes the graph's BC workspace pools hold right now (idle or in use:
 * one-source and batched workspaces with their level arrays, the
 * device-resident loop's pool and tables), for admission control alongside
 * bc_workspace_bytes.  Excludes the graph itself (bc_graph_info), the SSSP and
 * PageRank workspaces, and a call's transient buffers. */
bc_status bc_workspace_held(bc_graph_t g, size_t *bytes);

/*
 * Measurement support, for benchmark and profiling tools.  While enabled on a
 * graph, every run on it brackets each kernel launch with HIP events on the
 * run's stream and counts the work the kernels did; bc_profile_read returns
 * the totals accumulated since the last reset.  Classes:
 *   BC_PROF_FORWARD  forward level kernel (sigma sums and next-level marks)
 *   BC_PROF_COMPACT  compaction of the marks into the next level's queues
 *   BC_PROF_REVERSE  reverse level kernel (dependency sums, BC update)
 *   BC_PROF_FINISH   completion of vertices split into several chunks
 *   BC_PROF_SSSP     one pass of bc_sssp (owners = vertices whose arcs were
 *                    relaxed, arcs = arcs relaxed, hits = improved distances)
 *   BC_PROF_PAGERANK the sum step of one bc_pagerank iteration (timing only;
 *                    its bytes follow from the graph's size)
 *   BC_PROF_FUSED    device-resident level loop: one launch runs whole
 *                    batches (its forward and reverse work counters are
 *                    added to FORWARD and REVERSE, which then show no launches)
 * owners = vertices processed (for COMPACT: vertices queued), arcs = adjacency
 * entries read, hits = parent arcs (FORWARD) or child arcs (REVERSE).
 */
enum {
    BC_PROF_FORWARD = 0,
    BC_PROF_COMPACT = 1,
    BC_PROF_REVERSE = 2,
    BC_PROF_FINISH = 3,
    BC_PROF_FUSED = 4,
    BC_PROF_SSSP = 5,
    BC_PROF_PAGERANK = 6,
    BC_PROF_CLASSES = 7
};

typedef struct bc_profile {
    int64_t launches[BC_PROF_CLASSES];
    double ms[BC_PROF_CLASSES];
    int64_t owners[BC_PROF_CLASSES];
    int64_t arcs[BC_PROF_CLASSES];
    int64_t hits[BC_PROF_CLASSES];
    int64_t runs;
    int64_t vertices[BC_PROF_CLASSES]; /* FORWARD / REVERSE of the batched path:
                                          vertices examined (mask and offsets
                                          read) */
    int64_t levels;  /* level steps taken: for every source (one-source path) or
                        batch (batched path), depth + 1 forward and depth reverse
                        steps; with P > 1 below, every run still counts all */
} bc_profile;

/* Switch measurement off (on = 0) or on for runs on g.  With on = P > 1, the
 * one-source-at-a-time path measures only every P-th source of a run, and the
 * batched path's host-driven loop only the launches of every P-th level (the
 * work counters cover the same launches), so that the event records do not
 * slow short launches; with P = 1 every launch is measured. */
bc_status bc_profile_enable(bc_graph_t g, int32_t on);

/* Copy the accumulated totals to *out; with reset != 0, clear them. */
bc_status bc_profile_read(bc_graph_t g, bc_profile *out, int32_t reset);

/*
 * Autotuner (the choices the library makes for BC_MODE_AUTO).  Times, on the
 * first min(k, 128) of `sources`, the sparse_div values at width 64 (on up to
 * 64 of them), then on the same batch the degree thresholds of the batched
 * path's work items (the cut above which a vertex is split into chunk items:
 * the graph's current one, then 4, 8, 16, 32, 64, 128; the chunk size: the
 * current one, then 64, 128, 256, 512, 1024 arcs), then widths 64, 32 and
 * 128 on the whole sample, and the
 * one-source-at-a-time path on up to 4 sources; stores the fastest batched
 * settings in the graph, together with the source count from which
 * BC_MODE_AUTO takes the batched path (one batch's time over one plain
 * source's).  Later runs on g with BC_MODE_AUTO (and batch_width / sparse_div
 * 0) use them; results stay within the usual rounding of the settings chosen.
 * The choice is remembered for the process, keyed by the graph's shape (n, arc
 * count, direction, and its vertex counts per power-of-two degree class, each
 * in 64ths of n); a later call on a graph of the same shape takes it without
 * timing (out->cached = 1).  With the environment variable
 * BC_MI355X_TUNE_CACHE naming a file, choices are also read from and appended
 * to that file (one text line per shape), so they persist across processes.
 * Runs on `stream` and waits for it.
 *   sources  [k] host, k >= 1
 *   out      NULL or receives the choice and the measured times
 * Errors: BC_ERR_INVALID_ARG, BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE (the graph's
 * settings are unchanged).  BC_ERR_RANGE from the sample runs is not an error
 * here.  Not to be called while other runs on g are in flight.
 */
typedef struct bc_tuning {
    int32_t batch_width;        /* chosen sources per batch                          */
    int32_t sparse_div;         /* chosen sparse_div (-1 = never)                     */
    int32_t min_batched;        /* BC_MODE_AUTO is batched from this many sources
                                   (INT32_MAX: never)                                 */
    int32_t sample;             /* sources timed (0: taken from the cache)            */
    double plain_ms_per_source; /* one-source-at-a-time path, per source              */
    double batch_ms;            /* the sample with the chosen settings                */
    int32_t cached;             /* 1: the choice came from the tuning cache           */
    int32_t group_cut;          /* vertices of higher degree are split into chunk
                                   items; the rest go 64 to a group item             */
    int32_t chunk;              /* arcs per chunk item                                */
    int32_t reserved;
} bc_tuning;

bc_status bc_autotune(bc_graph_t g, const int32_t *sources, int32_t k, void *stream,
                      bc_tuning *out);

/*
 * Set the degree thresholds of the batched path's work items explicitly (the
 * ones bc_autotune chooses): vertices of degree above group_cut (for a
 * directed graph, of larger in- or out-degree above it) are split into chunk
 * items of `chunk` arcs, one wavefront each, the others are taken 64 to a
 * group item with their arcs flattened into runs of 64.  Defaults 64 and 512,
 * or 8 and 128 for a graph of fewer than 8192 groups of 64 vertices (fewer
 * than 524,225 vertices), which has too few group items to fill the device.
 * The host-driven level loop uses them; the device-resident loop (one
 * workgroup per batch) always works on 64 and 512.
 *   group_cut  >= 1
 *   chunk      a multiple of 64 in [64, 4096], >= group_cut
 * Frees the graph's idle pooled batched workspaces (their partial rows follow
 * the item count).  Results stay within the usual rounding of the settings.
 * Errors: BC_ERR_INVALID_ARG, BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE (the
 * previous thresholds stay).  Not to be called while other runs on g are in
 * flight.
 */
bc_status bc_set_work_items(bc_graph_t g, int32_t group_cut, int32_t chunk);

/*
 * Single-source shortest paths over weighted arcs, the paper's second
 * propagation algorithm (Sections "fixedPoint Construct" and "Min/Max
 * Constructs": passes over the vertices modified by the previous pass relax
 * their out-arcs with Min(nbr.dist, v.dist + w) until a pass modifies
 * nothing).  Uses the graph's out-arcs (for an undirected graph, both arcs of
 * an edge; give them the same weight).
 *
 * bc_set_weights attaches arc weights: weight [row_ptr[n]] host, non-negative
 * int32, in the order of the caller's col_idx (copied; the caller may free it).
 * Until it is called every arc weighs 1 (hop distances).  Errors:
 * BC_ERR_INVALID_ARG (NULL, a negative weight), BC_ERR_RANGE (the largest
 * weight times n-1 does not fit int32: distances are int32),
 * BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.
 *
 * bc_sssp writes dist_dev [n] (device, int32, caller vertex order): the
 * distance from `source`, -1 where unreachable, complete when the call
 * returns (it waits on `stream` once per 8 queued passes).  Calls on one graph
 * are serialised (one workspace per graph).  Errors: BC_ERR_INVALID_ARG,
 * BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.
 */
bc_status bc_set_weights(bc_graph_t g, const int32_t *weight);
bc_status bc_sssp(bc_graph_t g, int32_t source, int32_t *dist_dev, void *stream);

/*
 * PageRank, the paper's pull iteration (Section "Backend Optimizations", the
 * generated reduction loop): every vertex starts at 1/n; an iteration computes
 * for each v the sum over the arcs u->v of pr[u] / outdeg(u), the new rank
 * (1 - damping)/n + damping * sum, and the L1 change sum |new - old| (the
 * listing adds the signed change, which sums to zero whenever no rank leaks;
 * the L1 norm is the test used here); iterations stop when the change is at
 * most tol or after max_iter.  Vertices without out-arcs keep no share of their
 * rank (the formula's leak).  Arcs are the graph's out-arcs (an undirected
 * graph's edges count both ways); a directed graph's sums use its reversed CSR.
 *   damping     in [0, 1] (0.85 typically)
 *   tol         >= 0; 0 runs max_iter iterations unless a change is exactly 0
 *   max_iter    >= 1
 *   pr_dev      [n] device double, caller vertex order, written by the time the
 *               call returns (it waits on `stream` once per 8 queued iterations)
 *   iterations  host, may be NULL: iterations run
 * Calls on one graph are serialised.  Errors: BC_ERR_INVALID_ARG,
 * BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.
 */
bc_status bc_pagerank(bc_graph_t g, double damping, double tol, int32_t max_iter, double *pr_dev,
                      int32_t *iterations, void *stream);

/* Static description of a status code. */
const char *bc_status_str(bc_status s);

#ifdef __cplusplus
}
#endif

#endif /* BC_MI355X_BC_H */
