// Internal declarations shared by the library's HIP translation units.
// Not part of the public ABI (include/bc.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace bcx {

constexpr int kWave = 64;             // CDNA wavefront width
constexpr int kBlock = 256;           // threads per workgroup for the level kernels
constexpr int kWavesPerBlock = kBlock / kWave;

// Degree buckets of the frontier queues.  A vertex of degree d is processed by
//   bucket 0 (d <= kB0MaxDeg):   one lane,
//   bucket 1 (d <= kB1MaxDeg):   a group of kB1Lanes lanes,
//   bucket 2 (d <= kChunkArcs):  one wavefront,
//   bucket 3 (larger):           one wavefront per chunk of kChunkArcs arcs;
//                                the chunks' partial sums are combined in chunk
//                                order by the next kernel on the stream.
constexpr int kB0MaxDeg = 8;
constexpr int kB1MaxDeg = 64;
constexpr int kB1Lanes = 8;
constexpr int kChunkArcs = 2048;
constexpr int kBuckets = 4;

// Work counters of measured runs (device, 64-bit each): [0..2] forward
// owners / arcs / hits, [3] vertices queued by the plain compaction, [6..8]
// reverse owners / arcs / hits, [9..11] SSSP, [12] / [13] vertices whose
// arcs the batched forward / reverse kernels walked.
constexpr int kStatWords = 16;

// The library relabels vertices by degree, descending, when a graph is
// created, so the buckets are id ranges: [0, b3_end) bucket 3,
// [b3_end, b2_end) bucket 2, [b2_end, b1_end) bucket 1, the rest bucket 0.
__host__ __device__ inline int degree_bucket(int32_t d) {
    return d <= kB0MaxDeg ? 0 : (d <= kB1MaxDeg ? 1 : (d <= kChunkArcs ? 2 : 3));
}
__host__ __device__ inline uint32_t chunks_of(int32_t d) {
    return (uint32_t)((d + kChunkArcs - 1) / kChunkArcs);
}

// Per-level bookkeeping of the BFS queues.  Level L of bucket b < 3 occupies
// queue_b[start[b] .. start[b] + cnt[b]); bucket 3 occupies vertex slots
// vstart3 .. and chunk slots cstart3 ...  Counts are appended to atomically
// while the level is being discovered (by the compaction after level L-1),
// which also writes the starts before anything reads them.
struct LevelRec {
    uint32_t start[3];
    uint32_t vstart3, cstart3;
    uint32_t cnt[3];
    unsigned long long cnt3;    // (vertex count << 32) | chunk count
};
static_assert(sizeof(LevelRec) == 40, "LevelRec layout");

__host__ __device__ inline bool level_empty(const LevelRec &r) {
    return (r.cnt[0] | r.cnt[1] | r.cnt[2] | (uint32_t)(r.cnt3 >> 32)) == 0u;
}

// Device view of one plain (one source at a time) workspace.
struct PlainDev {
    int32_t n;
    int32_t b3_end, b2_end, b1_end;  // bucket id ranges (see degree_bucket)
    const int32_t *row_ptr;
    const int32_t *col_idx;
    uint32_t *lev3;       // 2 bits per vertex (16 per word): level mod 3, or 3 = not reached
    uint8_t *nextmap;     // 1 byte per vertex (padded to 16): marked for the next level
    double *sigma;        // shortest-path counts
    double *coef;         // (1 + delta[v]) / sigma[v], written by the reverse sweep
    int32_t *q[kBuckets]; // per-bucket queues (all levels back to back)
    int32_t *q3c;         // bucket 3: first chunk slot of the vertex
    double *partial;      // bucket 3: per-chunk partial sums
    LevelRec *lvl;        // [n + 2]
    int32_t *ctrl;        // [0] deepest non-empty level of the current source,
                          // [1] range flag, [2] current source truncated (more
                          // levels than launched), [3] deepest level of the run,
                          // [4] sum of the depths of the run's earlier sources
    unsigned long long *stats;  // NULL, or work counters when measuring:
                                // [0..2] forward owners/arcs/parent arcs,
                                // [3] vertices queued by the compaction,
                                // [6..8] reverse owners/arcs/child arcs
    double *bc;           // [n] accumulated BC
};

// Device view of one batched workspace (up to 64 sources, one per lane, with
// H = 1; up to 128 with H = 2, a wave running each work item once per half).
// Vertices [0, big_end) (degree > 64) are processed as chunk items of kChunk
// arcs; of those, [0, multi_end) (degree > kChunk) span several items.
// item_info[i] = (vertex, chunk index); item_first[v] = first item of v.  For
// a directed graph the degree is the larger of the in- and out-degree, and a
// vertex below big_end has at least one item in either direction.
constexpr int kChunk = 512;
// Host-loop work items of graphs with fewer than kFineGroups groups of 64
// vertices: a cut of kFineCut arcs and chunks of kFineChunk.  Such a graph has
// too few group items to fill the device (one wave each), and a dense group's
// arcs make a long chain of dependent gathers in its one wave; vertices of
// more than kFineCut arcs as chunk items spread the arcs over more waves.
// Measured on R-MAT (edge factor 16, 64 sources, host loop): scale 12 2.18 ->
// 0.74 ms, 14 2.14 -> 0.92, 16 2.52 -> 1.05, 18 3.52 -> 1.90; at scale 20
// (16K groups) the 64 / 512 items stay faster (6.1 against 7.6 ms).
constexpr int kFineCut = 8;
constexpr int kFineChunk = 128;
constexpr int kFineGroups = 8192;
// Default threshold of the batched forward step: a level whose frontier has
// fewer than nnz / kDefaultSparseDiv arcs expands from the frontier.
constexpr int kDefaultSparseDiv = 64;
// Most batches one call runs at once (each with its own workspace and stream).
constexpr int kMaxParts = 8;

struct BatchDev {
    int32_t n;
    int32_t H;             // lane words per vertex: 1 (up to 64 sources) or 2 (up to 128)
    int32_t lcap;          // levels the F array holds
    int32_t big_end, multi_end;
    int32_t chunk;         // arcs per chunk item (a multiple of 64, at most 4096)
    uint32_t items;        // chunk items of the vertices below big_end
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const int2 *item_info;
    const uint32_t *item_first;  // [big_end + 1]
    // The forward pass pulls over the arcs into each vertex: for a directed
    // graph the reversed CSR and its own chunk items, for an undirected one
    // the same arrays as above.
    uint32_t items_in;
    const int32_t *row_ptr_in;
    const int32_t *col_idx_in;
    const int2 *item_info_in;
    const uint32_t *item_first_in;
    // Per-source arrays have H lane words (or 64-value rows) per vertex,
    // interleaved: word h of vertex v at v*H + h, half h of its row at
    // (v*H + h)*64; bit / lane s of half h stands for source 64*h + s.
    uint64_t *vis;         // [n][H] sources that reached v
    uint64_t *F;           // [lcap][n][H] F[L][v]: sources at distance L from v
    double *sigma;         // [n][H][64] path counts as doubles (wide rows)
    uint32_t *sigma32;     // [n][H][64] the same memory as exact uint32 counts (narrow rows)
    int32_t narrow;        // 1: sigma32 rows are in use
    double *coef;          // [n][H][64] (1 + delta) / sigma
    uint64_t *reach;       // [multi_end][H] sources reaching a split vertex this iteration
    double *partial;       // [max(items, items_in)][H][64] per-chunk-item sums: the
                           // forward pass's parent counts of split vertices
                           // (items_in), the reverse pass's child sums (items)
    int32_t *ctrl;         // see kCtl* below
    // sparse forward step: cand marks the neighbours of the frontier (1 byte
    // per vertex, padded to 16); clist lists the marked vertices of degree
    // <= 64, ilist the chunk items of the larger ones
    uint8_t *cand;
    int32_t *clist;
    int32_t *ilist;
    unsigned long long *front;  // [kFrontSets][kFrontWaves][2]
    int64_t nnz;
    int64_t sparse_arcs;   // a level runs sparse when its frontier has fewer arcs
    unsigned long long *stats;  // NULL, or work counters when measuring (see
                                // kStatWords)
    double *bc;            // [H][n] accumulated BC per half (internal order), when nseg == 0
    // Several requests in one batch (nseg > 0): lanes [seg_start[g],
    // seg_start[g+1]) feed seg_out[g], an [n] array in caller vertex order.
    int32_t nseg;
    const int32_t *seg_start;
    double *const *seg_out;
    const int32_t *iperm;  // internal id -> caller id
    // Extended range (wide rows only; all three NULL otherwise).  Level L's
    // rows hold sigma * 2^-xe[L][s] for lane s; level L+1's counts are summed
    // from them and stored times xs[L][s] = 2^-k, k chosen from the largest
    // stored value of level L (xmax[L][s], the bits of a positive double) so
    // that counts of any size stay inside double's range.
    double *xs;                 // [lcap][H][64]
    int32_t *xe;                // [lcap][H][64]
    unsigned long long *xmax;   // [lcap][H][64]
};

// BatchDev::ctrl layout (int32 words).
enum {
    kCtlDeepest = 0,   // deepest level found
    kCtlRange = 1,     // some sigma (or scaled coefficient) out of range
    kCtlTrunc = 2,     // level array full: run the batch again with more room
    kCtlMode = 3,      // 1: the running iteration takes the sparse forward step
    kCtlCand = 4,      // candidates listed by the sparse step
    kCtlItems = 5,     // chunk items listed by the sparse step
    kCtlNarrow = 6,    // a path count does not fit the uint32 sigma rows
    kCtlLevel = 7,     // base level of a replayed chunk of level steps
    kCtlInts = 8
};

// A level argument of kRelLevel + i is relative: a chunk of level steps
// captured once (a HIP graph) and replayed for any base level reads the base
// from ctrl[kCtlLevel]; step i of a forward chunk runs level base + i, of a
// reverse chunk level base - i.  Smaller arguments are the level itself.
constexpr int32_t kRelLevel = 1 << 30;

// Per-wave frontier counts of one forward iteration: set 0 the scan-all step,
// set 1 the sparse step, set 2 the completion of split vertices; each wave of
// those kernels stores (vertices, arcs) of the new frontier it found in its
// own slot, and the bookkeeping kernel adds them up (no shared counter).
constexpr int kMaxGridBlocks = 2048;
// Waves per SIMD the batched level kernels (forward, sparse pull, reverse)
// are compiled for: at most 96 VGPRs each, a few values spilled.  Their waves
// mostly wait on memory, and the fifth wave per SIMD gave 6-7 % on the
// scale-22 R-MAT (no change on the ER and grid graphs); six spill too much.
constexpr int kLevelWaves = 5;
constexpr int kFrontWaves = kMaxGridBlocks * kWavesPerBlock;
constexpr int kFrontSets = 3;

#ifdef BC_CHECK_EXEC
// Check builds: each kernel file's count of cross-lane helper calls made with
// part of a wave inactive since the last read (see BC_FULL_EXEC in bc_wave.h).
unsigned int exec_partial_batched();
unsigned int exec_partial_plain();
unsigned int exec_partial_sssp();
unsigned int exec_partial_pagerank();
#endif

// Launchers (bc_batched.hip).  All are asynchronous on `stream`.
// Clear the batch state and seed source s with src_dev[s], s < nlanes (<= 64 H).
hipError_t batch_start(const BatchDev &d, const int32_t *src_dev, int32_t nlanes,
                       hipStream_t stream);
// Forward iteration L -> L+1 (nlanes sources in use), then batch_forward_done
// (completes split vertices, depth bookkeeping).
hipError_t batch_forward(const BatchDev &d, int32_t level, int32_t nlanes, hipStream_t stream);
hipError_t batch_forward_done(const BatchDev &d, int32_t level, hipStream_t stream);
// Reverse iteration of level L (>= 1): child sums (not for the deepest
// level), then batch_finalize (delta, c, BC).
hipError_t batch_reverse(const BatchDev &d, int32_t level, hipStream_t stream);
hipError_t batch_finalize(const BatchDev &d, int32_t level, bool deepest, hipStream_t stream);
// Replayed chunks: batch_finalize for a relative level (the kernel finds on
// the device whether it is the deepest one, or no level at all); the chunk's
// base moved by `delta` levels; the reverse pass's base set to the deepest
// level found.
hipError_t batch_finalize_rel(const BatchDev &d, int32_t level_rel, hipStream_t stream);
hipError_t batch_level_advance(const BatchDev &d, int32_t delta, hipStream_t stream);
hipError_t batch_level_from_deepest(const BatchDev &d, hipStream_t stream);
// dist [nlanes][n] (int32) and sigma [nlanes][n] of the batch, internal order.
// Every batch of a call in one launch, one workgroup per batch (graphs small
// enough for one compute unit per batch); devs_dev[b] is batch b's workspace,
// batches_dev[b] = (first lane in lanes_dev, lane count).
hipError_t batch_fused(const BatchDev *devs_dev, int32_t nbatches, bool narrow,
                       const int32_t *lanes_dev, const int2 *batches_dev, hipStream_t stream);
hipError_t batch_export(const BatchDev &d, int32_t deepest, int32_t nlanes, int32_t *dist,
                        double *sigma, hipStream_t stream);

// Device view of a single-source shortest-path run (bc_sssp.hip): the graph's
// out-arcs with their weights (NULL: every arc weighs 1), the same chunk items
// as the batched BC path, a distance and a pass stamp per vertex.
struct SsspDev {
    int32_t n;
    int32_t big_end;
    uint32_t items;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const int32_t *weight;
    const int2 *item_info;
    int32_t *dist;
    int32_t *stamp;               // pass that must relax the vertex's arcs
    unsigned long long *stats;    // NULL, or [0..2]: vertices relaxed, arcs, improvements
};

// Device view of a PageRank run (bc_pagerank.hip): the reversed CSR and its
// chunk items (for the pull), the out-offsets (out-degrees), two rank and
// two share buffers (iteration i reads [i & 1], writes [(i + 1) & 1]), chunk
// partials of the split vertices, per-wave change slots (2 sets) and the
// change of every iteration (-1 = not run).
struct PrDev {
    int32_t n;
    int32_t big_end, multi_end;
    uint32_t items_in;
    const int32_t *row_ptr;
    const int32_t *row_ptr_in;
    const int32_t *col_idx_in;
    const int2 *item_info_in;
    const uint32_t *item_first_in;
    double *pr[2];
    double *contrib[2];
    double *partial;
    double *slots;   // [2][kFrontWaves]
    double *diff;    // [max_iter]
    double damping, base, tol;  // base = (1 - damping) / n
};

hipError_t pagerank_init(const PrDev &d, int32_t max_iter, hipStream_t stream);
// One iteration = pagerank_pull (the sums, most of the work), then
// pagerank_finish (split vertices and the iteration's change).
hipError_t pagerank_pull(const PrDev &d, int32_t iter, hipStream_t stream);
hipError_t pagerank_finish(const PrDev &d, int32_t iter, hipStream_t stream);

hipError_t sssp_init(int32_t n, int32_t *dist, int32_t *stamp, int32_t src, hipStream_t stream);
hipError_t sssp_pass(const SsspDev &d, int32_t pass, const int32_t *prev, int32_t *cur,
                     hipStream_t stream);
hipError_t sssp_export(int32_t n, const int32_t *perm, const int32_t *dist, int32_t *out,
                       hipStream_t stream);
hipError_t permute_arc_values(int32_t n, int64_t nnz, const int32_t *old_rp,
                              const int32_t *old_vals, const int32_t *new_rp,
                              const int32_t *iperm, int32_t *new_vals, hipStream_t stream);

// Launchers (bc_plain.hip).  All are asynchronous on `stream`.
// Graph set-up (bc_graph.hip).
// new_ci[e] = perm[old_ci[old_rp[iperm[u]] + e - new_rp[u]]] for the internal
// vertex u owning arc e of the relabelled CSR.
hipError_t relabel_csr(int32_t n, int64_t nnz, const int32_t *old_rp, const int32_t *old_ci,
                       const int32_t *new_rp, const int32_t *perm, const int32_t *iperm,
                       int32_t *new_ci, hipStream_t stream);
// dst[o] = src[perm[o]] for o < n (internal order -> caller order).
hipError_t gather_f64(int32_t n, const int32_t *perm, const double *src, double *dst,
                      hipStream_t stream);
hipError_t sum_parts(int32_t n, const double *parts, int32_t nparts, double *out,
                     hipStream_t stream, bool accumulate = false);
hipError_t gather_i32(int32_t n, const int32_t *perm, const int32_t *src, int32_t *dst,
                      hipStream_t stream);

hipError_t plain_reset_run(const PlainDev &d, hipStream_t stream);
hipError_t plain_init_source(const PlainDev &d, int32_t s, hipStream_t stream);
// Forward step of level L: sigma of the level-L vertices and the marks of
// level L+1.  Then plain_compact turns the marks into the level L+1 queues
// (and completes the sigma of multi-chunk level-L vertices).
hipError_t plain_forward_level(const PlainDev &d, int32_t level, int grid, hipStream_t stream);
// `last` is the deepest level launched for this source: finding vertices
// below it marks the source truncated (ctrl[2], and *trunc_flag if given).
hipError_t plain_compact(const PlainDev &d, int32_t level, int32_t last, int32_t *trunc_flag,
                         hipStream_t stream);
// Reverse step of level L (>= 1); `deepest` = 1 marks the last level (no
// children), 0 not, -1 lets the kernel decide.  Then plain_finish_reverse
// completes the multi-chunk vertices.  Both do nothing for a truncated source.
hipError_t plain_backward_level(const PlainDev &d, int32_t level, int deepest, int grid,
                                double *delta_out, hipStream_t stream);
hipError_t plain_finish_reverse(const PlainDev &d, int32_t level, double *delta_out,
                                hipStream_t stream);
// Single-source export: fill dist = -1, sigma = 0, delta = 0 (any may be NULL),
// then write dist / sigma of every vertex on levels 0..deepest.
hipError_t plain_export_fill(int32_t n, int32_t *dist, double *sigma, double *delta,
                             hipStream_t stream);
hipError_t plain_export_levels(const PlainDev &d, int32_t deepest, int32_t *dist, double *sigma,
                               hipStream_t stream);

}  // namespace bcx
