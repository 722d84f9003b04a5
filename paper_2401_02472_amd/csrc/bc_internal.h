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
//   bucket 0 (d <= kB0MaxDeg):  one lane,
//   bucket 1 (d <= kB1MaxDeg):  a group of kB1Lanes lanes,
//   bucket 2 (larger):          one wavefront per chunk of kChunkArcs arcs;
//                               chunks of one vertex are combined in a fixed order.
constexpr int kB0MaxDeg = 8;
constexpr int kB1MaxDeg = 64;
constexpr int kB1Lanes = 8;
constexpr int kChunkArcs = 2048;

// The library relabels vertices by degree, descending, when a graph is
// created, so the buckets are id ranges: [0, b2_end) bucket 2,
// [b2_end, b1_end) bucket 1, the rest bucket 0.
__host__ __device__ inline int degree_bucket(int32_t d) {
    return d <= kB0MaxDeg ? 0 : (d <= kB1MaxDeg ? 1 : 2);
}
__host__ __device__ inline uint32_t chunks_of(int32_t d) {
    return (uint32_t)((d + kChunkArcs - 1) / kChunkArcs);
}

// Per-level bookkeeping of the BFS queues.  Level L of bucket b occupies
// queue_b[start_b .. start_b + cnt_b).  Counts are appended to atomically while
// the level is being discovered (during the kernel of level L-1); starts are
// written by the kernel of level L-1 as well, before anything reads them.
struct LevelRec {
    uint32_t start0, start1;
    uint32_t vstart2, cstart2;  // bucket 2: first vertex slot, first chunk slot
    uint32_t cnt0, cnt1;
    unsigned long long cnt2;    // (vertex count << 32) | chunk count
};
static_assert(sizeof(LevelRec) == 32, "LevelRec layout");

// Device view of one plain (one source at a time) workspace.
struct PlainDev {
    int32_t n;
    int32_t b2_end, b1_end;  // bucket id ranges (see degree_bucket)
    const int32_t *row_ptr;
    const int32_t *col_idx;
    uint32_t *lev3;       // 2 bits per vertex (16 per word): level mod 3, or 3 = not reached
    uint8_t *nextmap;     // 1 byte per vertex (padded to 16): marked for the next level
    double *sigma;        // shortest-path counts
    double *coef;         // (1 + delta[v]) / sigma[v], written by the reverse sweep
    int32_t *q0, *q1, *q2;  // per-bucket queues (all levels back to back)
    int32_t *q2c;         // bucket 2: first chunk slot of the vertex
    double *partial;      // bucket 2: per-chunk partial sums
    LevelRec *lvl;        // [n + 2]
    int32_t *ctrl;        // [0] deepest non-empty level, [1] range flag
    double *bc;           // [n] accumulated BC
};

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
hipError_t gather_i32(int32_t n, const int32_t *perm, const int32_t *src, int32_t *dst,
                      hipStream_t stream);

hipError_t plain_reset_run(const PlainDev &d, hipStream_t stream);
hipError_t plain_init_source(const PlainDev &d, int32_t s, hipStream_t stream);
// Forward step of level L: sigma of the level-L vertices and the marks of
// level L+1, then the compaction of the marks into the level L+1 queues.
hipError_t plain_forward_level(const PlainDev &d, int32_t level, int grid, hipStream_t stream);
// Reverse step of level L (>= 1); `deepest` marks the last level (no children).
hipError_t plain_backward_level(const PlainDev &d, int32_t level, bool deepest, int grid,
                                double *delta_out, hipStream_t stream);
// Single-source export: fill dist = -1, sigma = 0, delta = 0 (any may be NULL),
// then write dist / sigma of every vertex on levels 0..deepest.
hipError_t plain_export_fill(int32_t n, int32_t *dist, double *sigma, double *delta,
                             hipStream_t stream);
hipError_t plain_export_levels(const PlainDev &d, int32_t deepest, int32_t *dist, double *sigma,
                               hipStream_t stream);

}  // namespace bcx
