// One-source-at-a-time Brandes betweenness centrality on gfx950.
//
// Follows the paper's ComputeBC specification (Section "Background", the BC
// listing): per source, sigma = 0 and sigma[src] = 1, a forward breadth-first
// pass in which every vertex sums sigma over its neighbours one level closer to
// the source (iterateInBFS), then a reverse pass over the levels, skipping the
// source, in which every vertex sums over its neighbours one level further away
// (iterateInReverse) and adds its dependency to BC.
//
// Differences from the paper's generated code (Section "Code Generation", BFS
// traversal), which scans all n vertices every level and copies a `finished`
// flag between host and device after each level:
//   * Work-efficient queues: each level kernel touches only the vertices of
//     its level, kept in per-degree-bucket queues.
//   * One pass per level does both the sigma sum of a level-L vertex (over its
//     level L-1 neighbours) and the marking of its unreached neighbours for
//     level L+1, so each adjacency list is read once in the forward direction.
//     Marking is an idempotent byte store (no atomics per arc); a compaction
//     kernel then turns the marks into the level L+1 queues, one thread per 16
//     vertices, with one atomic per wavefront and bucket (positions from
//     wavefront prefix sums).
//   * Level tests read a 2-bit "level mod 3" code per vertex (n/4 bytes, small
//     enough for each XCD's L2) instead of an int32 level array: neighbours of a
//     reached vertex lie within one level of it, so level mod 3 tells parent,
//     sibling and child apart.
//   * The reverse pass sums c[w] = (1 + delta[w]) / sigma[w] over children w
//     and sets delta[v] = sigma[v] * sum, which equals the listing's
//     sum of (sigma[v] / sigma[w]) * (1 + delta[w]) up to rounding.
//   * Degree buckets pick one lane, an 8-lane group, one wavefront, or one
//     wavefront per 2048-arc chunk per vertex.  Each lane issues its arcs' loads in batches
//     of 8 independent loads (neighbour ids, then codes, then sigma or c) so
//     that memory latency overlaps.  Sums run in a fixed order (chunks of one
//     vertex are combined in chunk order by the next kernel on the stream, so
//     no device-scope fences are needed), and results are identical from run
//     to run.
#include "bc_internal.h"
#include "bc_wave.h"

namespace bcx {
namespace {

constexpr int kBatch = 8;  // independent loads in flight per lane and batch

__device__ __forceinline__ uint32_t lev_code(const uint32_t *lev3, int32_t v) {
    return (lev3[v >> 4] >> ((v & 15) << 1)) & 3u;
}

struct LevelCtx {
    PlainDev d;
    int32_t L;
    uint32_t code_parent;  // (L-1) mod 3, or 4 (matches nothing) at the source level
    uint32_t code_next;    // (L+1) mod 3
    LevelRec cur;
};

__device__ __forceinline__ LevelCtx make_ctx(const PlainDev &d, int32_t L) {
    LevelCtx c;
    c.d = d;
    c.L = L;
    c.code_parent = L > 0 ? (uint32_t)((L + 2) % 3) : 4u;
    c.code_next = (uint32_t)((L + 1) % 3);
    c.cur = d.lvl[L];
    return c;
}

// Arcs first + stride*j, j < count (count <= kBatch), of one owner vertex.
// Forward: acc += sigma of parents, unreached neighbours are marked.
// Reverse: acc += c of children.  Terms are added in j order.
// Per-lane work counters, reported only when measurement is switched on.
struct Work {
    uint32_t owners = 0, arcs = 0, hits = 0;
};

template <bool FWD>
__device__ __forceinline__ void arc_batch(const LevelCtx &c, int32_t first, int32_t stride,
                                          int32_t count, double &acc, Work &wk) {
    int32_t v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j)
        v[j] = (j < count) ? __builtin_nontemporal_load(&c.d.col_idx[first + stride * j]) : -1;
    uint32_t code[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) code[j] = (v[j] >= 0) ? lev_code(c.d.lev3, v[j]) : 4u;
    const uint32_t want = FWD ? c.code_parent : c.code_next;
    const double *val = FWD ? c.d.sigma : c.d.coef;
    double x[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) x[j] = (code[j] == want) ? val[v[j]] : 0.0;
    wk.arcs += (uint32_t)(count > 0 ? count : 0);
#pragma unroll
    for (int j = 0; j < kBatch; ++j) wk.hits += (code[j] == want) ? 1u : 0u;
#pragma unroll
    for (int j = 0; j < kBatch; ++j) acc += x[j];
    if (FWD) {
#pragma unroll
        for (int j = 0; j < kBatch; ++j)
            if (code[j] == 3u) c.d.nextmap[v[j]] = 1;
    }
}

__device__ __forceinline__ void set_sigma(const LevelCtx &c, int32_t w, double s) {
    if (c.L == 0) return;  // the source keeps sigma = 1
    c.d.sigma[w] = s;
    if (!isfinite(s)) atomicOr(&c.d.ctrl[1], 1);
}

__device__ __forceinline__ void set_delta(const LevelCtx &c, int32_t v, double acc,
                                          double *delta_out) {
    const double sv = c.d.sigma[v];
    const double delta = sv * acc;
    c.d.coef[v] = (1.0 + delta) / sv;
    if (delta != 0.0) c.d.bc[v] += delta;
    if (delta_out) delta_out[v] = delta;
}

// ---- bucket 0: one lane per vertex (degree <= 8) --------------------------
template <bool FWD>
__device__ __forceinline__ void
level_b0(const LevelCtx &c, uint32_t item, bool leaf, double *delta_out, Work &wk) {
    const uint32_t idx = item * kWave + (uint32_t)lane_id();
    if (idx >= c.cur.cnt[0]) return;
    const int32_t w = c.d.q[0][c.cur.start[0] + idx];
    double acc = 0.0;
    if (!leaf) {
        const int32_t rs = c.d.row_ptr[w], re = c.d.row_ptr[w + 1];
        arc_batch<FWD>(c, rs, 1, re - rs, acc, wk);
    }
    ++wk.owners;
    if (FWD) set_sigma(c, w, acc);
    else set_delta(c, w, acc, delta_out);
}

// ---- bucket 1: kB1Lanes lanes per vertex (degree <= 64) --------------------
template <bool FWD>
__device__ __forceinline__ void
level_b1(const LevelCtx &c, uint32_t item, bool leaf, double *delta_out, Work &wk) {
    const int lane = lane_id();
    const int sub = lane & (kB1Lanes - 1);
    const uint32_t idx = item * (kWave / kB1Lanes) + (uint32_t)(lane / kB1Lanes);
    const bool active = idx < c.cur.cnt[1];
    int32_t w = 0;
    double acc = 0.0;
    if (active) {
        w = c.d.q[1][c.cur.start[1] + idx];
        if (!leaf) {
            const int32_t rs = c.d.row_ptr[w], re = c.d.row_ptr[w + 1];
            const int32_t cnt = (re - rs - sub + kB1Lanes - 1) / kB1Lanes;
            arc_batch<FWD>(c, rs + sub, kB1Lanes, cnt, acc, wk);
        }
    }
#pragma unroll
    for (int off = kB1Lanes / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (active && sub == 0) {
        ++wk.owners;
        if (FWD) set_sigma(c, w, acc);
        else set_delta(c, w, acc, delta_out);
    }
}

// Arcs [cb, ce) of one vertex by one wavefront; returns the wave-wide sum.
template <bool FWD>
__device__ __forceinline__ double wave_arcs(const LevelCtx &c, int32_t cb, int32_t ce,
                                            Work &wk) {
    const int lane = lane_id();
    double acc = 0.0;
    const int32_t mine = (ce - cb - lane + kWave - 1) / kWave;  // arcs of this lane
    for (int32_t t = 0; t < mine; t += kBatch)
        arc_batch<FWD>(c, cb + lane + t * kWave, kWave, min(kBatch, mine - t), acc, wk);
    return wave_sum(acc);
}

// ---- bucket 2: one wavefront per vertex (degree <= kChunkArcs) ------------
template <bool FWD>
__device__ __forceinline__ void
level_b2(const LevelCtx &c, uint32_t item, bool leaf, double *delta_out, Work &wk) {
    const int32_t w = c.d.q[2][c.cur.start[2] + item];
    double acc = 0.0;
    if (!leaf) acc = wave_arcs<FWD>(c, c.d.row_ptr[w], c.d.row_ptr[w + 1], wk);
    if (lane_id() == 0) {
        ++wk.owners;
        if (FWD) set_sigma(c, w, acc);
        else set_delta(c, w, acc, delta_out);
    }
}

// ---- bucket 3: one wavefront per chunk of kChunkArcs arcs ----------------
template <bool FWD>
__device__ __forceinline__ void
level_b3(const LevelCtx &c, uint32_t item, bool leaf, double *delta_out, Work &wk) {
    const int lane = lane_id();
    const uint32_t nv = (uint32_t)(c.cur.cnt3 >> 32);
    const int32_t slot = (int32_t)(c.cur.cstart3 + item);
    // last vertex of the level whose first chunk slot is <= slot
    uint32_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (c.d.q3c[c.cur.vstart3 + mid] <= slot) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t qi = c.cur.vstart3 + lo;
    const int32_t w = c.d.q[3][qi];
    const int32_t first = c.d.q3c[qi];
    const int32_t j = slot - first;
    const int32_t rs = c.d.row_ptr[w], re = c.d.row_ptr[w + 1];
    if (leaf) {  // a leaf level has no partials: chunk 0 finishes the vertex
        if (lane == 0 && j == 0) {
            ++wk.owners;
            if (FWD) set_sigma(c, w, 0.0);
            else set_delta(c, w, 0.0, delta_out);
        }
        return;
    }
    const int32_t cb = rs + j * kChunkArcs;
    const double acc = wave_arcs<FWD>(c, cb, min(re, cb + kChunkArcs), wk);
    if (lane == 0) {
        if (j == 0) ++wk.owners;
        c.d.partial[first + j] = acc;
    }
}

// Sum the chunk partials of the bucket-3 vertices of level L in chunk order;
// one wavefront per vertex.  Runs in the kernel after the level kernel, so the
// partials are visible without fences.
template <bool FWD>
__device__ __forceinline__ void finish_chunks(const LevelCtx &c, uint32_t wave, uint32_t nwaves,
                              double *delta_out) {
    const int lane = lane_id();
    const uint32_t nv = (uint32_t)(c.cur.cnt3 >> 32);
    for (uint32_t k = wave; k < nv; k += nwaves) {
        const uint32_t qi = c.cur.vstart3 + k;
        const int32_t w = c.d.q[3][qi];
        const uint32_t nch = chunks_of(c.d.row_ptr[w + 1] - c.d.row_ptr[w]);
        const int32_t first = c.d.q3c[qi];
        double t = 0.0;
        for (uint32_t j = (uint32_t)lane; j < nch; j += kWave) t += c.d.partial[first + j];
        t = wave_sum(t);
        if (lane == 0) {
            if (FWD) set_sigma(c, w, t);
            else set_delta(c, w, t, delta_out);
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_finish_reverse(PlainDev d, int32_t L,
                                                           double *delta_out) {
    if (d.ctrl[2]) return;
    if (level_empty(d.lvl[L + 1])) return;  // a leaf level has no partials
    const LevelCtx c = make_ctx(d, L);
    finish_chunks<false>(c, (blockIdx.x * kBlock + threadIdx.x) / kWave,
                         gridDim.x * kWavesPerBlock, delta_out);
}

__device__ __forceinline__ void report_work(unsigned long long *out, const Work &wk) {
    unsigned long long o = wk.owners, a = wk.arcs, h = wk.hits;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        o += __shfl_xor(o, off);
        a += __shfl_xor(a, off);
        h += __shfl_xor(h, off);
    }
    if (lane_id() == 0 && (o | a | h)) {
        atomicAdd(&out[0], o);
        atomicAdd(&out[1], a);
        atomicAdd(&out[2], h);
    }
}

template <bool FWD>
__global__ __launch_bounds__(kBlock) void k_level(PlainDev d, int32_t L, int32_t leaf,
                                                  double *delta_out) {
    if (!FWD && d.ctrl[2]) return;  // truncated source: it is run again with more levels
    const LevelCtx c = make_ctx(d, L);
    if (!FWD && leaf < 0) leaf = level_empty(d.lvl[L + 1]) ? 1 : 0;  // deepest level?
    const uint32_t n3 = (uint32_t)(c.cur.cnt3 & 0xffffffffu);  // chunks
    const uint32_t n2 = c.cur.cnt[2];
    const uint32_t w1 = (c.cur.cnt[1] + (kWave / kB1Lanes) - 1) / (kWave / kB1Lanes);
    const uint32_t w0 = (c.cur.cnt[0] + kWave - 1) / kWave;
    const uint32_t total = n3 + n2 + w1 + w0;
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    for (uint32_t it = wave; it < total; it += nwaves) {
        if (it < n3) level_b3<FWD>(c, it, leaf != 0, delta_out, wk);
        else if (it < n3 + n2) level_b2<FWD>(c, it - n3, leaf != 0, delta_out, wk);
        else if (it < n3 + n2 + w1) level_b1<FWD>(c, it - n3 - n2, leaf != 0, delta_out, wk);
        else level_b0<FWD>(c, it - n3 - n2 - w1, leaf != 0, delta_out, wk);
    }
    if (d.stats) report_work(d.stats + (FWD ? 0 : 6), wk);
}

// Compaction after the forward step of level L: every marked vertex gets code
// (L+1) mod 3 and a slot in the level L+1 queue of its degree bucket; marks
// are cleared.  Thread t owns vertices 16t .. 16t+15 (one code word, one
// 16-byte mark group), so codes are written without atomics.  The kernel also
// completes the sigma of the level-L bucket-3 vertices.
__global__ __launch_bounds__(kBlock) void k_compact(PlainDev d, int32_t L, int32_t last,
                                                    int32_t *trunc_flag) {
    const LevelRec cur = d.lvl[L];
    if (level_empty(cur)) {
        // a level past the deepest one: nothing is marked
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            LevelRec *nn = &d.lvl[L + 2];
            nn->cnt[0] = nn->cnt[1] = nn->cnt[2] = 0u;
            nn->cnt3 = 0ull;
        }
        return;
    }
    {
        const LevelCtx c = make_ctx(d, L);
        finish_chunks<true>(c, (blockIdx.x * kBlock + threadIdx.x) / kWave,
                            gridDim.x * kWavesPerBlock, nullptr);
    }
    uint32_t ns[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) ns[b] = cur.start[b] + cur.cnt[b];
    const uint32_t nv3 = cur.vstart3 + (uint32_t)(cur.cnt3 >> 32);
    const uint32_t nc3 = cur.cstart3 + (uint32_t)(cur.cnt3 & 0xffffffffu);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        LevelRec *nx = &d.lvl[L + 1];
#pragma unroll
        for (int b = 0; b < 3; ++b) nx->start[b] = ns[b];
        nx->vstart3 = nv3;
        nx->cstart3 = nc3;
        LevelRec *nn = &d.lvl[L + 2];
        nn->cnt[0] = nn->cnt[1] = nn->cnt[2] = 0u;
        nn->cnt3 = 0ull;
    }
    const uint32_t code = (uint32_t)((L + 1) % 3);
    const int32_t words = (d.n + 15) >> 4;
    LevelRec *nx = &d.lvl[L + 1];
    const int lane = lane_id();
    // All lanes of a wave run the same number of iterations (ballots inside).
    const int32_t stride = gridDim.x * kBlock;
    const int32_t base0 = blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
    for (int32_t wb = base0; wb < words; wb += stride) {
        const int32_t i = wb + lane;
        uint4 m = make_uint4(0u, 0u, 0u, 0u);
        if (i < words) m = reinterpret_cast<const uint4 *>(d.nextmap)[i];
        const bool any = (m.x | m.y | m.z | m.w) != 0u;
        if (__ballot(any) == 0) continue;
        uint32_t bits = 0;  // bit j: vertex 16i+j is marked
        {
            const uint32_t wv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if ((wv[q] >> (8 * b)) & 0xffu) bits |= 1u << (4 * q + b);
        }
        uint32_t cb[4] = {0u, 0u, 0u, 0u}, ch3 = 0;
        uint32_t nch[16];
        if (bits) {
            const int32_t v0 = i << 4;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                nch[j] = 0;
                if ((bits >> j) & 1u) {
                    const int32_t v = v0 + j;
                    if (v < d.b3_end) {
                        ++cb[3];
                        nch[j] = chunks_of(d.row_ptr[v + 1] - d.row_ptr[v]);
                        ch3 += nch[j];
                    } else if (v < d.b2_end) {
                        ++cb[2];
                    } else if (v < d.b1_end) {
                        ++cb[1];
                    } else {
                        ++cb[0];
                    }
                }
            }
            // codes: fields of marked vertices go from 3 to `code`
            uint32_t clear = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if ((bits >> j) & 1u) clear |= ((~code) & 3u) << (2 * j);
            d.lev3[i] &= ~clear;
            reinterpret_cast<uint4 *>(d.nextmap)[i] = make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t off[4], tot[4], offc3, totc3;
#pragma unroll
        for (int b = 0; b < 4; ++b) off[b] = wave_excl_scan(cb[b], tot[b]);
        offc3 = wave_excl_scan(ch3, totc3);
        uint32_t base[4] = {0u, 0u, 0u, 0u}, basec3 = 0u;
        if (lane == 0) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                if (tot[b]) base[b] = atomicAdd(&nx->cnt[b], tot[b]);
            if (tot[3]) {
                const unsigned long long old = atomicAdd(
                    &nx->cnt3, ((unsigned long long)tot[3] << 32) | (unsigned long long)totc3);
                base[3] = (uint32_t)(old >> 32);
                basec3 = (uint32_t)(old & 0xffffffffu);
            }
            const uint32_t found = tot[0] + tot[1] + tot[2] + tot[3];
            if (found) {
                atomicMax(&d.ctrl[0], L + 1);
                atomicMax(&d.ctrl[3], L + 1);
                if (L == last) {  // more levels than were launched for this source
                    atomicOr(&d.ctrl[2], 1);
                    if (trunc_flag) atomicOr(trunc_flag, 1);
                }
                if (d.stats) atomicAdd(&d.stats[3], (unsigned long long)found);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) base[b] = __shfl(base[b], 0);
        basec3 = __shfl(basec3, 0);
        if (bits) {
            uint32_t p0 = ns[0] + base[0] + off[0], p1 = ns[1] + base[1] + off[1];
            uint32_t p2 = ns[2] + base[2] + off[2], p3 = nv3 + base[3] + off[3];
            uint32_t pc = nc3 + basec3 + offc3;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (!((bits >> j) & 1u)) continue;
                const int32_t v = (i << 4) + j;
                if (v >= d.b1_end) {
                    d.q[0][p0++] = v;
                } else if (v >= d.b2_end) {
                    d.q[1][p1++] = v;
                } else if (v >= d.b3_end) {
                    d.q[2][p2++] = v;
                } else {
                    d.q[3][p3] = v;
                    d.q3c[p3] = (int32_t)pc;
                    ++p3;
                    pc += nch[j];
                }
            }
        }
    }
}

__global__ void k_reset_run(PlainDev d) {
    const int32_t groups = (d.n + 15) >> 4;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < groups;
         i += gridDim.x * blockDim.x)
        reinterpret_cast<uint4 *>(d.nextmap)[i] = make_uint4(0u, 0u, 0u, 0u);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d.ctrl[0] = 0;
        d.ctrl[1] = 0;
        d.ctrl[2] = 0;
        d.ctrl[3] = 0;
        d.ctrl[4] = 0;
    }
}

// All codes to 3 (not reached) except the source's (0); the source becomes
// level 0 of its degree bucket.
__global__ void k_init_source(PlainDev d, int32_t s) {
    const int32_t words = (d.n + 15) >> 4;
    const int32_t sw = s >> 4;
    const uint32_t sval = ~(3u << ((s & 15) << 1));
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += gridDim.x * blockDim.x)
        d.lev3[i] = (i == sw) ? sval : 0xffffffffu;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        LevelRec r0 = {};
        if (s < d.b3_end) {
            r0.cnt3 = (1ull << 32) |
                      (unsigned long long)chunks_of(d.row_ptr[s + 1] - d.row_ptr[s]);
            d.q[3][0] = s;
            d.q3c[0] = 0;
        } else {
            const int b = s < d.b2_end ? 2 : (s < d.b1_end ? 1 : 0);
            r0.cnt[b] = 1;
            d.q[b][0] = s;
        }
        d.lvl[0] = r0;
        LevelRec r1 = {};
        d.lvl[1] = r1;
        d.sigma[s] = 1.0;
        d.ctrl[4] += d.ctrl[0];  // the previous source's depth
        d.ctrl[0] = 0;
        d.ctrl[2] = 0;
    }
}

__global__ void k_export_fill(int32_t n, int32_t *dist, double *sigma, double *delta) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (dist) dist[i] = -1;
        if (sigma) sigma[i] = 0.0;
        if (delta) delta[i] = 0.0;
    }
}

__global__ void k_export_levels(PlainDev d, int32_t deepest, int32_t *dist, double *sigma) {
    const int32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t L = 0; L <= deepest; ++L) {
        const LevelRec r = d.lvl[L];
        const uint32_t n3 = (uint32_t)(r.cnt3 >> 32);
        const uint32_t tot = r.cnt[0] + r.cnt[1] + r.cnt[2] + n3;
        for (uint32_t i = (uint32_t)tid; i < tot; i += (uint32_t)stride) {
            int32_t v;
            uint32_t k = i;
            if (k < r.cnt[0]) {
                v = d.q[0][r.start[0] + k];
            } else if ((k -= r.cnt[0]) < r.cnt[1]) {
                v = d.q[1][r.start[1] + k];
            } else if ((k -= r.cnt[1]) < r.cnt[2]) {
                v = d.q[2][r.start[2] + k];
            } else {
                v = d.q[3][r.vstart3 + k - r.cnt[2]];
            }
            if (dist) dist[v] = L;
            if (sigma) sigma[v] = d.sigma[v];
        }
    }
}

int grid_for(int64_t items, int cap) {
    int64_t g = (items + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace

#ifdef BC_CHECK_EXEC
unsigned int exec_partial_plain() { return exec_partial_take(); }
#endif

hipError_t plain_reset_run(const PlainDev &d, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset_run, dim3(grid_for((d.n + 15) / 16, 1024)), dim3(kBlock), 0,
                       stream, d);
    return hipGetLastError();
}

hipError_t plain_init_source(const PlainDev &d, int32_t s, hipStream_t stream) {
    hipLaunchKernelGGL(k_init_source, dim3(grid_for((d.n + 15) / 16, 1024)), dim3(kBlock), 0,
                       stream, d, s);
    return hipGetLastError();
}

hipError_t plain_forward_level(const PlainDev &d, int32_t level, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_level<true>, dim3(grid), dim3(kBlock), 0, stream, d, level, 0,
                       (double *)nullptr);
    return hipGetLastError();
}

hipError_t plain_compact(const PlainDev &d, int32_t level, int32_t last, int32_t *trunc_flag,
                         hipStream_t stream) {
    hipLaunchKernelGGL(k_compact, dim3(grid_for((d.n + 15) / 16, 2048)), dim3(kBlock), 0,
                       stream, d, level, last, trunc_flag);
    return hipGetLastError();
}

hipError_t plain_backward_level(const PlainDev &d, int32_t level, int deepest, int grid,
                                double *delta_out, hipStream_t stream) {
    hipLaunchKernelGGL(k_level<false>, dim3(grid), dim3(kBlock), 0, stream, d, level, deepest,
                       delta_out);
    return hipGetLastError();
}

hipError_t plain_finish_reverse(const PlainDev &d, int32_t level, double *delta_out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_finish_reverse, dim3(64), dim3(kBlock), 0, stream, d, level, delta_out);
    return hipGetLastError();
}

hipError_t plain_export_levels(const PlainDev &d, int32_t deepest, int32_t *dist, double *sigma,
                               hipStream_t stream) {
    hipLaunchKernelGGL(k_export_levels, dim3(256), dim3(kBlock), 0, stream, d, deepest, dist,
                       sigma);
    return hipGetLastError();
}

hipError_t plain_export_fill(int32_t n, int32_t *dist, double *sigma, double *delta,
                             hipStream_t stream) {
    hipLaunchKernelGGL(k_export_fill, dim3(grid_for(n, 2048)), dim3(kBlock), 0, stream, n, dist,
                       sigma, delta);
    return hipGetLastError();
}

}  // namespace bcx
