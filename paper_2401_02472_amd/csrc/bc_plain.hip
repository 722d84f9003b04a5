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
//     its level, kept in per-degree-bucket queues that the previous level's
//     kernel appended to with wavefront-aggregated atomics (one atomic per
//     wave and bucket, positions from ballot + mbcnt).
//   * One pass per level does both the sigma sum of a level-L vertex (over its
//     level L-1 neighbours) and the discovery of its unreached neighbours for
//     level L+1, so each adjacency list is read once in the forward direction.
//   * Level tests read a 2-bit "level mod 3" code per vertex (n/4 bytes, which
//     stays in each XCD's L2) instead of an int32 level array: neighbours of a
//     reached vertex lie within one level of it, so level mod 3 tells parent,
//     sibling and child apart.  Discovery turns the code from 3 (not reached)
//     into (L+1) mod 3 with one atomicAnd, which exactly one caller wins.
//   * The reverse pass sums c[w] = (1 + delta[w]) / sigma[w] over children w
//     and sets delta[v] = sigma[v] * sum, which equals the listing's
//     sum of (sigma[v] / sigma[w]) * (1 + delta[w]) up to rounding.
//   * Degree buckets pick one lane, an 8-lane group, or one wavefront per
//     2048-arc chunk per vertex; chunks of one vertex are combined in chunk
//     order by the last chunk to finish, so every sum has a fixed order and
//     results are identical from run to run.
#include "bc_internal.h"

namespace bcx {
namespace {

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t lev_code(const uint32_t *lev3, int32_t v) {
    return (lev3[v >> 4] >> ((v & 15) << 1)) & 3u;
}

// Turn v's code from 3 (not reached) into `code`; true for exactly one caller.
__device__ __forceinline__ bool lev_claim(uint32_t *lev3, int32_t v, uint32_t code) {
    const uint32_t sh = (uint32_t)(v & 15) << 1;
    const uint32_t clear = ((~code) & 3u) << sh;
    const uint32_t old = atomicAnd(&lev3[v >> 4], ~clear);
    return ((old >> sh) & 3u) == 3u;
}

struct LevelCtx {
    PlainDev d;
    int32_t L;
    uint32_t code_parent;  // (L-1) mod 3, or 4 (matches nothing) at the source level
    uint32_t code_next;    // (L+1) mod 3
    // first slots of level L+1 in each queue
    uint32_t ns0, ns1, nv2, nc2;
    LevelRec cur;
};

__device__ __forceinline__ LevelCtx make_ctx(const PlainDev &d, int32_t L) {
    LevelCtx c;
    c.d = d;
    c.L = L;
    c.code_parent = L > 0 ? (uint32_t)((L + 2) % 3) : 4u;
    c.code_next = (uint32_t)((L + 1) % 3);
    c.cur = d.lvl[L];
    c.ns0 = c.cur.start0 + c.cur.cnt0;
    c.ns1 = c.cur.start1 + c.cur.cnt1;
    c.nv2 = c.cur.vstart2 + (uint32_t)(c.cur.cnt2 >> 32);
    c.nc2 = c.cur.cstart2 + (uint32_t)(c.cur.cnt2 & 0xffffffffu);
    return c;
}

// Append the vertices this wave discovered (one per lane at most) to the
// level L+1 queues.  Called by all 64 lanes.
__device__ void append_discovered(const LevelCtx &c, bool found, int32_t v) {
    const uint64_t any = __ballot(found);
    if (any == 0) return;
    const int lane = lane_id();
    int32_t deg = 0;
    if (found) deg = c.d.row_ptr[v + 1] - c.d.row_ptr[v];
    const int b = found ? degree_bucket(deg) : -1;
    LevelRec *nx = &c.d.lvl[c.L + 1];

    const uint64_t m0 = __ballot(b == 0);
    if (m0) {
        const int leader = __ffsll((unsigned long long)m0) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&nx->cnt0, (uint32_t)__popcll(m0));
        base = __shfl(base, leader);
        if (b == 0) c.d.q0[c.ns0 + base + lanes_below(m0)] = v;
    }
    const uint64_t m1 = __ballot(b == 1);
    if (m1) {
        const int leader = __ffsll((unsigned long long)m1) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&nx->cnt1, (uint32_t)__popcll(m1));
        base = __shfl(base, leader);
        if (b == 1) c.d.q1[c.ns1 + base + lanes_below(m1)] = v;
    }
    const uint64_t m2 = __ballot(b == 2);
    if (m2) {
        const uint32_t nch = (b == 2) ? chunks_of(deg) : 0u;
        const uint32_t incl = wave_incl_scan(nch);
        const uint32_t total = __shfl(incl, kWave - 1);
        const int leader = __ffsll((unsigned long long)m2) - 1;
        uint32_t vb = 0, cb = 0;
        if (lane == leader) {
            const unsigned long long old = atomicAdd(
                &nx->cnt2, ((unsigned long long)__popcll(m2) << 32) | (unsigned long long)total);
            vb = (uint32_t)(old >> 32);
            cb = (uint32_t)(old & 0xffffffffu);
        }
        vb = __shfl(vb, leader);
        cb = __shfl(cb, leader);
        if (b == 2) {
            const uint32_t slot = c.nv2 + vb + lanes_below(m2);
            c.d.q2[slot] = v;
            c.d.q2c[slot] = (int32_t)(c.nc2 + cb + incl - nch);
            c.d.done2[slot] = 0;
        }
    }
    if (lane == __ffsll((unsigned long long)any) - 1) atomicMax(&c.d.ctrl[0], c.L + 1);
}

// Forward visit of arc (w -> v) for a level-L owner w.
__device__ __forceinline__ void fwd_arc(const LevelCtx &c, int32_t v, double &acc,
                                        bool &found) {
    const uint32_t code = lev_code(c.d.lev3, v);
    if (code == c.code_parent) {
        acc += c.d.sigma[v];
    } else if (code == 3u) {
        found = lev_claim(c.d.lev3, v, c.code_next);
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
    c.d.bc[v] += delta;
    if (delta_out) delta_out[v] = delta;
}

// ---- bucket 0: one lane per vertex -------------------------------------
template <bool FWD>
__device__ void level_b0(const LevelCtx &c, uint32_t item, double *delta_out) {
    const int lane = lane_id();
    const uint32_t idx = item * kWave + (uint32_t)lane;
    const bool active = idx < c.cur.cnt0;
    int32_t w = 0, rs = 0, re = 0;
    if (active) {
        w = c.d.q0[c.cur.start0 + idx];
        rs = c.d.row_ptr[w];
        re = c.d.row_ptr[w + 1];
    }
    double acc = 0.0;
    for (int32_t j = 0;; ++j) {
        const bool has = rs + j < re;
        if (__ballot(has) == 0) break;
        bool found = false;
        int32_t v = 0;
        if (has) {
            v = c.d.col_idx[rs + j];
            if (FWD) {
                fwd_arc(c, v, acc, found);
            } else if (lev_code(c.d.lev3, v) == c.code_next) {
                acc += c.d.coef[v];
            }
        }
        if (FWD) append_discovered(c, found, v);
    }
    if (active) {
        if (FWD) set_sigma(c, w, acc);
        else set_delta(c, w, acc, delta_out);
    }
}

// ---- bucket 1: kB1Lanes lanes per vertex --------------------------------
template <bool FWD>
__device__ void level_b1(const LevelCtx &c, uint32_t item, double *delta_out) {
    const int lane = lane_id();
    const int sub = lane & (kB1Lanes - 1);
    const uint32_t idx = item * (kWave / kB1Lanes) + (uint32_t)(lane / kB1Lanes);
    const bool active = idx < c.cur.cnt1;
    int32_t w = 0, rs = 0, re = 0;
    if (active) {
        w = c.d.q1[c.cur.start1 + idx];
        rs = c.d.row_ptr[w];
        re = c.d.row_ptr[w + 1];
    }
    double acc = 0.0;
    for (int32_t e = rs + sub;; e += kB1Lanes) {
        const bool has = e < re;
        if (__ballot(has) == 0) break;
        bool found = false;
        int32_t v = 0;
        if (has) {
            v = c.d.col_idx[e];
            if (FWD) {
                fwd_arc(c, v, acc, found);
            } else if (lev_code(c.d.lev3, v) == c.code_next) {
                acc += c.d.coef[v];
            }
        }
        if (FWD) append_discovered(c, found, v);
    }
#pragma unroll
    for (int off = kB1Lanes / 2; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (active && sub == 0) {
        if (FWD) set_sigma(c, w, acc);
        else set_delta(c, w, acc, delta_out);
    }
}

// ---- bucket 2: one wavefront per chunk of kChunkArcs arcs ----------------
template <bool FWD>
__device__ void level_b2(const LevelCtx &c, uint32_t item, double *delta_out) {
    const int lane = lane_id();
    const uint32_t nv = (uint32_t)(c.cur.cnt2 >> 32);
    const int32_t slot = (int32_t)(c.cur.cstart2 + item);
    // last vertex of the level whose first chunk slot is <= slot
    uint32_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (c.d.q2c[c.cur.vstart2 + mid] <= slot) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t qi = c.cur.vstart2 + lo;
    const int32_t w = c.d.q2[qi];
    const int32_t first = c.d.q2c[qi];
    const int32_t j = slot - first;
    const int32_t rs = c.d.row_ptr[w], re = c.d.row_ptr[w + 1];
    const uint32_t nch = chunks_of(re - rs);
    const int32_t cb = rs + j * kChunkArcs;
    const int32_t ce = min(re, cb + kChunkArcs);
    double acc = 0.0;
    for (int32_t e = cb + lane;; e += kWave) {
        const bool has = e < ce;
        if (__ballot(has) == 0) break;
        bool found = false;
        int32_t v = 0;
        if (has) {
            v = c.d.col_idx[e];
            if (FWD) {
                fwd_arc(c, v, acc, found);
            } else if (lev_code(c.d.lev3, v) == c.code_next) {
                acc += c.d.coef[v];
            }
        }
        if (FWD) append_discovered(c, found, v);
    }
    acc = wave_sum(acc);
    if (nch == 1) {
        if (lane == 0) {
            if (FWD) set_sigma(c, w, acc);
            else set_delta(c, w, acc, delta_out);
        }
        return;
    }
    // Several chunks: publish this chunk's partial; the last chunk to finish
    // adds all partials in chunk order.
    uint32_t prev = 0;
    if (lane == 0) {
        __hip_atomic_store(&c.d.partial[first + j], acc, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        prev = __hip_atomic_fetch_add((uint32_t *)&c.d.done2[qi], 1u, __ATOMIC_ACQ_REL,
                                      __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = __shfl(prev, 0);
    if (prev != nch - 1) return;
    double t = 0.0;
    for (uint32_t k = (uint32_t)lane; k < nch; k += kWave)
        t += __hip_atomic_load(&c.d.partial[first + k], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    t = wave_sum(t);
    if (lane == 0) {
        if (FWD) set_sigma(c, w, t);
        else set_delta(c, w, t, delta_out);
        c.d.done2[qi] = 0;
    }
}

template <bool FWD>
__global__ __launch_bounds__(kBlock) void k_level(PlainDev d, int32_t L, double *delta_out) {
    const LevelCtx c = make_ctx(d, L);
    if (FWD && blockIdx.x == 0 && threadIdx.x == 0) {
        LevelRec *nx = &d.lvl[L + 1];
        nx->start0 = c.ns0;
        nx->start1 = c.ns1;
        nx->vstart2 = c.nv2;
        nx->cstart2 = c.nc2;
        LevelRec *nn = &d.lvl[L + 2];
        nn->cnt0 = 0;
        nn->cnt1 = 0;
        nn->cnt2 = 0ull;
    }
    const uint32_t nch2 = (uint32_t)(c.cur.cnt2 & 0xffffffffu);
    const uint32_t w1 = (c.cur.cnt1 + (kWave / kB1Lanes) - 1) / (kWave / kB1Lanes);
    const uint32_t w0 = (c.cur.cnt0 + kWave - 1) / kWave;
    const uint32_t total = nch2 + w1 + w0;
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    for (uint32_t it = wave; it < total; it += nwaves) {
        if (it < nch2) level_b2<FWD>(c, it, delta_out);
        else if (it < nch2 + w1) level_b1<FWD>(c, it - nch2, delta_out);
        else level_b0<FWD>(c, it - nch2 - w1, delta_out);
    }
}

__global__ void k_reset_run(PlainDev d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        d.ctrl[0] = 0;
        d.ctrl[1] = 0;
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
        const int32_t deg = d.row_ptr[s + 1] - d.row_ptr[s];
        const int b = degree_bucket(deg);
        LevelRec r0 = {0u, 0u, 0u, 0u, 0u, 0u, 0ull};
        if (b == 0) {
            r0.cnt0 = 1;
            d.q0[0] = s;
        } else if (b == 1) {
            r0.cnt1 = 1;
            d.q1[0] = s;
        } else {
            r0.cnt2 = (1ull << 32) | (unsigned long long)chunks_of(deg);
            d.q2[0] = s;
            d.q2c[0] = 0;
            d.done2[0] = 0;
        }
        d.lvl[0] = r0;
        LevelRec r1 = {0u, 0u, 0u, 0u, 0u, 0u, 0ull};
        d.lvl[1] = r1;
        d.sigma[s] = 1.0;
        d.ctrl[0] = 0;
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
        const uint32_t n2 = (uint32_t)(r.cnt2 >> 32);
        const uint32_t tot = r.cnt0 + r.cnt1 + n2;
        for (uint32_t i = (uint32_t)tid; i < tot; i += (uint32_t)stride) {
            int32_t v;
            if (i < r.cnt0) v = d.q0[r.start0 + i];
            else if (i < r.cnt0 + r.cnt1) v = d.q1[r.start1 + i - r.cnt0];
            else v = d.q2[r.vstart2 + i - r.cnt0 - r.cnt1];
            if (dist) dist[v] = L;
            if (sigma) sigma[v] = d.sigma[v];
        }
    }
}

}  // namespace

hipError_t plain_reset_run(const PlainDev &d, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset_run, dim3(1), dim3(64), 0, stream, d);
    return hipGetLastError();
}

hipError_t plain_init_source(const PlainDev &d, int32_t s, hipStream_t stream) {
    const int32_t words = (d.n + 15) >> 4;
    int grid = (words + kBlock - 1) / kBlock;
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_init_source, dim3(grid), dim3(kBlock), 0, stream, d, s);
    return hipGetLastError();
}

hipError_t plain_forward_level(const PlainDev &d, int32_t level, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_level<true>, dim3(grid), dim3(kBlock), 0, stream, d, level,
                       (double *)nullptr);
    return hipGetLastError();
}

hipError_t plain_backward_level(const PlainDev &d, int32_t level, int grid, double *delta_out,
                                hipStream_t stream) {
    hipLaunchKernelGGL(k_level<false>, dim3(grid), dim3(kBlock), 0, stream, d, level,
                       delta_out);
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
    int grid = (n + kBlock - 1) / kBlock;
    if (grid < 1) grid = 1;
    if (grid > 2048) grid = 2048;
    hipLaunchKernelGGL(k_export_fill, dim3(grid), dim3(kBlock), 0, stream, n, dist, sigma,
                       delta);
    return hipGetLastError();
}

}  // namespace bcx
