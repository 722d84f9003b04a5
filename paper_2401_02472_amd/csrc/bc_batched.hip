// Batched Brandes betweenness centrality: up to 64 sources share every level
// step, one source per lane of a wavefront.
//
// The computation per source is the paper's (Section "Background", the
// ComputeBC listing): a forward breadth-first pass summing sigma over parents
// and a reverse pass over the levels summing over children.  The paper runs
// its source loop one source after another; here a batch of up to 64 sources
// advances level by level together:
//
//   F_L[v]   64-bit mask, bit s set when v is at distance L from source s
//   vis[v]   64-bit mask of the sources that have reached v
//   sigma[v][s], c[v][s]   lane-major rows of 64 doubles (512 bytes)
//
// Forward iteration L (pull): for every vertex w with lanes still unvisited
// and every neighbour v, m = F_L[v] & ~vis[w] are the sources for which v is a
// parent of w; lane s adds sigma[v][s] for s in m (a coalesced row read), and
// the union of the m is the set of sources reaching w at level L+1.  The
// neighbour ids and masks are probed once per arc for all 64 sources.
//
// Reverse iteration L: for every vertex v with F_L[v] != 0 and every neighbour
// w, m = F_{L+1}[w] & F_L[v] are the sources for which w is a child of v; lane
// s adds c[w][s].  A finalising pass then sets delta = sigma[v][s] * sum,
// c[v][s] = (1 + delta) / sigma[v][s], and adds the lanes' deltas to BC[v] in
// lane order (v != source always holds at levels >= 1).
//
// Work items: a vertex of degree > 64 is split into chunks of 512 arcs (8 per
// lane, loaded together), one wavefront per chunk; chunks of one vertex are
// combined by exact FP64 atomic adds of integer sigma (forward) or by partial
// rows summed in chunk order (reverse).  Vertices of degree <= 64 are taken 64
// at a time: the wavefront flattens their arcs into runs of 64 and walks the
// hits in vertex order.  Every sum has a fixed order except the forward
// combine of split vertices, which adds integers exactly; results are
// identical from run to run.
#include "bc_internal.h"

namespace bcx {
namespace {

constexpr int kProbe = 8;    // arcs per lane probed together in a chunk item
constexpr int kUnroll = 8;   // neighbour rows gathered concurrently

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x |= __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    const uint32_t lo = __shfl((uint32_t)x, src);
    const uint32_t hi = __shfl((uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    const int lane = lane_id();
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    total = __shfl(incl, kWave - 1);
    return incl - x;
}

// The last lane whose first flattened arc (exclusive prefix `excl`,
// non-decreasing over lanes) is <= a: the owner of flattened arc a.
__device__ __forceinline__ int owner_lane(uint32_t excl, uint32_t a) {
    int o = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t ex = __shfl(excl, o + step);  // o + step <= 63 at every step
        if (ex <= a) o += step;
    }
    return o;
}

// Per-lane work counters, reported only when measurement is switched on:
// owners = (vertex, source) pairs completed, arcs = arcs probed, hits =
// (arc, source) pairs whose row value was gathered.
struct Work {
    uint32_t owners = 0, arcs = 0, hits = 0;
};

__device__ void report_work(unsigned long long *out, const Work &wk) {
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

// Walk the lanes set in `hit` (each holding a neighbour id `nb` and a lane
// mask `m`), kUnroll rows at a time; lane s adds val[nb][s] when s is in m.
__device__ __forceinline__ void gather_hits(uint64_t hit, int32_t nb, uint64_t m,
                                            const double *val, double &acc, Work &wk) {
    const int lane = lane_id();
    while (hit) {
        int32_t vj[kUnroll];
        bool on[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int j = 0;
            if (hit) {
                j = __ffsll((unsigned long long)hit) - 1;
                hit &= hit - 1;
                vj[u] = __shfl(nb, j);
                on[u] = (shfl64(m, j) >> lane) & 1ull;
            } else {
                vj[u] = 0;
                on[u] = false;
            }
        }
        double x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x[u] = on[u] ? val[(size_t)vj[u] * kWave + lane] : 0.0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) wk.hits += on[u] ? 1u : 0u;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += x[u];
    }
}

// Probe the arcs first + 64*u + lane (u < kProbe, below `end`) of one vertex:
// m = mask[neighbour] & keep, then gather val rows for the hits.
__device__ __forceinline__ uint64_t probe_chunk(const BatchDev &d, int32_t first, int32_t end,
                                                const uint64_t *mask, uint64_t keep,
                                                const double *val, double &acc, Work &wk) {
    const int lane = lane_id();
    int32_t nb[kProbe];
    uint64_t m[kProbe];
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
        const int32_t e = first + u * kWave + lane;
        nb[u] = e < end ? d.col_idx[e] : -1;
        wk.arcs += e < end ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < kProbe; ++u) m[u] = nb[u] >= 0 ? (mask[nb[u]] & keep) : 0ull;
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
        any |= m[u];
        gather_hits(__ballot(m[u] != 0ull), nb[u], m[u], val, acc, wk);
    }
    return wave_or(any);
}

// ---- forward ---------------------------------------------------------------

// Size of the next frontier (vertices and arcs), counted per lane and added
// to the level's counters once per wavefront at the end of a kernel.
struct Front {
    uint32_t cnt = 0;
    unsigned long long arcs = 0;
};

__device__ void report_front(const BatchDev &d, int32_t L, const Front &fr) {
    unsigned long long c = fr.cnt, a = fr.arcs;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        c += __shfl_xor(c, off);
        a += __shfl_xor(a, off);
    }
    if (lane_id() == 0 && c) {
        const int nx = (L + 1) & 1;
        atomicAdd((uint32_t *)&d.ctrl[kCtlQCount + nx], (uint32_t)c);
        atomicAdd((unsigned long long *)&d.ctrl[kCtlQArcs + 2 * nx], a);
    }
}

// Chunk item of a vertex of degree > 64.
__device__ void fwd_chunk(const BatchDev &d, int32_t L, uint32_t item, uint64_t full,
                          uint64_t *found, Work &wk, Front &fr) {
    const int lane = lane_id();
    const int2 info = d.item_info[item];
    const int32_t w = info.x, j = info.y;
    const int32_t rs = d.row_ptr[w], re = d.row_ptr[w + 1];
    const bool multi = w < d.multi_end;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n;
    const uint64_t vis = d.vis[w];
    const uint64_t unvis = ~vis & full;
    if (unvis == 0ull) {
        if (!multi && lane == 0) FN[w] = 0ull;
        return;
    }
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n;
    const int32_t cb = rs + j * kChunk;
    double acc = 0.0;
    const uint64_t nw = probe_chunk(d, cb, min(re, cb + kChunk), FL, unvis, d.sigma, acc, wk);
    const bool mine = (nw >> lane) & 1ull;
    if (mine && (!multi || j == 0)) ++wk.owners;
    if (!multi) {
        if (mine) {
            d.sigma[(size_t)w * kWave + lane] = acc;
            if (!isfinite(acc)) atomicOr(&d.ctrl[kCtlRange], 1);
        }
        if (lane == 0) {
            FN[w] = nw;
            if (nw) {
                d.vis[w] = vis | nw;
                atomicOr((unsigned long long *)found, 1ull);
            }
        }
        if (lane == 0 && nw) {
            ++fr.cnt;
            fr.arcs += (unsigned long long)(re - rs);
        }
    } else if (nw) {
        // integer sums: the atomic adds are exact in any order
        if (mine) unsafeAtomicAdd(&d.sigma[(size_t)w * kWave + lane], acc);
        if (lane == 0) atomicOr((unsigned long long *)&d.reach[w], (unsigned long long)nw);
    }
}

// Group item: 64 vertices, either base .. base+63 (dense step: all of degree
// <= 64, F_{L+1} written for every one) or list[base .. base+63] (sparse step:
// candidates of any degree, F_{L+1} cleared beforehand).  The wave flattens
// the arcs of the vertices that still have unvisited lanes into runs of 64.
__device__ void fwd_group(const BatchDev &d, int32_t L, int32_t base, const int32_t *list,
                          int32_t count, uint64_t full, uint64_t *found, Work &wk, Front &fr) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n;
    int32_t me = -1;
    if (list) {
        if (base + lane < count) me = list[base + lane];
    } else if (base + lane < d.n) {
        me = base + lane;
    }
    uint64_t vis = full;
    int32_t rs = 0, cnt = 0;
    if (me >= 0) {
        vis = d.vis[me];
        if (!list) FN[me] = 0ull;
        if (vis != full) {
            rs = d.row_ptr[me];
            cnt = d.row_ptr[me + 1] - rs;
        }
    }
    uint32_t total;
    const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
    const uint64_t unvis = ~vis & full;
    int cur = -1;        // owner lane being accumulated
    double acc = 0.0;
    uint64_t nw = 0;
    uint64_t any_found = 0;
    auto flush = [&]() {
        if (cur >= 0 && nw) {
            const int32_t w = __shfl(me, cur);                   // all lanes active here
            const uint64_t w_vis = ~shfl64(unvis, cur) & full;
            const int32_t w_deg = __shfl(cnt, cur);
            if ((nw >> lane) & 1ull) {
                d.sigma[(size_t)w * kWave + lane] = acc;
                if (!isfinite(acc)) atomicOr(&d.ctrl[kCtlRange], 1);
                ++wk.owners;
            }
            if (lane == 0) {
                FN[w] = nw;
                d.vis[w] = w_vis | nw;
                ++fr.cnt;
                fr.arcs += (unsigned long long)w_deg;
            }
            any_found |= nw;
        }
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t a = c0 + (uint32_t)lane;
        const int o = owner_lane(excl, a);
        // cross-lane reads first, with every lane active
        const int32_t o_rs = __shfl(rs, o);
        const uint32_t o_excl = __shfl(excl, o);
        const uint64_t o_keep = shfl64(unvis, o);
        int32_t nb = -1;
        uint64_t m = 0;
        if (a < total) {
            nb = d.col_idx[o_rs + (int32_t)(a - o_excl)];
            m = FL[nb] & o_keep;
            ++wk.arcs;
        }
        uint64_t hit = __ballot(m != 0ull);
        while (hit) {
            // hits of one owner at a time, gathered kUnroll rows at once
            const int h0 = __ffsll((unsigned long long)hit) - 1;
            const int own = __shfl(o, h0);
            if (own != cur) {
                flush();
                cur = own;
                acc = 0.0;
                nw = 0;
            }
            const uint64_t same = __ballot(o == own) & hit;
            hit &= ~same;
            nw |= wave_or(((same >> lane) & 1ull) ? m : 0ull);
            gather_hits(same, nb, m, d.sigma, acc, wk);
        }
    }
    flush();
    if (lane == 0 && any_found) atomicOr((unsigned long long *)found, 1ull);
}

__global__ __launch_bounds__(kBlock) void k_batch_forward(BatchDev d, int32_t L, uint64_t full) {
    // nothing past the deepest level found so far (F_L is empty), no room, or
    // this level takes the sparse step
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || d.ctrl[kCtlMode]) return;
    uint64_t *found = (uint64_t *)&d.ctrl[kCtlFound];
    const uint32_t items = d.items;
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    Front fr;
    for (uint32_t it = wave; it < items + groups; it += nwaves) {
        if (it < items) fwd_chunk(d, L, it, full, found, wk, fr);
        else fwd_group(d, L, d.big_end + (int32_t)(it - items) * kWave, nullptr, 0, full, found,
                       wk, fr);
    }
    report_front(d, L, fr);
    if (d.stats) report_work(d.stats, wk);
}

// After a forward iteration: completes the split vertices, records the depth
// (or the truncation when the level array is full), clears the flag.
__global__ __launch_bounds__(kBlock) void k_batch_forward_finish(BatchDev d, int32_t L,
                                                                 uint64_t full) {
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap) return;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n;
    uint64_t *found = (uint64_t *)&d.ctrl[kCtlFound];
    Front fr;
    const int lane = lane_id();
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    for (int32_t w = wave; w < d.multi_end; w += nwaves) {
        const uint64_t nw = d.reach[w];
        if (lane == 0) FN[w] = nw;
        if (nw == 0ull) continue;
        if ((nw >> lane) & 1ull) {
            if (!isfinite(d.sigma[(size_t)w * kWave + lane])) atomicOr(&d.ctrl[kCtlRange], 1);
        }
        if (lane == 0) {
            d.vis[w] |= nw;
            d.reach[w] = 0ull;
            atomicOr((unsigned long long *)found, 1ull);
            ++fr.cnt;
            fr.arcs += (unsigned long long)(d.row_ptr[w + 1] - d.row_ptr[w]);
        }
    }
    report_front(d, L, fr);
    (void)full;
}

// Bookkeeping between iterations (one thread): depth (or truncation when the
// level array is full), the step the next iteration takes (sparse when the
// new frontier has few arcs), and the counters of the lists.
__global__ void k_batch_level_done(BatchDev d, int32_t L) {
    uint64_t *found = (uint64_t *)&d.ctrl[kCtlFound];
    if (*found) {
        d.ctrl[kCtlDeepest] = L + 1;
        if (L + 2 >= d.lcap) d.ctrl[kCtlTrunc] = 1;  // level L+2 would not fit
    }
    *found = 0ull;
    const int nx = (L + 1) & 1, cur = L & 1;
    const unsigned long long arcs = *(unsigned long long *)&d.ctrl[kCtlQArcs + 2 * nx];
    d.ctrl[kCtlMode] = (int64_t)arcs < d.sparse_arcs ? 1 : 0;
    // the list of level L is consumed: it receives level L+2
    d.ctrl[kCtlQCount + cur] = 0;
    *(unsigned long long *)&d.ctrl[kCtlQArcs + 2 * cur] = 0ull;
    d.ctrl[kCtlCand] = 0;
    d.ctrl[kCtlItems] = 0;
}

// ---- sparse forward step ------------------------------------------------------

// Mark every neighbour of the level-L frontier (the vertices with F_L != 0,
// found by scanning F_L 64 vertices per wave; their arcs 8 per lane per
// round).  Marks are idempotent byte stores.
__global__ __launch_bounds__(kBlock) void k_batch_sparse_mark(BatchDev d, int32_t L) {
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n;
    const int32_t groups = (d.n + kWave - 1) / kWave;
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    for (int32_t gi = wave; gi < groups; gi += nwaves) {
        const int32_t me = gi * kWave + lane;
        const bool on = me < d.n && FL[me] != 0ull;
        uint64_t todo = __ballot(on);
        while (todo) {
            const int t = __ffsll((unsigned long long)todo) - 1;
            todo &= todo - 1;
            const int32_t v = gi * kWave + t;
            const int32_t rs = d.row_ptr[v], re = d.row_ptr[v + 1];
            for (int32_t cb = rs; cb < re; cb += kProbe * kWave) {
                int32_t nb[kProbe];
#pragma unroll
                for (int u = 0; u < kProbe; ++u) {
                    const int32_t e = cb + u * kWave + lane;
                    nb[u] = e < re ? d.col_idx[e] : -1;
                }
#pragma unroll
                for (int u = 0; u < kProbe; ++u)
                    if (nb[u] >= 0) d.cand[nb[u]] = 1;
            }
        }
    }
}

// Turn the marks into the candidate lists (one thread per 16 vertices), clear
// them, and clear F_{L+1} (the sparse pull writes only the candidates').
__global__ __launch_bounds__(kBlock) void k_batch_sparse_compact(BatchDev d, int32_t L,
                                                                 uint64_t full) {
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    const int lane = lane_id();
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n;
    const int32_t groups = (d.n + 15) >> 4;
    const int32_t stride = gridDim.x * kBlock;
    const int32_t base0 = blockIdx.x * kBlock + (threadIdx.x & ~(kWave - 1));
    for (int32_t wb = base0; wb < groups; wb += stride) {
        const int32_t i = wb + lane;
        uint4 m = make_uint4(0u, 0u, 0u, 0u);
        if (i < groups) {
            m = reinterpret_cast<const uint4 *>(d.cand)[i];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if ((i << 4) + j < d.n) FN[(i << 4) + j] = 0ull;
        }
        const bool any = (m.x | m.y | m.z | m.w) != 0u;
        if (__ballot(any) == 0ull) continue;
        uint32_t bits = 0;
        {
            const uint32_t wv[4] = {m.x, m.y, m.z, m.w};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if ((wv[q] >> (8 * b)) & 0xffu) bits |= 1u << (4 * q + b);
        }
        if (bits) reinterpret_cast<uint4 *>(d.cand)[i] = make_uint4(0u, 0u, 0u, 0u);
        // vertices visited from every source have nothing to discover
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (((bits >> j) & 1u) && d.vis[(i << 4) + j] == full) bits &= ~(1u << j);
        // vertices of degree <= 64 go to the candidate list; larger ones
        // contribute their chunk items to the item list
        uint32_t nsmall = 0, nitems = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            const int32_t v = (i << 4) + j;
            if (v < d.big_end) nitems += d.item_first[v + 1] - d.item_first[v];
            else ++nsmall;
        }
        uint32_t tot, toti;
        const uint32_t off = wave_excl_scan(nsmall, tot);
        const uint32_t offi = wave_excl_scan(nitems, toti);
        uint32_t base = 0, basei = 0;
        if (lane == 0) {
            if (tot) base = atomicAdd((uint32_t *)&d.ctrl[kCtlCand], tot);
            if (toti) basei = atomicAdd((uint32_t *)&d.ctrl[kCtlItems], toti);
        }
        base = __shfl(base, 0);
        basei = __shfl(basei, 0);
        uint32_t p = base + off, pi = basei + offi;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            const int32_t v = (i << 4) + j;
            if (v < d.big_end) {
                for (uint32_t it = d.item_first[v]; it < d.item_first[v + 1]; ++it)
                    d.ilist[pi++] = it;
            } else {
                d.clist[p++] = v;
            }
        }
    }
}

// Pull over the candidates only (groups of 64 list entries).
__global__ __launch_bounds__(kBlock) void k_batch_sparse_pull(BatchDev d, int32_t L,
                                                              uint64_t full) {
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    uint64_t *found = (uint64_t *)&d.ctrl[kCtlFound];
    const int32_t c = d.ctrl[kCtlCand];
    const int32_t ni = d.ctrl[kCtlItems];
    const int32_t groups = (c + kWave - 1) / kWave;
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    Front fr;
    for (int32_t it = wave; it < ni + groups; it += nwaves) {
        if (it < ni) fwd_chunk(d, L, (uint32_t)d.ilist[it], full, found, wk, fr);
        else fwd_group(d, L, (it - ni) * kWave, d.clist, c, full, found, wk, fr);
    }
    report_front(d, L, fr);
    if (d.stats) report_work(d.stats, wk);
}

// ---- reverse ---------------------------------------------------------------

// Chunk item of a vertex of degree > 64: sums of c over children, written to
// the vertex's c row (one chunk) or to the item's partial row (split vertex).
__device__ void bwd_chunk(const BatchDev &d, int32_t L, uint32_t item, Work &wk) {
    const int lane = lane_id();
    const int2 info = d.item_info[item];
    const int32_t v = info.x, j = info.y;
    const uint64_t mv = d.F[(size_t)L * (size_t)d.n + v];
    if (mv == 0ull) return;
    const uint64_t *FC = d.F + (size_t)(L + 1) * (size_t)d.n;
    const int32_t rs = d.row_ptr[v], re = d.row_ptr[v + 1];
    const int32_t cb = rs + j * kChunk;
    double acc = 0.0;
    (void)probe_chunk(d, cb, min(re, cb + kChunk), FC, mv, d.coef, acc, wk);
    if (((mv >> lane) & 1ull) && j == 0) ++wk.owners;
    if (v < d.multi_end) d.partial[(size_t)item * kWave + lane] = acc;
    else if ((mv >> lane) & 1ull) d.coef[(size_t)v * kWave + lane] = acc;
}

__device__ void bwd_group(const BatchDev &d, int32_t L, int32_t base, Work &wk) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n;
    const uint64_t *FC = d.F + (size_t)(L + 1) * (size_t)d.n;
    const int32_t me = base + lane;
    uint64_t mv = 0;
    int32_t rs = 0, cnt = 0;
    if (me < d.n) {
        mv = FL[me];
        if (mv) {
            rs = d.row_ptr[me];
            cnt = d.row_ptr[me + 1] - rs;
        }
    }
    uint32_t total;
    const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
    wk.owners += (uint32_t)__popcll((unsigned long long)mv);
    // owners with lanes at level L but no children keep sum 0: written first
    uint64_t pending = __ballot(mv != 0ull);
    int cur = -1;
    double acc = 0.0;
    auto flush = [&]() {
        if (cur < 0) return;
        const uint64_t own_mv = shfl64(mv, cur);  // all lanes active here
        if ((own_mv >> lane) & 1ull) d.coef[(size_t)(base + cur) * kWave + lane] = acc;
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t a = c0 + (uint32_t)lane;
        const int o = owner_lane(excl, a);
        const int32_t o_rs = __shfl(rs, o);
        const uint32_t o_excl = __shfl(excl, o);
        const uint64_t o_keep = shfl64(mv, o);
        int32_t nb = -1;
        uint64_t m = 0;
        if (a < total) {
            nb = d.col_idx[o_rs + (int32_t)(a - o_excl)];
            m = FC[nb] & o_keep;
            ++wk.arcs;
        }
        uint64_t hit = __ballot(m != 0ull);
        while (hit) {
            const int h0 = __ffsll((unsigned long long)hit) - 1;
            const int own = __shfl(o, h0);
            if (own != cur) {
                flush();
                cur = own;
                acc = 0.0;
                pending &= ~(1ull << own);
            }
            const uint64_t same = __ballot(o == own) & hit;
            hit &= ~same;
            gather_hits(same, nb, m, d.coef, acc, wk);
        }
    }
    flush();
    // owners without any child: their sums are 0
    while (pending) {
        const int t = __ffsll((unsigned long long)pending) - 1;
        pending &= pending - 1;
        const uint64_t own_mv = shfl64(mv, t);
        if ((own_mv >> lane) & 1ull) d.coef[(size_t)(base + t) * kWave + lane] = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_reverse(BatchDev d, int32_t L) {
    const uint32_t items = d.items;
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    for (uint32_t it = wave; it < items + groups; it += nwaves) {
        if (it < items) bwd_chunk(d, L, it, wk);
        else bwd_group(d, L, d.big_end + (int32_t)(it - items) * kWave, wk);
    }
    if (d.stats) report_work(d.stats + 6, wk);
}

// Per-request outputs: lanes [seg_start[g], seg_start[g+1]) belong to request
// g of the batch.  Each segment's deltas are rotated down to lane 0 and summed
// with the same butterfly whatever the segment's position, so a request's sum
// does not depend on where in the batch its lanes sit; it is added to the
// request's output in caller vertex order.
__device__ void add_segments(const BatchDev &d, int32_t v, double delta) {
    const int lane = lane_id();
    for (int32_t g = 0; g < d.nseg; ++g) {
        const int32_t a = d.seg_start[g], len = d.seg_start[g + 1] - a;
        double x = __shfl(delta, (lane + a) & (kWave - 1));
        x = lane < len ? x : 0.0;
        x = wave_sum(x);
        if (lane == 0 && x != 0.0) d.seg_out[g][d.iperm[v]] += x;
    }
}

// Finalise level L: for every v and lane s with s in F_L[v], the child sum is
// in c[v][s] (or in the partial rows of a split vertex); delta = sigma * sum,
// c = (1 + delta) / sigma, BC[v] += sum of the lanes' deltas.  With leaf set
// (the deepest level), every sum is 0.
__global__ __launch_bounds__(kBlock) void k_batch_finalize(BatchDev d, int32_t L, int32_t leaf) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n;
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    const int32_t groups = (d.n + kWave - 1) / kWave;
    for (int32_t gi = wave; gi < groups; gi += nwaves) {
        const int32_t me = gi * kWave + lane;
        const uint64_t m_me = me < d.n ? FL[me] : 0ull;
        uint64_t todo = __ballot(m_me != 0ull);
        while (todo) {
            int32_t vj[4];
            uint64_t mj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (todo) {
                    const int t = __ffsll((unsigned long long)todo) - 1;
                    todo &= todo - 1;
                    vj[u] = gi * kWave + t;
                    mj[u] = shfl64(m_me, t);
                } else {
                    vj[u] = -1;
                    mj[u] = 0ull;
                }
            }
            double sig[4], sum[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool on = (mj[u] >> lane) & 1ull;
                const size_t at = (size_t)(vj[u] < 0 ? 0 : vj[u]) * kWave + lane;
                sig[u] = on ? d.sigma[at] : 1.0;
                sum[u] = 0.0;
                if (on && !leaf) {
                    if (vj[u] < d.multi_end) {
                        const int32_t v = vj[u];
                        const uint32_t i0 = d.item_first[v], i1 = d.item_first[v + 1];
                        double t = 0.0;
                        for (uint32_t i = i0; i < i1; ++i) t += d.partial[(size_t)i * kWave + lane];
                        sum[u] = t;
                    } else {
                        sum[u] = d.coef[at];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool on = (mj[u] >> lane) & 1ull;
                const double delta = on ? sig[u] * sum[u] : 0.0;
                if (on) d.coef[(size_t)vj[u] * kWave + lane] = (1.0 + delta) / sig[u];
                if (d.nseg == 0) {
                    const double tot = wave_sum(delta);
                    if (lane == 0 && vj[u] >= 0 && tot != 0.0) d.bc[vj[u]] += tot;
                } else if (vj[u] >= 0) {
                    add_segments(d, vj[u], delta);
                }
            }
        }
    }
}

// ---- batch set-up and export ------------------------------------------------

// vis = 0 and F_0 = 0 everywhere; the split vertices' sigma rows and reach
// masks are cleared for the atomic combine.
__global__ void k_batch_clear(BatchDev d) {
    const int32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int32_t i = tid; i < d.n; i += stride) {
        d.vis[i] = 0ull;
        d.F[i] = 0ull;
    }
    for (int32_t i = tid; i < d.multi_end; i += stride) d.reach[i] = 0ull;
    const int32_t groups = (d.n + 15) >> 4;
    for (int32_t i = tid; i < groups; i += stride)
        reinterpret_cast<uint4 *>(d.cand)[i] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t rows = (int64_t)d.multi_end * kWave;
    for (int64_t i = tid; i < rows; i += stride) d.sigma[i] = 0.0;
    if (blockIdx.x == 0 && threadIdx.x < kCtlInts) d.ctrl[threadIdx.x] = 0;
}

// Seed lane s with its source; the first iteration's step is chosen from the
// distinct sources' arc count.
__global__ void k_batch_seed(BatchDev d, const int32_t *src, int32_t nlanes) {
    const int lane = threadIdx.x;
    int32_t s = -1;
    bool first = false;
    if (lane < nlanes) {
        s = src[lane];
        atomicOr((unsigned long long *)&d.vis[s], 1ull << lane);
        const unsigned long long old =
            atomicOr((unsigned long long *)&d.F[s], 1ull << lane);
        first = old == 0ull;  // exactly one lane per distinct source
        d.sigma[(size_t)s * kWave + lane] = 1.0;
    }
    const int32_t deg = first ? d.row_ptr[s + 1] - d.row_ptr[s] : 0;
    unsigned long long arcs = (unsigned long long)deg;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) arcs += __shfl_xor(arcs, off);
    if (lane == 0) d.ctrl[kCtlMode] = (int64_t)arcs < d.sparse_arcs ? 1 : 0;
}

// dist[s][v] and sigma[s][v] of lane s (internal vertex order), s < nlanes.
__global__ void k_batch_export(BatchDev d, int32_t deepest, int32_t nlanes, int32_t *dist,
                               double *sigma) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n;
         v += gridDim.x * blockDim.x) {
        const uint64_t vis = d.vis[v];
        for (int32_t s = 0; s < nlanes; ++s) {
            int32_t lev = -1;
            if ((vis >> s) & 1ull) {
                for (int32_t L = 0; L <= deepest; ++L)
                    if ((d.F[(size_t)L * d.n + v] >> s) & 1ull) {
                        lev = L;
                        break;
                    }
            }
            if (dist) dist[(size_t)s * d.n + v] = lev;
            if (sigma)
                sigma[(size_t)s * d.n + v] = lev >= 0 ? d.sigma[(size_t)v * kWave + s] : 0.0;
        }
    }
}

int grid_of(int64_t waves) {
    int64_t g = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

}  // namespace

hipError_t batch_start(const BatchDev &d, const int32_t *src_dev, int32_t nlanes,
                       hipStream_t stream) {
    int grid = (d.n + kBlock - 1) / kBlock;
    grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
    hipLaunchKernelGGL(k_batch_clear, dim3(grid), dim3(kBlock), 0, stream, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_seed, dim3(1), dim3(kWave), 0, stream, d, src_dev, nlanes);
    return hipGetLastError();
}

hipError_t batch_forward(const BatchDev &d, int32_t level, uint64_t full, hipStream_t stream) {
    // both steps are launched; each returns at once unless the mode chosen on
    // the device for this level is its own
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    hipLaunchKernelGGL(k_batch_forward, dim3(grid_of(d.items + groups)), dim3(kBlock), 0, stream,
                       d, level, full);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_sparse_mark, dim3(2048), dim3(kBlock), 0, stream, d, level);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_sparse_compact, dim3(grid_of(((d.n + 15) / 16 + kWave - 1) / kWave)),
                       dim3(kBlock), 0, stream, d, level, full);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch_sparse_pull, dim3(2048), dim3(kBlock), 0, stream, d, level, full);
    return hipGetLastError();
}

hipError_t batch_forward_done(const BatchDev &d, int32_t level, uint64_t full,
                              hipStream_t stream) {
    if (d.multi_end > 0) {
        hipLaunchKernelGGL(k_batch_forward_finish, dim3(grid_of(d.multi_end)), dim3(kBlock), 0,
                           stream, d, level, full);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_level_done, dim3(1), dim3(1), 0, stream, d, level);
    return hipGetLastError();
}

hipError_t batch_reverse(const BatchDev &d, int32_t level, hipStream_t stream) {
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    hipLaunchKernelGGL(k_batch_reverse, dim3(grid_of(d.items + groups)), dim3(kBlock), 0, stream,
                       d, level);
    return hipGetLastError();
}

hipError_t batch_finalize(const BatchDev &d, int32_t level, bool deepest, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_finalize, dim3(grid_of((d.n + kWave - 1) / kWave)), dim3(kBlock),
                       0, stream, d, level, deepest ? 1 : 0);
    return hipGetLastError();
}

hipError_t batch_export(const BatchDev &d, int32_t deepest, int32_t nlanes, int32_t *dist,
                        double *sigma, hipStream_t stream) {
    int grid = (d.n + kBlock - 1) / kBlock;
    grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
    hipLaunchKernelGGL(k_batch_export, dim3(grid), dim3(kBlock), 0, stream, d, deepest, nlanes,
                       dist, sigma);
    return hipGetLastError();
}

}  // namespace bcx
