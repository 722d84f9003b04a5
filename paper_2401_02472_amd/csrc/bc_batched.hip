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
//   sigma[v][s]   lane-major rows of 64 counts: uint32 (256 bytes) while
//                 every count fits 32 bits, else doubles
//   c[v][s]       lane-major rows of 64 doubles (512 bytes)
//
// Forward iteration L (pull): for every vertex w with lanes still unvisited
// and every neighbour v, m = F_L[v] & ~vis[w] are the sources for which v is a
// parent of w; lane s adds sigma[v][s] for s in m (see the walks below), and
// the union of the m is the set of sources reaching w at level L+1.  The
// neighbour ids and masks are probed once per arc for all 64 sources.
//
// Reverse iteration L: for every vertex v with F_L[v] != 0 and every neighbour
// w, m = F_{L+1}[w] & F_L[v] are the sources for which w is a child of v; lane
// s adds c[w][s].  The wave owning v then sets delta = sigma[v][s] * sum,
// c[v][s] = (1 + delta) / sigma[v][s], and adds the lanes' deltas to BC[v] in
// lane order (v != source always holds at levels >= 1).  Vertices split over
// several work items, and the deepest level, are completed by a finalising
// pass.
//
// Work items: a vertex of degree above a cut (64 unless tuned) is split into
// chunks of arcs (512 unless tuned; 8 per lane loaded together per round), one
// wavefront per chunk; each chunk of a vertex with several chunks leaves a
// partial row of per-source sums (forward: parent counts, reverse: child
// coefficients), which the next kernel adds in chunk order.  Vertices at or
// below the cut are taken 64 at a time: the wavefront flattens their arcs into runs of 64 (one arc per
// lane) and walks the hits either arc by arc (one row for all sources per
// load) or, where arcs carry few sources each (deep, sparse levels), source by
// source: each run's 64 x 64 arc-by-source hit matrix is transposed with lane
// shuffles and each lane walks the arcs that count for its own source, so a
// load serves 64 sources on 64 different arcs.  Either way a lane adds its
// values in arc order.  Every sum has a fixed order, so results are identical
// from run to run, also where counts pass 2^53 and additions round.
#include "bc_internal.h"
#include "bc_wave.h"

namespace bcx {
namespace {

constexpr int kProbe = 8;    // arcs per lane probed together in a chunk item
constexpr int kUnroll = 8;   // neighbour rows gathered concurrently
constexpr int kRounds = 2;   // runs of 64 flattened arcs probed together in a group item
// a reverse group whose owners carry at least this many sources on average
// reads its children's c rows arc by arc (bwd_runs_rows), else source by
// source (bwd_runs_lanes)
constexpr int kDenseOwner = 8;
// a forward group whose first run's hit arcs carry at least this many
// sources on average reads parent rows arc by arc (fwd_runs_rows), else
// source by source (fwd_runs_lanes)
constexpr int kDenseArc = 4;

// Per-lane work counters, reported only when measurement is switched on:
// owners = (vertex, source) pairs completed, arcs = arcs probed, hits =
// (arc, source) pairs whose row value was gathered, verts = vertices
// examined (their mask and offsets read: every vertex of a group item, the
// first chunk of a chunked vertex).
struct Work {
    uint32_t owners = 0, arcs = 0, hits = 0, verts = 0;
};

// Adds a wave's counters to stats[base .. base + 2] and stats[vslot].
__device__ __forceinline__ void report_work(unsigned long long *stats, int base, int vslot,
                                            const Work &wk) {
    BC_FULL_EXEC();
    unsigned long long o = wk.owners, a = wk.arcs, h = wk.hits, v = wk.verts;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        o += __shfl_xor(o, off);
        a += __shfl_xor(a, off);
        h += __shfl_xor(h, off);
        v += __shfl_xor(v, off);
    }
    if (lane_id() == 0 && (o | a | h | v)) {
        atomicAdd(&stats[base], o);
        atomicAdd(&stats[base + 1], a);
        atomicAdd(&stats[base + 2], h);
        atomicAdd(&stats[vslot], v);
    }
}

// Walk the lanes set in `hit` (each holding a neighbour id `nb` and a lane
// mask `m`), kUnroll rows at a time; lane s adds val[nb][s] when s is in m.
template <int H, typename V>
__device__ __forceinline__ void gather_hits(uint64_t hit, int32_t nb, uint64_t m,
                                            const V *val, double &acc, Work &wk) {
    const int lane = lane_id();
    while (hit) {
        BC_FULL_EXEC();
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
        // raw loads first (all in flight), conversions after
        V raw[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            raw[u] = 0;
            if (on[u]) raw[u] = val[(size_t)vj[u] * (H * kWave) + lane];
        }
        double x[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x[u] = (double)raw[u];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) wk.hits += on[u] ? 1u : 0u;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) acc += x[u];
    }
}

// Take up to kUnroll of the lanes set in `hit` (lowest first; each holds a
// neighbour id `nb`, a lane mask `m` and an owner lane `o`) and load their
// rows together: x[u] = val[nb_u][lane] when lane is in m_u, else 0.  The
// owners and masks come back wave-uniform (oj[u] = -1 past the last hit), so
// the caller can fold the values into per-owner sums in arc order.
template <int H, typename V>
__device__ __forceinline__ void gather_run(uint64_t &hit, int32_t nb, uint64_t m, int o,
                                           const V *val, double (&x)[kUnroll],
                                           uint64_t (&mj)[kUnroll], int (&oj)[kUnroll],
                                           Work &wk) {
    BC_FULL_EXEC();
    const int lane = lane_id();
    int32_t vj[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        if (hit) {
            const int j = __ffsll((unsigned long long)hit) - 1;
            hit &= hit - 1;
            vj[u] = __shfl(nb, j);
            mj[u] = shfl64(m, j);
            oj[u] = __shfl(o, j);
        } else {
            vj[u] = 0;
            mj[u] = 0ull;
            oj[u] = -1;
        }
    }
    // raw loads first (all in flight), conversions after
    V raw[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const bool on = (mj[u] >> lane) & 1ull;
        raw[u] = 0;
        if (on) raw[u] = val[(size_t)vj[u] * (H * kWave) + lane];
        wk.hits += on ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) x[u] = (double)raw[u];
}

// Visit, in arc order, the arcs of one run of 64 flattened arcs that are this
// lane's: bit j of `col` set when arc j (neighbour id `nb` and owner lane `o`
// held by lane j) counts for this lane's source.  Up to kUnroll values
// val[nb_j][lane] are loaded at once, one neighbour per lane, then passed to
// take(owner, value) in arc order.  `col` comes from the transpose of the
// run's per-arc source masks, so a load serves 64 sources on different arcs
// instead of the sources of one arc.
template <int H, typename V, typename Take>
__device__ __forceinline__ void walk_own(uint64_t col, int32_t nb, int o, const V *val, Work &wk,
                                         Take &&take) {
    const int lane = lane_id();
    while (__ballot(col != 0ull)) {
        int j[kUnroll];
        bool on[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            on[u] = col != 0ull;
            j[u] = on[u] ? __ffsll((unsigned long long)col) - 1 : 0;
            col &= col - 1;
        }
        int32_t vj[kUnroll];
        int oj[kUnroll];
        BC_FULL_EXEC();
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            vj[u] = __shfl(nb, j[u]);  // every lane active here
            oj[u] = __shfl(o, j[u]);
        }
        V raw[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            raw[u] = 0;
            if (on[u]) raw[u] = val[(size_t)vj[u] * (H * kWave) + lane];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (on[u]) take(oj[u], (double)raw[u]);
            wk.hits += on[u] ? 1u : 0u;
        }
    }
}

// Probe the arcs first + 64*u + lane (u < kProbe, below `end`) of one vertex:
// m = mask[neighbour] & keep, then gather val rows for the hits.
template <int H, typename V>
__device__ __forceinline__ uint64_t probe_chunk(const int32_t *col, int32_t first, int32_t end,
                                                const uint64_t *mask, uint64_t keep,
                                                const V *val, double &acc, Work &wk) {
    const int lane = lane_id();
    int32_t nb[kProbe];
    uint64_t m[kProbe];
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
        const int32_t e = first + u * kWave + lane;
        nb[u] = e < end ? col[e] : -1;
        wk.arcs += e < end ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < kProbe; ++u) m[u] = nb[u] >= 0 ? (mask[(size_t)nb[u] * H] & keep) : 0ull;
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
        any |= m[u];
        gather_hits<H>(__ballot(m[u] != 0ull), nb[u], m[u], val, acc, wk);
    }
    return wave_or(any);
}

// ---- sigma rows ------------------------------------------------------------

// Shortest-path counts are integers.  They are kept as exact uint32 rows
// (narrow: half the bytes per gathered row) while every count fits; a count
// that does not fit raises kCtlNarrow and the batch is run again with double
// rows (wide), where a count beyond double's range raises kCtlRange.  A split
// vertex's chunks leave double partial rows, which the completion kernel adds
// in chunk order and stores into the vertex's sigma row.
template <bool N> struct SigRows;

template <> struct SigRows<true> {
    using T = uint32_t;
    __device__ static T *rows(const BatchDev &d) { return d.sigma32; }
    // a complete sum (exact in double)
    __device__ static void store(const BatchDev &d, size_t at, double acc) {
        if (acc >= 4294967296.0) atomicOr(&d.ctrl[kCtlNarrow], 1);
        d.sigma32[at] = (uint32_t)fmin(acc, 4294967295.0);
    }
};

template <> struct SigRows<false> {
    using T = double;
    __device__ static T *rows(const BatchDev &d) { return d.sigma; }
    // a complete sum: at least 1 unscaled, at least 2^-1000 scaled (below
    // that the extended range would lose precision), finite
    __device__ static void store(const BatchDev &d, size_t at, double acc) {
        d.sigma[at] = acc;
        if (!(acc >= 0x1p-1000 && acc <= 0x1.fffffffffffffp+1023))
            atomicOr(&d.ctrl[kCtlRange], 1);
    }
};

template <bool N>
__device__ __forceinline__ double sig_at(const BatchDev &d, size_t at) {
    return (double)SigRows<N>::rows(d)[at];
}

// Scale of level L for this lane: 1 unless the extended range is on.  Sums of
// level-L rows are multiplied by it when stored (forward) or completed
// (reverse); a power of two, so the product is exact.
template <bool N, int H>
__device__ __forceinline__ double level_scale(const BatchDev &d, int32_t L) {
    return (!N && d.xs) ? d.xs[(size_t)L * (H * kWave) + lane_id()] : 1.0;
}

// ---- batches of up to 128 sources ------------------------------------------

// A batch keeps H lane words per vertex: H = 1 for up to 64 sources, H = 2
// for up to 128.  Word h of vertex v's masks is at v*H + h (the words of a
// vertex share a cache line), half h of its rows at (v*H + h)*64 (a row of
// H*64 values), and each half has its own BC array.  A wave runs each work
// item once per half on the half's view of the workspace: the arc ids, offsets
// and the mask lines of the second pass come from cache.
template <int H>
__device__ __forceinline__ BatchDev half_view(const BatchDev &d, int h) {
    BatchDev e = d;
    if (H > 1 && h > 0) {
        e.vis += h;
        e.F += h;
        e.reach += h;
        e.sigma += (size_t)h * kWave;
        e.sigma32 += (size_t)h * kWave;
        e.coef += (size_t)h * kWave;
        e.partial += (size_t)h * kWave;
        e.bc += (size_t)h * (size_t)d.n;
        if (e.xs) {
            e.xs += (size_t)h * kWave;
            e.xmax += (size_t)h * kWave;
            e.xe += (size_t)h * kWave;
        }
    }
    return e;
}

// The lanes of half h in use: lane s stands for source 64*h + s of the batch.
__device__ __forceinline__ uint64_t half_full(int32_t nlanes, int h) {
    const int32_t k = nlanes - kWave * h;
    return k >= kWave ? ~0ull : (k <= 0 ? 0ull : ((1ull << k) - 1ull));
}

// The level a kernel argument names (dir +1 forward, -1 reverse; see
// kRelLevel).
__device__ __forceinline__ int32_t level_arg(const BatchDev &d, int32_t L, int32_t dir) {
    return L < kRelLevel ? L : d.ctrl[kCtlLevel] + dir * (L - kRelLevel);
}

// ---- forward ---------------------------------------------------------------

// Size of the next frontier (vertices and arcs), counted per lane and stored
// by every wave of a kernel in its own slot of frontier set `set`: no counter
// is shared between waves (atomics on one address from every wave of the
// device serialise).
struct Front {
    uint32_t cnt = 0;
    unsigned long long arcs = 0;
    double smax = 0.0;  // the lane's largest stored count (wide rows)
};

// Also records, in extended range, each half's lane's largest count stored
// for level L+1 (one atomic max per lane, half and wave that stored any).
// d is the whole workspace (not a half's view).
template <bool N, int H>
__device__ __forceinline__ void report_front(const BatchDev &d, int set, int32_t L,
                                             const Front (&fr)[H]) {
    BC_FULL_EXEC();
    unsigned long long c = 0, a = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        if (!N && d.xmax && fr[h].smax > 0.0)
            atomicMax(&d.xmax[((size_t)(L + 1) * H + h) * kWave + lane_id()],
                      (unsigned long long)__double_as_longlong(fr[h].smax));
        c += fr[h].cnt;
        a += fr[h].arcs;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        c += __shfl_xor(c, off);
        a += __shfl_xor(a, off);
    }
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (lane_id() == 0) {
        unsigned long long *slot = d.front + ((size_t)set * kFrontWaves + wave) * 2;
        slot[0] = c;
        slot[1] = a;
    }
}

// A complete count of level L+1 (already scaled): stored, and kept for the
// lane's largest value.
template <bool N>
__device__ __forceinline__ void store_sigma(const BatchDev &d, size_t at, double acc, Front &fr) {
    SigRows<N>::store(d, at, acc);
    if (!N) fr.smax = fmax(fr.smax, acc);
}

// Chunk item of a vertex of degree > 64 (xsc: the lane's scale of level L).
template <bool N, int H>
__device__ __forceinline__ void fwd_chunk(const BatchDev &d, int32_t L, uint32_t item,
                                          uint64_t full, double xsc, Work &wk, Front &fr) {
    const int lane = lane_id();
    const int2 info = d.item_info_in[item];
    const int32_t w = info.x, j = info.y;
    const int32_t rs = d.row_ptr_in[w], re = d.row_ptr_in[w + 1];
    const bool multi = w < d.multi_end;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    const uint64_t vis = d.vis[(size_t)w * H];
    const uint64_t unvis = ~vis & full;
    if (lane == 0 && j == 0) ++wk.verts;
    // (vis of a split vertex changes only in the completion kernel, so all of
    // its chunks agree here; with nothing to discover none writes a row and
    // the completion skips the vertex)
    if (unvis == 0ull) {
        if (!multi && lane == 0) FN[(size_t)w * H] = 0ull;
        return;
    }
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n * H;
    // the item's arcs, kProbe * 64 per round (an item holds d.chunk of them)
    const int32_t cb = rs + j * d.chunk, ce = min(re, cb + d.chunk);
    double acc = 0.0;
    uint64_t nw = 0;
    for (int32_t c0 = cb; c0 < ce; c0 += kProbe * kWave)
        nw |= probe_chunk<H>(d.col_idx_in, c0, min(ce, c0 + kProbe * kWave), FL, unvis,
                             SigRows<N>::rows(d), acc, wk);
    const bool mine = (nw >> lane) & 1ull;
    if (mine && (!multi || j == 0)) ++wk.owners;
    if (!multi) {
        if (mine) store_sigma<N>(d, (size_t)w * (H * kWave) + lane, acc * xsc, fr);
        if (lane == 0) {
            FN[(size_t)w * H] = nw;
            if (nw) {
                d.vis[(size_t)w * H] = vis | nw;
                ++fr.cnt;
                fr.arcs += (unsigned long long)(re - rs);
            }
        }
    } else {
        // every lane's sum (0 without parents in this chunk), for the
        // completion kernel to add in chunk order
        d.partial[(size_t)item * (H * kWave) + lane] = acc;
        if (nw && lane == 0) atomicOr((unsigned long long *)&d.reach[(size_t)w * H], (unsigned long long)nw);
    }
}

// Forward runs of a group item, arc by arc: up to kUnroll hit arcs' sigma
// rows loaded for all 64 sources at once and folded into one owner's sum at a
// time (the wave switches owner in arc order); an owner's counts, F_{L+1} and
// vis entries are stored when the next owner starts.  For groups whose arcs
// carry many sources each.
template <bool N, int H>
__device__ __forceinline__ void fwd_runs_rows(const BatchDev &d, const uint64_t *FL, uint64_t *FN,
                                              int32_t me, int32_t rs, int32_t cnt, uint32_t excl,
                                              uint32_t total, uint64_t unvis, uint64_t full,
                                              double xsc, Work &wk, Front &fr) {
    const int lane = lane_id();
    int cur = -1;        // owner lane being accumulated
    double acc = 0.0;
    uint64_t nw = 0;
    auto flush = [&]() {
        if (cur >= 0 && nw) {
            BC_FULL_EXEC();
            const int32_t w = __shfl(me, cur);                   // all lanes active here
            const uint64_t w_vis = ~shfl64(unvis, cur) & full;
            const int32_t w_deg = __shfl(cnt, cur);
            if ((nw >> lane) & 1ull) {
                store_sigma<N>(d, (size_t)w * (H * kWave) + lane, acc * xsc, fr);
                ++wk.owners;
            }
            if (lane == 0) {
                FN[(size_t)w * H] = nw;
                d.vis[(size_t)w * H] = w_vis | nw;
                ++fr.cnt;
                fr.arcs += (unsigned long long)w_deg;
            }
        }
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave * kRounds) {
        // kRounds runs of 64 arcs: ids, then masks, loaded together
        int o[kRounds];
        int32_t nb[kRounds];
        uint64_t m[kRounds];
        bool live[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t a = c0 + (uint32_t)(r * kWave + lane);
            o[r] = owner_lane(excl, a);
            // cross-lane reads first, with every lane active
            const int32_t o_rs = __shfl(rs, o[r]);
            const uint32_t o_excl = __shfl(excl, o[r]);
            live[r] = a < total;
            nb[r] = live[r] ? d.col_idx_in[o_rs + (int32_t)(a - o_excl)] : 0;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint64_t o_keep = shfl64(unvis, o[r]);
            m[r] = live[r] ? FL[(size_t)nb[r] * H] & o_keep : 0ull;
            wk.arcs += live[r] ? 1u : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            uint64_t hit = __ballot(m[r] != 0ull);
            while (hit) {
                // kUnroll parent rows in flight at once, whatever their
                // owners; then folded into the owners' sums in arc order
                double x[kUnroll];
                uint64_t mj[kUnroll];
                int oj[kUnroll];
                gather_run<H>(hit, nb[r], m[r], o[r], SigRows<N>::rows(d), x, mj, oj, wk);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    if (oj[u] < 0) break;
                    if (oj[u] != cur) {
                        flush();
                        cur = oj[u];
                        acc = 0.0;
                        nw = 0;
                    }
                    acc += x[u];
                    nw |= mj[u];
                }
            }
        }
    }
    flush();
}

// Forward runs of a group item, source by source: each lane keeps its own
// running sum and owner and walks its parent arcs in arc order (owners
// ascending; see walk_own); F_{L+1} and vis are written per vertex at the end.
// For groups whose arcs carry few sources each (deep, sparse levels).
template <bool N, int H>
__device__ __forceinline__ void fwd_runs_lanes(const BatchDev &d, const uint64_t *FL, uint64_t *FN,
                                               int32_t base, const int32_t *list, int32_t me,
                                               uint64_t vis, int32_t rs, int32_t cnt,
                                               uint32_t excl, uint32_t total, uint64_t unvis,
                                               double xsc, Work &wk, Front &fr) {
    const int lane = lane_id();
    int cur = -1;             // owner lane being summed by this lane
    double acc = 0.0;
    uint64_t owners = 0;      // owner lanes this lane found parents for
    auto flush = [&]() {
        if (cur >= 0) {
            const int32_t w = list ? list[base + cur] : base + cur;
            store_sigma<N>(d, (size_t)w * (H * kWave) + lane, acc * xsc, fr);
            ++wk.owners;
        }
    };
    auto take = [&](int ow, double x) {
        if (ow != cur) {
            flush();
            cur = ow;
            acc = 0.0;
            owners |= 1ull << cur;
        }
        acc += x;
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave * kRounds) {
        // kRounds runs of 64 arcs: ids, then masks, loaded together
        int o[kRounds];
        int32_t nb[kRounds];
        uint64_t m[kRounds];
        bool live[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t a = c0 + (uint32_t)(r * kWave + lane);
            o[r] = owner_lane(excl, a);
            // cross-lane reads first, with every lane active
            const int32_t o_rs = __shfl(rs, o[r]);
            const uint32_t o_excl = __shfl(excl, o[r]);
            live[r] = a < total;
            nb[r] = live[r] ? d.col_idx_in[o_rs + (int32_t)(a - o_excl)] : 0;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint64_t o_keep = shfl64(unvis, o[r]);
            m[r] = live[r] ? FL[(size_t)nb[r] * H] & o_keep : 0ull;
            wk.arcs += live[r] ? 1u : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r)
            if (__ballot(m[r] != 0ull))
                walk_own<H>(transpose64(m[r]), nb[r], o[r], SigRows<N>::rows(d), wk, take);
    }
    flush();
    // lane i: the sources that reached its vertex at L+1
    const uint64_t nw = transpose64(owners);
    if (me >= 0) {
        FN[(size_t)me * H] = nw;
        if (nw) {
            d.vis[(size_t)me * H] = vis | nw;
            ++fr.cnt;
            fr.arcs += (unsigned long long)cnt;
        }
    }
}

// Group item: 64 vertices, either base .. base+63 (dense step: all of degree
// <= 64, F_{L+1} written for every one) or list[base .. base+63] (sparse step:
// the step's candidates of degree <= 64, F_{L+1} cleared beforehand; larger
// candidates come as chunk items).  The wave flattens
// the arcs of the vertices that still have unvisited lanes into runs of 64;
// the first run's masks choose the walk: by rows when its hit arcs carry at
// least kDenseArc sources on average, else by lanes.
template <bool N, int H>
__device__ __forceinline__ void
fwd_group(const BatchDev &d, int32_t L, int32_t base, const int32_t *list, int32_t count,
          uint64_t full, double xsc, Work &wk, Front &fr) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n * H;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    int32_t me = -1;
    if (list) {
        if (base + lane < count) me = list[base + lane];
    } else if (base + lane < d.n) {
        me = base + lane;
    }
    uint64_t vis = full;
    int32_t rs = 0, cnt = 0;
    if (me >= 0) {
        vis = d.vis[(size_t)me * H];
        rs = d.row_ptr_in[me];
        const int32_t re = d.row_ptr_in[me + 1];
        cnt = vis != full ? re - rs : 0;
    }
    wk.verts += me >= 0 ? 1u : 0u;
    uint32_t total;
    const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
    const uint64_t unvis = ~vis & full;
    bool rows = true;
    if (total > 0) {
        const uint32_t a = (uint32_t)lane;
        const int o = owner_lane(excl, a);
        const int32_t o_rs = __shfl(rs, o);
        const uint32_t o_excl = __shfl(excl, o);
        const uint64_t o_keep = shfl64(unvis, o);
        uint64_t m = 0ull;
        if (a < total) m = FL[(size_t)d.col_idx_in[o_rs + (int32_t)(a - o_excl)] * H] & o_keep;
        const int hits = __popcll((unsigned long long)__ballot(m != 0ull));
        rows = wave_sum_int(__popcll((unsigned long long)m)) >= kDenseArc * hits;
    }
    if (rows) {
        if (!list && me >= 0) FN[(size_t)me * H] = 0ull;
        fwd_runs_rows<N, H>(d, FL, FN, me, rs, cnt, excl, total, unvis, full, xsc, wk, fr);
    } else {
        fwd_runs_lanes<N, H>(d, FL, FN, base, list, me, vis, rs, cnt, excl, total, unvis, xsc, wk,
                          fr);
    }
}

template <bool N, int H>
__global__ __launch_bounds__(kBlock, kLevelWaves) void k_batch_forward(BatchDev d, int32_t L, int32_t nlanes) {
    L = level_arg(d, L, 1);
    // nothing past the deepest level found so far (F_L is empty), no room, or
    // this level takes the sparse step
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || d.ctrl[kCtlMode]) return;
    const uint32_t items = d.items_in;
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    Front fr[H];
    // one pass per half over the item (constant h: the step is inlined twice)
    const double x0 = level_scale<N, H>(half_view<H>(d, 0), L);
    const double x1 = H > 1 ? level_scale<N, H>(half_view<H>(d, H - 1), L) : 1.0;
    auto step = [&](uint32_t it, int h, double xsc, Front &f) __attribute__((always_inline)) {
        const BatchDev dh = half_view<H>(d, h);
        const uint64_t full = half_full(nlanes, h);
        if (it < items) fwd_chunk<N, H>(dh, L, it, full, xsc, wk, f);
        else fwd_group<N, H>(dh, L, d.big_end + (int32_t)(it - items) * kWave, nullptr, 0, full,
                             xsc, wk, f);
    };
    for (uint32_t it = wave; it < items + groups; it += nwaves) {
        step(it, 0, x0, fr[0]);
        if (H > 1) step(it, 1, x1, fr[H - 1]);
    }
    report_front<N, H>(d, 0, L, fr);
    if (d.stats) report_work(d.stats, 0, 12, wk);
}

// After a forward iteration: completes the split vertices (their counts = the
// chunks' partial rows added in chunk order, F_{L+1}, vis) and counts them
// into the new frontier.
template <bool N, int H>
__device__ __forceinline__ void finish_split(const BatchDev &d, int32_t L, int32_t wave,
                                             int32_t nwaves, double xsc, Front &fr) {
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    const int lane = lane_id();
    for (int32_t w = wave; w < d.multi_end; w += nwaves) {
        const uint64_t nw = d.reach[(size_t)w * H];
        if (lane == 0) FN[(size_t)w * H] = nw;
        if (nw == 0ull) continue;
        const uint32_t i0 = d.item_first_in[w], i1 = d.item_first_in[w + 1];
        double t = 0.0;
        uint32_t i = i0;
        for (; i + 8 <= i1; i += 8) {  // 8 rows in flight
            double x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = d.partial[(size_t)(i + q) * (H * kWave) + lane];
#pragma unroll
            for (int q = 0; q < 8; ++q) t += x[q];
        }
        for (; i < i1; ++i) t += d.partial[(size_t)i * (H * kWave) + lane];
        if ((nw >> lane) & 1ull) store_sigma<N>(d, (size_t)w * (H * kWave) + lane, t * xsc, fr);
        if (lane == 0) {
            d.vis[(size_t)w * H] |= nw;
            d.reach[(size_t)w * H] = 0ull;
            ++fr.cnt;
            fr.arcs += (unsigned long long)(d.row_ptr[w + 1] - d.row_ptr[w]);
        }
    }
}

template <bool N, int H>
__global__ __launch_bounds__(kBlock) void k_batch_forward_finish(BatchDev d, int32_t L) {
    L = level_arg(d, L, 1);
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap) return;
    Front fr[H];
    auto step = [&](int h, Front &f) __attribute__((always_inline)) {
        const BatchDev dh = half_view<H>(d, h);
        finish_split<N, H>(dh, L, (blockIdx.x * kBlock + threadIdx.x) / kWave,
                           gridDim.x * kWavesPerBlock, level_scale<N, H>(dh, L), f);
    };
    step(0, fr[0]);
    if (H > 1) step(1, fr[H - 1]);
    report_front<N, H>(d, 2, L, fr);
}

// Bookkeeping between iterations (one block): adds up the frontier slots of
// the kernels that ran, records the depth (or the truncation when the level
// array is full), picks the step of the next iteration (sparse when the new
// frontier has few arcs) and clears the list counters.  waves[s] = the waves
// of the kernel of frontier set s.
constexpr int kDoneBlock = 1024;

template <int H>
__global__ __launch_bounds__(kDoneBlock) void k_batch_level_done(BatchDev d, int32_t L,
                                                                 int32_t w0, int32_t w1,
                                                                 int32_t w2) {
    __shared__ unsigned long long sc[kDoneBlock], sa[kDoneBlock];
    L = level_arg(d, L, 1);
    const int t = threadIdx.x;
    const bool live = !(L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap);
    const int mode = d.ctrl[kCtlMode];
    unsigned long long c = 0, a = 0;
    if (live) {
        const int32_t waves[kFrontSets] = {mode ? 0 : w0, mode ? w1 : 0, w2};
        for (int set = 0; set < kFrontSets; ++set) {
            const unsigned long long *slot = d.front + (size_t)set * kFrontWaves * 2;
            for (int32_t w = t; w < waves[set]; w += kDoneBlock) {
                c += slot[2 * w];
                a += slot[2 * w + 1];
            }
        }
    }
    sc[t] = c;
    sa[t] = a;
    __syncthreads();
    for (int h = kDoneBlock / 2; h >= 1; h >>= 1) {
        if (t < h) {
            sc[t] += sc[t + h];
            sa[t] += sa[t + h];
        }
        __syncthreads();
    }
    // extended range: level L+1's scale from its largest stored counts (k = 0
    // below 2^512, so ordinary counts are never rescaled), and its exponent
    if (live && d.xs && t < H * kWave) {
        const size_t at = (size_t)(L + 1) * (H * kWave) + t;
        const double m = __longlong_as_double((long long)d.xmax[at]);
        const int k = m >= 0x1p512 ? ilogb(m) : 0;
        d.xs[at] = ldexp(1.0, -k);
        d.xe[at] = d.xe[at - H * kWave] - ilogb(d.xs[at - H * kWave]);
    }
    if (t == 0) {
        if (live && sc[0] != 0) {
            d.ctrl[kCtlDeepest] = L + 1;
            if (L + 2 >= d.lcap) d.ctrl[kCtlTrunc] = 1;  // level L+2 would not fit
        }
        if (live) d.ctrl[kCtlMode] = (int64_t)sa[0] < d.sparse_arcs ? 1 : 0;
        d.ctrl[kCtlCand] = 0;
        d.ctrl[kCtlItems] = 0;
    }
}

// ---- sparse forward step ------------------------------------------------------

// Mark every neighbour of the level-L frontier (the vertices with F_L != 0,
// found by scanning F_L 64 vertices per wave).  The arcs of a wave's frontier
// vertices are flattened into runs of 64 (one arc per lane, kProbe runs per
// round), so a group with many small frontier vertices (a deep graph's
// frontier rings) takes as many rounds as it has arcs / 512, not one round
// per vertex.  Marks are idempotent byte stores.
template <int H>
__global__ __launch_bounds__(kBlock) void k_batch_sparse_mark(BatchDev d, int32_t L) {
    L = level_arg(d, L, 1);
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n * H;
    const int32_t groups = (d.n + kWave - 1) / kWave;
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    for (int32_t gi = wave; gi < groups; gi += nwaves) {
        const int32_t me = gi * kWave + lane;
        int32_t rs = 0, cnt = 0;
        uint64_t f = 0ull;
        if (me < d.n) {
#pragma unroll
            for (int h = 0; h < H; ++h) f |= FL[(size_t)me * H + h];
        }
        if (f != 0ull) {
            rs = d.row_ptr[me];
            cnt = d.row_ptr[me + 1] - rs;
        }
        uint32_t total;
        const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
        for (uint32_t c0 = 0; c0 < total; c0 += kWave * kProbe) {
            int32_t nb[kProbe];
#pragma unroll
            for (int u = 0; u < kProbe; ++u) {
                const uint32_t a = c0 + (uint32_t)(u * kWave + lane);
                const int o = owner_lane(excl, a);
                // cross-lane reads first, with every lane active
                const int32_t o_rs = __shfl(rs, o);
                const uint32_t o_excl = __shfl(excl, o);
                nb[u] = a < total ? d.col_idx[o_rs + (int32_t)(a - o_excl)] : -1;
            }
#pragma unroll
            for (int u = 0; u < kProbe; ++u)
                if (nb[u] >= 0) d.cand[nb[u]] = 1;
        }
    }
}

// Turn the marks into the candidate lists (one thread per 16 vertices), clear
// them, and clear F_{L+1} (the sparse pull writes only the candidates').
template <int H>
__global__ __launch_bounds__(kBlock) void k_batch_sparse_compact(BatchDev d, int32_t L,
                                                                 int32_t nlanes) {
    L = level_arg(d, L, 1);
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    // list space is taken once per block (the waves' counts added in LDS):
    // one atomic per block and list instead of one per wave
    __shared__ uint32_t s_small[kWavesPerBlock], s_items[kWavesPerBlock], s_base[2];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    uint64_t *FN = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    const int32_t groups = (d.n + 15) >> 4;
    const int32_t stride = gridDim.x * kBlock;
    // the loop runs the same number of times in every wave of the block
    for (int32_t bb = blockIdx.x * kBlock; bb < groups; bb += stride) {
        const int32_t wb = bb + wib * kWave;
        const int32_t i = wb + lane;
        uint4 m = make_uint4(0u, 0u, 0u, 0u);
        if (i < groups) m = reinterpret_cast<const uint4 *>(d.cand)[i];
        // the wave's 1024 vertices of F_{L+1}, cleared with coalesced stores
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int32_t v = (wb << 4) + j * kWave + lane;
            if (v < d.n) {
#pragma unroll
                for (int h = 0; h < H; ++h) FN[(size_t)v * H + h] = 0ull;
            }
        }
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
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            bool all = true;
#pragma unroll
            for (int h = 0; h < H; ++h)
                all = all && d.vis[(size_t)((i << 4) + j) * H + h] == half_full(nlanes, h);
            if (all) bits &= ~(1u << j);
        }
        // vertices of degree <= 64 go to the candidate list; larger ones
        // contribute their chunk items to the item list
        uint32_t nsmall = 0, nitems = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            const int32_t v = (i << 4) + j;
            if (v < d.big_end) nitems += d.item_first_in[v + 1] - d.item_first_in[v];
            else ++nsmall;
        }
        uint32_t tot, toti;
        const uint32_t off = wave_excl_scan(nsmall, tot);
        const uint32_t offi = wave_excl_scan(nitems, toti);
        if (lane == 0) {
            s_small[wib] = tot;
            s_items[wib] = toti;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t a = 0, b = 0;
            for (int w = 0; w < kWavesPerBlock; ++w) {
                a += s_small[w];
                b += s_items[w];
            }
            s_base[0] = a ? atomicAdd((uint32_t *)&d.ctrl[kCtlCand], a) : 0u;
            s_base[1] = b ? atomicAdd((uint32_t *)&d.ctrl[kCtlItems], b) : 0u;
        }
        __syncthreads();
        uint32_t p = s_base[0] + off, pi = s_base[1] + offi;
        for (int w = 0; w < wib; ++w) {
            p += s_small[w];
            pi += s_items[w];
        }
        __syncthreads();  // the shared counts are rewritten by the next round
        uint32_t big = 0;  // bit j: vertex 16i+j is a listed candidate of degree > 64
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            if (!((bits >> j) & 1u)) continue;
            const int32_t v = (i << 4) + j;
            if (v < d.big_end) big |= 1u << j;
            else d.clist[p++] = v;
        }
        // chunk items of the large candidates, written by the whole wave (a
        // hub has hundreds of items)
        uint64_t owners = __ballot(big != 0u);
        while (owners) {
            const int src = __ffsll((unsigned long long)owners) - 1;
            owners &= owners - 1;
            uint32_t sbig = __shfl(big, src);
            uint32_t spi = __shfl(pi, src);
            const int32_t sv0 = __shfl(i, src) << 4;
            while (sbig) {
                const int j = __ffs(sbig) - 1;
                sbig &= sbig - 1;
                const uint32_t f0 = d.item_first_in[sv0 + j], cnt = d.item_first_in[sv0 + j + 1] - f0;
                for (uint32_t q = (uint32_t)lane; q < cnt; q += kWave) d.ilist[spi + q] = f0 + q;
                spi += cnt;
            }
        }
    }
}

// Pull over the candidates only (groups of 64 list entries).
template <bool N, int H>
__global__ __launch_bounds__(kBlock, kLevelWaves) void k_batch_sparse_pull(BatchDev d, int32_t L,
                                                              int32_t nlanes) {
    L = level_arg(d, L, 1);
    if (L > d.ctrl[kCtlDeepest] || L + 1 >= d.lcap || !d.ctrl[kCtlMode]) return;
    const int32_t c = d.ctrl[kCtlCand];
    const int32_t ni = d.ctrl[kCtlItems];
    const int32_t groups = (c + kWave - 1) / kWave;
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    Front fr[H];
    const double x0 = level_scale<N, H>(half_view<H>(d, 0), L);
    const double x1 = H > 1 ? level_scale<N, H>(half_view<H>(d, H - 1), L) : 1.0;
    auto step = [&](int32_t it, int h, double xsc, Front &f) __attribute__((always_inline)) {
        const BatchDev dh = half_view<H>(d, h);
        const uint64_t full = half_full(nlanes, h);
        if (it < ni) fwd_chunk<N, H>(dh, L, (uint32_t)d.ilist[it], full, xsc, wk, f);
        else fwd_group<N, H>(dh, L, (it - ni) * kWave, d.clist, c, full, xsc, wk, f);
    };
    for (int32_t it = wave; it < ni + groups; it += nwaves) {
        step(it, 0, x0, fr[0]);
        if (H > 1) step(it, 1, x1, fr[H - 1]);
    }
    report_front<N, H>(d, 1, L, fr);
    if (d.stats) report_work(d.stats, 0, 12, wk);
}

// ---- reverse ---------------------------------------------------------------

// Per-request outputs: lanes [seg_start[g], seg_start[g+1]) belong to request
// g of the batch.  Each segment's deltas are rotated down to lane 0 and summed
// with the same butterfly whatever the segment's position, so a request's sum
// does not depend on where in the batch its lanes sit; it is added to the
// request's output in caller vertex order.
__device__ __forceinline__ void add_segments(const BatchDev &d, int32_t v, double delta) {
    BC_FULL_EXEC();
    const int lane = lane_id();
    for (int32_t g = 0; g < d.nseg; ++g) {
        const int32_t a = d.seg_start[g], len = d.seg_start[g + 1] - a;
        double x = __shfl(delta, (lane + a) & (kWave - 1));
        x = lane < len ? x : 0.0;
        x = wave_sum(x);
        if (lane == 0 && x != 0.0) d.seg_out[g][d.iperm[v]] += x;
    }
}

// Complete (v, lanes mv) at level L from its children sums acc (already
// times the level's scale) and its sigma (lane s meaningful for s in mv):
// delta = sigma * acc, c = (1 + delta) / sigma, and the lanes' deltas added
// to BC[v] (or to the requests' outputs).  Called with every lane active.
// This form returns BC[v]'s share (the lanes' delta sum, the same in every
// lane) for the caller to add later; segments are added at once.  With wide
// rows a c beyond double's range (possible only with scaled counts) raises
// the range flag.
template <bool N, int H>
__device__ __forceinline__ double settle_deferred(const BatchDev &d, int32_t v, uint64_t mv,
                                                  double sig, double acc) {
    BC_FULL_EXEC();
    const int lane = lane_id();
    const bool on = (mv >> lane) & 1ull;
    const double delta = on ? sig * acc : 0.0;
    if (on) {
        const double c = (1.0 + delta) / sig;
        d.coef[(size_t)v * (H * kWave) + lane] = c;
        if (!N && !(c <= 0x1.fffffffffffffp+1023)) atomicOr(&d.ctrl[kCtlRange], 1);
    }
    if (d.nseg == 0) return wave_sum(delta);
    add_segments(d, v, delta);
    return 0.0;
}

template <bool N, int H>
__device__ __forceinline__ void settle(const BatchDev &d, int32_t v, uint64_t mv, double sig,
                                       double acc) {
    const double tot = settle_deferred<N, H>(d, v, mv, sig, acc);
    if (lane_id() == 0 && tot != 0.0) d.bc[v] += tot;
}

// Chunk item of a vertex of degree > 64: sums of c over children; a vertex
// with one chunk is completed here, a split vertex leaves the item's partial
// row for the finalising pass.
template <bool N, int H>
__device__ __forceinline__ void bwd_chunk(const BatchDev &d, int32_t L, uint32_t item,
                                          double xsc, Work &wk) {
    const int lane = lane_id();
    const int2 info = d.item_info[item];
    const int32_t v = info.x, j = info.y;
    const uint64_t mv = d.F[((size_t)L * (size_t)d.n + v) * H];
    if (lane == 0 && j == 0) ++wk.verts;
    if (mv == 0ull) return;
    const uint64_t *FC = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    const int32_t rs = d.row_ptr[v], re = d.row_ptr[v + 1];
    const int32_t cb = rs + j * d.chunk, ce = min(re, cb + d.chunk);
    const bool on = (mv >> lane) & 1ull;
    const double sig = (on && v >= d.multi_end) ? sig_at<N>(d, (size_t)v * (H * kWave) + lane) : 1.0;
    double acc = 0.0;
    for (int32_t c0 = cb; c0 < ce; c0 += kProbe * kWave)
        (void)probe_chunk<H>(d.col_idx, c0, min(ce, c0 + kProbe * kWave), FC, mv, d.coef, acc, wk);
    if (on && j == 0) ++wk.owners;
    if (v < d.multi_end) d.partial[(size_t)item * (H * kWave) + lane] = acc;
    else settle<N, H>(d, v, mv, sig, acc * xsc);
}

// The runs of a reverse group, arc by arc: up to kUnroll hit arcs' c rows
// loaded for all 64 sources at once, folded into one owner's sum at a time
// (the wave switches owner in arc order) and each owner completed when the
// next one starts.  For groups whose owners carry many sources each.
template <bool N, int H>
__device__ __forceinline__ void bwd_runs_rows(const BatchDev &d, const uint64_t *FC, int32_t base,
                                              uint64_t mv, int32_t rs, uint32_t excl,
                                              uint32_t total, double xsc, Work &wk,
                                              uint64_t &pending, double &my_bc) {
    const int lane = lane_id();
    int cur = -1;
    double acc = 0.0;
    double cur_sig = 1.0;   // sigma of the owner being accumulated (its lanes)
    auto flush = [&]() {
        if (cur < 0) return;
        const double tot = settle_deferred<N, H>(d, base + cur, shfl64(mv, cur), cur_sig, acc * xsc);
        if (lane == cur) my_bc = tot;  // all lanes active here
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave * kRounds) {
        int o[kRounds];
        int32_t nb[kRounds];
        uint64_t m[kRounds];
        bool live[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t a = c0 + (uint32_t)(r * kWave + lane);
            o[r] = owner_lane(excl, a);
            const int32_t o_rs = __shfl(rs, o[r]);
            const uint32_t o_excl = __shfl(excl, o[r]);
            live[r] = a < total;
            nb[r] = live[r] ? d.col_idx[o_rs + (int32_t)(a - o_excl)] : 0;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint64_t o_keep = shfl64(mv, o[r]);
            m[r] = live[r] ? FC[(size_t)nb[r] * H] & o_keep : 0ull;
            wk.arcs += live[r] ? 1u : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            uint64_t hit = __ballot(m[r] != 0ull);
            while (hit) {
                double x[kUnroll];
                uint64_t mj[kUnroll];
                int oj[kUnroll];
                gather_run<H>(hit, nb[r], m[r], o[r], d.coef, x, mj, oj, wk);
#pragma unroll
                for (int u = 0; u < kUnroll; ++u) {
                    if (oj[u] < 0) break;
                    if (oj[u] != cur) {
                        flush();
                        cur = oj[u];
                        acc = 0.0;
                        pending &= ~(1ull << cur);
                        const bool on = (shfl64(mv, cur) >> lane) & 1ull;
                        cur_sig = on ? sig_at<N>(d, (size_t)(base + cur) * (H * kWave) + lane) : 1.0;
                    }
                    acc += x[u];
                }
            }
        }
    }
    flush();
}

// The runs of a reverse group, source by source: each lane sums c over its
// own children arcs in arc order (see walk_own); a finished sum (times the
// level's scale) is parked in the owner's c entry, which no wave reads during
// this level (it is read only where the owner sits at level L + 1, and
// written only where it sits at L).  The owners are completed afterwards, one
// wave-wide settle each, from those sums and their sigma rows.  For groups
// whose owners carry few sources each (deep, sparse levels).
template <bool N, int H>
__device__ __forceinline__ void bwd_runs_lanes(const BatchDev &d, const uint64_t *FC, int32_t base,
                                               uint64_t mv, int32_t rs, uint32_t excl,
                                               uint32_t total, double xsc, Work &wk,
                                               uint64_t &pending, double &my_bc) {
    const int lane = lane_id();
    int cur = -1;
    double acc = 0.0;
    uint64_t owners = 0;      // owner lanes this lane found children for
    auto flush = [&]() {
        if (cur >= 0) d.coef[(size_t)(base + cur) * (H * kWave) + lane] = acc * xsc;
    };
    auto take = [&](int ow, double x) {
        if (ow != cur) {
            flush();
            cur = ow;
            acc = 0.0;
            owners |= 1ull << cur;
        }
        acc += x;
    };
    for (uint32_t c0 = 0; c0 < total; c0 += kWave * kRounds) {
        int o[kRounds];
        int32_t nb[kRounds];
        uint64_t m[kRounds];
        bool live[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint32_t a = c0 + (uint32_t)(r * kWave + lane);
            o[r] = owner_lane(excl, a);
            const int32_t o_rs = __shfl(rs, o[r]);
            const uint32_t o_excl = __shfl(excl, o[r]);
            live[r] = a < total;
            nb[r] = live[r] ? d.col_idx[o_rs + (int32_t)(a - o_excl)] : 0;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const uint64_t o_keep = shfl64(mv, o[r]);
            m[r] = live[r] ? FC[(size_t)nb[r] * H] & o_keep : 0ull;
            wk.arcs += live[r] ? 1u : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r)
            if (__ballot(m[r] != 0ull))
                walk_own<H>(transpose64(m[r]), nb[r], o[r], d.coef, wk, take);
    }
    flush();
    // lane t: the sources for which owner t has children
    const uint64_t touched = transpose64(owners);
    uint64_t busy = __ballot(touched != 0ull);
    pending &= ~busy;
    while (busy) {
        int t[kUnroll];
        uint64_t mt[kUnroll];
        double x[kUnroll], sg[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            t[u] = -1;
            if (busy) {
                t[u] = __ffsll((unsigned long long)busy) - 1;
                busy &= busy - 1;
            }
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int tt = t[u] < 0 ? 0 : t[u];
            mt[u] = t[u] < 0 ? 0ull : shfl64(mv, tt);
            const uint64_t tu = shfl64(touched, tt);
            const bool on = (mt[u] >> lane) & 1ull;
            const size_t at = (size_t)(base + tt) * (H * kWave) + lane;
            x[u] = (on && ((tu >> lane) & 1ull)) ? d.coef[at] : 0.0;
            sg[u] = on ? sig_at<N>(d, at) : 1.0;
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            if (t[u] < 0) break;  // wave-uniform
            const double tot = settle_deferred<N, H>(d, base + t[u], mt[u], sg[u], x[u]);
            if (lane == t[u]) my_bc = tot;
        }
    }
}

template <bool N, int H>
__device__ __forceinline__ void bwd_group(const BatchDev &d, int32_t L, int32_t base, double xsc,
                                          Work &wk) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n * H;
    const uint64_t *FC = d.F + (size_t)(L + 1) * (size_t)d.n * H;
    const int32_t me = base + lane;
    uint64_t mv = 0;
    int32_t rs = 0, cnt = 0;
    if (me < d.n) {
        mv = FL[(size_t)me * H];
        rs = d.row_ptr[me];
        const int32_t re = d.row_ptr[me + 1];
        cnt = mv ? re - rs : 0;
    }
    uint32_t total;
    const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
    const int pairs = wave_sum_int(__popcll((unsigned long long)mv));
    wk.owners += (uint32_t)__popcll((unsigned long long)mv);
    wk.verts += me < d.n ? 1u : 0u;
    // owners with lanes at level L but no children are completed at the end
    uint64_t pending = __ballot(mv != 0ull);
    // BC shares of the group's owners, held by the owner's lane and added in
    // one parallel read-modify-write at the end (a load per owner otherwise
    // stalls the wave)
    double my_bc = 0.0;
    if (pairs >= kDenseOwner * __popcll(pending))
        bwd_runs_rows<N, H>(d, FC, base, mv, rs, excl, total, xsc, wk, pending, my_bc);
    else
        bwd_runs_lanes<N, H>(d, FC, base, mv, rs, excl, total, xsc, wk, pending, my_bc);
    // owners without any child: delta = 0, c = 1 / sigma, nothing for BC
    while (pending) {
        int32_t vj[kUnroll];
        bool on[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            vj[u] = -1;
            on[u] = false;
            if (pending) {
                const int t = __ffsll((unsigned long long)pending) - 1;
                pending &= pending - 1;
                vj[u] = base + t;
                on[u] = (shfl64(mv, t) >> lane) & 1ull;
            }
        }
        double sig[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            sig[u] = on[u] ? sig_at<N>(d, (size_t)vj[u] * (H * kWave) + lane) : 1.0;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (on[u]) d.coef[(size_t)vj[u] * (H * kWave) + lane] = 1.0 / sig[u];
    }
    if (my_bc != 0.0) d.bc[base + lane] += my_bc;
}

template <bool N, int H>
__global__ __launch_bounds__(kBlock, kLevelWaves) void k_batch_reverse(BatchDev d, int32_t L) {
    // levels 1 .. deepest-1 have children (a replayed chunk passes others)
    L = level_arg(d, L, -1);
    if (L < 1 || L >= d.ctrl[kCtlDeepest]) return;
    const uint32_t items = d.items;
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Work wk;
    const double x0 = level_scale<N, H>(half_view<H>(d, 0), L);
    const double x1 = H > 1 ? level_scale<N, H>(half_view<H>(d, H - 1), L) : 1.0;
    auto step = [&](uint32_t it, int h, double xsc) __attribute__((always_inline)) {
        const BatchDev dh = half_view<H>(d, h);
        if (it < items) bwd_chunk<N, H>(dh, L, it, xsc, wk);
        else bwd_group<N, H>(dh, L, d.big_end + (int32_t)(it - items) * kWave, xsc, wk);
    };
    for (uint32_t it = wave; it < items + groups; it += nwaves) {
        step(it, 0, x0);
        if (H > 1) step(it, 1, x1);
    }
    if (d.stats) report_work(d.stats, 6, 13, wk);
}

// Finalise level L for the vertices the reverse kernel leaves open: the split
// vertices (v < multi_end, one wave each), whose child sums are the partial
// rows of their chunks added in chunk order, or, with leaf set (the deepest
// level), every vertex, with sum 0.  delta = sigma * sum, c = (1 + delta) /
// sigma, BC[v] += the lanes' deltas.
template <bool N, int H>
__device__ __forceinline__ void
finalize_level(const BatchDev &d, int32_t L, int32_t leaf, int32_t wave, int32_t nwaves) {
    const int lane = lane_id();
    const uint64_t *FL = d.F + (size_t)L * (size_t)d.n * H;
    if (!leaf) {
        // split vertices, one wave each: the chunks' partial rows added in
        // chunk order (8 rows in flight), then delta, c and BC
        for (int32_t v = wave; v < d.multi_end; v += nwaves) {
            const uint64_t mv = FL[(size_t)v * H];
            if (mv == 0ull) continue;
            const bool on = (mv >> lane) & 1ull;
            const double sig = on ? sig_at<N>(d, (size_t)v * (H * kWave) + lane) : 1.0;
            const uint32_t i0 = d.item_first[v], i1 = d.item_first[v + 1];
            double t = 0.0;
            uint32_t i = i0;
            for (; i + 8 <= i1; i += 8) {
                double x[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) x[q] = d.partial[(size_t)(i + q) * (H * kWave) + lane];
#pragma unroll
                for (int q = 0; q < 8; ++q) t += x[q];
            }
            for (; i < i1; ++i) t += d.partial[(size_t)i * (H * kWave) + lane];
            settle<N, H>(d, v, mv, sig, t * level_scale<N, H>(d, L));
        }
        return;
    }
    const int32_t vend = d.n;
    const int32_t groups = (vend + kWave - 1) / kWave;
    for (int32_t gi = wave; gi < groups; gi += nwaves) {
        const int32_t me = gi * kWave + lane;
        const uint64_t m_me = me < vend ? FL[(size_t)me * H] : 0ull;
        uint64_t todo = __ballot(m_me != 0ull);
        while (todo) {
            // kFinal vertices per round: their rows are loaded together and
            // their BC updates made by kFinal lanes at once
            constexpr int kFinal = 8;
            int32_t vj[kFinal];
            uint64_t mj[kFinal];
#pragma unroll
            for (int u = 0; u < kFinal; ++u) {
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
            double sig[kFinal], sum[kFinal];
#pragma unroll
            for (int u = 0; u < kFinal; ++u) {
                const bool on = (mj[u] >> lane) & 1ull;
                const size_t at = (size_t)(vj[u] < 0 ? 0 : vj[u]) * (H * kWave) + lane;
                sig[u] = on ? sig_at<N>(d, at) : 1.0;
                sum[u] = 0.0;  // the deepest level has no children
            }
            double delta[kFinal];
#pragma unroll
            for (int u = 0; u < kFinal; ++u) {
                const bool on = (mj[u] >> lane) & 1ull;
                delta[u] = on ? sig[u] * sum[u] : 0.0;
                if (on) d.coef[(size_t)vj[u] * (H * kWave) + lane] = (1.0 + delta[u]) / sig[u];
            }
            if (d.nseg == 0) {
                // lane u receives vertex u's sum over the lanes
                double my_tot = 0.0;
                int32_t my_v = -1;
#pragma unroll
                for (int u = 0; u < kFinal; ++u) {
                    const double tot = wave_sum(delta[u]);
                    if (lane == u) {
                        my_tot = tot;
                        my_v = vj[u];
                    }
                }
                if (my_v >= 0 && my_tot != 0.0) d.bc[my_v] += my_tot;
            } else {
#pragma unroll
                for (int u = 0; u < kFinal; ++u)
                    if (vj[u] >= 0) add_segments(d, vj[u], delta[u]);
            }
        }
    }
}

template <bool N, int H>
__global__ __launch_bounds__(kBlock) void k_batch_finalize(BatchDev d, int32_t L, int32_t leaf) {
    if (leaf < 0) {  // relative level: levels 1 .. deepest, the deepest a leaf
        L = level_arg(d, L, -1);
        if (L < 1 || L > d.ctrl[kCtlDeepest]) return;
        leaf = L == d.ctrl[kCtlDeepest] ? 1 : 0;
    }
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    finalize_level<N, H>(half_view<H>(d, 0), L, leaf, wave, gridDim.x * kWavesPerBlock);
    if (H > 1)
        finalize_level<N, H>(half_view<H>(d, H - 1), L, leaf, wave, gridDim.x * kWavesPerBlock);
}

// ---- device-resident level loop (small graphs) -----------------------------

// One workgroup runs one whole batch: clear, seed, every forward level, every
// reverse level and the completion, with a workgroup barrier between steps
// (the waves of a workgroup share one compute unit and its L1, so the barrier
// orders their global-memory accesses).  A call's batches run as the
// workgroups of one launch.  The per-wave step code is the one the grid-wide
// kernels run, inlined here as there: no kernel of this library makes calls
// (with the steps as out-of-line calls, this kernel's dependency sums came
// out wrong on gfx950, varying from run to run, while the level masks and
// path counts stayed exact).  ctrl of the batch receives the depth and the flags
// (truncation: the host runs the call again with a longer level array).  No
// extended range and no 128-source batches here: the host runs those on its
// own loop.
constexpr int kFusedBlock = 1024;
constexpr int kFusedWaves = kFusedBlock / kWave;

template <bool N>
__global__ __launch_bounds__(kFusedBlock) void k_batch_fused(const BatchDev *devs,
                                                             const int32_t *lanes,
                                                             const int2 *batches) {
    const BatchDev &d = devs[blockIdx.x];
    const int2 bt = batches[blockIdx.x];  // (first lane in `lanes`, lane count)
    const int t = threadIdx.x;
    const int lane = lane_id();
    const int32_t wave = t / kWave;
    __shared__ uint32_t s_found;
    // clear
    for (int32_t i = t; i < d.n; i += kFusedBlock) {
        d.vis[i] = 0ull;
        d.F[i] = 0ull;
        if (d.nseg == 0) d.bc[i] = 0.0;
    }
    for (int32_t i = t; i < d.multi_end; i += kFusedBlock) d.reach[i] = 0ull;
    if (t < kCtlInts) d.ctrl[t] = 0;
    __syncthreads();
    // seed
    const int32_t nl = bt.y;
    if (wave == 0 && lane < nl) {
        const int32_t s = lanes[bt.x + lane];
        atomicOr((unsigned long long *)&d.vis[s], 1ull << lane);
        atomicOr((unsigned long long *)&d.F[s], 1ull << lane);
        SigRows<N>::rows(d)[(size_t)s * kWave + lane] = 1;
    }
    __syncthreads();
    const uint64_t full = nl >= 64 ? ~0ull : ((1ull << nl) - 1ull);
    const uint32_t items = d.items;         // reverse (arcs out of a vertex)
    const uint32_t items_in = d.items_in;   // forward (arcs into a vertex)
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    // forward
    int32_t deepest = 0;
    bool trunc = false;
    Work wkf, wkr;
    for (int32_t L = 0;; ++L) {
        if (L + 1 >= d.lcap) {  // level L+1 does not fit
            trunc = true;
            break;
        }
        if (t == 0) s_found = 0;
        Front fr;
        for (uint32_t it = wave; it < items_in + groups; it += kFusedWaves) {
            if (it < items_in) fwd_chunk<N, 1>(d, L, it, full, 1.0, wkf, fr);
            else fwd_group<N, 1>(d, L, d.big_end + (int32_t)(it - items_in) * kWave, nullptr, 0,
                              full, 1.0, wkf, fr);
        }
        __syncthreads();
        finish_split<N, 1>(d, L, wave, kFusedWaves, 1.0, fr);
        uint32_t c = fr.cnt;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0 && c) atomicAdd(&s_found, c);
        __syncthreads();
        const uint32_t found = s_found;
        __syncthreads();  // s_found is reset by the next iteration
        if (found == 0) break;
        deepest = L + 1;
    }
    if (t == 0) {
        d.ctrl[kCtlDeepest] = deepest;
        if (trunc) d.ctrl[kCtlTrunc] = 1;
    }
    if (trunc) return;
    // reverse
    for (int32_t L = deepest; L >= 1; --L) {
        if (L != deepest) {
            for (uint32_t it = wave; it < items + groups; it += kFusedWaves) {
                if (it < items) bwd_chunk<N, 1>(d, L, it, 1.0, wkr);
                else bwd_group<N, 1>(d, L, d.big_end + (int32_t)(it - items) * kWave, 1.0, wkr);
            }
            __syncthreads();
        }
        finalize_level<N, 1>(d, L, L == deepest ? 1 : 0, wave, kFusedWaves);
        __syncthreads();
    }
    if (d.stats) {
        report_work(d.stats, 0, 12, wkf);
        report_work(d.stats, 6, 13, wkr);
    }
}

// ---- batch set-up and export ------------------------------------------------

// vis = 0 and F_0 = 0 everywhere; the split vertices' reach masks cleared.
template <bool N, int H>
__global__ void k_batch_clear(BatchDev d) {
    const int32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t stride = gridDim.x * blockDim.x;
    for (int64_t i = tid; i < (int64_t)d.n * H; i += stride) {
        d.vis[i] = 0ull;
        d.F[i] = 0ull;
    }
    for (int64_t i = tid; i < (int64_t)d.multi_end * H; i += stride) d.reach[i] = 0ull;
    const int32_t groups = (d.n + 15) >> 4;
    for (int32_t i = tid; i < groups; i += stride)
        reinterpret_cast<uint4 *>(d.cand)[i] = make_uint4(0u, 0u, 0u, 0u);
    // the range flag stays set over the run's batches (the host clears it)
    if (blockIdx.x == 0 && threadIdx.x < kCtlInts && threadIdx.x != kCtlRange)
        d.ctrl[threadIdx.x] = 0;
    if (d.xmax) {  // extended range: no maxima yet, level 0 (the sources) unscaled
        for (int64_t i = tid; i < (int64_t)d.lcap * (H * kWave); i += stride) d.xmax[i] = 0ull;
        if (tid < H * kWave) {
            d.xs[tid] = 1.0;
            d.xe[tid] = 0;
        }
    }
}

// Seed lane s with its source; the first iteration's step is chosen from the
// distinct sources' arc count.
template <bool N, int H>
__global__ void k_batch_seed(BatchDev d, const int32_t *src, int32_t nlanes) {
    const int lane = threadIdx.x;  // source lane + 64 h of half h
    unsigned long long arcs = 0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int32_t t = lane + kWave * h;
        if (t < nlanes) {
            const int32_t s = src[t];
            atomicOr((unsigned long long *)&d.vis[(size_t)s * H + h], 1ull << lane);
            const unsigned long long old =
                atomicOr((unsigned long long *)&d.F[(size_t)s * H + h], 1ull << lane);
            // exactly one lane per distinct source of the half
            if (old == 0ull) arcs += (unsigned long long)(d.row_ptr[s + 1] - d.row_ptr[s]);
            SigRows<N>::rows(d)[((size_t)s * H + h) * kWave + lane] = 1;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) arcs += __shfl_xor(arcs, off);
    if (lane == 0) d.ctrl[kCtlMode] = (int64_t)arcs < d.sparse_arcs ? 1 : 0;
}

// dist[s][v] and sigma[s][v] of lane s (internal vertex order), s < nlanes.
template <bool N, int H>
__global__ void k_batch_export(BatchDev d, int32_t deepest, int32_t nlanes, int32_t *dist,
                               double *sigma) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n;
         v += gridDim.x * blockDim.x) {
        for (int32_t s = 0; s < nlanes; ++s) {
            const int h = s / kWave, b = s % kWave;  // half and lane of source s
            int32_t lev = -1;
            if ((d.vis[(size_t)v * H + h] >> b) & 1ull) {
                for (int32_t L = 0; L <= deepest; ++L)
                    if ((d.F[((size_t)L * d.n + v) * H + h] >> b) & 1ull) {
                        lev = L;
                        break;
                    }
            }
            if (dist) dist[(size_t)s * d.n + v] = lev;
            if (sigma) {
                // extended range: the stored value times 2^xe (infinite past
                // double's range)
                const size_t at = ((size_t)v * H + h) * kWave + b;
                double x = lev >= 0 ? sig_at<N>(d, at) : 0.0;
                if (lev >= 0 && d.xe) x = ldexp(x, d.xe[((size_t)lev * H + h) * kWave + b]);
                sigma[(size_t)s * d.n + v] = x;
            }
        }
    }
}

int grid_of(int64_t waves) {
    int64_t g = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int)(g < 1 ? 1 : (g > kMaxGridBlocks ? kMaxGridBlocks : g));
}

constexpr int kSparseGrid = kMaxGridBlocks;  // blocks of the sparse mark / pull kernels

}  // namespace

#ifdef BC_CHECK_EXEC
unsigned int exec_partial_batched() { return exec_partial_take(); }
#endif

// The kernel instance for the workspace's row format (narrow uint32 or wide
// double sigma rows) and lane words per vertex (1: up to 64 sources, 2: up to
// 128).
#define BC_PICK(k, d)                                                    \
    ((d).H == 2 ? ((d).narrow ? k<true, 2> : k<false, 2>)                \
                : ((d).narrow ? k<true, 1> : k<false, 1>))
#define BC_PICK_H(k, d) ((d).H == 2 ? k<2> : k<1>)

hipError_t batch_start(const BatchDev &d, const int32_t *src_dev, int32_t nlanes,
                       hipStream_t stream) {
    int grid = (int)(((int64_t)d.n * d.H + kBlock - 1) / kBlock);
    grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
    hipLaunchKernelGGL(BC_PICK(k_batch_clear, d), dim3(grid), dim3(kBlock), 0, stream, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(BC_PICK(k_batch_seed, d), dim3(1), dim3(kWave), 0, stream, d, src_dev,
                       nlanes);
    return hipGetLastError();
}

hipError_t batch_forward(const BatchDev &d, int32_t level, int32_t nlanes, hipStream_t stream) {
    // both steps are launched; each returns at once unless the mode chosen on
    // the device for this level is its own
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    hipLaunchKernelGGL(BC_PICK(k_batch_forward, d), dim3(grid_of(d.items_in + groups)),
                       dim3(kBlock), 0, stream, d, level, nlanes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (d.sparse_arcs == 0) return hipSuccess;  // the sparse step is switched off
    hipLaunchKernelGGL(BC_PICK_H(k_batch_sparse_mark, d), dim3(kSparseGrid), dim3(kBlock), 0,
                       stream, d, level);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(BC_PICK_H(k_batch_sparse_compact, d),
                       dim3(grid_of(((d.n + 15) / 16 + kWave - 1) / kWave)), dim3(kBlock), 0,
                       stream, d, level, nlanes);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(BC_PICK(k_batch_sparse_pull, d), dim3(kSparseGrid), dim3(kBlock), 0, stream,
                       d, level, nlanes);
    return hipGetLastError();
}

hipError_t batch_forward_done(const BatchDev &d, int32_t level, hipStream_t stream) {
    if (d.multi_end > 0) {
        hipLaunchKernelGGL(BC_PICK(k_batch_forward_finish, d), dim3(grid_of(d.multi_end)),
                           dim3(kBlock), 0, stream, d, level);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    const int32_t w0 = grid_of(d.items_in + groups) * kWavesPerBlock;
    const int32_t w1 = kSparseGrid * kWavesPerBlock;
    const int32_t w2 = d.multi_end > 0 ? grid_of(d.multi_end) * kWavesPerBlock : 0;
    hipLaunchKernelGGL(BC_PICK_H(k_batch_level_done, d), dim3(1), dim3(kDoneBlock), 0, stream, d,
                       level, w0, w1, w2);
    return hipGetLastError();
}

hipError_t batch_reverse(const BatchDev &d, int32_t level, hipStream_t stream) {
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    hipLaunchKernelGGL(BC_PICK(k_batch_reverse, d), dim3(grid_of(d.items + groups)), dim3(kBlock),
                       0, stream, d, level);
    return hipGetLastError();
}

hipError_t batch_finalize(const BatchDev &d, int32_t level, bool deepest, hipStream_t stream) {
    // deepest level: every vertex, 64 per wave; otherwise one wave per split vertex
    const int64_t waves = deepest ? (d.n + kWave - 1) / kWave : d.multi_end;
    if (waves == 0) return hipSuccess;
    hipLaunchKernelGGL(BC_PICK(k_batch_finalize, d), dim3(grid_of(waves)), dim3(kBlock), 0, stream,
                       d, level, deepest ? 1 : 0);
    return hipGetLastError();
}

__global__ void k_level_advance(int32_t *ctrl, int32_t delta) { ctrl[kCtlLevel] += delta; }

__global__ void k_level_from_deepest(int32_t *ctrl) { ctrl[kCtlLevel] = ctrl[kCtlDeepest]; }

hipError_t batch_finalize_rel(const BatchDev &d, int32_t level_rel, hipStream_t stream) {
    // grid for the deepest level (every vertex); other levels use its first
    // multi_end waves
    const int64_t waves = std::max<int64_t>((d.n + kWave - 1) / kWave, d.multi_end);
    hipLaunchKernelGGL(BC_PICK(k_batch_finalize, d), dim3(grid_of(waves)), dim3(kBlock), 0, stream,
                       d, level_rel, -1);
    return hipGetLastError();
}

hipError_t batch_level_advance(const BatchDev &d, int32_t delta, hipStream_t stream) {
    hipLaunchKernelGGL(k_level_advance, dim3(1), dim3(1), 0, stream, d.ctrl, delta);
    return hipGetLastError();
}

hipError_t batch_level_from_deepest(const BatchDev &d, hipStream_t stream) {
    hipLaunchKernelGGL(k_level_from_deepest, dim3(1), dim3(1), 0, stream, d.ctrl);
    return hipGetLastError();
}

hipError_t batch_fused(const BatchDev *devs_dev, int32_t nbatches, bool narrow,
                       const int32_t *lanes_dev, const int2 *batches_dev, hipStream_t stream) {
    if (nbatches <= 0) return hipSuccess;
    hipLaunchKernelGGL(narrow ? k_batch_fused<true> : k_batch_fused<false>, dim3(nbatches),
                       dim3(kFusedBlock), 0, stream, devs_dev, lanes_dev, batches_dev);
    return hipGetLastError();
}

hipError_t batch_export(const BatchDev &d, int32_t deepest, int32_t nlanes, int32_t *dist,
                        double *sigma, hipStream_t stream) {
    int grid = (d.n + kBlock - 1) / kBlock;
    grid = grid < 1 ? 1 : (grid > 4096 ? 4096 : grid);
    hipLaunchKernelGGL(BC_PICK(k_batch_export, d), dim3(grid), dim3(kBlock), 0, stream, d,
                       deepest, nlanes, dist, sigma);
    return hipGetLastError();
}

}  // namespace bcx
