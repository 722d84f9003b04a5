// Single-source shortest paths over weighted arcs: the paper's fixed-point
// formulation (Sections "fixedPoint Construct" and "Min/Max Constructs").  A
// pass relaxes the out-arcs of every vertex modified in the previous pass,
// <nbr.dist, nbr.modified> = <Min(nbr.dist, v.dist + w), true>, with an atomic
// min on the distance; the passes repeat until one modifies nothing.
//
// Instead of two modified arrays that must be cleared, a vertex carries the
// number of the pass that must process it (stamp): a pass p takes the
// vertices stamped p and stamps p + 1 on the ones it improves.  Passes are
// launched over the same work items as the batched BC kernels: chunk items of
// 512 arcs for vertices of degree > 64, and 64-vertex groups whose arcs are
// flattened into runs of 64 (one arc per lane).  Distances are exact integers,
// so the result does not depend on the order of the relaxations.
#include "bc_internal.h"
#include "bc_wave.h"

namespace bcx {
namespace {

constexpr int kPerLane = kChunk / kWave;  // arcs per lane in a chunk item
static_assert(kPerLane * kWave == kChunk, "a chunk item is kPerLane arcs per lane");

constexpr int32_t kInf = 0x7fffffff;

struct Relax {
    uint32_t active = 0, arcs = 0, better = 0;  // work counters (per lane)
    bool changed = false;
};

// Relax arc e of a vertex at distance dv: a shorter distance is installed
// with an atomic min and the neighbour is stamped for the next pass.
__device__ __forceinline__ void relax(const SsspDev &d, int32_t nb, int32_t nd, int32_t pass,
                                      Relax &r) {
    if (nd < d.dist[nb]) {
        const int32_t old = atomicMin(&d.dist[nb], nd);
        if (nd < old) {
            d.stamp[nb] = pass + 1;
            r.changed = true;
            ++r.better;
        }
    }
}

__device__ __forceinline__ int32_t weight_of(const SsspDev &d, int64_t e) {
    return d.weight ? d.weight[e] : 1;
}

// Chunk item (vertex of degree > 64): kPerLane arcs per lane, loads issued together.
__device__ __forceinline__ void sssp_chunk(const SsspDev &d, int32_t pass, uint32_t item,
                                           Relax &r) {
    const int lane = lane_id();
    const int2 info = d.item_info[item];
    const int32_t v = info.x, j = info.y;
    if (d.stamp[v] != pass) return;
    const int32_t dv = d.dist[v];
    const int32_t rs = d.row_ptr[v], re = d.row_ptr[v + 1];
    const int32_t cb = rs + j * kChunk, ce = min(re, cb + kChunk);
    if (lane == 0 && j == 0) ++r.active;
    int32_t nb[kPerLane], nd[kPerLane];
#pragma unroll
    for (int u = 0; u < kPerLane; ++u) {
        const int32_t e = cb + u * kWave + lane;
        nb[u] = e < ce ? d.col_idx[e] : -1;
        nd[u] = e < ce ? dv + weight_of(d, e) : 0;
        r.arcs += e < ce ? 1u : 0u;
    }
#pragma unroll
    for (int u = 0; u < kPerLane; ++u)
        if (nb[u] >= 0) relax(d, nb[u], nd[u], pass, r);
}

// 64 vertices of degree <= 64: the arcs of the ones stamped for this pass,
// flattened into runs of 64.
__device__ __forceinline__ void sssp_group(const SsspDev &d, int32_t pass, int32_t base,
                                           Relax &r) {
    const int lane = lane_id();
    const int32_t me = base + lane;
    int32_t rs = 0, cnt = 0, dv = 0;
    if (me < d.n && d.stamp[me] == pass) {
        dv = d.dist[me];
        rs = d.row_ptr[me];
        cnt = d.row_ptr[me + 1] - rs;
        ++r.active;
    }
    uint32_t total;
    const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
    for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
        const uint32_t a = c0 + (uint32_t)lane;
        const int o = owner_lane(excl, a);
        const int32_t o_rs = __shfl(rs, o);
        const uint32_t o_excl = __shfl(excl, o);
        const int32_t o_dv = __shfl(dv, o);
        if (a < total) {
            const int32_t e = o_rs + (int32_t)(a - o_excl);
            ++r.arcs;
            relax(d, d.col_idx[e], o_dv + weight_of(d, e), pass, r);
        }
    }
}

// One pass.  prev: the previous pass's "modified something" flag (NULL for
// the first pass); a pass after a quiet one returns at once, so that several
// passes can be queued without a host wait.  cur receives 1 if this pass
// improved a distance (a plain store of 1 by each wave that did).
__global__ __launch_bounds__(kBlock) void k_sssp_pass(SsspDev d, int32_t pass,
                                                      const int32_t *prev, int32_t *cur) {
    if (prev && *prev == 0) return;
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    Relax r;
    for (uint32_t it = wave; it < d.items + groups; it += nwaves) {
        if (it < d.items) sssp_chunk(d, pass, it, r);
        else sssp_group(d, pass, d.big_end + (int32_t)(it - d.items) * kWave, r);
    }
    if (__ballot(r.changed) && lane_id() == 0) *cur = 1;
    if (d.stats) {
        unsigned long long a = r.active, b = r.arcs, c = r.better;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off);
            b += __shfl_xor(b, off);
            c += __shfl_xor(c, off);
        }
        if (lane_id() == 0 && (a | b | c)) {
            atomicAdd(&d.stats[0], a);
            atomicAdd(&d.stats[1], b);
            atomicAdd(&d.stats[2], c);
        }
    }
}

__global__ void k_sssp_init(int32_t n, int32_t *dist, int32_t *stamp, int32_t src) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        dist[v] = v == src ? 0 : kInf;
        stamp[v] = v == src ? 1 : 0;
    }
}

// dist in caller order, -1 where unreachable.
__global__ void k_sssp_export(int32_t n, const int32_t *perm, const int32_t *dist,
                              int32_t *out) {
    for (int32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x) {
        const int32_t x = dist[perm[o]];
        out[o] = x == kInf ? -1 : x;
    }
}

// new_vals[e] = old_vals[e'] where e' is the same arc in the caller's CSR
// (rows are permuted, the arcs of a row keep their order).
__global__ void k_permute_arcs(int32_t n, int64_t nnz, const int32_t *old_rp,
                               const int32_t *old_vals, const int32_t *new_rp,
                               const int32_t *iperm, int32_t *new_vals) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if ((int64_t)new_rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        new_vals[e] = old_vals[(int64_t)old_rp[iperm[lo]] + (e - new_rp[lo])];
    }
}

int blocks_for(int64_t n) {
    int64_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

#ifdef BC_CHECK_EXEC
unsigned int exec_partial_sssp() { return exec_partial_take(); }
#endif

hipError_t sssp_init(int32_t n, int32_t *dist, int32_t *stamp, int32_t src, hipStream_t stream) {
    hipLaunchKernelGGL(k_sssp_init, dim3(blocks_for(n)), dim3(kBlock), 0, stream, n, dist, stamp,
                       src);
    return hipGetLastError();
}

hipError_t sssp_pass(const SsspDev &d, int32_t pass, const int32_t *prev, int32_t *cur,
                     hipStream_t stream) {
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    int64_t blocks = (d.items + groups + kWavesPerBlock - 1) / kWavesPerBlock;
    blocks = blocks < 1 ? 1 : (blocks > kMaxGridBlocks ? kMaxGridBlocks : blocks);
    hipLaunchKernelGGL(k_sssp_pass, dim3((int)blocks), dim3(kBlock), 0, stream, d, pass, prev,
                       cur);
    return hipGetLastError();
}

hipError_t sssp_export(int32_t n, const int32_t *perm, const int32_t *dist, int32_t *out,
                       hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sssp_export, dim3(blocks_for(n)), dim3(kBlock), 0, stream, n, perm, dist,
                       out);
    return hipGetLastError();
}

hipError_t permute_arc_values(int32_t n, int64_t nnz, const int32_t *old_rp,
                              const int32_t *old_vals, const int32_t *new_rp,
                              const int32_t *iperm, int32_t *new_vals, hipStream_t stream) {
    if (n == 0 || nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_arcs, dim3(blocks_for(nnz)), dim3(kBlock), 0, stream, n, nnz,
                       old_rp, old_vals, new_rp, iperm, new_vals);
    return hipGetLastError();
}

}  // namespace bcx
