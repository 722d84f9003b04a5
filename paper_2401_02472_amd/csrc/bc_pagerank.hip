// PageRank: the paper's pull iteration (the generated loop of Section "Backend
// Optimizations", OpenACC reduction).  Every vertex starts at 1/n; an
// iteration computes sum = sum over the arcs u->v of pr[u] / outdeg(u),
// val = (1 - d)/n + d * sum and the L1 change sum |val - pr[v]|, into a second
// buffer; iterations stop when the change is at most tol or after max_iter.
//
// pr[u] / outdeg(u) is kept per vertex (contrib, written with the rank), so
// an arc costs one 8-byte gather.  Sums run over the reversed CSR in the
// work layout of the batched BC kernels: vertices of degree <= 64 64 at a
// time with their arcs flattened into runs of 64 (a segmented scan per run),
// vertices up to 512 arcs one wave each (tree sum),
// larger ones one wave per 512-arc chunk with the chunks' partial sums added
// in chunk order by a second kernel.  The change is summed per wave into
// slots that a third kernel adds in slot order, so every result repeats bit
// for bit.
#include "bc_internal.h"
#include "bc_wave.h"

namespace bcx {
namespace {

constexpr int kPerLane = kChunk / kWave;  // arcs per lane in a chunk item
static_assert(kPerLane * kWave == kChunk, "a chunk item is kPerLane arcs per lane");

constexpr int kDiffBlock = 1024;

__device__ __forceinline__ bool converged(const PrDev &d, int32_t iter) {
    return iter > 0 && d.diff[iter - 1] >= 0.0 && d.diff[iter - 1] <= d.tol;
}

// New rank of v from its sum: rank, its per-arc share and the change.
__device__ __forceinline__ double settle_rank(const PrDev &d, int32_t v, double sum,
                                              const double *pr, double *pr_next,
                                              double *contrib_next) {
    const double val = d.base + d.damping * sum;
    pr_next[v] = val;
    const int32_t od = d.row_ptr[v + 1] - d.row_ptr[v];
    contrib_next[v] = od > 0 ? val / (double)od : 0.0;
    return fabs(val - pr[v]);
}

__device__ __forceinline__ void report_diff(const PrDev &d, int set, double x) {
    x = wave_sum(x);
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (lane_id() == 0) d.slots[(size_t)set * kFrontWaves + wave] = x;
}

// Pull step: groups of 64 small vertices (one lane each), chunk items of the
// big ones (one wave each; a split vertex leaves a partial sum).
__global__ __launch_bounds__(kBlock) void k_pr_pull(PrDev d, int32_t iter) {
    if (converged(d, iter)) return;
    const double *pr = d.pr[iter & 1];
    const double *contrib = d.contrib[iter & 1];
    double *pr_next = d.pr[(iter + 1) & 1];
    double *contrib_next = d.contrib[(iter + 1) & 1];
    const int lane = lane_id();
    const uint32_t groups = (uint32_t)((d.n - d.big_end + kWave - 1) / kWave);
    const uint32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const uint32_t nwaves = gridDim.x * kWavesPerBlock;
    double change = 0.0;
    for (uint32_t it = wave; it < d.items_in + groups; it += nwaves) {
        if (it < d.items_in) {
            const int2 info = d.item_info_in[it];
            const int32_t v = info.x, j = info.y;
            const int32_t rs = d.row_ptr_in[v], re = d.row_ptr_in[v + 1];
            const int32_t cb = rs + j * kChunk, ce = min(re, cb + kChunk);
            double x[kPerLane];
#pragma unroll
            for (int u = 0; u < kPerLane; ++u) {
                const int32_t e = cb + u * kWave + lane;
                x[u] = e < ce ? contrib[d.col_idx_in[e]] : 0.0;
            }
            double s = 0.0;
#pragma unroll
            for (int u = 0; u < kPerLane; ++u) s += x[u];
            s = wave_sum(s);
            if (v < d.multi_end) {
                if (lane == 0) d.partial[it] = s;
            } else if (lane == 0) {
                change += settle_rank(d, v, s, pr, pr_next, contrib_next);
            }
        } else {
            // 64 vertices of degree <= 64: their arcs flattened into runs of 64
            // (coalesced index reads, 64 gathers per load), each run summed per
            // vertex by a segmented scan and added to the vertex's lane
            const int32_t v = d.big_end + (int32_t)(it - d.items_in) * kWave + lane;
            int32_t rs = 0, cnt = 0;
            if (v < d.n) {
                rs = d.row_ptr_in[v];
                cnt = d.row_ptr_in[v + 1] - rs;
            }
            uint32_t total;
            const uint32_t excl = wave_excl_scan((uint32_t)cnt, total);
            double s = 0.0;
            for (uint32_t c0 = 0; c0 < total; c0 += kWave) {
                const uint32_t a = c0 + (uint32_t)lane;
                const int o = owner_lane(excl, a);
                const int32_t o_rs = __shfl(rs, o);
                const uint32_t o_excl = __shfl(excl, o);
                double x = a < total ? contrib[d.col_idx_in[o_rs + (int32_t)(a - o_excl)]] : 0.0;
#pragma unroll
                for (int off = 1; off < kWave; off <<= 1) {
                    const double y = __shfl_up(x, off);
                    const int oy = __shfl_up(o, off);
                    if (lane >= off && oy == o) x += y;
                }
                // the vertex's arcs in this run end at lane hi - 1 - c0
                const uint32_t lo = excl > c0 ? excl : c0;
                const uint32_t hi = min(excl + (uint32_t)cnt, c0 + (uint32_t)kWave);
                const double part = __shfl(x, hi > lo ? (int)(hi - 1 - c0) : 0);
                if (hi > lo) s += part;
            }
            if (v < d.n) change += settle_rank(d, v, s, pr, pr_next, contrib_next);
        }
    }
    report_diff(d, 0, change);
}

// Split vertices: their chunks' partial sums added in chunk order, one wave each.
__global__ __launch_bounds__(kBlock) void k_pr_finish(PrDev d, int32_t iter) {
    if (converged(d, iter)) return;
    const double *pr = d.pr[iter & 1];
    double *pr_next = d.pr[(iter + 1) & 1];
    double *contrib_next = d.contrib[(iter + 1) & 1];
    const int32_t wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int32_t nwaves = gridDim.x * kWavesPerBlock;
    double change = 0.0;
    for (int32_t v = wave; v < d.multi_end; v += nwaves) {
        double s = 0.0;
        for (uint32_t i = d.item_first_in[v]; i < d.item_first_in[v + 1]; ++i)
            s += d.partial[i];
        if (lane_id() == 0) change += settle_rank(d, v, s, pr, pr_next, contrib_next);
    }
    report_diff(d, 1, change);
}

// diff[iter] = the slots of both steps added in order (one block).
__global__ __launch_bounds__(kDiffBlock) void k_pr_diff(PrDev d, int32_t iter, int32_t w0,
                                                        int32_t w1) {
    if (converged(d, iter)) return;
    __shared__ double s[kDiffBlock];
    const int t = threadIdx.x;
    double x = 0.0;
    for (int32_t w = t; w < w0; w += kDiffBlock) x += d.slots[w];
    for (int32_t w = t; w < w1; w += kDiffBlock) x += d.slots[(size_t)kFrontWaves + w];
    s[t] = x;
    __syncthreads();
    for (int h = kDiffBlock / 2; h >= 1; h >>= 1) {
        if (t < h) s[t] += s[t + h];
        __syncthreads();
    }
    if (t == 0) d.diff[iter] = s[0];
}

__global__ void k_pr_init(PrDev d, int32_t max_iter) {
    const double r = 1.0 / (double)d.n;
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < d.n;
         v += gridDim.x * blockDim.x) {
        d.pr[0][v] = r;
        const int32_t od = d.row_ptr[v + 1] - d.row_ptr[v];
        d.contrib[0][v] = od > 0 ? r / (double)od : 0.0;
    }
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < max_iter;
         i += gridDim.x * blockDim.x)
        d.diff[i] = -1.0;  // iterations not run
}

int waves_blocks(int64_t waves) {
    int64_t b = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    return (int)(b < 1 ? 1 : (b > kMaxGridBlocks ? kMaxGridBlocks : b));
}

}  // namespace

#ifdef BC_CHECK_EXEC
unsigned int exec_partial_pagerank() { return exec_partial_take(); }
#endif

hipError_t pagerank_init(const PrDev &d, int32_t max_iter, hipStream_t stream) {
    const int64_t m = d.n > max_iter ? d.n : max_iter;
    int64_t b = (m + kBlock - 1) / kBlock;
    b = b < 1 ? 1 : (b > 4096 ? 4096 : b);
    hipLaunchKernelGGL(k_pr_init, dim3((int)b), dim3(kBlock), 0, stream, d, max_iter);
    return hipGetLastError();
}

hipError_t pagerank_pull(const PrDev &d, int32_t iter, hipStream_t stream) {
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    hipLaunchKernelGGL(k_pr_pull, dim3(waves_blocks(d.items_in + groups)), dim3(kBlock), 0, stream,
                       d, iter);
    return hipGetLastError();
}

hipError_t pagerank_finish(const PrDev &d, int32_t iter, hipStream_t stream) {
    const int64_t groups = (d.n - d.big_end + kWave - 1) / kWave;
    const int g0 = waves_blocks(d.items_in + groups);
    int g1 = 0;
    if (d.multi_end > 0) {
        g1 = waves_blocks(d.multi_end);
        hipLaunchKernelGGL(k_pr_finish, dim3(g1), dim3(kBlock), 0, stream, d, iter);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_pr_diff, dim3(1), dim3(kDiffBlock), 0, stream, d, iter,
                       g0 * kWavesPerBlock, g1 * kWavesPerBlock);
    return hipGetLastError();
}

}  // namespace bcx
