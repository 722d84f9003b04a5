// Allocation-free BC run (bc_run_async_noalloc): the batched path's
// host-driven level loop with its whole workspace carved out of one fixed
// device array, for callers that cannot allocate device memory.
//
// The array below is the workspace of every such call on a device.  Host code
// never uses its name as an address: at a device's first call the device
// address is looked up once (hipGetSymbolAddress, that device current) and
// kept per device; kernels receive pointers derived from it.  Calls that
// overlap on one device share the array and race; the array keeps the last
// call's contents, so everything a run reads before writing is cleared by
// the run itself (the batch-start kernel clears the masks, a fill kernel the
// BC total and the control words).
#include "bc_runtime.h"

namespace bcx {
namespace {

constexpr size_t kScratchBytes = (size_t)BC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

// Device address of this device's array (the device must be current).
hipError_t scratch_of(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

__global__ void k_zero_words(uint32_t *p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Clear `bytes` (a multiple of 4) at p with a kernel.
hipError_t zero_bytes(void *p, size_t bytes, hipStream_t stream) {
    const size_t words = bytes / 4;
    if (words == 0) return hipSuccess;
    size_t grid = (words + kBlock - 1) / kBlock;
    grid = grid > 1024 ? 1024 : grid;
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)grid), dim3(kBlock), 0, stream,
                       (uint32_t *)p, words);
    return hipGetLastError();
}

// Where the workspace of one run on g lies in the array (byte offsets), and
// how many levels the level array then holds.
struct Layout {
    size_t vis, sigma, coef, ctrl, bc, reach, partial, clist, ilist, cand, front, lanes, levels;
    int32_t lcap = 0;
};

// false: not even two levels fit.
bool layout_of(const bc_graph_s *g, Layout &L) {
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    size_t at = 0;
    auto take = [&](size_t bytes) {
        const size_t r = at;
        at += align_up(bytes);
        return r;
    };
    L.vis = take(n * sizeof(uint64_t));
    L.sigma = take(n * kWave * sizeof(double));
    L.coef = take(n * kWave * sizeof(double));
    L.ctrl = take(kBatchCtrlInts * sizeof(int32_t));
    L.bc = take(n * sizeof(double));
    // the host-driven loop's work items, as in bc_run_async
    L.reach = take((size_t)std::max(g->bci.multi_end, 1) * sizeof(uint64_t));
    L.partial = take(partial_rows(g) * kWave * sizeof(double));
    L.clist = take(n * sizeof(int32_t));
    L.ilist = take((size_t)std::max<uint32_t>(g->bci.items_in, 1) * sizeof(int32_t));
    L.cand = take(((n + 15) / 16) * 16);
    L.front = take((size_t)kFrontSets * kFrontWaves * 2 * sizeof(unsigned long long));
    L.lanes = take(kWave * sizeof(int32_t));
    L.levels = at;
    if (at >= kScratchBytes) return false;
    const size_t per_level = batch_level_bytes(g, 1, 1);
    // a graph's depth is at most n - 1: n + 1 levels always suffice
    const size_t fit = (kScratchBytes - at) / per_level;
    L.lcap = (int32_t)std::min<size_t>(fit, (size_t)g->n + 1);
    return L.lcap >= 2;
}

}  // namespace
}  // namespace bcx

using namespace bcx;

extern "C" bc_status bc_run_async_noalloc(bc_graph_t g, const int32_t *sources, int32_t k,
                                          double *bc_out_dev, void *stream_) {
    if (!g || (!bc_out_dev && g->n > 0)) return BC_ERR_INVALID_ARG;
    bc_status st = check_sources(g, sources, k);
    if (st != BC_OK) return st;
    if (g->n == 0) return BC_OK;
    Layout L;
    if (!layout_of(g, L)) return BC_ERR_TOO_LARGE;
    DeviceGuard dg(g->device);
    hipStream_t stream = (hipStream_t)stream_;
    void *base_v = nullptr;
    BC_TRY_HIP(scratch_of(g->device, &base_v));
    char *base = (char *)base_v;
    const size_t n = (size_t)g->n;

    // the workspace, as batch_ws_create lays it out, inside the array
    BatchDev d{};
    d.n = g->n;
    d.H = 1;
    d.row_ptr = g->d_row_ptr;
    d.col_idx = g->d_col_idx;
    set_items(g, d);
    d.row_ptr_in = g->d_row_ptr_in;
    d.col_idx_in = g->d_col_idx_in;
    d.vis = (uint64_t *)(base + L.vis);
    d.sigma = (double *)(base + L.sigma);
    d.sigma32 = reinterpret_cast<uint32_t *>(d.sigma);
    d.coef = (double *)(base + L.coef);
    d.ctrl = (int32_t *)(base + L.ctrl);
    d.bc = (double *)(base + L.bc);
    d.reach = (uint64_t *)(base + L.reach);
    d.partial = (double *)(base + L.partial);
    d.clist = (int32_t *)(base + L.clist);
    d.ilist = (int32_t *)(base + L.ilist);
    d.cand = (uint8_t *)(base + L.cand);
    d.front = (unsigned long long *)(base + L.front);
    d.nnz = g->nnz;
    const int32_t sdiv = sparse_div_of(g, nullptr);
    d.sparse_arcs = sdiv < 0 ? 0 : g->nnz / std::max(sdiv, 1);
    d.stats = nullptr;
    d.nseg = 0;
    d.iperm = g->d_iperm;
    d.lcap = L.lcap;
    d.F = (uint64_t *)(base + L.levels);
    ExtTables ext;
    ext.xs = (double *)(d.F + (size_t)L.lcap * n);
    ext.xmax = (unsigned long long *)(ext.xs + (size_t)L.lcap * kWave);
    ext.xe = (int32_t *)(ext.xmax + (size_t)L.lcap * kWave);
    int32_t *d_lanes = (int32_t *)(base + L.lanes);

    hipError_t e = zero_bytes(d.bc, n * sizeof(double), stream);
    if (e == hipSuccess) e = zero_bytes(d.ctrl, kBatchCtrlInts * sizeof(int32_t), stream);
    if (e != hipSuccess) return from_hip(e);
    // host mirrors on the stack: no host allocation either
    int32_t h_ctrl[kBatchCtrlInts] = {};
    int32_t lanes[kWave];
    LaunchTimer timer;  // off: no events
    const int32_t width = std::min(batch_width_of(g, nullptr, k), (int32_t)kWave);
    int32_t range = 0, run_depth = 0;
    for (int32_t b0 = 0; b0 < k;) {
        const int32_t nl = std::min(width, k - b0);
        for (int32_t i = 0; i < nl; ++i) lanes[i] = g->h_perm[(size_t)sources[b0 + i]];
        // ordered after the previous batch's kernels; drive_batch waits on the
        // stream before it returns, so the stack copy outlives the transfer
        e = hipMemcpyAsync(d_lanes, lanes, (size_t)nl * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream);
        if (e != hipSuccess) return from_hip(e);
        BatchOutcome how = BatchOutcome::Done;
        int32_t deepest = 0;
        // (the array's sigma rows are double-sized)
        e = drive_batch(g, d, ext, d_lanes, nl, h_ctrl, stream, timer, nullptr, 1, how, deepest,
                        nullptr, true);
        if (e != hipSuccess) return from_hip(e);
        if (how == BatchOutcome::Rerun) continue;           // same memory, wider rows
        if (how == BatchOutcome::Grow) return BC_ERR_TOO_LARGE;  // deeper than the array holds
        range |= h_ctrl[kCtlRange];
        run_depth = std::max(run_depth, deepest);
        b0 += nl;
    }
    e = gather_f64(g->n, g->d_perm, d.bc, bc_out_dev, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_ctrl, d.ctrl, kBatchCtrlInts * sizeof(int32_t), hipMemcpyDeviceToHost,
                           stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return from_hip(e);
    range |= h_ctrl[kCtlRange];
    if (k > 0) g->batch_depth_hint.store(run_depth);
    return range ? BC_ERR_RANGE : BC_OK;
}
