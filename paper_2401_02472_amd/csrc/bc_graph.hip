// Graph set-up kernels: relabelling of the CSR into the library's internal
// vertex order, and gathers from internal order back to the caller's order.
#include "bc_internal.h"

namespace bcx {
namespace {

__global__ __launch_bounds__(kBlock) void k_relabel(int32_t n, int64_t nnz,
                                                    const int32_t *old_rp,
                                                    const int32_t *old_ci,
                                                    const int32_t *new_rp,
                                                    const int32_t *perm,
                                                    const int32_t *iperm, int32_t *new_ci) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += stride) {
        // owner u: last vertex with new_rp[u] <= e
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo + 1) / 2;
            if ((int64_t)new_rp[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        const int32_t o = iperm[lo];
        new_ci[e] = perm[old_ci[(int64_t)old_rp[o] + (e - new_rp[lo])]];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int32_t n, const int32_t *perm, const T *src,
                                                   T *dst) {
    for (int32_t o = blockIdx.x * blockDim.x + threadIdx.x; o < n; o += gridDim.x * blockDim.x)
        dst[o] = src[perm[o]];
}

int grid_for(int64_t items) {
    int64_t g = (items + kBlock - 1) / kBlock;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t relabel_csr(int32_t n, int64_t nnz, const int32_t *old_rp, const int32_t *old_ci,
                       const int32_t *new_rp, const int32_t *perm, const int32_t *iperm,
                       int32_t *new_ci, hipStream_t stream) {
    if (nnz == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_relabel, dim3(grid_for(nnz)), dim3(kBlock), 0, stream, n, nnz, old_rp,
                       old_ci, new_rp, perm, iperm, new_ci);
    return hipGetLastError();
}

hipError_t gather_f64(int32_t n, const int32_t *perm, const double *src, double *dst,
                      hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<double>, dim3(grid_for(n)), dim3(kBlock), 0, stream, n, perm,
                       src, dst);
    return hipGetLastError();
}

// out[v] = (accumulate ? out[v] : 0) + parts[0][v] + parts[1][v] + ... (in
// part order), parts stored [nparts][n].
__global__ void k_sum_parts(int32_t n, const double *parts, int32_t nparts, double *out,
                            int32_t accumulate) {
    for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        double t = accumulate ? out[v] : 0.0;
        for (int32_t i = 0; i < nparts; ++i) t += parts[(size_t)i * n + v];
        out[v] = t;
    }
}

hipError_t sum_parts(int32_t n, const double *parts, int32_t nparts, double *out,
                     hipStream_t stream, bool accumulate) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_parts, dim3(grid_for(n)), dim3(kBlock), 0, stream, n, parts, nparts,
                       out, accumulate ? 1 : 0);
    return hipGetLastError();
}

hipError_t gather_i32(int32_t n, const int32_t *perm, const int32_t *src, int32_t *dst,
                      hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<int32_t>, dim3(grid_for(n)), dim3(kBlock), 0, stream, n, perm,
                       src, dst);
    return hipGetLastError();
}

}  // namespace bcx
