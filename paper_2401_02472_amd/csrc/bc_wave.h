// Wavefront-level helpers shared by the library's kernels (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bc_internal.h"

namespace bcx {

// Cross-lane helpers read other lanes' registers, so every lane of the wave
// must be active where they run.  Check builds (BC_CHECK_EXEC) count every
// call made with part of the wave inactive, per translation unit; normal
// builds compile the check away.
#ifdef BC_CHECK_EXEC
static __device__ unsigned int exec_partial_count;
#define BC_FULL_EXEC()                                                   \
    do {                                                                 \
        if (__builtin_amdgcn_read_exec() != ~0ull)                       \
            atomicAdd(&::bcx::exec_partial_count, 1u);                   \
    } while (0)
// The translation unit's count since the last call (host side).
static inline unsigned int exec_partial_take() {
    unsigned int v = 0, zero = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(exec_partial_count), sizeof(v)) != hipSuccess)
        return ~0u;
    (void)hipMemcpyToSymbol(HIP_SYMBOL(exec_partial_count), &zero, sizeof(zero));
    return v;
}
#else
#define BC_FULL_EXEC() \
    do {               \
    } while (0)
#endif

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ double wave_sum(double x) {
    BC_FULL_EXEC();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
    BC_FULL_EXEC();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x |= __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int src) {
    BC_FULL_EXEC();
    const uint32_t lo = __shfl((uint32_t)x, src);
    const uint32_t hi = __shfl((uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t x, uint32_t &total) {
    BC_FULL_EXEC();
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
    BC_FULL_EXEC();
    int o = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t ex = __shfl(excl, o + step);  // o + step <= 63 at every step
        if (ex <= a) o += step;
    }
    return o;
}

__device__ __forceinline__ int wave_sum_int(int x) {
    BC_FULL_EXEC();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

// Transpose of a 64x64 bit matrix held one row per lane (bit j of lane i's
// value = entry (i, j)): lane i receives column i.  Six butterfly stages, each
// swapping the off-diagonal k x k blocks of every 2k x 2k block.
__device__ __forceinline__ uint64_t transpose64(uint64_t row) {
    BC_FULL_EXEC();
    const int lane = lane_id();
    const uint64_t keep[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                              0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0, k = 32; st < 6; ++st, k >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)row, k);
        const uint32_t hi = __shfl_xor((uint32_t)(row >> 32), k);
        const uint64_t p = ((uint64_t)hi << 32) | lo;
        if (lane & k) row = (row & ~keep[st]) | ((p >> k) & keep[st]);
        else row = (row & keep[st]) | ((p & keep[st]) << k);
    }
    return row;
}

}  // namespace bcx
