// Wavefront-level helpers shared by the library's kernels (64-lane waves).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bc_internal.h"

namespace bcx {

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

}  // namespace bcx
