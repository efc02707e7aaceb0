// Device helpers shared by the kernel files of the sgm library (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sgm_internal.h"

namespace sgm {

__device__ __forceinline__ bool bit_test(const uint64_t *bits, int32_t x) {
    return (bits[x >> 6] >> (x & 63)) & 1ull;
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) { return (1ull << lane) - 1ull; }

// Candidate predicate (Def. 3.3 + pin + incoming degree).
__device__ __forceinline__ bool vinfo_ok(const VPred &p, int2 vi) {
    return (p.label < 0 || vi.x == p.label) && (vi.y & 255) >= p.qout && (vi.y >> 8) >= p.qin;
}

__device__ __forceinline__ bool vpred(const DevGraph &g, const VPred &p, int32_t v) {
    if (p.pin >= 0 && v != p.pin) return false;
    return vinfo_ok(p, g.vinfo[v]);
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ int32_t wave_incl_scan32(int32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// Block-wide exclusive scan of one int64 per thread. Returns the exclusive
// prefix; *total receives the block sum. `sh` holds >= blockDim/64 entries.
// Contains two barriers, the last one after every read of `sh`.
__device__ __forceinline__ int64_t block_excl_scan(int64_t x, int64_t *sh, int64_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int64_t inc = wave_incl_scan(x, lane);
    if (lane == 63) sh[wid] = inc;
    __syncthreads();
    int64_t wo = 0, tot = 0;
    for (int w = 0; w < nw; ++w) {
        const int64_t s = sh[w];
        if (w < wid) wo += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wo + inc - x;
}

// First index i in [lo, hi) with v[i] >= x (hi if none).
__device__ __forceinline__ int32_t lower_bound_i32(const int32_t *v, int32_t lo, int32_t hi,
                                                   int32_t x) {
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

}  // namespace sgm
