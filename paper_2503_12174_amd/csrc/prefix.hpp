// prefix.hpp -- workgroup and grid prefix sums shared by the BVH builders (device code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpcs {
namespace {

constexpr int SCAN_TB = 256;   // workgroup size block_exclusive is written for

// exclusive prefix of v over a 256-thread workgroup (every thread must call), the
// workgroup's total in *total; two 32-bit counters packed into one 64-bit value add
// without carrying into each other as long as each stays below 2^32
__device__ __forceinline__ uint64_t block_exclusive(uint64_t v, uint64_t* wsum, uint64_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)x, off), hi = __shfl_up((uint32_t)(x >> 32), off);
        if (lane >= off) x += ((uint64_t)hi << 32) | lo;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int k = 0; k < SCAN_TB / 64; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    *total = all;
    __syncthreads();   // wsum may be reused by the next call
    return before + x - v;
}

// exclusive scan of per-workgroup totals in place, one workgroup of 1024 threads; the
// grand total into *total
__global__ void __launch_bounds__(1024) k_scan_blocks(uint64_t* __restrict__ sums, int n, uint64_t* __restrict__ total) {
    __shared__ uint64_t part[1024];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per;
    const int e = min(b + per, n);
    uint64_t s = 0;
    for (int i = b; i < e; ++i) s += sums[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint64_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    for (int i = b; i < e; ++i) {
        const uint64_t v = sums[i];
        sums[i] = run;
        run += v;
    }
    if (threadIdx.x == 1023) *total = part[1023];
}

}  // namespace
}  // namespace dpcs
