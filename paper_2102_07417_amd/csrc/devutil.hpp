// Device helpers for gfx950 (64-wide wavefronts, 8 XCDs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace camg {

constexpr int kWave = 64;

// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  Renumber them so that each XCD works on one contiguous range of
// logical blocks: neighbouring rows then share the XCD's L2 for the
// gathered vector entries.  gridDim.x must be a multiple of 8.
__device__ __forceinline__ int xcd_block() {
    const int g = gridDim.x, b = blockIdx.x;
    return (b & 7) * (g >> 3) + (b >> 3);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

template <int W, class T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Sum over a block of NT threads in a fixed order (wave shuffles, then the
// waves in index order).  Result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[NT / kWave];
    v = wave_sum(v);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / kWave; ++i) t += ws[i];
    }
    __syncthreads();
    return t;
}

// Block-wide integer sum / unsigned max; result valid in thread 0.
template <int NT>
__device__ __forceinline__ long long block_sum_ll(long long v) {
    __shared__ long long ws[NT / kWave];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / kWave; ++i) t += ws[i];
    __syncthreads();
    return t;
}

template <int NT>
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v) {
    __shared__ unsigned long long ws[NT / kWave];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long x = __shfl_xor(v, o, kWave);
        v = x > v ? x : v;
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < NT / kWave; ++i) t = ws[i] > t ? ws[i] : t;
    __syncthreads();
    return t;
}

// Deterministic sum of partials[0..n) by one block of NT threads: thread t
// adds t, t+NT, ... in order, then the fixed block tree.  Thread 0 gets it.
template <int NT>
__device__ __forceinline__ double sum_partials(const double *partials, int n) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v += partials[i];
    return block_sum<NT>(v);
}

// splitmix64 (Steele, Lea, Flood 2014): draw number c (from 0) of a
// generator seeded with `seed`.
__device__ __host__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int find_col(const int32_t *ci, int lo, int hi, int j) {
    // position of j in the sorted ci[lo, hi) or -1
    hi -= 1;
    while (lo <= hi) {
        int mid = lo + ((hi - lo) >> 1);
        int c = ci[mid];
        if (c == j) return mid;
        if (c < j) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

}  // namespace camg
