// dms_scan.hpp -- device-wide exclusive prefix sum (reduce, scan of block
// partials, downsweep), used by the radix passes and the critical-cell
// compaction.  Three plain launches; no inter-block waiting.
#pragma once
#include "dms_common.hpp"

namespace dms {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;  // elements per block

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over a kBlock-thread block; returns
// the exclusive prefix, writes the block total to *total.
template <typename T, int kBlock = kScanThreads>
__device__ __forceinline__ T block_exclusive_scan(T v, T *total)
{
    __shared__ T wsum[kBlock / kWave];
    const int lane = lane_id(), wave = threadIdx.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) wsum[wave] = inc;
    __syncthreads();
    T before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kBlock / kWave; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

// Sum of each chunk (order-free, so the loads are striped across the block
// and coalesced).  Loads past the end re-read the last element and are
// dropped, so that none waits behind a branch (every block's chunk starts
// inside the data).
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const T *in, int64_t len, T *partials)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    T x[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k * kScanThreads + threadIdx.x;
        x[k] = in[i < len ? i : len - 1];
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k * kScanThreads + threadIdx.x < len) s += x[k];
    T total;
    block_exclusive_scan(s, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// One block scans all partials (exclusive, in place), looping with a carry.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(T *partials, int64_t len)
{
    T carry = 0;
    for (int64_t start = 0; start < len; start += kScanChunk) {
        const int64_t base = start + (int64_t)threadIdx.x * kScanItems;
        T v[kScanItems];
        T s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < len ? partials[base + k] : T(0);
            s += v[k];
        }
        T total;
        T run = carry + block_exclusive_scan(s, &total);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < len) partials[base + k] = run;
            run += v[k];
        }
        carry += total;
    }
}

// Downsweep: the chunk is loaded and stored striped (coalesced) through LDS;
// each thread scans its kScanItems consecutive elements there.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(T *data, int64_t len, const T *partials)
{
    __shared__ T buf[kScanChunk];
    const int64_t base = (int64_t)blockIdx.x * kScanChunk;
    const int tid = threadIdx.x;
    T x[kScanItems];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {  // unconditional loads, as in k_scan_reduce
        const int64_t i = base + k * kScanThreads + tid;
        x[k] = data[i < len ? i : len - 1];
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kScanThreads + tid;
        buf[j] = base + j < len ? x[k] : T(0);
    }
    __syncthreads();
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = buf[tid * kScanItems + k];
        s += v[k];
    }
    T total;
    T run = partials[blockIdx.x] + block_exclusive_scan(s, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        buf[tid * kScanItems + k] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int j = k * kScanThreads + tid;
        if (base + j < len) data[base + j] = buf[j];
    }
}

constexpr size_t scan_partials_bytes(int64_t len, size_t elem)
{
    const int64_t blocks = (len + kScanChunk - 1) / kScanChunk;
    return align_up((size_t)(blocks > 0 ? blocks : 1) * elem, 256);
}

// Exclusive scan of data[0, len) in place; partials needs
// scan_partials_bytes(len, sizeof(T)) bytes.
template <typename T>
inline void exclusive_scan(T *data, int64_t len, T *partials, hipStream_t s)
{
    if (len <= 0) return;
    const int64_t blocks = (len + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, data, len,
                       partials);
    hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(kScanThreads), 0, s, partials, blocks);
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, data, len,
                       partials);
}

}  // namespace dms
