// Device-wide exclusive prefix sum: reduce tiles, scan the tile sums (recursively),
// then scan each tile with its offset.  Deterministic (fixed tile order).
#pragma once

#include "common.hpp"

namespace tcl {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr size_t kScanTile = (size_t)kScanThreads * kScanItems;

// Exclusive scan of one value per thread across a 256-thread block; *total gets the block sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* lds /*[kScanThreads/kWave]*/, T* total) {
    constexpr int NW = kScanThreads / kWave;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    T incl = wave_inclusive_scan(x);
    if (lane == kWave - 1) lds[w] = incl;
    __syncthreads();
    T base = 0, sum = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T s = lds[i];
        if (i < w) base += s;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return base + incl - x;
}

template <typename T>
struct ArrayIn {
    const T* p;
    size_t n;
    __device__ T operator()(size_t i) const { return i < n ? p[i] : T(0); }
};

// Tiles are read and written in striped order (element i * 256 + thread), so every
// global access is coalesced; the per-thread runs of 16 consecutive elements are
// formed through LDS, padded by one slot per 32 to avoid bank conflicts.
template <typename T, typename In>
__global__ __launch_bounds__(kScanThreads) void k_reduce_tiles(In in, size_t n, T* partials) {
    __shared__ T lds[kScanThreads / kWave];
    const size_t base = (size_t)blockIdx.x * kScanTile + threadIdx.x;
    T s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t e = base + (size_t)i * kScanThreads;
        if (e < n) s += in(e);
    }
    s = wave_sum(s);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int i = 0; i < kScanThreads / kWave; ++i) t += lds[i];
        partials[blockIdx.x] = t;
    }
}

__device__ __forceinline__ int scan_pad(int e) { return e + (e >> 5); }

template <typename T, typename In>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(In in, size_t n, const T* tile_off, T* out) {
    __shared__ T lds[kScanThreads / kWave];
    __shared__ T buf[kScanTile + kScanTile / 32];
    const size_t tile = (size_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanThreads + threadIdx.x;
        buf[scan_pad(e)] = (tile + e < n) ? in(tile + e) : T(0);
    }
    __syncthreads();
    T v[kScanItems];
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = buf[scan_pad(threadIdx.x * kScanItems + j)];
        s += v[j];
    }
    T total;
    T run = block_exclusive_scan(s, lds, &total) + (tile_off ? tile_off[blockIdx.x] : T(0));
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        buf[scan_pad(threadIdx.x * kScanItems + j)] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanThreads + threadIdx.x;
        if (tile + e < n) out[tile + e] = buf[scan_pad(e)];
    }
}

// Scratch elements needed by exclusive_scan for n items.
inline size_t scan_scratch_elems(size_t n) {
    size_t s = 0;
    while (n > kScanTile) {
        n = (n + kScanTile - 1) / kScanTile;
        s += n;
    }
    return s + 1;
}

// out[i] = sum of in(j) for j < i, for i in [0, n).  out may alias the array `in` reads.
template <typename T, typename In>
hipError_t exclusive_scan(In in, size_t n, T* out, T* scratch, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const size_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        k_scan_tiles<T, In><<<1, kScanThreads, 0, st>>>(in, n, nullptr, out);
        return hipGetLastError();
    }
    T* partials = scratch;
    k_reduce_tiles<T, In><<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, partials);
    hipError_t e = exclusive_scan<T>(ArrayIn<T>{partials, tiles}, tiles, partials, scratch + tiles, st);
    if (e != hipSuccess) return e;
    k_scan_tiles<T, In><<<(unsigned)tiles, kScanThreads, 0, st>>>(in, n, partials, out);
    return hipGetLastError();
}

}  // namespace tcl
