// LSD radix sort of 64-bit keys, 8-bit digits, three kernels per digit pass:
//   1. per-tile digit histogram            (reads the keys once)
//   2. digit-major exclusive scan of the (digit, tile) counts
//   3. stable scatter: each wave ranks its keys with ballot-based peer masks,
//      the tile is staged in LDS in digit order and written out in runs.
// Stability within a tile comes from processing keys in index order: wave w
// owns a contiguous quarter of the tile, its 64-key chunks go in order, and
// within a chunk the rank among equal digits is the count of lower lanes.
#include "internal.hpp"
#include "scan.hpp"

namespace tcl {

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;                                   // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;             // 4096 keys per tile
constexpr int kWaveSpan = kSortTile / kSortWaves;                // 1024 keys per wave

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys, size_t n,
                                                             int shift, uint32_t* __restrict__ counts,
                                                             unsigned ntiles) {
    __shared__ uint32_t h[kSortWaves][256];
    const int w = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&h[0][0])[i] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int i = 0; i < kSortItems; ++i) {
        size_t idx = base + (size_t)i * kSortThreads + threadIdx.x;
        if (idx < n) atomicAdd(&h[w][(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int d = threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kSortWaves; ++k) s += h[k][d];
    counts[(size_t)d * ntiles + blockIdx.x] = s;
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ in,
                                                                uint64_t* __restrict__ out, size_t n,
                                                                int shift,
                                                                const uint32_t* __restrict__ offsets,
                                                                unsigned ntiles) {
    __shared__ uint32_t wcnt[kSortWaves][256];
    __shared__ uint32_t wbase[kSortWaves][256];
    __shared__ uint32_t gbase[256];
    __shared__ uint32_t tstart[256];
    __shared__ uint32_t scan_lds[kSortThreads / kWave];
    __shared__ uint64_t stage[kSortTile];

    const int lane = lane_id(), w = threadIdx.x / kWave;
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const size_t tile0 = (size_t)blockIdx.x * kSortTile;
    const size_t wbeg = tile0 + (size_t)w * kWaveSpan;
    const unsigned long long lt = lanemask_lt();
    uint64_t k[kSortItems];
    uint32_t r[kSortItems];
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
        const size_t idx = wbeg + (size_t)c * kWave + lane;
        const bool valid = idx < n;
        const uint64_t key = valid ? in[idx] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t before = wcnt[w][d];
        if (valid && below == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        k[c] = key;
        r[c] = before + below;
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) {
            wbase[q][d] = run;
            run += wcnt[q][d];
        }
        gbase[d] = offsets[(size_t)d * ntiles + blockIdx.x];
        uint32_t tot;
        tstart[d] = block_exclusive_scan(run, scan_lds, &tot);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
        const size_t idx = wbeg + (size_t)c * kWave + lane;
        if (idx < n) {
            const uint32_t d = (uint32_t)(k[c] >> shift) & 255u;
            stage[tstart[d] + wbase[w][d] + r[c]] = k[c];
        }
    }
    __syncthreads();
    const size_t rem = n - tile0;
    const int tile_n = rem < (size_t)kSortTile ? (int)rem : kSortTile;
    for (int i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const uint64_t key = stage[i];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        out[(size_t)gbase[d] + (uint32_t)i - tstart[d]] = key;
    }
}

size_t radix_sort_scratch_bytes(size_t n) {
    const size_t tiles = (n + kSortTile - 1) / kSortTile;
    const size_t cnt = 256 * (tiles ? tiles : 1);
    const size_t bytes = sizeof(uint32_t) * (cnt + scan_scratch_elems(cnt)) + 256;
    return (bytes + 255) & ~(size_t)255;
}

// Stable sort of n keys by bits [lo_bit, lo_bit + nbits).  Ping-pongs between keys and
// alt; *result points at whichever holds the sorted keys.
hipError_t radix_sort_u64(uint64_t* keys, uint64_t* alt, size_t n, int lo_bit, int nbits, void* scratch,
                          hipStream_t st, uint64_t** result) {
    *result = keys;
    if (n <= 1 || nbits <= 0) return hipSuccess;
    if (n >= (1ull << 32)) return hipErrorInvalidValue;
    const unsigned tiles = (unsigned)((n + kSortTile - 1) / kSortTile);
    const size_t cnt = 256 * (size_t)tiles;
    uint32_t* counts = (uint32_t*)scratch;
    uint32_t* sscratch = counts + cnt;
    uint64_t* a = keys;
    uint64_t* b = alt;
    for (int shift = lo_bit; shift < lo_bit + nbits; shift += 8) {
        k_radix_hist<<<tiles, kSortThreads, 0, st>>>(a, n, shift, counts, tiles);
        hipError_t e = exclusive_scan<uint32_t>(ArrayIn<uint32_t>{counts, cnt}, cnt, counts, sscratch, st);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<tiles, kSortThreads, 0, st>>>(a, b, n, shift, counts, tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* t = a;
        a = b;
        b = t;
    }
    *result = a;
    return hipSuccess;
}

}  // namespace tcl
