// LSD radix sort of 32- or 64-bit keys, 8-bit digits, one scatter kernel per digit pass.
//
// Before the passes, one kernel counts the digits of every pass in a single read of the
// keys and a second turns those counts into the first output position of each digit,
// per pass.  Each pass is then one kernel over tiles of kSortTile keys:
//   * a block takes the next tile number from a counter, so tiles are numbered in the
//     order their blocks started;
//   * it ranks the tile's keys per digit, stably: wave w owns a contiguous stretch of
//     the tile, its 64-key chunks go in index order, and within a chunk the rank among
//     equal digits is the number of lower lanes with that digit (ballot peer masks);
//   * it publishes the tile's count of each digit and finds the count of that digit in
//     all earlier tiles by walking back over their published values until it meets a
//     tile that has already published its running total (decoupled look-back).  A tile
//     only waits on tiles with lower numbers, whose blocks started before it, so every
//     wait ends; as a guard, a wait longer than a fixed number of polls raises the
//     error flag and gives up (the result is then wrong and the caller reports it);
//   * the tile is staged in LDS in digit order and written out in runs.
#include "digits.hpp"
#include "internal.hpp"
#include "scan.hpp"

namespace tcl {

constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kSortItems = 16;                        // keys per thread
constexpr int kSortTile = kSortThreads * kSortItems;  // 16384 keys per tile (128 KiB staged in LDS)
constexpr int kWaveSpan = kSortTile / kSortWaves;     // 1024 keys per wave
constexpr uint64_t kAggregate = 1ull << 62;  // status: the tile's own count is published
constexpr uint64_t kInclusive = 2ull << 62;  // status: the running total through the tile
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;

__global__ void k_sort_zero(uint64_t* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Digit counts of every pass: hist[p][d] for digit d of bits [lo_bit + 8p, lo_bit + 8p + 8).
constexpr int kCountItems = 4;  // keys per thread and round, loaded before any is counted

template <typename K>
__global__ __launch_bounds__(256) void k_radix_count_all(const K* __restrict__ keys, size_t n, int lo_bit,
                                                          int passes, uint32_t* __restrict__ hist) {
    __shared__ DigitCounts dc;
    dc.clear(passes);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i0 < n; i0 += stride * kCountItems) {
        K kk[kCountItems];
#pragma unroll
        for (int q = 0; q < kCountItems; ++q) {
            const size_t i = i0 + (size_t)q * stride;
            kk[q] = i < n ? keys[i] : K(0);
        }
#pragma unroll
        for (int q = 0; q < kCountItems; ++q) {
            if (i0 + (size_t)q * stride >= n) break;
            dc.add(kk[q], lo_bit, passes);
        }
    }
    dc.flush(hist, passes);
}

// First output position of each digit, per pass (one block of 256 threads).
__global__ __launch_bounds__(256) void k_radix_bases(const uint32_t* __restrict__ hist, int passes,
                                                      uint32_t* __restrict__ base) {
    __shared__ uint32_t lds[256 / kWave];
    for (int p = 0; p < passes; ++p) {
        uint32_t tot;
        base[p * 256 + threadIdx.x] = block_exclusive_scan(hist[p * 256 + threadIdx.x], lds, &tot);
    }
}

__device__ __forceinline__ uint64_t status_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_radix_pass(const K* __restrict__ in, K* __restrict__ out, size_t n,
                                                             int shift,
                                                             const uint32_t* __restrict__ base,
                                                             uint64_t* __restrict__ status,
                                                             unsigned int* __restrict__ ticket,
                                                             unsigned int* __restrict__ err) {
    __shared__ uint32_t wcnt[kSortWaves][256];  // per-wave digit counts, then per-wave bases
    __shared__ uint32_t tstart[256];            // first slot of each digit in the staged tile
    __shared__ uint32_t gstart[256];            // output position of the tile's first key of each digit
    __shared__ uint32_t scan_lds[256 / kWave];
    __shared__ unsigned int s_tile;
    __shared__ K stage[kSortTile];

    const int lane = lane_id(), w = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    const size_t tile = s_tile;

    const size_t tile0 = tile * kSortTile;
    const size_t wbeg = tile0 + (size_t)w * kWaveSpan;
    const unsigned long long lt = lanemask_lt();
    K k[kSortItems];
    uint32_t r[kSortItems];
    // every load is issued before any key is ranked (lanes past the end re-read the last key
    // and are left out of the peer masks)
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) k[c] = in[min(wbeg + (size_t)c * kWave + lane, n - 1)];
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
        const size_t idx = wbeg + (size_t)c * kWave + lane;
        const bool valid = idx < n;
        const K key = k[c];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        // peers: valid lanes whose digit equals this lane's, one bit of the digit at a time
        unsigned long long peers = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const unsigned long long bb = __builtin_amdgcn_ballot_w64((d >> b) & 1u);
            const unsigned long long mybit = (unsigned long long)(long long)(((int)(d << (31 - b))) >> 31);
            peers &= ~(bb ^ mybit);
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t before = wcnt[w][d];
        if (valid && below == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        r[c] = before + below;
    }
    __syncthreads();
    uint32_t cnt = 0, incl = 0;
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
#pragma unroll
        for (int q = 0; q < kSortWaves; ++q) {
            const uint32_t c = wcnt[q][d];
            wcnt[q][d] = cnt;
            cnt += c;
        }
        incl = wave_inclusive_scan(cnt);
        if (lane == kWave - 1) scan_lds[w] = incl;
    }
    __syncthreads();
    if (threadIdx.x < 256) {
        const int d = threadIdx.x;
        uint32_t off = 0;
        for (int i = 0; i < w; ++i) off += scan_lds[i];
        tstart[d] = off + incl - cnt;
        // publish this tile's count of digit d, then look back for the earlier tiles' total
        uint64_t* mine = status + tile * 256 + d;
        uint64_t excl = 0;
        if (tile == 0) {
            status_store(mine, kInclusive | cnt);
        } else {
            status_store(mine, kAggregate | cnt);
            size_t t = tile - 1;
            uint32_t spins = 0;
            for (;;) {
                const uint64_t s = status_load(status + t * 256 + d);
                if ((s >> 62) == 0) {
                    if (++spins > kSpinLimit) {
                        atomicOr(err, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += s & kValueMask;
                if (s & kInclusive) break;
                --t;  // tile 0 always publishes its running total, so t stays >= 0
            }
            status_store(mine, kInclusive | (excl + cnt));
        }
        gstart[d] = base[d] + (uint32_t)excl;
    }
    __syncthreads();
    // per wave and digit: the staged slot of the wave's first key of that digit; per digit: its
    // output position less its staged position (modulo 2^32), so that each key reads one word
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] += tstart[i & 255];
    __syncthreads();
    if (threadIdx.x < 256) gstart[threadIdx.x] -= tstart[threadIdx.x];
#pragma unroll
    for (int c = 0; c < kSortItems; ++c) {
        const size_t idx = wbeg + (size_t)c * kWave + lane;
        if (idx < n) {
            const uint32_t d = (uint32_t)(k[c] >> shift) & 255u;
            stage[wcnt[w][d] + r[c]] = k[c];
        }
    }
    __syncthreads();
    const size_t rem = n - tile0;
    const int tile_n = rem < (size_t)kSortTile ? (int)rem : kSortTile;
    for (int i = threadIdx.x; i < tile_n; i += kSortThreads) {
        const K key = stage[i];
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        out[(size_t)(uint32_t)(gstart[d] + (uint32_t)i)] = key;  // n < 2^32
    }
}

namespace {
constexpr size_t kHeadWords = 2 * kMaxPasses * 256 + 64;  // hist, bases, tickets (uint32)
size_t sort_tiles(size_t n) { return (n + kSortTile - 1) / kSortTile; }
}  // namespace

size_t radix_sort_scratch_bytes(size_t n) {
    const size_t tiles = std::max<size_t>(sort_tiles(n), 1);
    const size_t bytes = kHeadWords * sizeof(uint32_t) + tiles * 256 * sizeof(uint64_t);
    return (bytes + 255) & ~(size_t)255;
}

// Stable sort of n keys by bits [lo_bit, lo_bit + nbits) (digits of 8 bits: bits above
// the range up to the next multiple of 8 take part, so callers keep them zero).
// Ping-pongs between keys and alt; *result points at whichever holds the sorted keys.
// err (device) is raised if a look-back wait gave up.
template <typename K>
static hipError_t radix_sort(K* keys, K* alt, size_t n, int lo_bit, int nbits, void* scratch, unsigned int* err,
                             hipStream_t st, K** result, bool counted) {
    *result = keys;
    if (n <= 1 || nbits <= 0) return hipSuccess;
    if (n >= (1ull << 32)) return hipErrorInvalidValue;
    const int passes = (nbits + 7) / 8;
    if (passes > kMaxPasses || lo_bit + 8 * passes > (int)(8 * sizeof(K))) return hipErrorInvalidValue;
    const size_t tiles = sort_tiles(n);
    uint32_t* hist = (uint32_t*)scratch;
    uint32_t* bases = hist + kMaxPasses * 256;
    unsigned int* tickets = bases + kMaxPasses * 256;
    uint64_t* status = (uint64_t*)((uint8_t*)scratch + kHeadWords * sizeof(uint32_t));
    if (counted) {
        // the digit counts are already in place: clear bases and tickets only
        k_sort_zero<<<4, 256, 0, st>>>((uint64_t*)(hist + kMaxPasses * 256), (kHeadWords - kMaxPasses * 256) / 2);
    } else {
        k_sort_zero<<<4, 256, 0, st>>>((uint64_t*)scratch, kHeadWords / 2);
        k_radix_count_all<K><<<(unsigned)std::min<size_t>((n + 16383) / 16384, 1024), 256, 0, st>>>(keys, n, lo_bit,
                                                                                               passes, hist);
    }
    k_radix_bases<<<1, 256, 0, st>>>(hist, passes, bases);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    K* a = keys;
    K* b = alt;
    for (int p = 0; p < passes; ++p) {
        k_sort_zero<<<(unsigned)std::min<size_t>((tiles * 256 + 255) / 256, 4096), 256, 0, st>>>(status, tiles * 256);
        k_radix_pass<K><<<(unsigned)tiles, kSortThreads, 0, st>>>(a, b, n, lo_bit + 8 * p, bases + p * 256, status,
                                                                  tickets + p, err);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        K* t = a;
        a = b;
        b = t;
    }
    *result = a;
    return hipSuccess;
}

hipError_t radix_sort_u64(uint64_t* keys, uint64_t* alt, size_t n, int lo_bit, int nbits, void* scratch,
                          unsigned int* err, hipStream_t st, uint64_t** result, bool counted) {
    return radix_sort<uint64_t>(keys, alt, n, lo_bit, nbits, scratch, err, st, result, counted);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* alt, size_t n, int lo_bit, int nbits, void* scratch,
                          unsigned int* err, hipStream_t st, uint32_t** result, bool counted) {
    return radix_sort<uint32_t>(keys, alt, n, lo_bit, nbits, scratch, err, st, result, counted);
}

uint32_t* radix_counts(void* scratch) { return (uint32_t*)scratch; }

hipError_t radix_counts_clear(void* scratch, hipStream_t st) {
    k_sort_zero<<<4, 256, 0, st>>>((uint64_t*)scratch, kMaxPasses * 256 / 2);
    return hipGetLastError();
}

}  // namespace tcl
