// Graph builder (CSR with sorted, deduplicated, loop-free lists; Sec. II-A/II-B) and
// the degree-binned schedule of the count kernels.  Every step is a stable radix
// sort, a scan, a gather or a run-boundary pass; no global atomics are used, so
// hub vertices cause no contention.
//
//   raw pairs -> canonical 64-bit keys (lo << b | hi, loops marked) -> sort -> unique
//   degrees   -> lo-side counts from runs of the sorted keys, hi-side counts from runs
//                after sorting the hi ends (stable sort on bits [32, 32 + b))
//   rank      -> sort (degree << b | id): rank r = position, order[r] = id
//   orient    -> keys (min(rank) << b | max(rank)) -> sort -> oriented CSR N+(r) in rank
//                space with ascending lists; |N+(r)| from runs, offsets by a scan
//   reverse   -> for each oriented edge i = (u -> v) whose tail N+(u) after v is nonempty
//                (and N+(v) nonempty): word (v << 32 | i), stable sort on the v bits
//                -> in-edge lists of v ordered by u; tail start i + 1, tail length
//                out_off[u + 1] - i - 1; per-vertex probe counts from a scan of lengths.
//
// Ranking by (degree, id) orients each edge towards the higher-degree end, so
// |N+(r)| <= sqrt(2m), and relabelling by rank keeps every list sorted by rank: the
// entries of N+(u) after v are exactly the candidates w > v that close a triangle
// (u, v, w), the rank-space form of the upper-triangle offset of Sec. II-C.
#include "digits.hpp"
#include "internal.hpp"
#include "scan.hpp"

namespace tcl {

constexpr int kB = 256;

#define GRID_STRIDE(i, n) \
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)(n); i += (size_t)gridDim.x * blockDim.x)

// Canonical keys (lo << bits | hi); a self-loop gets the all-ones key, dropped after the sort.
// (Their digits are counted by the sort itself: six LDS counts per key cost more here than
// the extra read there.)
__global__ void k_make_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, size_t m_in,
                            int64_t n, int bits, uint64_t* __restrict__ keys, int* __restrict__ bad) {
    const uint64_t loop = (1ull << (2 * bits)) - 1;
    GRID_STRIDE(i, m_in) {
        const int32_t a = src[i], b = dst[i];
        uint64_t key = loop;
        if (a < 0 || a >= n || b < 0 || b >= n) {
            *bad = 1;
        } else if (a != b) {
            const uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
            key = (lo << bits) | hi;
        }
        keys[i] = key;
    }
}

struct UniqueFlag {
    const uint64_t* k;
    size_t n;
    uint64_t loop;
    __device__ uint32_t operator()(size_t i) const {
        if (i >= n) return 0;
        const uint64_t x = k[i];
        return (x != loop && (i == 0 || k[i - 1] != x)) ? 1u : 0u;
    }
};

// Unique keys of one tile of kScanTile sorted keys, written at the tile's offset (the
// exclusive sum of the earlier tiles' unique counts), with the hi end of each (32 bits) for the
// hi-side degree sort.  Element i * 256 + t of the tile is thread t's i-th: one ballot per wave
// and round gives the ranks, one scan over the 16 x 4 (round, wave) counts the bases.
__global__ __launch_bounds__(kScanThreads) void k_unique_tiles(const uint64_t* __restrict__ k, size_t n, int bits,
                                                               const uint32_t* __restrict__ tile_off,
                                                               uint64_t* __restrict__ out,
                                                               uint32_t* __restrict__ hi_ends) {
    constexpr int NW = kScanThreads / kWave;
    static_assert(kScanItems * NW == kWave, "one lane per (round, wave) count");
    __shared__ uint32_t base[kScanItems][NW];
    const uint64_t loop = (1ull << (2 * bits)) - 1, mask = (1ull << bits) - 1;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const unsigned long long lt = lanemask_lt();
    const size_t tile = (size_t)blockIdx.x * kScanTile;
    uint64_t x[kScanItems];
    unsigned long long bal[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t e = tile + (size_t)i * kScanThreads + threadIdx.x;
        x[i] = e < n ? k[e] : loop;
        uint64_t prev = __shfl_up(x[i], 1, kWave);
        if (lane == 0) prev = (e > 0 && e < n) ? k[e - 1] : ~x[i];
        bal[i] = __builtin_amdgcn_ballot_w64(x[i] != loop && (e == 0 || prev != x[i]));
        if (lane == 0) base[i][w] = (uint32_t)__popcll(bal[i]);
    }
    __syncthreads();
    if (w == 0) {
        const uint32_t c = base[lane / NW][lane % NW];
        base[lane / NW][lane % NW] = wave_inclusive_scan(c) - c;
    }
    __syncthreads();
    const uint32_t t0 = tile_off[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if ((bal[i] >> lane) & 1ull) {
            const uint32_t p = t0 + base[i][w] + (uint32_t)__popcll(bal[i] & lt);
            out[p] = x[i];
            hi_ends[p] = (uint32_t)(x[i] & mask);
        }
    }
}

// Run boundaries of a sorted array grouped by g(i): first[g] = start, last[g] = one past the
// end.  Groups that do not occur keep the zeros the caller stored.  A wave takes kBoundItems
// rows of 64 consecutive entries at a time, all loads in flight at once; an entry's neighbours
// come from the lanes beside it, across rows from the edge lanes, and past the wave's span from
// one extra load on each side.
constexpr int kBoundItems = 4;

template <typename G>
__global__ void k_run_bounds(G g, size_t N, uint32_t* __restrict__ first, uint32_t* __restrict__ last) {
    const int lane = lane_id();
    const size_t span = (size_t)kBoundItems * kWave;
    const size_t wpb = blockDim.x / kWave;
    const size_t stride = (size_t)gridDim.x * wpb * span;
    for (size_t b = (blockIdx.x * wpb + threadIdx.x / kWave) * span; b < N; b += stride) {
        uint32_t gv[kBoundItems];
#pragma unroll
        for (int q = 0; q < kBoundItems; ++q) {
            const size_t i = b + (size_t)q * kWave + lane;
            gv[q] = g(i < N ? i : N - 1);
        }
        const uint32_t before = b > 0 ? g(b - 1) : 0u;
        const uint32_t after = b + span < N ? g(b + span) : 0u;
#pragma unroll
        for (int q = 0; q < kBoundItems; ++q) {
            const size_t i = b + (size_t)q * kWave + lane;
            const uint32_t left = q > 0 ? (uint32_t)__builtin_amdgcn_readlane(gv[q > 0 ? q - 1 : 0], kWave - 1) : before;
            const uint32_t right =
                q + 1 < kBoundItems ? (uint32_t)__builtin_amdgcn_readlane(gv[q + 1 < kBoundItems ? q + 1 : q], 0) : after;
            uint32_t prev = __shfl_up(gv[q], 1, kWave);
            uint32_t next = __shfl_down(gv[q], 1, kWave);
            if (lane == 0) prev = left;
            if (lane == kWave - 1) next = right;
            if (i < N) {
                if (i == 0 || prev != gv[q]) first[gv[q]] = (uint32_t)i;
                if (i + 1 == N || next != gv[q]) last[gv[q]] = (uint32_t)(i + 1);
            }
        }
    }
}

struct GroupShift {
    const uint64_t* k;
    int shift;
    __device__ uint32_t operator()(size_t i) const { return (uint32_t)(k[i] >> shift); }
};

// deg[v] = (lo-side run length) + (hi-side count)
__global__ void k_degrees(const uint32_t* __restrict__ f1, const uint32_t* __restrict__ l1,
                          const uint32_t* __restrict__ hi_count, int64_t n, int32_t* __restrict__ deg) {
    GRID_STRIDE(v, n) deg[v] = (int32_t)((l1[v] - f1[v]) + hi_count[v]);
}

// Hi-side counts from the hi ends sorted by their bits above kBucketBits: block b counts the
// ends in [b << kBucketBits, (b + 1) << kBucketBits) in LDS (many ends of one vertex only
// contend in LDS) and writes the counts of its range, which no other block touches.
constexpr int kBucketBits = 15;  // 32768 counters, 128 KiB of LDS
constexpr int kBucketThreads = 1024;

__device__ __forceinline__ size_t lower_bound_u32(const uint32_t* a, size_t n, uint64_t x) {
    size_t lo = 0, hi = n;
    while (lo < hi) {
        const size_t mid = (lo + hi) >> 1;
        if ((uint64_t)a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_counts(const uint32_t* __restrict__ ends, size_t m,
                                                                  int64_t n, uint32_t* __restrict__ count) {
    __shared__ uint32_t c[1u << kBucketBits];
    __shared__ size_t range[2];
    const uint64_t b0 = (uint64_t)blockIdx.x << kBucketBits;
    for (int i = threadIdx.x; i < (1 << kBucketBits); i += blockDim.x) c[i] = 0;
    if (threadIdx.x < 2) range[threadIdx.x] = lower_bound_u32(ends, m, b0 + ((uint64_t)threadIdx.x << kBucketBits));
    __syncthreads();
    const size_t e0 = range[0], e1 = range[1];
    for (size_t i = e0 + threadIdx.x; i < e1; i += blockDim.x)
        atomicAdd(&c[ends[i] & ((1u << kBucketBits) - 1)], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << kBucketBits); i += blockDim.x)
        if ((int64_t)(b0 + i) < n) count[b0 + i] = c[i];
}

__global__ void k_rank_keys(const int32_t* __restrict__ deg, int64_t n, int bits, uint64_t* __restrict__ rk) {
    GRID_STRIDE(v, n) rk[v] = ((uint64_t)(uint32_t)deg[v] << bits) | (uint64_t)v;
}

__global__ void k_rank_scatter(const uint64_t* __restrict__ rk, int64_t n, int bits, int32_t* __restrict__ order,
                               int32_t* __restrict__ rank, int32_t* __restrict__ deg_r) {
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(r, n) {
        const uint64_t x = rk[r];
        const int32_t v = (int32_t)(x & mask);
        order[r] = v;
        rank[v] = (int32_t)r;
        deg_r[r] = (int32_t)(x >> bits);
    }
}

// Oriented keys in rank space (lower rank << bits | higher rank), with the digits of the
// source rank counted for the sort by source that follows.
__global__ __launch_bounds__(kB) void k_relabel(const uint64_t* __restrict__ uk, size_t m, int bits,
                                                const int32_t* __restrict__ rank, uint64_t* __restrict__ ok,
                                                uint32_t* __restrict__ hist) {
    __shared__ DigitCounts dc;
    const int passes = digit_passes(bits);
    dc.clear(passes);
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(i, m) {
        const uint64_t x = uk[i];
        const uint32_t ra = (uint32_t)rank[x >> bits], rb = (uint32_t)rank[x & mask];
        const uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        const uint64_t key = ((uint64_t)lo << bits) | hi;
        ok[i] = key;
        dc.add(key, bits, passes);
    }
    dc.flush(hist, passes);
}

__global__ void k_run_counts(const uint32_t* __restrict__ f, const uint32_t* __restrict__ l, int64_t n,
                             int32_t* __restrict__ cnt) {
    GRID_STRIDE(v, n) cnt[v] = (int32_t)(l[v] - f[v]);
}

template <typename OffT>
struct I32In {
    const int32_t* p;
    int64_t n;
    __device__ OffT operator()(size_t i) const { return (int64_t)i < n ? (OffT)p[i] : OffT(0); }
};

// ---- rows of the oriented CSR: after the sort by source rank, each row's entries are in
// the order the relabel wrote them; these kernels sort every row by target rank in place.

constexpr int kRowSortMax = 4096;  // longest row sorted in registers (one wave, 64 entries per lane)

// x as held by lane l ^ J.  J = 1, 2 are quad permutes and J = 8 a rotation of each 16-lane row
// (DPP: plain VALU, no LDS); J = 4, 16 a swizzle within 32 lanes; J = 32 a permute by address.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x) {
    if constexpr (J == 1) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
    else if constexpr (J == 2) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
    else if constexpr (J == 8) return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);
    else if constexpr (J < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (J << 10) | 0x1F);
    else return (uint32_t)__shfl_xor((int)x, J, kWave);
}

// The same for a j known once the caller's loop is unrolled.
__device__ __forceinline__ uint32_t xor_lane(uint32_t x, int j) {
    switch (j) {
        case 1: return xor_lane<1>(x);
        case 2: return xor_lane<2>(x);
        case 4: return xor_lane<4>(x);
        case 8: return xor_lane<8>(x);
        case 16: return xor_lane<16>(x);
        default: return xor_lane<32>(x);
    }
}

// Ascending bitonic sort of one value per lane within each group of G lanes (G a power of two
// up to 64): the usual network, with every group's last merge ascending.
template <int G>
__device__ __forceinline__ uint32_t group_bitonic_sort(uint32_t x) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t y = xor_lane(x, j);
            // within an ascending run of k lanes the lower lane of a pair keeps the smaller value
            const bool up = (k == G) || ((lane & k) == 0);
            const bool keep_min = up == ((lane & j) == 0);
            x = keep_min ? min(x, y) : max(x, y);
        }
    }
    return x;
}

template <typename OffT>
__device__ __forceinline__ OffT shfl_off(OffT x, int src) {
    if constexpr (sizeof(OffT) == 8) {
        const uint64_t y = (uint64_t)x;
        const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)y, src, kWave);
        const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(y >> 32), src, kWave);
        return (OffT)(((uint64_t)hi << 32) | lo);
    } else {
        return (OffT)__shfl((int)x, src, kWave);
    }
}

// The rows of `todo` (bits = lanes of the 64-row group starting at r0; lane j holds row
// r0 + j's start and length), each of at most G entries: 64 / G rows at a time, one per group
// of G lanes.
template <int G, typename OffT>
__device__ __forceinline__ void sort_rows_by_group(uint64_t* __restrict__ keys, uint64_t todo, OffT beg, int32_t d,
                                                   int64_t r0, int bits) {
    constexpr int R = kWave / G;
    const int lane = lane_id(), grp = lane / G, e = lane % G;
    const uint64_t mask = (1ull << bits) - 1;
    while (todo) {
        int js[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            js[q] = todo ? (int)__builtin_ctzll(todo) : -1;
            todo &= todo - 1;  // no-op once empty
        }
        int jg = js[0];
#pragma unroll
        for (int q = 1; q < R; ++q) jg = grp == q ? js[q] : jg;
        const int jl = jg >= 0 ? jg : 0;
        const OffT s = shfl_off(beg, jl);
        const int32_t dj = __shfl(d, jl, kWave);
        const bool valid = jg >= 0 && e < dj;
        uint32_t x = valid ? (uint32_t)(keys[s + e] & mask) : 0xffffffffu;
        x = group_bitonic_sort<G>(x);
        if (valid) keys[s + e] = ((uint64_t)(r0 + jl) << bits) | x;
    }
}

// One wave per 64 consecutive rows; rows of 2..64 entries, sorted in registers: rows of up to
// 16 entries four at a time, up to 32 two at a time, longer ones by the whole wave.  Longer rows
// are left to k_row_sort_long.
template <typename OffT>
__global__ __launch_bounds__(256) void k_row_sort_short(uint64_t* __restrict__ keys, const OffT* __restrict__ out_off,
                                                        int64_t n, int bits) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r0 = wave * kWave; r0 < n; r0 += nwaves * kWave) {
        const int64_t r = r0 + lane;
        OffT beg = 0;
        int32_t d = 0;
        if (r < n) {
            beg = out_off[r];
            d = (int32_t)(out_off[r + 1] - beg);
        }
        sort_rows_by_group<16>(keys, __builtin_amdgcn_ballot_w64(d > 1 && d <= 16), beg, d, r0, bits);
        sort_rows_by_group<32>(keys, __builtin_amdgcn_ballot_w64(d > 16 && d <= 32), beg, d, r0, bits);
        sort_rows_by_group<64>(keys, __builtin_amdgcn_ballot_w64(d > 32 && d <= kWave), beg, d, r0, bits);
    }
}

// Ascending bitonic sort of 64·E values held E per lane, element e of lane l being entry
// 64·e + l.  Steps between entries 64 or more apart are compare-exchanges between a lane's own
// registers; shorter ones exchange with lane l ^ j.
template <int E, int JE>
__device__ __forceinline__ void reg_step(uint32_t (&v)[E], int k) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if ((e & JE) == 0) {
            const int f = e | JE;
            const bool up = ((e << 6) & k) == 0;  // entry 64·e + l: bit k is in e, as k >= 128
            const uint32_t lo = min(v[e], v[f]), hi = max(v[e], v[f]);
            v[e] = up ? lo : hi;
            v[f] = up ? hi : lo;
        }
    }
}

// Steps between lanes J apart (J < 64) of stage k.
template <int E, int J>
__device__ __forceinline__ void lane_step(uint32_t (&v)[E], int k) {
    const int lane = lane_id();
    const bool lower = (lane & J) == 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t y = xor_lane<J>(v[e]);
        const bool up = (((e << 6) | lane) & k) == 0;
        v[e] = (up == lower) ? min(v[e], y) : max(v[e], y);
    }
}

template <int E>
__device__ void reg_bitonic(uint32_t (&v)[E]) {
#pragma unroll 1
    for (int k = 2; k <= kWave * E; k <<= 1) {
#pragma unroll 1
        for (int j = k >> 1; j >= kWave; j >>= 1) {
            switch (j / kWave) {
                case 1: if constexpr (E > 1) reg_step<E, 1>(v, k); break;
                case 2: if constexpr (E > 2) reg_step<E, 2>(v, k); break;
                case 4: if constexpr (E > 4) reg_step<E, 4>(v, k); break;
                case 8: if constexpr (E > 8) reg_step<E, 8>(v, k); break;
                case 16: if constexpr (E > 16) reg_step<E, 16>(v, k); break;
                default: if constexpr (E > 32) reg_step<E, 32>(v, k); break;
            }
        }
        // then the steps between lanes, j = min(k / 2, 32) down to 1
        if (k >= 64) lane_step<E, 32>(v, k);
        if (k >= 32) lane_step<E, 16>(v, k);
        if (k >= 16) lane_step<E, 8>(v, k);
        if (k >= 8) lane_step<E, 4>(v, k);
        if (k >= 4) lane_step<E, 2>(v, k);
        lane_step<E, 1>(v, k);
    }
}

template <int E, typename OffT>
__device__ __forceinline__ void sort_long_row(uint64_t* __restrict__ keys, OffT s, int32_t d, uint64_t hi,
                                              uint64_t mask) {
    const int lane = lane_id();
    uint32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * kWave + lane;
        v[e] = i < d ? (uint32_t)(keys[s + i] & mask) : 0xffffffffu;
    }
    reg_bitonic<E>(v);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * kWave + lane;
        if (i < d) keys[s + i] = hi | v[e];
    }
}

// Rows listed in `rows` with LO < length <= HI (65 <= LO, HI <= kRowSortMax): one wave per row,
// sorted in registers over the row padded to a power of two.  Two launches split the lengths
// at 1024, so the register budget of the longest rows does not limit the many shorter ones.
template <typename OffT, int LO, int HI>
__global__ __launch_bounds__(256) void k_row_sort_long(uint64_t* __restrict__ keys, const OffT* __restrict__ out_off,
                                                       const int32_t* __restrict__ rows, int64_t count, int bits) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const uint64_t mask = (1ull << bits) - 1;
    for (int64_t it = wave; it < count; it += nwaves) {
        const int32_t r = rows[it];
        const OffT s = out_off[r];
        const int32_t d = (int32_t)(out_off[r + 1] - s);
        if (d <= LO || d > HI) continue;
        const uint64_t hi = (uint64_t)r << bits;
        if constexpr (HI <= 1024) {
            if (d <= 128) sort_long_row<2>(keys, s, d, hi, mask);
            else if (d <= 256) sort_long_row<4>(keys, s, d, hi, mask);
            else if (d <= 512) sort_long_row<8>(keys, s, d, hi, mask);
            else sort_long_row<16>(keys, s, d, hi, mask);
        } else {
            if (d <= 2048) sort_long_row<32>(keys, s, d, hi, mask);
            else sort_long_row<64>(keys, s, d, hi, mask);
        }
    }
}

// rows of more than lim entries (flag for the scan that lists them)
struct LongRow {
    const int32_t* dplus;
    int64_t n;
    int32_t lim;
    __device__ uint32_t operator()(size_t i) const { return ((int64_t)i < n && dplus[i] > lim) ? 1u : 0u; }
};

__global__ void k_list_rows(const int32_t* __restrict__ dplus, int64_t n, int32_t lim,
                            const uint32_t* __restrict__ pos, int32_t* __restrict__ rows) {
    GRID_STRIDE(r, n) if (dplus[r] > lim) rows[pos[r]] = (int32_t)r;
}

__global__ void k_max_i32(const int32_t* __restrict__ x, int64_t n, int* __restrict__ out) {
    int mx = 0;
    GRID_STRIDE(i, n) mx = max(mx, x[i]);
    for (int d = kWave / 2; d >= 1; d >>= 1) mx = max(mx, __shfl_xor(mx, d, kWave));
    if (lane_id() == 0) atomicMax(out, mx);
}

// One bit per vertex r: N+(r) is nonempty (bit r % 32 of word r / 32).  A megabyte at 2^23
// vertices, which the L2 holds while the edges look their targets up in it.
__global__ void k_nonempty_bits(const int32_t* __restrict__ dplus, int64_t n, uint32_t* __restrict__ bits) {
    GRID_STRIDE(r, n) {
        const unsigned long long b = __builtin_amdgcn_ballot_w64(dplus[r] > 0);
        const int lane = lane_id();
        // lanes hold consecutive r and a wave starts at a multiple of 64
        if (lane == 0) bits[r >> 5] = (uint32_t)b;
        else if (lane == 32) bits[r >> 5] = (uint32_t)(b >> 32);
    }
}

// What the reverse lists need of oriented edge i = (u -> v), besides its tail start i + 1:
// u and the tail length.
struct EdgePay {
    int32_t u;
    int32_t len;
};

// Layout of the word by which the in-edges are sorted: the key (v, or 2^bits for an edge that
// cannot close a triangle) at bit vshift and up, under it either u and the edge's position in
// N+(u) (packed: u << pbits | position; vshift = 64 minus the key's digit passes) or, where
// those do not fit, the edge index with the rest in an 8-byte payload array (vshift = 32).
struct InWord {
    int vshift;
    int pbits;
    bool packed;
    __host__ __device__ uint64_t low_mask() const { return (1ull << vshift) - 1; }
};

// Per oriented edge i = (u -> v) at position i of N+(u) (its tail is adj[i+1 .. out_off[u+1])):
// the adjacency entry and the in-edge word (with the payload where the word cannot hold it).
// An edge that cannot close a triangle (empty tail, or N+(v) empty) gets the key 2^bits,
// above every vertex, so it sorts after all in-edges that are kept.
template <typename OffT>
__global__ __launch_bounds__(kB) void k_edge_emit(const uint64_t* __restrict__ ok, size_t m, int bits, InWord iw,
                                                  const OffT* __restrict__ out_off, const uint32_t* __restrict__ nonempty,
                                                  int32_t* __restrict__ adj, uint64_t* __restrict__ words,
                                                  EdgePay* __restrict__ pay, uint32_t* __restrict__ hist) {
    __shared__ DigitCounts dc;
    const int passes = digit_passes(bits + 1);
    dc.clear(passes);
    const uint64_t mask = (1ull << bits) - 1;
    GRID_STRIDE(i, m) {
        const uint64_t x = ok[i];
        const int64_t u = (int64_t)(x >> bits), v = (int64_t)(x & mask);
        adj[i] = (int32_t)v;
        const int64_t len = (int64_t)out_off[u + 1] - (int64_t)i - 1;
        const bool kept = len > 0 && ((nonempty[v >> 5] >> (v & 31)) & 1u);
        const uint64_t key = kept ? (uint64_t)v : (1ull << bits);
        uint64_t w;
        if (iw.packed) {
            const uint64_t pos = (uint64_t)((int64_t)i - (int64_t)out_off[u]);
            w = (key << iw.vshift) | ((uint64_t)u << iw.pbits) | pos;
        } else {
            w = (key << iw.vshift) | (uint64_t)i;
            pay[i] = EdgePay{(int32_t)u, (int32_t)len};
        }
        words[i] = w;
        dc.add(w, iw.vshift, passes);
    }
    dc.flush(hist, passes);
}

// Number of leading words whose key is below 2^bits (the kept in-edges), by bisection.
__global__ void k_count_kept(const uint64_t* __restrict__ words, size_t m, int bits, int vshift,
                             uint32_t* __restrict__ out) {
    const uint64_t cut = (1ull << bits) << vshift;
    size_t lo = 0, hi = m;
    while (lo < hi) {
        const size_t mid = (lo + hi) >> 1;
        if (words[mid] < cut) lo = mid + 1;
        else hi = mid;
    }
    *out = (uint32_t)lo;
}

// In-edge k (sorted by v, then by edge position, so by u): u, its tail's start and length, from
// the packed word and the row bounds of u, or from the payload of the word's edge index.
// Also work[v] = sum of the tail lengths of v's in-edges (zeroed by the caller): lanes of a wave
// hold consecutive k, so each run of equal v within the wave is summed by a scan and added with
// one atomic by its last lane.
template <typename OffT>
__global__ void k_in_fill(const uint64_t* __restrict__ words, size_t kept, InWord iw, const OffT* __restrict__ out_off,
                          const EdgePay* __restrict__ pay, int32_t* __restrict__ in_u, OffT* __restrict__ in_start,
                          int32_t* __restrict__ in_len, unsigned long long* __restrict__ work) {
    const int lane = lane_id();
    GRID_STRIDE(k, kept) {
        const uint64_t wd = words[k];
        const uint32_t v = (uint32_t)(wd >> iw.vshift);
        const uint64_t low = wd & iw.low_mask();
        int32_t u, len;
        OffT start;
        if (iw.packed) {
            u = (int32_t)(low >> iw.pbits);
            const OffT pos = (OffT)(low & ((1ull << iw.pbits) - 1));
            const OffT o0 = out_off[u], o1 = out_off[u + 1];
            start = o0 + pos + 1;
            len = (int32_t)(o1 - start);
        } else {
            const EdgePay e = pay[low];
            u = e.u;
            start = (OffT)low + 1;
            len = e.len;
        }
        in_u[k] = u;
        in_start[k] = start;
        in_len[k] = len;
        // lanes past the end are inactive; lane l's run starts at the last head at or below l
        const uint32_t vp = (uint32_t)__shfl_up((int)v, 1, kWave);
        const uint32_t vn = (uint32_t)__shfl_down((int)v, 1, kWave);
        const bool head = lane == 0 || vp != v;
        const bool tail = lane == kWave - 1 || k + 1 == kept || vn != v;
        const unsigned long long incl = wave_inclusive_scan((unsigned long long)(uint32_t)len);
        const unsigned long long heads = __builtin_amdgcn_ballot_w64(head);
        const int start_lane = 63 - __builtin_clzll(heads & (~0ull >> (kWave - 1 - lane)));
        const unsigned long long before = __shfl(incl, start_lane > 0 ? start_lane - 1 : 0, kWave);
        if (tail) atomicAdd(&work[v], incl - (start_lane > 0 ? before : 0ull));
    }
}

// stats[0] = max |N+|, stats[1] = max degree, stats[2] = sum of work (wedges),
// stats[3] = sum of |N+(v)| over vertices with work (entries staged in LDS),
// stats[4] = sum over oriented edges (u -> v) of |N+(v)| = sum_v (d(v) - |N+(v)|) |N+(v)|
__global__ void k_stats(const int32_t* __restrict__ dplus, const int32_t* __restrict__ deg_r,
                        const unsigned long long* __restrict__ work, int64_t n, unsigned long long* stats) {
    __shared__ unsigned long long s[5][kB / kWave];
    unsigned long long a = 0, b = 0, c = 0, e = 0, f = 0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long wr = work[r];
        const unsigned long long dp = (unsigned long long)dplus[r];
        a = max(a, dp);
        b = max(b, (unsigned long long)deg_r[r]);
        c += wr;
        if (wr) e += dp;
        f += ((unsigned long long)deg_r[r] - dp) * dp;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        a = max(a, (unsigned long long)__shfl_xor(a, d, kWave));
        b = max(b, (unsigned long long)__shfl_xor(b, d, kWave));
        c += __shfl_xor(c, d, kWave);
        e += __shfl_xor(e, d, kWave);
        f += __shfl_xor(f, d, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s[0][w] = a;
        s[1][w] = b;
        s[2][w] = c;
        s[3][w] = e;
        s[4][w] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0;
        b = 0;
        c = 0;
        e = 0;
        f = 0;
        for (int i = 0; i < kB / kWave; ++i) {
            a = max(a, s[0][i]);
            b = max(b, s[1][i]);
            c += s[2][i];
            e += s[3][i];
            f += s[4][i];
        }
        atomicMax(&stats[0], a);
        atomicMax(&stats[1], b);
        atomicAdd(&stats[2], c);
        atomicAdd(&stats[3], e);
        atomicAdd(&stats[4], f);
    }
}

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
    GRID_STRIDE(i, n) p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, size_t n, T v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_fill<T><<<grid_for(n, kB, 4096), kB, 0, st>>>(p, n, v);
    return hipGetLastError();
}

// ------------------------------------------------------------------ direction bits (Eq. 1)

// Directed keys (src << bits | dst); a self-loop gets the all-ones key, dropped by the unique.
__global__ void k_make_dkeys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, size_t m_in, int bits,
                             uint64_t* __restrict__ keys) {
    const uint64_t loop = (1ull << (2 * bits)) - 1;
    GRID_STRIDE(i, m_in) {
        const int32_t a = src[i], b = dst[i];
        keys[i] = a == b ? loop : (((uint64_t)a << bits) | (uint64_t)b);
    }
}

// out-degree of rank r: the length of its id's run of directed keys
__global__ void k_dout(const int32_t* __restrict__ order, const uint32_t* __restrict__ f,
                       const uint32_t* __restrict__ l, int64_t n, int32_t* __restrict__ dout_r) {
    GRID_STRIDE(r, n) {
        const int32_t v = order[r];
        dout_r[r] = (int32_t)(l[v] - f[v]);
    }
}

__device__ __forceinline__ bool run_has(const uint64_t* __restrict__ k, uint32_t a, uint32_t b, uint64_t key) {
    const uint32_t end = b;
    while (a < b) {
        const uint32_t mid = a + ((b - a) >> 1);
        if (k[mid] < key) a = mid + 1;
        else b = mid;
    }
    return a < end && k[a] == key;
}

// Direction bits of oriented edge e = (u -> adj[e]) (u: the row holding e, by a search of
// out_off): the ids' runs of the sorted, unique directed keys are searched for both directions.
template <typename OffT>
__global__ void k_dir(const OffT* __restrict__ out_off, int64_t n, const int32_t* __restrict__ adj, size_t m,
                      const int32_t* __restrict__ order, const uint64_t* __restrict__ dk,
                      const uint32_t* __restrict__ f, const uint32_t* __restrict__ l, int bits,
                      uint8_t* __restrict__ dir) {
    GRID_STRIDE(e, m) {
        int64_t lo = 0, hi = n;  // last row r with out_off[r] <= e
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((size_t)out_off[mid] <= e) lo = mid;
            else hi = mid;
        }
        const uint64_t x = (uint64_t)order[lo], y = (uint64_t)order[adj[e]];
        const bool fw = run_has(dk, f[x], l[x], (x << bits) | y);
        const bool bw = run_has(dk, f[y], l[y], (y << bits) | x);
        dir[e] = (uint8_t)((fw ? 1u : 0u) | (bw ? 2u : 0u));
    }
}

// ------------------------------------------------------------------ host orchestration

namespace {

struct Temps {
    Pool* pool;
    std::vector<void*> held;
    ~Temps() {
        for (void* p : held) pool->release(p);
    }
    template <typename T>
    tc_lcc_status get(size_t count, T** out) {
        void* p = nullptr;
        tc_lcc_status s = pool->alloc(count * sizeof(T) + 16, &p);
        if (s != TC_LCC_OK) return s;
        held.push_back(p);
        *out = (T*)p;
        return TC_LCC_OK;
    }
};

template <typename T>
tc_lcc_status keep(tc_lcc_graph g, size_t count, T** out) {
    void* p = nullptr;
    const size_t bytes = count * sizeof(T) + 16;
    tc_lcc_status s = g->ctx->pool->alloc(bytes, &p);
    if (s != TC_LCC_OK) return s;
    g->blocks.push_back(p);
    g->d.device_bytes += Pool::round(bytes);
    *out = (T*)p;
    return TC_LCC_OK;
}

#define TCL_TRY(x)                           \
    do {                                     \
        tc_lcc_status _s = (x);              \
        if (_s != TC_LCC_OK) return _s;      \
    } while (0)

template <typename G>
hipError_t run_bounds(G g, size_t N, uint32_t* first, uint32_t* last, int64_t n, hipStream_t st) {
    hipError_t e = fill<uint32_t>(first, (size_t)n, 0u, st);
    if (e == hipSuccess) e = fill<uint32_t>(last, (size_t)n, 0u, st);
    if (e != hipSuccess || N == 0) return e;
    k_run_bounds<G><<<grid_for((N + kBoundItems - 1) / kBoundItems, kB, 16384), kB, 0, st>>>(g, N, first, last);
    return hipGetLastError();
}

template <typename OffT>
tc_lcc_status build_typed(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                          int on_device, int row_max, bool directed, hipStream_t st, tc_lcc_graph g) {
    GraphDev& d = g->d;
    Temps tmp{ctx->pool.get(), {}};
    const int bits = std::max(1, ceil_log2((uint64_t)n));
    d.n = n;
    d.bits = bits;
    const size_t M = (size_t)m_in;
    const size_t N = (size_t)n;

    const int32_t* s_dev = src;
    const int32_t* d_dev = dst;
    if (!on_device && M > 0) {
        int32_t *a, *b;
        TCL_TRY(tmp.get(M, &a));
        TCL_TRY(tmp.get(M, &b));
        TCL_HIP(hipMemcpyAsync(a, src, M * sizeof(int32_t), hipMemcpyHostToDevice, st));
        TCL_HIP(hipMemcpyAsync(b, dst, M * sizeof(int32_t), hipMemcpyHostToDevice, st));
        s_dev = a;
        d_dev = b;
    }

    // three K-word buffers rotate through the sorts; K >= every array they hold (+2 spare words)
    const size_t K = std::max<size_t>({M, N, 1});
    uint64_t *ka, *kb, *kc;
    uint32_t* pos;
    void* sort_scratch;
    TCL_TRY(tmp.get(K + 1, &ka));
    TCL_TRY(tmp.get(K + 1, &kb));
    TCL_TRY(tmp.get(K + 1, &kc));
    TCL_TRY(tmp.get(M + 1, &pos));
    const size_t rs_bytes = radix_sort_scratch_bytes(K);
    TCL_TRY(tmp.get(rs_bytes + sizeof(uint64_t) * scan_scratch_elems(K + 1) + 1024, (uint8_t**)&sort_scratch));
    uint32_t* scan32 = (uint32_t*)((uint8_t*)sort_scratch + rs_bytes);
    OffT* scanO = (OffT*)scan32;
    int* bad;  // [0]: an endpoint outside [0, n); [1]: a sort's look-back wait gave up
    TCL_TRY(tmp.get(16, &bad));
    TCL_HIP(fill<int>(bad, 16, 0, st));
    unsigned int* sort_err = (unsigned int*)(bad + 1);
    uint32_t *f1, *l1, *f2, *l2;
    TCL_TRY(tmp.get(N, &f1));
    TCL_TRY(tmp.get(N, &l1));
    TCL_TRY(tmp.get(N, &f2));
    TCL_TRY(tmp.get(N, &l2));
    int32_t* deg;
    TCL_TRY(tmp.get(N, &deg));

    mark(d, 0, st);
    // 1. canonical keys, sort, unique
    uint64_t* sorted = ka;
    uint64_t* ukeys = kb;
    uint32_t m32 = 0;
    if (M > 0) {
        k_make_keys<<<grid_for(M, kB, 8192), kB, 0, st>>>(s_dev, d_dev, M, n, bits, ka, bad);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(ka, kb, M, 0, 2 * bits, sort_scratch, sort_err, st, &sorted));
        ukeys = (sorted == ka) ? kb : ka;
        // unique counts per tile, their exclusive sums (tiles + 1 entries: the last is m), then
        // the unique keys written straight to their positions
        const size_t tiles = (M + kScanTile - 1) / kScanTile;
        uint32_t* toff = pos;
        k_reduce_tiles<uint32_t, UniqueFlag><<<(unsigned)tiles, kScanThreads, 0, st>>>(
            UniqueFlag{sorted, M, (1ull << (2 * bits)) - 1}, M, toff);
        TCL_HIP(hipGetLastError());
        TCL_HIP(exclusive_scan<uint32_t>(ArrayIn<uint32_t>{toff, tiles}, tiles + 1, toff, scan32, st));
        k_unique_tiles<<<(unsigned)tiles, kScanThreads, 0, st>>>(sorted, M, bits, toff, ukeys, (uint32_t*)kc);
        TCL_HIP(hipGetLastError());
        int hb = 0;
        TCL_HIP(hipMemcpyAsync(&m32, toff + tiles, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (hb) {
            set_error("tc_lcc_build_csr: an endpoint lies outside [0, %lld)", (long long)n);
            return TC_LCC_INVALID_ARGUMENT;
        }
    }
    const size_t m = m32;
    d.m = (int64_t)m;
    if (sizeof(OffT) == 4 && m >= (1ull << 31)) {
        set_error("tc_lcc_build_csr: %zu edges do not fit 4-byte offsets", m);
        return TC_LCC_INVALID_ARGUMENT;
    }
    uint64_t* spare = (ukeys == ka) ? kb : ka;  // held the raw sorted keys, free from here on
    // degrees: lo ends are runs of the (lo, hi)-sorted unique keys; hi ends are counted per
    // 2^15-vertex range in LDS after a sort of the 32-bit hi ends by their bits above that
    // (one pass at 2^23 vertices)
    TCL_HIP(run_bounds(GroupShift{ukeys, bits}, m, f1, l1, n, st));
    uint32_t* hi_count = f2;
    {
        uint32_t* hs = (uint32_t*)kc;
        if (m > 0 && bits > kBucketBits)
            TCL_HIP(radix_sort_u32((uint32_t*)kc, (uint32_t*)spare, m, kBucketBits, bits - kBucketBits, sort_scratch,
                                   sort_err, st, &hs));
        const size_t buckets = ((size_t)n + (1u << kBucketBits) - 1) >> kBucketBits;
        k_bucket_counts<<<(unsigned)buckets, kBucketThreads, 0, st>>>(hs, m, n, hi_count);
        TCL_HIP(hipGetLastError());
    }
    k_degrees<<<grid_for(N, kB, 8192), kB, 0, st>>>(f1, l1, hi_count, n, deg);
    TCL_HIP(hipGetLastError());

    mark(d, 1, st);
    // 2. rank by (degree, id)
    int32_t* rank;
    TCL_TRY(tmp.get(N, &rank));
    TCL_TRY(keep(g, N, &d.order));
    TCL_TRY(keep(g, N, &d.deg_r));
    {
        uint64_t* rs = spare;
        k_rank_keys<<<grid_for(N, kB, 8192), kB, 0, st>>>(deg, n, bits, spare);
        TCL_HIP(hipGetLastError());
        // the keys are written in vertex order, so a stable sort on the degree bits alone
        // (degrees are below n <= 2^bits) orders them by (degree, id)
        TCL_HIP(radix_sort_u64(spare, kc, N, bits, bits, sort_scratch, sort_err, st, &rs));
        k_rank_scatter<<<grid_for(N, kB, 8192), kB, 0, st>>>(rs, n, bits, d.order, rank, d.deg_r);
        TCL_HIP(hipGetLastError());
    }

    mark(d, 2, st);
    // 3. relabel + orient, sort by source rank, oriented CSR; then each row by target rank
    uint64_t* okeys = spare;
    uint64_t* osorted = okeys;
    TCL_TRY(keep(g, N, &d.dplus));
    OffT* out_off;
    TCL_TRY(keep(g, N + 1, &out_off));
    d.out_off = out_off;
    TCL_TRY(keep(g, std::max<size_t>(m, 1), &d.adj));
    if (m > 0) {
        TCL_HIP(radix_counts_clear(sort_scratch, st));
        k_relabel<<<grid_for(m, kB, 1024), kB, 0, st>>>(ukeys, m, bits, rank, okeys, radix_counts(sort_scratch));
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(okeys, kc, m, bits, bits, sort_scratch, sort_err, st, &osorted, true));
    }
    TCL_HIP(run_bounds(GroupShift{osorted, bits}, m, f1, l1, n, st));
    k_run_counts<<<grid_for(N, kB, 8192), kB, 0, st>>>(f1, l1, n, d.dplus);
    TCL_HIP(hipGetLastError());
    TCL_HIP(exclusive_scan<OffT>(I32In<OffT>{d.dplus, n}, N + 1, out_off, scanO, st));
    int dmax = 0;  // longest row of N+
    if (m > 0) {
        int* mx = bad + 4;
        k_max_i32<<<grid_for(N, kB, 1024), kB, 0, st>>>(d.dplus, n, mx);
        TCL_HIP(hipGetLastError());
        // the rows longer than a wave and those longer than 1024, listed (scans of their flags)
        constexpr int32_t kMid = 1024;
        uint32_t *rpos, *rpos2;
        TCL_TRY(tmp.get(N + 1, &rpos));
        TCL_TRY(tmp.get(N + 1, &rpos2));
        TCL_HIP(exclusive_scan<uint32_t>(LongRow{d.dplus, n, kWave}, N + 1, rpos, scan32, st));
        TCL_HIP(exclusive_scan<uint32_t>(LongRow{d.dplus, n, kMid}, N + 1, rpos2, scan32, st));
        uint32_t nlong = 0, nlong2 = 0;
        TCL_HIP(hipMemcpyAsync(&dmax, mx, sizeof(int), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipMemcpyAsync(&nlong, rpos + N, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipMemcpyAsync(&nlong2, rpos2 + N, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (dmax <= row_max) {
            const size_t groups = (N + kWave - 1) / kWave;
            k_row_sort_short<OffT><<<grid_for(groups * kWave, kB, 8192), kB, 0, st>>>(osorted, out_off, n, bits);
            TCL_HIP(hipGetLastError());
            if (nlong > 0) {
                int32_t* rows;
                TCL_TRY(tmp.get(nlong, &rows));
                k_list_rows<<<grid_for(N, kB, 8192), kB, 0, st>>>(d.dplus, n, kWave, rpos, rows);
                TCL_HIP(hipGetLastError());
                k_row_sort_long<OffT, kWave, kMid><<<grid_for((size_t)nlong * kWave, kB, 8192), kB, 0, st>>>(
                    osorted, out_off, rows, (int64_t)nlong, bits);
                TCL_HIP(hipGetLastError());
            }
            if (nlong2 > 0) {
                int32_t* rows2;
                TCL_TRY(tmp.get(nlong2, &rows2));
                k_list_rows<<<grid_for(N, kB, 8192), kB, 0, st>>>(d.dplus, n, kMid, rpos2, rows2);
                TCL_HIP(hipGetLastError());
                k_row_sort_long<OffT, kMid, kRowSortMax><<<grid_for((size_t)nlong2 * kWave, kB, 4096), kB, 0, st>>>(
                    osorted, out_off, rows2, (int64_t)nlong2, bits);
                TCL_HIP(hipGetLastError());
            }
        } else {
            // a row too long for the LDS sort: sort the keys by (source, target) in full instead
            // (an LSD sort over all digits, whatever order the keys are in)
            uint64_t* full = osorted;
            TCL_HIP(radix_sort_u64(osorted, osorted == kc ? okeys : kc, m, 0, 2 * bits, sort_scratch, sort_err, st,
                                   &full));
            osorted = full;
        }
    }

    mark(d, 3, st);
    // 4. reverse lists (in-edges with a nonempty tail), sorted by v then by position (so by u)
    uint64_t* wa = nullptr;
    uint64_t* wb = nullptr;
    for (uint64_t* b : {ka, kb, kc})
        if (b != osorted) (wa ? wb : wa) = b;
    uint32_t kept = 0;
    EdgePay* pay = nullptr;
    uint64_t* ws = wa;
    // the in-edge word: u and the row position packed under the key when they fit
    InWord iw;
    iw.pbits = dmax > 1 ? ceil_log2((uint64_t)dmax) : 0;
    iw.vshift = 64 - 8 * digit_passes(bits + 1);
    iw.packed = bits + iw.pbits <= iw.vshift;
    if (!iw.packed) {
        iw.vshift = 32;
        TCL_TRY(tmp.get(std::max<size_t>(m, 1), &pay));
    }
    if (m > 0) {
        // the kept test looks targets up in a bitmap of nonempty lists that the L2 holds
        uint32_t* nonempty;
        TCL_TRY(tmp.get((N + 63) / 32, &nonempty));
        k_nonempty_bits<<<grid_for(N, kB, 4096), kB, 0, st>>>(d.dplus, n, nonempty);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_counts_clear(sort_scratch, st));
        k_edge_emit<OffT><<<grid_for(m, kB, 1024), kB, 0, st>>>(osorted, m, bits, iw, out_off, nonempty, d.adj, wa,
                                                                pay, radix_counts(sort_scratch));
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(wa, wb, m, iw.vshift, bits + 1, sort_scratch, sort_err, st, &ws, true));
        uint32_t* kc_dev = (uint32_t*)(bad + 5);
        k_count_kept<<<1, 1, 0, st>>>(ws, m, bits, iw.vshift, kc_dev);
        TCL_HIP(hipGetLastError());
        TCL_HIP(hipMemcpyAsync(&kept, kc_dev, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
    }
    d.m_in_kept = (int64_t)kept;
    const size_t KE = std::max<size_t>((size_t)kept, 1);
    TCL_TRY(keep(g, KE, &d.in_u));
    OffT* in_start;
    TCL_TRY(keep(g, KE, &in_start));
    d.in_start = in_start;
    TCL_TRY(keep(g, KE, &d.in_len));
    OffT* in_off;
    TCL_TRY(keep(g, N + 1, &in_off));
    d.in_off = in_off;
    TCL_TRY(keep(g, N, &d.work));
    TCL_HIP(run_bounds(GroupShift{ws, iw.vshift}, kept, f2, l2, n, st));
    int32_t* din = deg;  // degrees by vertex are not needed any more (deg_r keeps them by rank)
    k_run_counts<<<grid_for(N, kB, 8192), kB, 0, st>>>(f2, l2, n, din);
    TCL_HIP(hipGetLastError());
    TCL_HIP(exclusive_scan<OffT>(I32In<OffT>{din, n}, N + 1, in_off, scanO, st));
    TCL_HIP(fill<uint64_t>(d.work, N, 0ull, st));
    if (kept > 0) {
        k_in_fill<OffT><<<grid_for(kept, kB, 8192), kB, 0, st>>>(ws, kept, iw, out_off, pay, d.in_u, in_start,
                                                                 d.in_len, (unsigned long long*)d.work);
        TCL_HIP(hipGetLastError());
    }

    mark(d, 4, st);
    // 5. run scratch and statistics
    TCL_TRY(keep(g, N, &d.t_rank));
    TCL_TRY(keep(g, 64, &d.counters));
    TCL_TRY(keep(g, N, &d.vlist));
    unsigned long long* stats;
    TCL_TRY(tmp.get(8, &stats));
    TCL_HIP(fill<unsigned long long>(stats, 8, 0ull, st));
    k_stats<<<grid_for(N, kB, 2048), kB, 0, st>>>(d.dplus, d.deg_r, (const unsigned long long*)d.work, n, stats);
    TCL_HIP(hipGetLastError());
    unsigned long long hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int serr = 0;
    TCL_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipMemcpyAsync(&serr, bad + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    if (serr) {
        set_error("tc_lcc_build_csr: a radix sort pass gave up waiting for an earlier tile");
        return TC_LCC_DEVICE_ERROR;
    }
    d.max_dplus = (int32_t)hs[0];
    d.max_deg = (int64_t)hs[1];
    d.wedges = hs[2];
    d.staged = hs[3];
    d.push_words = hs[4];

    // 6. a directed input (Eq. 1): the skeleton above is its undirected graph; each oriented
    // edge gets the directions the input held, and each vertex its out-degree
    if (directed) {
        TCL_TRY(keep(g, N, &d.dout_r));
        TCL_TRY(keep(g, std::max<size_t>(m, 1), &d.dir));
        if (M > 0) {
            k_make_dkeys<<<grid_for(M, kB, 8192), kB, 0, st>>>(s_dev, d_dev, M, bits, ka);
            TCL_HIP(hipGetLastError());
            uint64_t* dsorted = ka;
            TCL_HIP(radix_sort_u64(ka, kb, M, 0, 2 * bits, sort_scratch, sort_err, st, &dsorted));
            uint64_t* du = (dsorted == ka) ? kb : ka;
            const size_t tiles = (M + kScanTile - 1) / kScanTile;
            uint32_t* toff = pos;
            k_reduce_tiles<uint32_t, UniqueFlag><<<(unsigned)tiles, kScanThreads, 0, st>>>(
                UniqueFlag{dsorted, M, (1ull << (2 * bits)) - 1}, M, toff);
            TCL_HIP(hipGetLastError());
            TCL_HIP(exclusive_scan<uint32_t>(ArrayIn<uint32_t>{toff, tiles}, tiles + 1, toff, scan32, st));
            k_unique_tiles<<<(unsigned)tiles, kScanThreads, 0, st>>>(dsorted, M, bits, toff, du, (uint32_t*)kc);
            TCL_HIP(hipGetLastError());
            uint32_t md = 0;
            TCL_HIP(hipMemcpyAsync(&md, toff + tiles, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            TCL_HIP(hipStreamSynchronize(st));
            TCL_HIP(run_bounds(GroupShift{du, bits}, md, f1, l1, n, st));
            k_dout<<<grid_for(N, kB, 8192), kB, 0, st>>>(d.order, f1, l1, n, d.dout_r);
            TCL_HIP(hipGetLastError());
            if (m > 0) {
                k_dir<OffT><<<grid_for(m, kB, 16384), kB, 0, st>>>(out_off, n, d.adj, m, d.order, du, f1, l1, bits,
                                                                  d.dir);
                TCL_HIP(hipGetLastError());
            }
        } else {
            TCL_HIP(fill<int32_t>(d.dout_r, N, 0, st));
        }
        TCL_HIP(hipMemcpyAsync(&serr, bad + 1, sizeof(int), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (serr) {
            set_error("tc_lcc_build_directed: a radix sort pass gave up waiting for an earlier tile");
            return TC_LCC_DEVICE_ERROR;
        }
        d.directed = true;
    }
    return TC_LCC_OK;
}

}  // namespace

tc_lcc_status build_graph(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                          int on_device, int offset_bytes, const tc_lcc_tuning& tn, hipStream_t st, tc_lcc_graph g,
                          bool directed) {
    // offsets index the m oriented edges; m <= m_in, so 4 bytes suffice when m_in < 2^31
    int ob = offset_bytes;
    if (ob == 0) ob = (m_in < (1ll << 31)) ? 4 : 8;
    g->d.off_bytes = ob;
    const int row_max = tn.row_sort_max > 0 ? std::min(tn.row_sort_max, kRowSortMax) : kRowSortMax;
    tc_lcc_status s = (ob == 4) ? build_typed<int32_t>(ctx, n, m_in, src, dst, on_device, row_max, directed, st, g)
                                : build_typed<int64_t>(ctx, n, m_in, src, dst, on_device, row_max, directed, st, g);
    if (s != TC_LCC_OK) return s;
    s = build_schedule(g, tn, st);
    mark(g->d, 5, st);
    return s;
}

// ------------------------------------------------------------------ schedule (degree/work bins)

constexpr int kClassWave = 48, kClassList = 49, kClassGlobal = 50, kClassNone = 63;

// bitmap_ok: the vertex's rank bitmap fits a block's table (region_bytes), so the block kernel
// probes it there whatever the list's length (only lists beyond the block's hash need to know).
template <typename OffT>
__global__ void k_classify(const unsigned long long* __restrict__ work, const int32_t* __restrict__ dplus,
                           const OffT* __restrict__ out_off, const int32_t* __restrict__ adj, int64_t n, int bits,
                           int64_t wave_work_max, int32_t wave_cap, int32_t block_cap, int32_t list_cap,
                           uint32_t region_bytes, int group, uint64_t* __restrict__ keys,
                           unsigned long long* __restrict__ counts) {
    __shared__ unsigned int c[64];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) c[i] = 0;
    __syncthreads();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long w = work[v];
        const int32_t dp = dplus[v];
        bool bitmap_ok = false;
        if (region_bytes > 0 && dp > block_cap) {
            const uint32_t span = (uint32_t)(adj[out_off[v + 1] - 1] - (int32_t)v);
            bitmap_ok = bitmap_bytes((span + 31u) >> 5, dp) <= region_bytes;
        }
        int cls;
        if (w == 0) {
            cls = kClassNone;
        } else if (dp > list_cap && !bitmap_ok) {
            cls = kClassGlobal;
        } else if (dp > block_cap && !bitmap_ok) {
            cls = kClassList;
        } else if (dp <= wave_cap && (group == 1 || (group == 0 && (int64_t)w <= wave_work_max))) {
            cls = kClassWave;
        } else {
            // block bin, heaviest first: class 0 holds work >= 2^40
            const int bl = 64 - __clzll(w);
            cls = bl >= 40 ? 0 : 40 - bl;
        }
        keys[v] = ((uint64_t)cls << bits) | (uint64_t)v;
        atomicAdd(&c[cls], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 64; i += blockDim.x)
        if (c[i]) atomicAdd(&counts[i], (unsigned long long)c[i]);
}

__global__ void k_vlist(const uint64_t* __restrict__ keys, int64_t cnt, int bits, int32_t* __restrict__ vlist) {
    const uint64_t mask = (1ull << bits) - 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += (int64_t)gridDim.x * blockDim.x)
        vlist[i] = (int32_t)(keys[i] & mask);
}

// LDS slots of one block's table: the sorted list itself (binary search or hybrid), or a hash
// table for the longest list.
int32_t table_slots(int probe, int32_t dplus_max) {
    const bool sorted = probe == TC_LCC_PROBE_SORTED || probe == TC_LCC_PROBE_MERGE;
    int32_t need = sorted ? dplus_max : hash_table_slots(dplus_max);
    // every wave's slice of the table holds at least the 64 slots of the smallest hash table
    int32_t s = 64 * kWavesPerBlock;
    while (s < need && s < kMaxTableSlots) s <<= 1;
    return s;
}

tc_lcc_status build_schedule(tc_lcc_graph g, const tc_lcc_tuning& tn, hipStream_t st) {
    GraphDev& d = g->d;
    const int probe = resolve_probe(tn.probe, d.n);
    // the graph's schedule fields change only once the new schedule is complete, so a failed
    // rebuild leaves the previous one whole
    const int32_t slots = table_slots(probe, d.max_dplus);
    const bool sorted = probe == TC_LCC_PROBE_SORTED || probe == TC_LCC_PROBE_MERGE;
    const int32_t block_cap = sorted ? slots : hash_capacity(slots);
    // beyond the hash, a block's table still holds a sorted list of as many entries as it has
    // slots (not with the hash-only probe): such vertices get a launch of their own
    const int32_t list_cap = probe == TC_LCC_PROBE_HASH ? block_cap : slots;
    int32_t wave_cap = sorted ? slots / kWavesPerBlock : hash_capacity(slots / kWavesPerBlock);
    if (tn.wave_outdeg_max > 0 && tn.wave_outdeg_max < wave_cap) wave_cap = tn.wave_outdeg_max;
    Temps tmp{g->ctx->pool.get(), {}};
    const size_t n = (size_t)d.n;
    uint64_t *ka, *kb, *res;
    unsigned long long* counts;
    unsigned int* sort_err;
    void* scr;
    TCL_TRY(tmp.get(std::max<size_t>(n, 1), &ka));
    TCL_TRY(tmp.get(std::max<size_t>(n, 1), &kb));
    TCL_TRY(tmp.get(64, &counts));
    TCL_TRY(tmp.get(64, &sort_err));
    TCL_TRY(tmp.get(radix_sort_scratch_bytes(std::max<size_t>(n, 1)), (uint8_t**)&scr));
    TCL_HIP(fill<unsigned long long>(counts, 64, 0ull, st));
    TCL_HIP(fill<unsigned int>(sort_err, 64, 0u, st));
    const int group = tn.group;
    // the bitmap is taken wherever it fits with the automatic probe (not with hash, sorted or
    // merge), so there a long list whose bitmap fits the block's table stays in the block bins
    const uint32_t bm_region = probe == TC_LCC_PROBE_AUTO ? (uint32_t)slots * 8u : 0u;
    if (d.compact || d.off_bytes == 8)
        k_classify<int64_t><<<grid_for(n, kB, 4096), kB, 0, st>>>(
            (const unsigned long long*)d.work, d.dplus, (const int64_t*)d.out_off, d.adj, d.n, d.bits,
            tn.wave_work_max, wave_cap, block_cap, list_cap, bm_region, group, ka, counts);
    else
        k_classify<int32_t><<<grid_for(n, kB, 4096), kB, 0, st>>>(
            (const unsigned long long*)d.work, d.dplus, (const int32_t*)d.out_off, d.adj, d.n, d.bits,
            tn.wave_work_max, wave_cap, block_cap, list_cap, bm_region, group, ka, counts);
    TCL_HIP(hipGetLastError());
    // keys are written in vertex order: a stable sort on the 6 class bits keeps vertices
    // ascending within a class
    TCL_HIP(radix_sort_u64(ka, kb, n, d.bits, 6, scr, sort_err, st, &res));
    unsigned long long hc[64];
    unsigned int herr = 0;
    TCL_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipMemcpyAsync(&herr, sort_err, sizeof(herr), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    if (herr) {
        set_error("schedule: a radix sort pass gave up waiting for an earlier tile");
        return TC_LCC_DEVICE_ERROR;
    }
    int64_t nb = 0;
    for (int c = 0; c < kClassWave; ++c) nb += (int64_t)hc[c];
    const int64_t active = nb + (int64_t)hc[kClassWave] + (int64_t)hc[kClassList] + (int64_t)hc[kClassGlobal];
    if (active > 0) {
        k_vlist<<<grid_for(active, kB, 4096), kB, 0, st>>>(res, active, d.bits, d.vlist);
        TCL_HIP(hipGetLastError());
    }
    TCL_HIP(hipStreamSynchronize(st));
    for (int c = 0; c < kClassWave; ++c) d.class_count[c] = (int64_t)hc[c];
    d.n_block = nb;
    d.n_wave = (int64_t)hc[kClassWave];
    d.n_list = (int64_t)hc[kClassList];
    d.n_global = (int64_t)hc[kClassGlobal];
    d.hash_slots = slots;
    d.sched_probe = probe;
    return TC_LCC_OK;
}


// ------------------------------------------------------------------ streamed build
//
// A graph whose raw pairs do not fit HBM beside the build (R-MAT scale 30: 1.7e10 pairs, 137 GB
// as int32) is built from a pair source the library calls for consecutive chunks, once per
// pass.  The passes:
//   0. a histogram of the pairs' lower ends (top 12 bits) sets partitions of the id range that
//      each hold at most `partition_pairs` pairs;
//   1. per partition: the canonical keys of its pairs (lower end in the partition) are
//      gathered, sorted and made unique; the higher ends are appended to the upper lists of
//      the canonical CSR (lower id -> higher ids), which is all that is kept of them;
//      degrees from the run lengths (lower ends) and one atomic per unique edge (higher end);
//   2. rank by (degree, id) as in the one-pass build;
//   3. orientation: each canonical edge adds 1 to the out-degree of its lower-ranked end; the
//      oriented lists are filled through per-row cursors and then sorted row by row;
//   4. reverse lists in compact form: per kept in-edge (u -> v), u and the position of v in
//      N+(u) (16 bits; the tail start and length follow from out_off[u] and out_off[u + 1]),
//      placed through per-vertex cursors.  6 bytes per in-edge instead of 16;
//   5. statistics and the schedule as in the one-pass build.
// Peak memory at scale 30 is about 215 GB for the graph plus one phase's temporaries.

namespace {

constexpr int kHistBits = 12;
constexpr int kEdgeTile = 4096;  // edges per block in the passes over a CSR's entries

// Histogram of the pairs' lower ends by their top kHistBits bits, counted in LDS; blocks stride
// over the chunk so that each flushes its counts once.
__global__ __launch_bounds__(kB) void k_stream_hist(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                                                    size_t cnt, int64_t n, int shift,
                                                    unsigned long long* __restrict__ hist, int* __restrict__ bad) {
    __shared__ unsigned int h[1 << kHistBits];
    for (int i = threadIdx.x; i < (1 << kHistBits); i += blockDim.x) h[i] = 0;
    __syncthreads();
    bool out = false;
    GRID_STRIDE(i, cnt) {
        const int32_t a = src[i], b = dst[i];
        if (a < 0 || a >= n || b < 0 || b >= n) {
            out = true;
        } else if (a != b) {
            atomicAdd(&h[(uint32_t)(a < b ? a : b) >> shift], 1u);
        }
    }
    if (out) *bad = 1;
    __syncthreads();
    for (int i = threadIdx.x; i < (1 << kHistBits); i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

// Canonical keys ((lower - lo0) << bits | higher) of the pairs whose lower end lies in
// [lo0, lo1), appended behind a counter: a block takes kScanTile pairs at a time (element
// i * 256 + t is thread t's i-th), ranks its keys by ballots and one scan over the (round, wave)
// counts, and reserves their places with one atomic per tile.  At most `cap` keys are written;
// the counter still counts every one.  A pair with an end outside [0, n) (a source that changed
// since the histogram pass) is not taken and raises *bad.
__global__ __launch_bounds__(kScanThreads) void k_stream_keys(const int32_t* __restrict__ src,
                                                              const int32_t* __restrict__ dst, size_t cnt, int64_t n,
                                                              int bits, int64_t lo0, int64_t lo1,
                                                              uint64_t* __restrict__ keys,
                                                              unsigned long long* __restrict__ count,
                                                              unsigned long long cap, int* __restrict__ bad) {
    constexpr int NW = kScanThreads / kWave;
    static_assert(kScanItems * NW == kWave, "one lane per (round, wave) count");
    __shared__ uint32_t base[kScanItems][NW];
    __shared__ unsigned long long s_base;
    const int lane = lane_id(), w = threadIdx.x / kWave;
    const unsigned long long lt = lanemask_lt();
    for (size_t tile = (size_t)blockIdx.x * kScanTile; tile < cnt; tile += (size_t)gridDim.x * kScanTile) {
        uint64_t key[kScanItems];
        unsigned long long bal[kScanItems];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const size_t e = tile + (size_t)i * kScanThreads + threadIdx.x;
            bool take = false;
            key[i] = 0;
            if (e < cnt) {
                const int32_t a = src[e], b = dst[e];
                const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
                if (lo < 0 || hi >= n) *bad = 1;
                take = a != b && lo >= lo0 && lo < lo1 && hi < n;
                key[i] = ((uint64_t)(lo - lo0) << bits) | (uint64_t)hi;
            }
            bal[i] = __builtin_amdgcn_ballot_w64(take);
            if (lane == 0) base[i][w] = (uint32_t)__popcll(bal[i]);
        }
        __syncthreads();
        if (w == 0) {
            const uint32_t c = base[lane / NW][lane % NW];
            const uint32_t incl = wave_inclusive_scan(c);
            base[lane / NW][lane % NW] = incl - c;
            const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
            if (lane == 0) s_base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
        }
        __syncthreads();
        const unsigned long long b0 = s_base;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if ((bal[i] >> lane) & 1ull) {
                const unsigned long long p = b0 + base[i][w] + (unsigned long long)__popcll(bal[i] & lt);
                if (p < cap) keys[p] = key[i];
            }
        }
        __syncthreads();  // base and s_base are rewritten by the next tile
    }
}

__global__ void k_hi_degree(const uint32_t* __restrict__ hi, size_t cnt, int32_t* __restrict__ deg) {
    GRID_STRIDE(i, cnt) atomicAdd(&deg[hi[i]], 1);
}

__global__ void k_add_i32(int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n) {
    GRID_STRIDE(i, n) a[i] += b[i];
}

// The row r of a CSR entry e: the last r in [lo, hi] with off[r] <= e.
template <typename OffT>
__device__ __forceinline__ int64_t row_of(const OffT* __restrict__ off, int64_t lo, int64_t hi, size_t e) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo + 1) >> 1);
        if ((size_t)off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Rows spanned by the entries [e0, e1) of a block (found once per block), so that each entry's
// row is a short search in cached offsets.
template <typename OffT>
__device__ __forceinline__ void block_rows(const OffT* __restrict__ off, int64_t n, size_t e0, size_t e1,
                                           int64_t* r0, int64_t* r1) {
    __shared__ int64_t s_r[2];
    if (threadIdx.x == 0) {
        s_r[0] = row_of(off, 0, n - 1, e0);
        s_r[1] = row_of(off, s_r[0], n - 1, e1 - 1);
    }
    __syncthreads();
    *r0 = s_r[0];
    *r1 = s_r[1];
    __syncthreads();
}

// Pass 3a: for each canonical edge (x < y) of the upper lists, +1 to the out-degree of the end
// of lower rank.
__global__ __launch_bounds__(256) void k_orient_count(const int64_t* __restrict__ uoff, const int32_t* __restrict__ uadj,
                                                      int64_t n, size_t m, const int32_t* __restrict__ rank,
                                                      int32_t* __restrict__ dplus) {
    for (size_t e0 = (size_t)blockIdx.x * kEdgeTile; e0 < m; e0 += (size_t)gridDim.x * kEdgeTile) {
        const size_t e1 = e0 + kEdgeTile < m ? e0 + kEdgeTile : m;
        int64_t r0, r1;
        block_rows(uoff, n, e0, e1, &r0, &r1);
        for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int64_t x = row_of(uoff, r0, r1, e);
            const int32_t rx = rank[x], ry = rank[uadj[e]];
            atomicAdd(&dplus[rx < ry ? rx : ry], 1);
        }
    }
}

// Pass 3b: each canonical edge written into its lower-ranked end's oriented list, at the next
// free place of that row (per-row cursors); the rows are sorted afterwards.
__global__ __launch_bounds__(256) void k_orient_fill(const int64_t* __restrict__ uoff, const int32_t* __restrict__ uadj,
                                                     int64_t n, size_t m, const int32_t* __restrict__ rank,
                                                     const int64_t* __restrict__ out_off, int32_t* __restrict__ cursor,
                                                     int32_t* __restrict__ adj) {
    for (size_t e0 = (size_t)blockIdx.x * kEdgeTile; e0 < m; e0 += (size_t)gridDim.x * kEdgeTile) {
        const size_t e1 = e0 + kEdgeTile < m ? e0 + kEdgeTile : m;
        int64_t r0, r1;
        block_rows(uoff, n, e0, e1, &r0, &r1);
        for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int64_t x = row_of(uoff, r0, r1, e);
            const int32_t rx = rank[x], ry = rank[uadj[e]];
            const int32_t lo = rx < ry ? rx : ry, hi = rx < ry ? ry : rx;
            const int32_t slot = atomicAdd(&cursor[lo], 1);
            adj[out_off[lo] + slot] = hi;
        }
    }
}

// Rows of up to 64 int32 entries sorted in registers, G lanes per row (as sort_rows_by_group).
template <int G>
__device__ __forceinline__ void sort_rows32_by_group(int32_t* __restrict__ adj, uint64_t todo, int64_t beg, int32_t d) {
    constexpr int R = kWave / G;
    const int lane = lane_id(), grp = lane / G, e = lane % G;
    while (todo) {
        int js[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            js[q] = todo ? (int)__builtin_ctzll(todo) : -1;
            todo &= todo - 1;
        }
        int jg = js[0];
#pragma unroll
        for (int q = 1; q < R; ++q) jg = grp == q ? js[q] : jg;
        const int jl = jg >= 0 ? jg : 0;
        const int64_t s = shfl_off(beg, jl);
        const int32_t dj = __shfl(d, jl, kWave);
        const bool valid = jg >= 0 && e < dj;
        uint32_t x = valid ? (uint32_t)adj[s + e] : 0xffffffffu;
        x = group_bitonic_sort<G>(x);
        if (valid) adj[s + e] = (int32_t)x;
    }
}

__global__ __launch_bounds__(256) void k_sort_rows32_short(int32_t* __restrict__ adj, const int64_t* __restrict__ off,
                                                           int64_t n) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r0 = wave * kWave; r0 < n; r0 += nwaves * kWave) {
        const int64_t r = r0 + lane;
        int64_t beg = 0;
        int32_t d = 0;
        if (r < n) {
            beg = off[r];
            d = (int32_t)(off[r + 1] - beg);
        }
        sort_rows32_by_group<16>(adj, __builtin_amdgcn_ballot_w64(d > 1 && d <= 16), beg, d);
        sort_rows32_by_group<32>(adj, __builtin_amdgcn_ballot_w64(d > 16 && d <= 32), beg, d);
        sort_rows32_by_group<64>(adj, __builtin_amdgcn_ballot_w64(d > 32 && d <= kWave), beg, d);
    }
}

template <int E>
__device__ __forceinline__ void sort_long_row32(int32_t* __restrict__ adj, int64_t s, int32_t d) {
    const int lane = lane_id();
    uint32_t v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * kWave + lane;
        v[e] = i < d ? (uint32_t)adj[s + i] : 0xffffffffu;
    }
    reg_bitonic<E>(v);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int i = e * kWave + lane;
        if (i < d) adj[s + i] = (int32_t)v[e];
    }
}

// Listed rows of 65 .. 4096 entries: one wave per row, in registers.
__global__ __launch_bounds__(256) void k_sort_rows32_long(int32_t* __restrict__ adj, const int64_t* __restrict__ off,
                                                          const int32_t* __restrict__ rows, int64_t count) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t it = wave; it < count; it += nwaves) {
        const int32_t r = rows[it];
        const int64_t s = off[r];
        const int32_t d = (int32_t)(off[r + 1] - s);
        if (d <= kWave || d > kRowSortMax) continue;
        if (d <= 128) sort_long_row32<2>(adj, s, d);
        else if (d <= 256) sort_long_row32<4>(adj, s, d);
        else if (d <= 512) sort_long_row32<8>(adj, s, d);
        else if (d <= 1024) sort_long_row32<16>(adj, s, d);
        else if (d <= 2048) sort_long_row32<32>(adj, s, d);
        else sort_long_row32<64>(adj, s, d);
    }
}

// Rows longer than the register sort: their entries as (row list index << 32 | value) keys,
// sorted together, and written back.
__global__ void k_long_gather(int32_t* __restrict__ adj, const int64_t* __restrict__ off,
                              const int32_t* __restrict__ rows, const int64_t* __restrict__ kpos, int64_t count,
                              uint64_t* __restrict__ keys, bool back) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t it = wave; it < count; it += nwaves) {
        const int32_t r = rows[it];
        const int64_t s = off[r], d = off[r + 1] - s, k0 = kpos[it];
        for (int64_t i = lane_id(); i < d; i += kWave) {
            if (!back) keys[k0 + i] = ((uint64_t)it << 32) | (uint32_t)adj[s + i];
            else adj[s + i] = (int32_t)(uint32_t)keys[k0 + i];
        }
    }
}

__global__ void k_row_len64(const int32_t* __restrict__ rows, int64_t count, const int32_t* __restrict__ dplus,
                            int64_t* __restrict__ len) {
    GRID_STRIDE(i, count) len[i] = dplus[rows[i]];
}

// Pass 4a: per oriented edge e = (u -> v) at position p of N+(u): an in-edge of v is kept if its
// tail (the entries of N+(u) after v) and N+(v) are nonempty; counts per v, probes of v, and a
// flag if a position does not fit 16 bits.
__global__ __launch_bounds__(256) void k_in_count_compact(const int64_t* __restrict__ out_off,
                                                          const int32_t* __restrict__ adj, int64_t n, size_t m,
                                                          const int32_t* __restrict__ dplus, int32_t* __restrict__ din,
                                                          unsigned long long* __restrict__ work, int* __restrict__ wide) {
    for (size_t e0 = (size_t)blockIdx.x * kEdgeTile; e0 < m; e0 += (size_t)gridDim.x * kEdgeTile) {
        const size_t e1 = e0 + kEdgeTile < m ? e0 + kEdgeTile : m;
        int64_t r0, r1;
        block_rows(out_off, n, e0, e1, &r0, &r1);
        for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int64_t u = row_of(out_off, r0, r1, e);
            const int64_t pos = (int64_t)e - out_off[u];
            const int64_t tail = (int64_t)dplus[u] - pos - 1;
            const int32_t v = adj[e];
            if (tail > 0 && dplus[v] > 0) {
                if (pos > 0xffff) *wide = 1;
                atomicAdd(&din[v], 1);
                atomicAdd(&work[v], (unsigned long long)tail);
            }
        }
    }
}

// Pass 4b: the kept in-edges placed through per-vertex cursors: u and the position of v in N+(u).
__global__ __launch_bounds__(256) void k_in_fill_compact(const int64_t* __restrict__ out_off,
                                                         const int32_t* __restrict__ adj, int64_t n, size_t m,
                                                         const int32_t* __restrict__ dplus,
                                                         const int64_t* __restrict__ in_off, int32_t* __restrict__ cursor,
                                                         int32_t* __restrict__ in_u, uint16_t* __restrict__ in_pos) {
    for (size_t e0 = (size_t)blockIdx.x * kEdgeTile; e0 < m; e0 += (size_t)gridDim.x * kEdgeTile) {
        const size_t e1 = e0 + kEdgeTile < m ? e0 + kEdgeTile : m;
        int64_t r0, r1;
        block_rows(out_off, n, e0, e1, &r0, &r1);
        for (size_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const int64_t u = row_of(out_off, r0, r1, e);
            const int64_t pos = (int64_t)e - out_off[u];
            const int64_t tail = (int64_t)dplus[u] - pos - 1;
            const int32_t v = adj[e];
            if (tail > 0 && dplus[v] > 0) {
                const int64_t k = in_off[v] + atomicAdd(&cursor[v], 1);
                in_u[k] = (int32_t)u;
                in_pos[k] = (uint16_t)pos;
            }
        }
    }
}

unsigned edge_grid(size_t m) {
    const size_t b = (m + kEdgeTile - 1) / kEdgeTile;
    return (unsigned)std::max<size_t>(1, std::min<size_t>(b, 65536));
}

}  // namespace

tc_lcc_status build_streamed(tc_lcc_ctx ctx, int64_t n, uint64_t m_in, const StreamSource& source,
                             uint64_t chunk, uint64_t part_cap, const tc_lcc_tuning& tn, hipStream_t st,
                             tc_lcc_graph g) {
    GraphDev& d = g->d;
    Pool* pool = ctx->pool.get();
    Temps tmp{pool, {}};
    // give a temporary back before the build ends (the stream is idle when this is called)
    auto drop = [&](void* p) {
        for (auto it = tmp.held.begin(); it != tmp.held.end(); ++it)
            if (*it == p) {
                pool->release(p);
                tmp.held.erase(it);
                return;
            }
    };
    const int bits = std::max(1, ceil_log2((uint64_t)n));
    const size_t N = (size_t)n;
    d.n = n;
    d.bits = bits;
    d.off_bytes = 8;
    d.compact = true;
    chunk = std::max<uint64_t>(1, std::min<uint64_t>(chunk, std::max<uint64_t>(m_in, 1)));
    part_cap = std::max<uint64_t>(part_cap ? part_cap : m_in, 1);

    int32_t *cs, *cd;
    TCL_TRY(tmp.get(chunk, &cs));
    TCL_TRY(tmp.get(chunk, &cd));
    int* bad;  // [0] id outside [0, n), [1] sort gave up, [2] a row position beyond 16 bits
    TCL_TRY(tmp.get(16, &bad));
    TCL_HIP(fill<int>(bad, 16, 0, st));
    unsigned int* sort_err = (unsigned int*)(bad + 1);
    auto each_chunk = [&](auto&& fn) -> tc_lcc_status {
        for (uint64_t first = 0; first < m_in; first += chunk) {
            const uint64_t cnt = std::min<uint64_t>(chunk, m_in - first);
            const tc_lcc_status s = source(first, cnt, cs, cd, st);
            if (s != TC_LCC_OK) return s;
            fn(cnt);
            TCL_HIP(hipGetLastError());
        }
        return TC_LCC_OK;
    };

    mark(d, 0, st);
    // 0. histogram of the lower ends -> partitions of at most part_cap pairs
    const int shift = std::max(0, bits - kHistBits);
    unsigned long long* hist;
    TCL_TRY(tmp.get(1 << kHistBits, &hist));
    TCL_HIP(fill<unsigned long long>(hist, 1 << kHistBits, 0ull, st));
    TCL_TRY(each_chunk([&](uint64_t cnt) {
        k_stream_hist<<<grid_for(cnt, kB, 512), kB, 0, st>>>(cs, cd, cnt, n, shift, hist, bad);
    }));
    std::vector<unsigned long long> hh(1 << kHistBits);
    int hbad = 0;
    TCL_HIP(hipMemcpyAsync(hh.data(), hist, hh.size() * 8, hipMemcpyDeviceToHost, st));
    TCL_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    if (hbad) {
        set_error("tc_lcc_build_streamed: an endpoint lies outside [0, %lld)", (long long)n);
        return TC_LCC_INVALID_ARGUMENT;
    }
    // partitions: consecutive bins while they hold at most part_cap pairs together (a single
    // bin above part_cap is a partition of its own)
    std::vector<int64_t> bounds{0};
    unsigned long long kmax = 0;
    int64_t span_max = 1;
    {
        unsigned long long acc = 0;
        for (size_t b = 0; b < hh.size(); ++b) {
            if (acc > 0 && acc + hh[b] > part_cap) {
                bounds.push_back(std::min<int64_t>((int64_t)b << shift, n));
                kmax = std::max(kmax, acc);
                acc = 0;
            }
            acc += hh[b];
        }
        bounds.push_back(n);
        kmax = std::max(kmax, acc);
        for (size_t p = 0; p + 1 < bounds.size(); ++p) span_max = std::max(span_max, bounds[p + 1] - bounds[p]);
    }
    if (kmax >= (1ull << 32)) {
        set_error("tc_lcc_build_streamed: %llu pairs fall into one partition (at most 2^32 - 1)", kmax);
        return TC_LCC_UNSUPPORTED;
    }
    drop(hist);

    // 1. per partition: keys, sort, unique, upper lists, degrees
    const size_t K = std::max<size_t>((size_t)kmax, 1);
    int32_t* uadj;
    TCL_TRY(tmp.get(std::max<uint64_t>(m_in, 1), &uadj));
    int32_t *ucnt, *deg;
    TCL_TRY(tmp.get(N, &ucnt));
    TCL_TRY(tmp.get(N, &deg));
    TCL_HIP(fill<int32_t>(ucnt, N, 0, st));
    TCL_HIP(fill<int32_t>(deg, N, 0, st));
    uint64_t *ka, *kb, *kc;
    uint32_t *hi_ends, *toff, *f1, *l1;
    TCL_TRY(tmp.get(K + 1, &ka));
    TCL_TRY(tmp.get(K + 1, &kb));
    TCL_TRY(tmp.get(K + 1, &kc));
    TCL_TRY(tmp.get(K + 1, &hi_ends));
    const size_t tiles_max = (K + kScanTile - 1) / kScanTile;
    TCL_TRY(tmp.get(tiles_max + 2, &toff));
    TCL_TRY(tmp.get((size_t)span_max + 1, &f1));
    TCL_TRY(tmp.get((size_t)span_max + 1, &l1));
    void* sort_scratch;
    const size_t rs_bytes = radix_sort_scratch_bytes(std::max(K, N));
    const size_t scan_elems = scan_scratch_elems(std::max(K, N) + 1);
    TCL_TRY(tmp.get(rs_bytes + sizeof(uint64_t) * scan_elems + 1024, (uint8_t**)&sort_scratch));
    uint32_t* scan32 = (uint32_t*)((uint8_t*)sort_scratch + rs_bytes);
    int64_t* scan64 = (int64_t*)scan32;
    unsigned long long* kcount;
    TCL_TRY(tmp.get(2, &kcount));
    size_t mtot = 0;
    for (size_t p = 0; p + 1 < bounds.size(); ++p) {
        const int64_t lo0 = bounds[p], lo1 = bounds[p + 1];
        if (lo1 <= lo0) continue;
        TCL_HIP(fill<unsigned long long>(kcount, 2, 0ull, st));
        TCL_TRY(each_chunk([&](uint64_t cnt) {
            const size_t ktiles = (cnt + kScanTile - 1) / kScanTile;
            k_stream_keys<<<(unsigned)std::min<size_t>(ktiles, 8192), kScanThreads, 0, st>>>(
                cs, cd, cnt, n, bits, lo0, lo1, ka, kcount, K, bad);
        }));
        unsigned long long kp = 0;
        int pbad = 0;
        TCL_HIP(hipMemcpyAsync(&kp, kcount, 8, hipMemcpyDeviceToHost, st));
        TCL_HIP(hipMemcpyAsync(&pbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (kp > K || pbad) {
            set_error("tc_lcc_build_streamed: the pair source gave different pairs on two passes");
            return TC_LCC_INVALID_ARGUMENT;
        }
        if (kp == 0) continue;
        const int lbits = std::max(1, ceil_log2((uint64_t)(lo1 - lo0)));
        uint64_t* sorted = ka;
        TCL_HIP(radix_sort_u64(ka, kb, kp, 0, bits + lbits, sort_scratch, sort_err, st, &sorted));
        const size_t tiles = (kp + kScanTile - 1) / kScanTile;
        k_reduce_tiles<uint32_t, UniqueFlag><<<(unsigned)tiles, kScanThreads, 0, st>>>(
            UniqueFlag{sorted, (size_t)kp, (1ull << (2 * bits)) - 1}, kp, toff);
        TCL_HIP(hipGetLastError());
        TCL_HIP(exclusive_scan<uint32_t>(ArrayIn<uint32_t>{toff, tiles}, tiles + 1, toff, scan32, st));
        k_unique_tiles<<<(unsigned)tiles, kScanThreads, 0, st>>>(sorted, kp, bits, toff, kc, hi_ends);
        TCL_HIP(hipGetLastError());
        uint32_t up = 0;
        TCL_HIP(hipMemcpyAsync(&up, toff + tiles, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (mtot + up > m_in) {
            set_error("tc_lcc_build_streamed: the pair source gave different pairs on two passes");
            return TC_LCC_INVALID_ARGUMENT;
        }
        TCL_HIP(hipMemcpyAsync(uadj + mtot, hi_ends, (size_t)up * 4, hipMemcpyDeviceToDevice, st));
        // run lengths per lower end: the upper-list lengths of the partition's ids
        TCL_HIP(run_bounds(GroupShift{kc, bits}, up, f1, l1, lo1 - lo0, st));
        k_run_counts<<<grid_for((size_t)(lo1 - lo0), kB, 8192), kB, 0, st>>>(f1, l1, lo1 - lo0, ucnt + lo0);
        k_hi_degree<<<grid_for(up, kB, 8192), kB, 0, st>>>(hi_ends, up, deg);
        TCL_HIP(hipGetLastError());
        mtot += up;
    }
    TCL_HIP(hipStreamSynchronize(st));
    for (void* p : {(void*)ka, (void*)kb, (void*)kc, (void*)hi_ends, (void*)cs, (void*)cd, (void*)f1, (void*)l1}) drop(p);
    const size_t m = mtot;
    d.m = (int64_t)m;
    int64_t* uoff;
    TCL_TRY(tmp.get(N + 1, &uoff));
    TCL_HIP(exclusive_scan<int64_t>(I32In<int64_t>{ucnt, n}, N + 1, uoff, scan64, st));
    k_add_i32<<<grid_for(N, kB, 8192), kB, 0, st>>>(deg, ucnt, n);
    TCL_HIP(hipGetLastError());
    TCL_HIP(hipStreamSynchronize(st));
    drop(ucnt);

    mark(d, 1, st);
    // 2. rank by (degree, id)
    int32_t* rank;
    TCL_TRY(tmp.get(N, &rank));
    TCL_TRY(keep(g, N, &d.order));
    TCL_TRY(keep(g, N, &d.deg_r));
    {
        uint64_t *ra, *rb2;
        TCL_TRY(tmp.get(N + 1, &ra));
        TCL_TRY(tmp.get(N + 1, &rb2));
        uint64_t* rs = ra;
        k_rank_keys<<<grid_for(N, kB, 8192), kB, 0, st>>>(deg, n, bits, ra);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(ra, rb2, N, bits, bits, sort_scratch, sort_err, st, &rs));
        k_rank_scatter<<<grid_for(N, kB, 8192), kB, 0, st>>>(rs, n, bits, d.order, rank, d.deg_r);
        TCL_HIP(hipGetLastError());
        TCL_HIP(hipStreamSynchronize(st));
        drop(ra);
        drop(rb2);
    }
    drop(deg);

    mark(d, 2, st);
    // 3. orientation: out-degrees, offsets, fill through cursors, sort the rows
    TCL_TRY(keep(g, N, &d.dplus));
    int64_t* out_off;
    TCL_TRY(keep(g, N + 1, &out_off));
    d.out_off = out_off;
    TCL_TRY(keep(g, std::max<size_t>(m, 1), &d.adj));
    int32_t* cursor;
    TCL_TRY(tmp.get(N, &cursor));
    TCL_HIP(fill<int32_t>(d.dplus, N, 0, st));
    TCL_HIP(fill<int32_t>(cursor, N, 0, st));
    if (m > 0) {
        k_orient_count<<<edge_grid(m), 256, 0, st>>>(uoff, uadj, n, m, rank, d.dplus);
        TCL_HIP(hipGetLastError());
    }
    TCL_HIP(exclusive_scan<int64_t>(I32In<int64_t>{d.dplus, n}, N + 1, out_off, scan64, st));
    if (m > 0) {
        k_orient_fill<<<edge_grid(m), 256, 0, st>>>(uoff, uadj, n, m, rank, out_off, cursor, d.adj);
        TCL_HIP(hipGetLastError());
    }
    TCL_HIP(hipStreamSynchronize(st));
    drop(uadj);
    drop(uoff);
    drop(rank);
    int dmax = 0;
    if (m > 0) {
        int* mx = bad + 4;
        k_max_i32<<<grid_for(N, kB, 1024), kB, 0, st>>>(d.dplus, n, mx);
        TCL_HIP(hipGetLastError());
        TCL_HIP(hipMemcpyAsync(&dmax, mx, sizeof(int), hipMemcpyDeviceToHost, st));
        const size_t groups = (N + kWave - 1) / kWave;
        k_sort_rows32_short<<<grid_for(groups * kWave, kB, 8192), kB, 0, st>>>(d.adj, out_off, n);
        TCL_HIP(hipGetLastError());
        // the longer rows, listed by a scan of their flags
        uint32_t* rpos;
        TCL_TRY(tmp.get(N + 1, &rpos));
        TCL_HIP(exclusive_scan<uint32_t>(LongRow{d.dplus, n, kWave}, N + 1, rpos, scan32, st));
        uint32_t nlong = 0;
        TCL_HIP(hipMemcpyAsync(&nlong, rpos + N, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        TCL_HIP(hipStreamSynchronize(st));
        if (nlong > 0) {
            int32_t* rows;
            TCL_TRY(tmp.get(nlong, &rows));
            k_list_rows<<<grid_for(N, kB, 8192), kB, 0, st>>>(d.dplus, n, kWave, rpos, rows);
            k_sort_rows32_long<<<grid_for((size_t)nlong * kWave, kB, 8192), kB, 0, st>>>(d.adj, out_off, rows,
                                                                                        (int64_t)nlong);
            TCL_HIP(hipGetLastError());
        }
        if (dmax > kRowSortMax) {
            // rows beyond the register sort: gathered as (list index << 32 | value), sorted, put back
            uint32_t* rpos2;
            TCL_TRY(tmp.get(N + 1, &rpos2));
            TCL_HIP(exclusive_scan<uint32_t>(LongRow{d.dplus, n, kRowSortMax}, N + 1, rpos2, scan32, st));
            uint32_t nvery = 0;
            TCL_HIP(hipMemcpyAsync(&nvery, rpos2 + N, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            TCL_HIP(hipStreamSynchronize(st));
            int32_t* vrows;
            int64_t *vlen, *vpos;
            TCL_TRY(tmp.get(std::max<uint32_t>(nvery, 1), &vrows));
            TCL_TRY(tmp.get(std::max<uint32_t>(nvery, 1), &vlen));
            TCL_TRY(tmp.get((size_t)nvery + 1, &vpos));
            k_list_rows<<<grid_for(N, kB, 8192), kB, 0, st>>>(d.dplus, n, kRowSortMax, rpos2, vrows);
            k_row_len64<<<grid_for(nvery, kB, 1024), kB, 0, st>>>(vrows, nvery, d.dplus, vlen);
            TCL_HIP(hipGetLastError());
            TCL_HIP(exclusive_scan<int64_t>(ArrayIn<int64_t>{vlen, nvery}, (size_t)nvery + 1, vpos, scan64, st));
            int64_t tot = 0;
            TCL_HIP(hipMemcpyAsync(&tot, vpos + nvery, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            TCL_HIP(hipStreamSynchronize(st));
            uint64_t *va, *vb;
            TCL_TRY(tmp.get((size_t)tot + 1, &va));
            TCL_TRY(tmp.get((size_t)tot + 1, &vb));
            void* vscr;
            TCL_TRY(tmp.get(radix_sort_scratch_bytes((size_t)tot), (uint8_t**)&vscr));
            k_long_gather<<<grid_for((size_t)nvery * kWave, kB, 4096), kB, 0, st>>>(d.adj, out_off, vrows, vpos,
                                                                                    nvery, va, false);
            uint64_t* vs = va;
            TCL_HIP(radix_sort_u64(va, vb, (size_t)tot, 0, 32 + std::max(1, ceil_log2(nvery)), vscr, sort_err, st,
                                   &vs));
            k_long_gather<<<grid_for((size_t)nvery * kWave, kB, 4096), kB, 0, st>>>(d.adj, out_off, vrows, vpos,
                                                                                    nvery, vs, true);
            TCL_HIP(hipGetLastError());
        }
    }
    TCL_HIP(hipStreamSynchronize(st));
    drop(cursor);

    mark(d, 3, st);
    // 4. reverse lists in compact form
    int32_t* din;
    TCL_TRY(tmp.get(N, &din));
    TCL_HIP(fill<int32_t>(din, N, 0, st));
    TCL_TRY(keep(g, N, &d.work));
    TCL_HIP(fill<uint64_t>(d.work, N, 0ull, st));
    if (m > 0) {
        k_in_count_compact<<<edge_grid(m), 256, 0, st>>>(out_off, d.adj, n, m, d.dplus, din,
                                                         (unsigned long long*)d.work, bad + 2);
        TCL_HIP(hipGetLastError());
    }
    int64_t* in_off;
    TCL_TRY(keep(g, N + 1, &in_off));
    d.in_off = in_off;
    TCL_HIP(exclusive_scan<int64_t>(I32In<int64_t>{din, n}, N + 1, in_off, scan64, st));
    int64_t kept = 0;
    int wide = 0;
    TCL_HIP(hipMemcpyAsync(&kept, in_off + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipMemcpyAsync(&wide, bad + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    if (wide) {
        set_error("tc_lcc_build_streamed: an oriented list longer than 65536 entries (compact in-edges hold "
                  "16-bit positions)");
        return TC_LCC_UNSUPPORTED;
    }
    d.m_in_kept = kept;
    const size_t KE = std::max<size_t>((size_t)kept, 1);
    TCL_TRY(keep(g, KE, &d.in_u));
    TCL_TRY(keep(g, KE, &d.in_pos));
    TCL_HIP(fill<int32_t>(din, N, 0, st));  // the cursors
    if (m > 0) {
        k_in_fill_compact<<<edge_grid(m), 256, 0, st>>>(out_off, d.adj, n, m, d.dplus, in_off, din, d.in_u, d.in_pos);
        TCL_HIP(hipGetLastError());
    }
    TCL_HIP(hipStreamSynchronize(st));
    drop(din);

    mark(d, 4, st);
    // 5. run scratch and statistics
    TCL_TRY(keep(g, N, &d.t_rank));
    TCL_TRY(keep(g, 64, &d.counters));
    TCL_TRY(keep(g, N, &d.vlist));
    unsigned long long* stats;
    TCL_TRY(tmp.get(8, &stats));
    TCL_HIP(fill<unsigned long long>(stats, 8, 0ull, st));
    k_stats<<<grid_for(N, kB, 2048), kB, 0, st>>>(d.dplus, d.deg_r, (const unsigned long long*)d.work, n, stats);
    TCL_HIP(hipGetLastError());
    unsigned long long hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int serr = 0;
    TCL_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipMemcpyAsync(&serr, bad + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    if (serr) {
        set_error("tc_lcc_build_streamed: a radix sort pass gave up waiting for an earlier tile");
        return TC_LCC_DEVICE_ERROR;
    }
    d.max_dplus = (int32_t)hs[0];
    d.max_deg = (int64_t)hs[1];
    d.wedges = hs[2];
    d.staged = hs[3];
    d.push_words = hs[4];
    tc_lcc_status s = build_schedule(g, tn, st);
    mark(d, 5, st);
    return s;
}

}  // namespace tcl
