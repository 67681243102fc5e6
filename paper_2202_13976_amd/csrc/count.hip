// Triangle count kernels, the per-triangle scatter and the FP64 LCC epilogue.
//
// Every triangle has ranks u < v < w with oriented edges u->v, u->w, v->w.  It is
// found exactly once, at its middle vertex v: for every in-edge (u -> v), the tail
// of N+(u) after v holds the candidates w > v (rank-space form of the
// upper-triangle offset of Sec. II-C), and each candidate is probed against N+(v),
// which is staged once per v in LDS.  One candidate probe is one oriented wedge
// (u; v, w), so the work is the number of oriented wedges, sum_u C(|N+(u)|, 2).
//
// Scatter (each triangle adds 1 to t(u), t(v), t(w); Alg. 3 accumulates t):
//   t(v): summed in registers, one atomic per wave and vertex;
//   t(u): one LDS counter per in-edge, one global atomic per in-edge that closed any;
//   t(w): one LDS counter per entry of N+(v), one global atomic per entry that hit.
// So there are at most 2m + n global atomics whatever the triangle count.
//
// Load balance: a persistent grid pulls vertices from device queues.  Heavy
// vertices (by probe count, heaviest first) take a whole block; light ones take
// one wave with a slice of the block's LDS.  Each wave takes 64 in-edges at a
// time and walks their tails one after the other in windows of 64 candidates
// (lane i reads candidate base + i: coalesced), with all loop bounds wave-uniform
// (scalar).  A ring of kUnroll windows is prefetched, so that many loads stay in
// flight across tail boundaries.  Hits per tail are popcounts of ballots.
#include "internal.hpp"

namespace tcl {

constexpr int kUnroll = 4;  // prefetched windows of 64 candidates

template <typename OffT>
struct CountArgs {
    const OffT* out_off;
    const int32_t* adj;
    const OffT* in_off;
    const int32_t* in_u;
    const OffT* in_start;
    const int32_t* in_len;
    const int32_t* vlist;
    int64_t n_block, n_wave, n_global;
    unsigned long long* t;
    unsigned int* ctr;
    int32_t slots;  // table slots of a block (power of two, >= 256)
};

// bucket hash: high bits of a 24x24-bit product (one full-rate multiply)
__device__ __forceinline__ uint32_t hash32(int32_t x) { return __umul24((uint32_t)x, 0x9E3779u); }

template <int NWAVES>
__device__ __forceinline__ void group_sync() {
    if constexpr (NWAVES > 1) __syncthreads();
    else wave_lds_sync();
}

// Bucketed open addressing: 4 slots per bucket read with one 16-byte LDS load; a key
// lives in the first bucket with room from its hash bucket on.  Returns slot or -1.
__device__ __forceinline__ int hash_find(const int32_t* keys, uint32_t nb_mask, int logNB, int32_t x) {
    uint32_t b = logNB ? (hash32(x) >> (32 - logNB)) : 0u;
    for (;;) {
        const int4 k = *reinterpret_cast<const int4*>(keys + 4 * b);
        if (k.x == x) return (int)(4 * b);
        if (k.y == x) return (int)(4 * b + 1);
        if (k.z == x) return (int)(4 * b + 2);
        if (k.w == x) return (int)(4 * b + 3);
        if ((k.x | k.y | k.z | k.w) < 0) return -1;  // a free slot: x is absent
        b = (b + 1) & nb_mask;
    }
}

// continue a lookup at bucket b (after the first bucket was full and did not hold x)
__device__ __forceinline__ int hash_find_from(const int32_t* keys, uint32_t nb_mask, uint32_t b, int32_t x) {
    for (;;) {
        const int4 k = *reinterpret_cast<const int4*>(keys + 4 * b);
        if (k.x == x) return (int)(4 * b);
        if (k.y == x) return (int)(4 * b + 1);
        if (k.z == x) return (int)(4 * b + 2);
        if (k.w == x) return (int)(4 * b + 3);
        if ((k.x | k.y | k.z | k.w) < 0) return -1;
        b = (b + 1) & nb_mask;
    }
}

__device__ __forceinline__ void hash_insert(int32_t* keys, uint32_t nb_mask, int logNB, int32_t x) {
    uint32_t b = logNB ? (hash32(x) >> (32 - logNB)) : 0u;
    for (;;) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (atomicCAS(&keys[4 * b + k], -1, x) == -1) return;
        b = (b + 1) & nb_mask;
    }
}

__device__ __forceinline__ int sorted_find(const int32_t* keys, int32_t T, int32_t x) {
    int lo = 0, hi = T;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return (lo < T && keys[lo] == x) ? lo : -1;
}

// A window: 64 consecutive candidates of one tail (lane i takes candidate base + i).
template <typename OffT>
struct Win {
    OffT st;      // tail start in adj
    int32_t len;  // tail length
    int32_t base; // first candidate of the window within the tail
    int32_t j;    // tail index within the wave's chunk (-1: no window)
};

// LDS view of the staged N+(v) for one probe method.
//   hash:   keys[T] (-1 = empty) and cnt[T], 4-slot buckets
//   sorted: keys[dv] = N+(v) and cnt[dv], binary search
//   bitmap: bm[words] over ranks (v, vmax], first[words] = index in N+(v) of the first
//           entry in each word, cnt[dv]; the entry index of a hit is first + popcount
struct Table {
    int32_t* keys;
    uint32_t* cnt;
    uint32_t* bm;
    uint16_t* first;
    int32_t T;
    uint32_t nb_mask;
    int logNB;
    int32_t base;   // bitmap: rank v + 1 is bit 0
    uint32_t span;  // bitmap: ranks v + 1 .. vmax
    uint32_t words;
};

template <int MODE>
__device__ __forceinline__ bool probe_one(const Table& tb, int32_t x, bool val) {
    bool hit = false;
    if constexpr (MODE == TC_LCC_PROBE_BITMAP) {
        const uint32_t i = (uint32_t)(x - tb.base);  // candidates are ranks above v
        const uint32_t wi = min(i >> 5, tb.words - 1u);
        const uint32_t word = tb.bm[wi];
        const uint32_t bit = i & 31u;
        hit = val && i < tb.span && ((word >> bit) & 1u);
        if (hit) {
            const uint32_t pos = (uint32_t)tb.first[wi] + (uint32_t)__popc(word & ((1u << bit) - 1u));
            atomicAdd(&tb.cnt[pos], 1u);
        }
    } else if constexpr (MODE == TC_LCC_PROBE_HASH) {
        // bucket chain from the home bucket; each matching key bumps its own counter (the
        // slot is the bucket address plus an immediate offset)
        uint32_t b = hash32(x) >> (32 - tb.logNB);
        bool pending = val;
        for (;;) {
            const int4 kk = *reinterpret_cast<const int4*>(tb.keys + 4 * b);
            uint32_t* cb = tb.cnt + 4 * b;
            if (pending) {
                if (kk.x == x) {
                    atomicAdd(cb, 1u);
                    hit = true;
                }
                if (kk.y == x) {
                    atomicAdd(cb + 1, 1u);
                    hit = true;
                }
                if (kk.z == x) {
                    atomicAdd(cb + 2, 1u);
                    hit = true;
                }
                if (kk.w == x) {
                    atomicAdd(cb + 3, 1u);
                    hit = true;
                }
            }
            // keep looking only past a full bucket that did not hold x
            pending = pending && !hit && min(min(kk.x, kk.y), min(kk.z, kk.w)) >= 0;
            if (!__ballot(pending)) break;
            b = pending ? ((b + 1) & tb.nb_mask) : b;
        }
    } else {
        const int sl = sorted_find(tb.keys, tb.T, x);
        hit = val && sl >= 0;
        if (hit) atomicAdd(&tb.cnt[sl], 1u);
    }
    return hit;
}

// Each wave walks the tails of its chunks of 64 in-edges of v and probes every candidate.
template <typename OffT, int MODE, int NWAVES>
__device__ void walk_tails(const CountArgs<OffT>& a, int32_t v, const Table& tb, int wig, uint32_t& local) {
    const int lane = lane_id();
    const OffT i0 = a.in_off[v], i1 = a.in_off[v + 1];
    for (OffT cb = i0 + (OffT)wig * kWave; cb < i1; cb += (OffT)NWAVES * kWave) {
        const OffT k = cb + lane;
        const bool ok = k < i1;
        int32_t u = 0;
        OffT st = 0;
        int32_t len = 0;
        if (ok) {
            u = a.in_u[k];
            st = a.in_start[k];
            len = a.in_len[k];
        }
        const int nk = (int)__builtin_amdgcn_readfirstlane((int)min((OffT)kWave, i1 - cb));
        uint32_t mine = 0;  // hits of the tail this lane owns (tail index == lane)

        // window generator over the chunk, all state scalar: tail gj, next base gbase
        int gj = 0, gbase = 0;
        OffT gst = 0;
        int32_t glen = 0;
        auto fetch_tail = [&]() {
            if (gj < nk) {
                const uint32_t lo32 = __builtin_amdgcn_readlane((uint32_t)((uint64_t)st & 0xffffffffu), gj);
                OffT s = (OffT)lo32;
                if constexpr (sizeof(OffT) == 8) {
                    const uint32_t hi32 = __builtin_amdgcn_readlane((uint32_t)((uint64_t)st >> 32), gj);
                    s = (OffT)(((uint64_t)hi32 << 32) | lo32);
                }
                gst = s;
                glen = __builtin_amdgcn_readlane(len, gj);
            }
        };
        fetch_tail();
        auto next_win = [&](Win<OffT>& w) {
            if (gj >= nk) {
                w.j = -1;
                w.st = 0;
                w.len = 1;
                w.base = 0;
                return;
            }
            w.st = gst;
            w.len = glen;
            w.base = gbase;
            w.j = gj;
            gbase += kWave;
            if (gbase >= glen) {
                gbase = 0;
                ++gj;
                fetch_tail();
            }
        };
        // unconditional load (a spent generator yields adj[0]) so that the compiler can wait
        // for the oldest window only; lanes past the tail re-read its last candidate
        auto load_win = [&](const Win<OffT>& w) -> int32_t {
            const int32_t* tp = a.adj + w.st;
            const uint32_t off = (uint32_t)min(w.base + lane, w.len - 1);
            return tp[off];
        };

        // ring of kUnroll windows: slot q holds windows q, q + kUnroll, ...; a slot is probed
        // and refilled in place, so each load keeps its register until it is consumed
        Win<OffT> win[kUnroll];
        int32_t xs[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
            next_win(win[q]);
            xs[q] = load_win(win[q]);
        }
        int cur_j = 0;       // tail whose hits accumulate in cur_c (windows come in tail order)
        uint32_t cur_c = 0;  // scalar
        uint32_t vsum = 0;   // scalar: hits of this wave for t(v)
        while (win[0].j >= 0) {
#pragma unroll
            for (int q = 0; q < kUnroll; ++q) {
                const Win<OffT> w = win[q];
                const int32_t x = xs[q];
                next_win(win[q]);
                xs[q] = load_win(win[q]);
                if (w.j >= 0) {
                    const bool val = w.base + lane < w.len;
                    const bool hit = probe_one<MODE>(tb, x, val);
                    const unsigned long long H = __ballot(hit);
                    if (w.j != cur_j) {
                        mine = (lane == cur_j) ? mine + cur_c : mine;
                        cur_j = w.j;
                        cur_c = 0;
                    }
                    if (H) {
                        const uint32_t c = (uint32_t)__popcll(H);
                        cur_c += c;
                        vsum += c;
                    }
                }
            }
        }
        mine = (lane == cur_j) ? mine + cur_c : mine;
        local += (lane == 0) ? vsum : 0u;
        if (ok && mine) atomicAdd(&a.t[u], (unsigned long long)mine);
    }
}

// Bytes of the bitmap layout for `words` bitmap words and dv counters.
__device__ __forceinline__ uint32_t bitmap_bytes(uint32_t words, int32_t dv) {
    return ((6u * words + 3u) & ~3u) + 4u * (uint32_t)dv;
}

// One vertex v, processed by a group of NWAVES waves (gtid = thread index in the group,
// wig = wave index in the group) with an LDS region of region_bytes.  The probe method is
// chosen per vertex: the rank bitmap when it fits (AUTO or BITMAP), else the hash; or the
// sorted list when asked for.  Returns this lane's share of t(v) in `local`.
template <typename OffT, int PROBE, int NWAVES>
__device__ void process_vertex(const CountArgs<OffT>& a, int32_t v, uint8_t* region, uint32_t region_bytes,
                               int gtid, int wig, uint32_t& local) {
    constexpr int gsize = NWAVES * kWave;
    const OffT b0 = a.out_off[v];
    const int32_t dv = (int32_t)(a.out_off[v + 1] - b0);
    const int32_t* nv = a.adj + b0;

    Table tb;
    tb.base = v + 1;
    int mode;
    if constexpr (PROBE == TC_LCC_PROBE_SORTED) {
        mode = TC_LCC_PROBE_SORTED;
    } else {
        tb.span = (uint32_t)(nv[dv - 1] - v);
        tb.words = (tb.span + 31u) >> 5;
        mode = (PROBE != TC_LCC_PROBE_HASH && bitmap_bytes(tb.words, dv) <= region_bytes) ? TC_LCC_PROBE_BITMAP
                                                                                           : TC_LCC_PROBE_HASH;
    }

    // ---- stage N+(v)
    if (mode == TC_LCC_PROBE_BITMAP) {
        tb.bm = (uint32_t*)region;
        tb.first = (uint16_t*)(tb.bm + tb.words);
        tb.cnt = (uint32_t*)(region + ((6u * tb.words + 3u) & ~3u));
        for (uint32_t s = gtid; s < tb.words; s += gsize) tb.bm[s] = 0u;
        for (int j = gtid; j < dv; j += gsize) tb.cnt[j] = 0u;
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t i = (uint32_t)(nv[j] - tb.base);
            atomicOr(&tb.bm[i >> 5], 1u << (i & 31u));
            if (j == 0 || ((uint32_t)(nv[j - 1] - tb.base) >> 5) != (i >> 5)) tb.first[i >> 5] = (uint16_t)j;
        }
    } else if (mode == TC_LCC_PROBE_HASH) {
        int32_t T = 64;
        while (T < 2 * dv) T <<= 1;
        const uint32_t nb = (uint32_t)T >> 2;
        tb.T = T;
        tb.nb_mask = nb - 1;
        tb.logNB = 31 - __clz(nb);
        tb.keys = (int32_t*)region;
        tb.cnt = (uint32_t*)(tb.keys + T);
        for (int s = gtid; s < T; s += gsize) {
            tb.keys[s] = -1;
            tb.cnt[s] = 0;
        }
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) hash_insert(tb.keys, tb.nb_mask, tb.logNB, nv[j]);
    } else {
        tb.T = dv;
        tb.keys = (int32_t*)region;
        tb.cnt = (uint32_t*)(tb.keys + dv);
        for (int j = gtid; j < dv; j += gsize) {
            tb.keys[j] = nv[j];
            tb.cnt[j] = 0;
        }
    }
    group_sync<NWAVES>();

    // ---- probe the tails of the in-edges
    if (mode == TC_LCC_PROBE_BITMAP) walk_tails<OffT, TC_LCC_PROBE_BITMAP, NWAVES>(a, v, tb, wig, local);
    else if (mode == TC_LCC_PROBE_HASH) walk_tails<OffT, TC_LCC_PROBE_HASH, NWAVES>(a, v, tb, wig, local);
    else walk_tails<OffT, TC_LCC_PROBE_SORTED, NWAVES>(a, v, tb, wig, local);
    group_sync<NWAVES>();

    // ---- flush the per-entry counters of N+(v)
    if (mode == TC_LCC_PROBE_HASH) {
        for (int s = gtid; s < tb.T; s += gsize) {
            const uint32_t c = tb.cnt[s];
            if (c) atomicAdd(&a.t[tb.keys[s]], (unsigned long long)c);
        }
    } else {
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t c = tb.cnt[j];
            if (c) atomicAdd(&a.t[nv[j]], (unsigned long long)c);
        }
    }
    group_sync<NWAVES>();
}

template <typename OffT, int PROBE>
__global__ __launch_bounds__(kCountThreads) void k_count(CountArgs<OffT> a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int64_t s_item;
    const uint32_t block_bytes = (uint32_t)a.slots * 8u;
    const uint32_t wave_bytes = block_bytes / kWavesPerBlock;
    const int w = threadIdx.x / kWave, lane = lane_id();

    // phase 1: heavy vertices, one block each, heaviest first
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(&a.ctr[0], 1u);
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();
        if (it >= a.n_block) break;
        const int32_t v = a.vlist[it];
        uint32_t local = 0;
        process_vertex<OffT, PROBE, kWavesPerBlock>(a, v, lds, block_bytes, threadIdx.x, w, local);
        const uint32_t ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], (unsigned long long)ws);
    }
    // phase 2: light vertices, one wave each with its own slice of the LDS
    uint8_t* wregion = lds + (size_t)w * wave_bytes;
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(&a.ctr[1], 1u);
        it = __shfl(it, 0, kWave);
        if ((int64_t)it >= a.n_wave) break;
        const int32_t v = a.vlist[a.n_block + it];
        uint32_t local = 0;
        process_vertex<OffT, PROBE, 1>(a, v, wregion, wave_bytes, lane, 0, local);
        const uint32_t ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], (unsigned long long)ws);
    }
}

// Vertices whose N+(v) exceeds the LDS table: binary search straight in N+(v) in
// global memory, one wave per in-edge chunk of 64, per-entry counts go to t(w)
// directly.  Only taken when |N+(v)| > 2048 (hash) or 4096 (sorted).
template <typename OffT>
__global__ __launch_bounds__(256) void k_count_global(CountArgs<OffT> a) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int64_t it = blockIdx.x; it < a.n_global; it += gridDim.x) {
        const int32_t v = a.vlist[a.n_block + a.n_wave + it];
        const OffT b0 = a.out_off[v];
        const int32_t dv = (int32_t)(a.out_off[v + 1] - b0);
        const int32_t* nv = a.adj + b0;
        const OffT i0 = a.in_off[v], i1 = a.in_off[v + 1];
        uint32_t local = 0;
        for (OffT cb = i0 + (OffT)w * kWave; cb < i1; cb += (OffT)4 * kWave) {
            const OffT k = cb + lane;
            const bool ok = k < i1;
            int32_t u = 0;
            OffT st = 0;
            int32_t len = 0;
            if (ok) {
                u = a.in_u[k];
                st = a.in_start[k];
                len = a.in_len[k];
            }
            // each lane walks its own tail (rare path, kept simple)
            uint32_t hits = 0;
            for (int32_t j = 0; j < len; ++j) {
                const int32_t x = a.adj[st + j];
                int lo = 0, hi = dv;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (nv[mid] < x) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < dv && nv[lo] == x) {
                    atomicAdd(&a.t[x], 1ull);
                    ++hits;
                }
            }
            if (hits) atomicAdd(&a.t[u], (unsigned long long)hits);
            local += hits;
        }
        const uint32_t ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], (unsigned long long)ws);
    }
}

// AUTO and BITMAP both take the rank bitmap where it fits and the hash elsewhere.
int resolve_probe(int probe, int64_t n) {
    (void)n;
    if (probe == TC_LCC_PROBE_SORTED) return TC_LCC_PROBE_SORTED;
    if (probe == TC_LCC_PROBE_HASH) return TC_LCC_PROBE_HASH;
    return TC_LCC_PROBE_AUTO;
}

template <typename OffT>
static tc_lcc_status launch_typed(tc_lcc_graph g, hipStream_t st) {
    GraphDev& d = g->d;
    CountArgs<OffT> a;
    a.out_off = (const OffT*)d.out_off;
    a.adj = d.adj;
    a.in_off = (const OffT*)d.in_off;
    a.in_u = d.in_u;
    a.in_start = (const OffT*)d.in_start;
    a.in_len = d.in_len;
    a.vlist = d.vlist;
    a.n_block = d.n_block;
    a.n_wave = d.n_wave;
    a.n_global = d.n_global;
    a.t = d.t_rank;
    a.ctr = d.counters;
    a.slots = d.hash_slots;
    if (d.n_block + d.n_wave > 0) {
        if (d.hash_slots < 64 * kWavesPerBlock || (d.hash_slots & (d.hash_slots - 1)) != 0) {
            set_error("count: table of %d slots cannot be split into %d wave slices", d.hash_slots, kWavesPerBlock);
            return TC_LCC_DEVICE_ERROR;
        }
        const size_t lds = (size_t)d.hash_slots * 8;  // keys and counters
        auto kern = (d.sched_probe == TC_LCC_PROBE_SORTED) ? k_count<OffT, TC_LCC_PROBE_SORTED>
                    : (d.sched_probe == TC_LCC_PROBE_HASH) ? k_count<OffT, TC_LCC_PROBE_HASH>
                                                           : k_count<OffT, TC_LCC_PROBE_AUTO>;
        int per_cu = 0;
        TCL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kCountThreads, lds));
        if (per_cu < 1) per_cu = 1;
        const int64_t want = d.n_block + (d.n_wave + kWavesPerBlock - 1) / kWavesPerBlock;
        int64_t grid = (int64_t)g->ctx->cu_count * per_cu;
        if (grid > want) grid = want;
        if (grid < 1) grid = 1;
        kern<<<(unsigned)grid, kCountThreads, lds, st>>>(a);
        TCL_HIP(hipGetLastError());
        d.count_grid = (int32_t)grid;
        d.count_lds = (int32_t)lds;
        d.count_per_cu = per_cu;
    }
    if (d.n_global > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(d.n_global, (int64_t)g->ctx->cu_count * 4);
        k_count_global<OffT><<<grid, 256, 0, st>>>(a);
        TCL_HIP(hipGetLastError());
    }
    return TC_LCC_OK;
}

tc_lcc_status launch_count(tc_lcc_graph g, const tc_lcc_tuning& tn, hipStream_t st) {
    (void)tn;
    return g->d.off_bytes == 4 ? launch_typed<int32_t>(g, st) : launch_typed<int64_t>(g, st);
}

// ------------------------------------------------------------------ zeroing and epilogue

__global__ void k_zero(unsigned long long* t, int64_t n, unsigned int* ctr, int nctr) {
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) t[i] = 0ull;
    if (i0 < nctr) ctr[i0] = 0u;
}

tc_lcc_status launch_zero_counts(tc_lcc_graph g, hipStream_t st) {
    const int64_t n = std::max<int64_t>(g->d.n, 64);
    k_zero<<<grid_for((size_t)n, 256, 4096), 256, 0, st>>>(g->d.t_rank, g->d.n, g->d.counters, 64);
    TCL_HIP(hipGetLastError());
    return TC_LCC_OK;
}

// Eq. 2 with exact integers: numerator 2 t(v) and denominator d(v) (d(v) - 1) are formed in
// 64-bit integers (exactly representable in binary64 while d < 9.4e7) and divided once,
// IEEE round to nearest.  d < 2 gives +0.0.  Outputs are written in original vertex order.
__global__ void k_epilogue(int64_t n, const int32_t* __restrict__ order, const int32_t* __restrict__ deg_r,
                           const unsigned long long* __restrict__ t_rank, unsigned long long* __restrict__ tri,
                           double* __restrict__ lcc) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = order[r];
        const unsigned long long tv = t_rank[r];
        const int64_t d = deg_r[r];
        tri[v] = tv;
        if (lcc) {
            double x = 0.0;
            if (d >= 2) x = (double)(2ull * tv) / (double)((unsigned long long)d * (unsigned long long)(d - 1));
            lcc[v] = x;
        }
    }
}

tc_lcc_status launch_epilogue(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st) {
    if (g->d.n == 0) return TC_LCC_OK;
    k_epilogue<<<grid_for((size_t)g->d.n, 256, 8192), 256, 0, st>>>(g->d.n, g->d.order, g->d.deg_r, g->d.t_rank,
                                                                    (unsigned long long*)tri, lcc);
    TCL_HIP(hipGetLastError());
    return TC_LCC_OK;
}

}  // namespace tcl
