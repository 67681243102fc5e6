// Triangle count kernels, the per-triangle scatter and the FP64 LCC epilogue.
//
// Every triangle has ranks u < v < w with oriented edges u->v, u->w, v->w.  It is
// found exactly once, at its middle vertex v: for every in-edge (u -> v), the tail
// of N+(u) after v holds the candidates w > v (rank-space form of the
// upper-triangle offset of Sec. II-C), and each candidate is probed against N+(v),
// which is staged once per v in LDS.  So one candidate probe is one oriented wedge
// (u; v, w), and the total work is the number of oriented wedges, sum_u C(|N+(u)|, 2).
//
// Scatter (each triangle adds 1 to t(u), t(v), t(w); Alg. 3 accumulates t):
//   t(v): summed in registers, one atomic per wave and vertex;
//   t(u): one LDS counter per in-edge, one global atomic per in-edge that closed any;
//   t(w): one LDS counter per entry of N+(v), one global atomic per entry that hit.
// So the number of global atomics is at most 2m + n whatever the triangle count.
//
// Load balance: a persistent grid pulls vertices from device queues.  Heavy
// vertices (by probe count, heaviest first) take a whole 256-thread block; light
// ones take one wave with a quarter of the block's LDS table.  Inside a group,
// each wave takes 64 in-edges at a time and flattens their tails so that the 64
// lanes read consecutive candidates (coalesced), mapping a flat index back to its
// in-edge by a 6-step binary search over the wave's prefix sums in LDS.
#include "internal.hpp"

namespace tcl {

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
    int32_t slots;  // table slots of a block (power of two)
};

// per-wave LDS: prefix P[64], per-in-edge hit counters E[64], tail starts S[64]
template <typename OffT>
struct WaveMeta {
    uint32_t P[kWave];
    uint32_t E[kWave];
    OffT S[kWave];
};

__device__ __forceinline__ uint32_t hash_slot(int32_t x, int logT) {
    return ((uint32_t)x * 0x9E3779B1u) >> (32 - logT);
}

template <int NWAVES>
__device__ __forceinline__ void group_sync() {
    if constexpr (NWAVES > 1) __syncthreads();
    else wave_lds_sync();
}

// One vertex v, processed by a group of NWAVES waves (gtid/gsize = thread index/size in the group).
template <typename OffT, int PROBE, int NWAVES>
__device__ void process_vertex(const CountArgs<OffT>& a, int32_t v, int32_t* keys, uint32_t* cnt,
                               WaveMeta<OffT>* meta, int gtid, int wig) {
    constexpr int gsize = NWAVES * kWave;
    const int lane = lane_id();
    const OffT b0 = a.out_off[v];
    const int32_t dv = (int32_t)(a.out_off[v + 1] - b0);
    const int32_t* nv = a.adj + b0;

    // ---- stage N+(v)
    int32_t T;
    int logT = 0;
    if constexpr (PROBE == TC_LCC_PROBE_HASH) {
        T = 64;
        while (T < 2 * dv) T <<= 1;
        logT = 31 - __clz(T);
        for (int s = gtid; s < T; s += gsize) {
            keys[s] = -1;
            cnt[s] = 0;
        }
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) {
            const int32_t x = nv[j];
            uint32_t h = hash_slot(x, logT);
            while (atomicCAS(&keys[h], -1, x) != -1) h = (h + 1) & (uint32_t)(T - 1);
        }
    } else {
        T = dv;
        for (int j = gtid; j < dv; j += gsize) {
            keys[j] = nv[j];
            cnt[j] = 0;
        }
    }
    group_sync<NWAVES>();

    // ---- probe the tails of the in-edges
    const OffT i0 = a.in_off[v], i1 = a.in_off[v + 1];
    uint32_t local = 0;
    for (OffT cb = i0 + (OffT)wig * kWave; cb < i1; cb += (OffT)NWAVES * kWave) {
        const OffT k = cb + lane;
        const bool ok = k < i1;
        int32_t u = 0;
        OffT st = 0;
        uint32_t len = 0;
        if (ok) {
            u = a.in_u[k];
            st = a.in_start[k];
            len = (uint32_t)a.in_len[k];
        }
        const uint32_t incl = wave_inclusive_scan(len);
        const uint32_t total = __shfl(incl, kWave - 1, kWave);
        meta->P[lane] = incl - len;
        meta->S[lane] = st;
        meta->E[lane] = 0;
        wave_lds_sync();
        for (uint32_t f = lane; f < total; f += kWave) {
            int s = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (meta->P[s + step] <= f) s += step;
            const int32_t x = a.adj[meta->S[s] + (OffT)(f - meta->P[s])];
            int slot = -1;
            if constexpr (PROBE == TC_LCC_PROBE_HASH) {
                uint32_t h = hash_slot(x, logT);
                for (;;) {
                    const int32_t kk = keys[h];
                    if (kk == x) {
                        slot = (int)h;
                        break;
                    }
                    if (kk < 0) break;
                    h = (h + 1) & (uint32_t)(T - 1);
                }
            } else {
                int lo = 0, hi = T;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (keys[mid] < x) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < T && keys[lo] == x) slot = lo;
            }
            if (slot >= 0) {
                atomicAdd(&cnt[slot], 1u);
                atomicAdd(&meta->E[s], 1u);
                ++local;
            }
        }
        wave_lds_sync();
        const uint32_t c = meta->E[lane];
        if (ok && c) atomicAdd(&a.t[u], (unsigned long long)c);
        wave_lds_sync();
    }
    const uint32_t wsum = wave_sum(local);
    if (lane == 0 && wsum) atomicAdd(&a.t[v], (unsigned long long)wsum);
    group_sync<NWAVES>();

    // ---- flush the per-entry counters of N+(v)
    for (int s = gtid; s < T; s += gsize) {
        const uint32_t c = cnt[s];
        if (c) atomicAdd(&a.t[keys[s]], (unsigned long long)c);
    }
    group_sync<NWAVES>();
}

template <typename OffT, int PROBE>
__global__ __launch_bounds__(kCountThreads) void k_count(CountArgs<OffT> a) {
    extern __shared__ __align__(16) uint8_t lds[];
    int32_t* keys = (int32_t*)lds;
    uint32_t* cnt = (uint32_t*)(keys + a.slots);
    WaveMeta<OffT>* metas = (WaveMeta<OffT>*)(cnt + a.slots);
    __shared__ int64_t s_item;
    const int w = threadIdx.x / kWave, lane = lane_id();
    WaveMeta<OffT>* meta = metas + w;

    // phase 1: heavy vertices, one block each, heaviest first
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(&a.ctr[0], 1u);
        __syncthreads();
        const int64_t it = s_item;
        __syncthreads();
        if (it >= a.n_block) break;
        process_vertex<OffT, PROBE, kWavesPerBlock>(a, a.vlist[it], keys, cnt, meta, threadIdx.x, w);
    }
    // phase 2: light vertices, one wave each with its own quarter of the table
    const int32_t wslots = a.slots / kWavesPerBlock;
    int32_t* wkeys = keys + w * wslots;
    uint32_t* wcnt = cnt + w * wslots;
    for (;;) {
        unsigned int it = 0;
        if (lane == 0) it = atomicAdd(&a.ctr[1], 1u);
        it = __shfl(it, 0, kWave);
        if ((int64_t)it >= a.n_wave) break;
        process_vertex<OffT, PROBE, 1>(a, a.vlist[a.n_block + it], wkeys, wcnt, meta, lane, 0);
    }
}

// Vertices whose N+(v) exceeds the LDS table: binary search straight in N+(v) in
// global memory, per-entry counts go to t(w) directly.  Never taken when
// |N+(v)| <= 4096 (hash) or 8192 (sorted).
template <typename OffT>
__global__ __launch_bounds__(kCountThreads) void k_count_global(CountArgs<OffT> a) {
    __shared__ WaveMeta<OffT> metas[kWavesPerBlock];
    const int w = threadIdx.x / kWave, lane = lane_id();
    WaveMeta<OffT>* meta = metas + w;
    for (int64_t it = blockIdx.x; it < a.n_global; it += gridDim.x) {
        const int32_t v = a.vlist[a.n_block + a.n_wave + it];
        const OffT b0 = a.out_off[v];
        const int32_t dv = (int32_t)(a.out_off[v + 1] - b0);
        const int32_t* nv = a.adj + b0;
        const OffT i0 = a.in_off[v], i1 = a.in_off[v + 1];
        uint32_t local = 0;
        for (OffT cb = i0 + (OffT)w * kWave; cb < i1; cb += (OffT)kWavesPerBlock * kWave) {
            const OffT k = cb + lane;
            const bool ok = k < i1;
            int32_t u = 0;
            OffT st = 0;
            uint32_t len = 0;
            if (ok) {
                u = a.in_u[k];
                st = a.in_start[k];
                len = (uint32_t)a.in_len[k];
            }
            const uint32_t incl = wave_inclusive_scan(len);
            const uint32_t total = __shfl(incl, kWave - 1, kWave);
            meta->P[lane] = incl - len;
            meta->S[lane] = st;
            meta->E[lane] = 0;
            wave_lds_sync();
            for (uint32_t f = lane; f < total; f += kWave) {
                int s = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (meta->P[s + step] <= f) s += step;
                const int32_t x = a.adj[meta->S[s] + (OffT)(f - meta->P[s])];
                int lo = 0, hi = dv;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if (nv[mid] < x) lo = mid + 1;
                    else hi = mid;
                }
                if (lo < dv && nv[lo] == x) {
                    atomicAdd(&a.t[x], 1ull);
                    atomicAdd(&meta->E[s], 1u);
                    ++local;
                }
            }
            wave_lds_sync();
            const uint32_t c = meta->E[lane];
            if (ok && c) atomicAdd(&a.t[u], (unsigned long long)c);
            wave_lds_sync();
        }
        const uint32_t wsum = wave_sum(local);
        if (lane == 0 && wsum) atomicAdd(&a.t[v], (unsigned long long)wsum);
        __syncthreads();
    }
}

int resolve_probe(int probe, int64_t n) {
    (void)n;
    if (probe == TC_LCC_PROBE_SORTED) return TC_LCC_PROBE_SORTED;
    return TC_LCC_PROBE_HASH;
}

template <typename OffT>
static tc_lcc_status launch_typed(tc_lcc_graph g, hipStream_t st) {
    const GraphDev& d = g->d;
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
        const size_t lds = (size_t)d.hash_slots * 8 + sizeof(WaveMeta<OffT>) * kWavesPerBlock;
        int per_cu = 0;
        if (d.sched_probe == TC_LCC_PROBE_SORTED) {
            TCL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count<OffT, TC_LCC_PROBE_SORTED>,
                                                                 kCountThreads, lds));
        } else {
            TCL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_count<OffT, TC_LCC_PROBE_HASH>,
                                                                 kCountThreads, lds));
        }
        if (per_cu < 1) per_cu = 1;
        const int64_t want = d.n_block + (d.n_wave + kWavesPerBlock - 1) / kWavesPerBlock;
        int64_t grid = (int64_t)g->ctx->cu_count * per_cu;
        if (grid > want) grid = want;
        if (grid < 1) grid = 1;
        if (d.sched_probe == TC_LCC_PROBE_SORTED)
            k_count<OffT, TC_LCC_PROBE_SORTED><<<(unsigned)grid, kCountThreads, lds, st>>>(a);
        else
            k_count<OffT, TC_LCC_PROBE_HASH><<<(unsigned)grid, kCountThreads, lds, st>>>(a);
        TCL_HIP(hipGetLastError());
    }
    if (d.n_global > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>(d.n_global, (int64_t)g->ctx->cu_count * 4);
        k_count_global<OffT><<<grid, kCountThreads, 0, st>>>(a);
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
