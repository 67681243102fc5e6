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
//   t(u): counted in the register lane that holds the in-edge, one global atomic per
//         in-edge that closed any;
//   t(w): one LDS counter per entry of N+(v), one global atomic per entry that hit.
// So there are at most 2m + n global atomics whatever the triangle count.
//
// Load balance: a persistent grid pulls vertices from device queues.  Heavy
// vertices (by probe count, heaviest first) take a whole block; light ones take
// one wave with a slice of the block's LDS, kLightGrab at a time.  The first item
// of every block (and the first grab of every wave) is fixed by its index and only
// later ones come from the queue counter: device-wide atomics on one address are
// serialized, so a small graph runs without any and a large one needs few.
// Each wave takes 64 of its in-edges at a time (in a block, every fourth in-edge of the
// vertex) and walks their tails one after the other in windows of 64 candidates (lane i
// reads candidate base + i: coalesced), with all loop bounds wave-uniform (scalar).  A ring
// of 2 * kUnroll windows is prefetched, so that many loads stay in flight across tail
// boundaries, and the next 64 in-edges are loaded while these are walked.  Hits per tail
// are popcounts of ballots.  Block vertices whose N+(v) is too long for the hash take the
// table as a sorted list in a launch of their own; lists beyond the table are searched in
// HBM (k_count_global).
#include "count_device.hpp"

namespace tcl {

constexpr int kLightGrab = 8;       // light vertices a wave takes per queue access (large graphs)
constexpr int kLightGrabLarge = 16;  // ... and for the largest graphs

// Light vertices per grab: 16 when there are at least four grabs of 16 per wave, 8 when there
// are four of 8, single ones when few (so that a small graph spreads its light vertices over
// all waves, and a mid-size one still takes several per queue access).
__host__ __device__ __forceinline__ int light_grab(int64_t n_light, int64_t waves) {
    return n_light >= waves * (int64_t)kLightGrabLarge * 4 ? kLightGrabLarge
           : n_light >= waves * (int64_t)kLightGrab * 4    ? kLightGrab
                                                           : 1;
}

template <typename OffT, int PROBE>
__global__ __launch_bounds__(kCountThreads) void k_count(CountArgs<OffT> a) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int64_t s_item;
    const uint32_t block_bytes = (uint32_t)a.slots * 8u;
    const uint32_t wave_bytes = block_bytes / kWavesPerBlock;
    const int w = threadIdx.x / kWave, lane = lane_id();

    // phase 1: heavy vertices, one block each, heaviest first
    const int64_t grid = gridDim.x;
    for (int64_t it = blockIdx.x;;) {
        if (it >= a.n_block) break;
        // the next item is taken from the queue before this one is worked on, so the atomic's
        // round trip overlaps the work (every thread has read the previous one by now)
        if (threadIdx.x == 0 && grid < a.n_block) s_item = grid + (int64_t)atomicAdd(&a.ctr[0], 1u);
        const int32_t v = a.vlist[it];
        unsigned long long local = 0;
        process_vertex<OffT, PROBE, kWavesPerBlock>(a, v, lds, block_bytes, threadIdx.x, w, local);
        const unsigned long long ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], ws);
        if (grid >= a.n_block) break;
        __syncthreads();
        it = s_item;
        __syncthreads();
    }
    // phase 2: light vertices, one wave each with its own slice of the LDS; the fixed first
    // grabs go to the last blocks first, which hold no heavy vertex
    uint8_t* wregion = lds + (size_t)w * wave_bytes;
    const int64_t waves = grid * kWavesPerBlock;
    const int grab = light_grab(a.n_wave, waves);
    for (int64_t it = ((grid - 1 - blockIdx.x) * (int64_t)kWavesPerBlock + w) * grab;;) {
        if (it >= a.n_wave) break;
        const int64_t end = min(it + (int64_t)grab, a.n_wave);
        // the grab's vertices and their list bounds, lane q holding vertex it + q, loaded at once
        int32_t hv = 0;
        OffT hb0 = 0, hb1 = 0, hi0 = 0, hi1 = 0;
        if (it + lane < end) {
            hv = a.vlist[a.n_block + it + lane];
            hb0 = a.out_off[hv];
            hb1 = a.out_off[hv + 1];
            hi0 = a.in_off[hv];
            hi1 = a.in_off[hv + 1];
        }
        for (int q = 0; it < end; ++it, ++q) {
            const VertexHead<OffT> hd{__builtin_amdgcn_readlane(hv, q), lane_value(hb0, q), lane_value(hb1, q),
                                      lane_value(hi0, q), lane_value(hi1, q)};
            unsigned long long local = 0;
            process_vertex<OffT, PROBE, 1>(a, hd, wregion, wave_bytes, lane, 0, local);
            const unsigned long long ws = wave_sum(local);
            if (lane == 0 && ws) atomicAdd(&a.t[hd.v], ws);
        }
        if (waves * grab >= a.n_wave) break;
        unsigned int q = 0;
        if (lane == 0) q = atomicAdd(&a.ctr[1], 1u);
        q = __shfl(q, 0, kWave);
        it = (waves + (int64_t)q) * grab;
    }
}

// Vertices whose N+(v) exceeds the LDS table: one block each, walking the tails in windows as
// the LDS kernel does, each candidate binary-searched in N+(v) where it lies in HBM (the list
// stays in the caches while the block works on it) and each hit added to t(w) at once.  Only
// taken when |N+(v)| exceeds the largest table: 4096 keys (the table as a sorted list), or
// 2048 with the hash-only probe (4096 slots at load 1/2).
template <typename OffT>
__global__ __launch_bounds__(kCountThreads) void k_count_global(CountArgs<OffT> a) {
    const int w = threadIdx.x / kWave, lane = lane_id();
    for (int64_t it = blockIdx.x; it < a.n_global; it += gridDim.x) {
        const int32_t v = a.vlist[a.n_block + a.n_wave + it];
        const OffT b0 = a.out_off[v];
        Table tb;
        tb.gkeys = a.adj + b0;
        tb.T = (int32_t)(a.out_off[v + 1] - b0);
        tb.tg = a.t;
        unsigned long long local = 0;
        walk_tails<OffT, kProbeGlobal, kWavesPerBlock>(a, first_in_edges<kWavesPerBlock>(a, v, w), tb, w, local);
        const unsigned long long ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], ws);
    }
}

// AUTO and BITMAP both take the rank bitmap where it fits and the hash elsewhere.
int resolve_probe(int probe, int64_t n) {
    (void)n;
    if (probe == TC_LCC_PROBE_SORTED) return TC_LCC_PROBE_SORTED;
    if (probe == TC_LCC_PROBE_MERGE) return TC_LCC_PROBE_MERGE;
    if (probe == TC_LCC_PROBE_HASH) return TC_LCC_PROBE_HASH;
    return TC_LCC_PROBE_AUTO;
}

template <typename OffT>
static tc_lcc_status launch_typed(tc_lcc_graph g, int merge_x100, int spare_per_cu, hipStream_t st) {
    GraphDev& d = g->d;
    CountArgs<OffT> a;
    a.out_off = (const OffT*)d.out_off;
    a.adj = d.adj;
    a.in_off = (const OffT*)d.in_off;
    a.in_u = d.in_u;
    a.in_start = (const OffT*)d.in_start;
    a.in_len = d.in_len;
    a.in_pos = d.in_pos;
    a.vlist = d.vlist;
    a.n_block = d.n_block;
    a.n_wave = d.n_wave;
    a.n_global = d.n_global;
    a.t = d.t_rank;
    a.ctr = d.counters;
    a.slots = d.hash_slots;
    a.merge_x100 = merge_x100 > 0 ? merge_x100 : 100;
    if (d.n_block + d.n_wave > 0) {
        if (d.hash_slots < 64 * kWavesPerBlock || (d.hash_slots & (d.hash_slots - 1)) != 0) {
            set_error("count: table of %d slots cannot be split into %d wave slices", d.hash_slots, kWavesPerBlock);
            return TC_LCC_DEVICE_ERROR;
        }
        const size_t lds = (size_t)d.hash_slots * 8;  // keys and counters
        auto kern = (d.sched_probe == TC_LCC_PROBE_SORTED)  ? k_count<OffT, TC_LCC_PROBE_SORTED>
                    : (d.sched_probe == TC_LCC_PROBE_MERGE) ? k_count<OffT, TC_LCC_PROBE_MERGE>
                    : (d.sched_probe == TC_LCC_PROBE_HASH)  ? k_count<OffT, TC_LCC_PROBE_HASH>
                                                            : k_count<OffT, TC_LCC_PROBE_AUTO>;
        int per_cu = 0;
        TCL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kCountThreads, lds));
        if (per_cu - spare_per_cu >= 1) per_cu -= spare_per_cu;
        if (per_cu < 1) per_cu = 1;
        // enough blocks for one heavy vertex or one grab per wave each, up to a full GPU; the
        // grab size follows from the grid actually launched
        int64_t grid = (int64_t)g->ctx->cu_count * per_cu;
        const int64_t want = d.n_block + (d.n_wave + kWavesPerBlock - 1) / kWavesPerBlock;
        if (grid > want) grid = want;
        if (grid < 1) grid = 1;
        kern<<<(unsigned)grid, kCountThreads, lds, st>>>(a);
        TCL_HIP(hipGetLastError());
        d.count_grid = (int32_t)grid;
        d.count_lds = (int32_t)lds;
        d.count_per_cu = per_cu;
    }
    if (d.n_list > 0) {
        // block vertices whose lists exceed the hash: the block's table as a sorted list, one
        // block each, with queue counters of their own (vlist: blocks, waves, these, global)
        CountArgs<OffT> al = a;
        al.vlist = d.vlist + d.n_block + d.n_wave;
        al.n_block = d.n_list;
        al.n_wave = 0;
        al.ctr = d.counters + 2;
        const size_t lds = (size_t)d.hash_slots * 8;
        const unsigned grid = (unsigned)std::min<int64_t>(d.n_list, (int64_t)g->ctx->cu_count * 4);
        k_count<OffT, TC_LCC_PROBE_SORTED><<<grid, kCountThreads, lds, st>>>(al);
        TCL_HIP(hipGetLastError());
    }
    if (d.n_global > 0) {
        CountArgs<OffT> ag = a;
        ag.vlist = d.vlist + d.n_list;  // k_count_global reads past the block and wave vertices
        const unsigned grid = (unsigned)std::min<int64_t>(d.n_global, (int64_t)g->ctx->cu_count * 4);
        k_count_global<OffT><<<grid, kCountThreads, 0, st>>>(ag);
        TCL_HIP(hipGetLastError());
    }
    return TC_LCC_OK;
}

tc_lcc_status launch_count(tc_lcc_graph g, const tc_lcc_tuning& tn, int spare_per_cu, hipStream_t st) {
    if (g->d.compact) return launch_typed<OffCompact>(g, tn.merge_ratio_x100, spare_per_cu, st);
    return g->d.off_bytes == 4 ? launch_typed<int32_t>(g, tn.merge_ratio_x100, spare_per_cu, st)
                               : launch_typed<int64_t>(g, tn.merge_ratio_x100, spare_per_cu, st);
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
