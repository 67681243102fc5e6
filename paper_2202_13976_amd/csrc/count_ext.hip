// Count kernels that carry more per triangle than the three +1s of k_count:
//
//   kExtEdges     the triangles of every edge, c(e) = |adj(i) ∩ adj(j)| for e = {i, j}: the
//                 entries of C = A A o A (Sec. V-B), besides t;
//   kExtDirected  the numerator of Eq. 1 for a directed graph: at vertex i, the edges e_jk
//                 with v_j, v_k out-neighbours of v_i.
//
// The triangles are found as in k_count: every triangle has ranks u < v < w (oriented edges
// u->v, u->w, v->w of the undirected skeleton) and is found once, at its middle vertex v,
// when candidate w of the tail of N+(u) after v is found in N+(v), staged in LDS.
//
// Edges.  An oriented edge e = (a -> b) lies on the triangles {a, b, x} with
//   x < a  (x -> a, x -> b): found at a, from in-edge x -> a, hit b: a's LDS counter of b;
//   a < x < b (a -> x, x -> b): found at x, from in-edge a -> x, hit b: the tail entry b of
//          N+(a) (one atomic on e per hit);
//   x > b  (a -> x, b -> x): found at b, from in-edge a -> b: the hits of that tail.
// So c(e) is the sum of the three; every one is added to a counter per position of adj.
//
// Directed.  Each oriented edge carries two bits: bit 0 if the input held it from the lower
// rank to the higher, bit 1 if the other way.  For a triangle u < v < w with bits
// (f_uv, b_uv), (f_uw, b_uw), (f_vw, b_vw) the numerator of vertex i counts the ordered pairs
// (j, k) of its other two vertices with i -> j, i -> k and j -> k:
//   u: f_uv f_uw (f_vw + b_vw)     v: b_uv f_vw (f_uw + b_uw)     w: b_uw b_vw (f_uv + b_uv).
// u's share is summed per tail and multiplied by f_uv at the tail's end, v's in registers,
// w's LDS counter takes b_uw (f_uv + b_uv) per hit and is multiplied by b_vw when flushed.
//
// The probe structure per vertex: the rank bitmap of N+(v) when it fits the LDS region (the
// entry index of a hit is the word's first index plus the popcount of the bits below), else
// N+(v) as a sorted list in LDS (binary search), else (lists longer than the table) a binary
// search in N+(v) where it lies in HBM.  The schedule is the graph's own: block vertices and
// sorted-list vertices take a block, light ones a wave with a quarter of its LDS, the rest
// (beyond the table) a block that searches HBM.
#include "count_device.hpp"

namespace tcl {

enum { kExtEdges = 1, kExtDirected = 2 };

template <typename OffT>
struct ExtArgs {
    const OffT* out_off;
    const int32_t* adj;
    const OffT* in_off;
    const int32_t* in_u;
    const OffT* in_start;
    const int32_t* in_len;
    const int32_t* vlist;
    int64_t n_block, n_wave, n_list, n_global;
    unsigned long long* t;
    unsigned int* ctr;   // [0] block items, [1] wave items taken beyond the first of each
    uint32_t* ce;        // kExtEdges: per position of adj
    const uint8_t* dir;  // kExtDirected: per position of adj
};

// LDS bytes per entry of N+(v) beyond the keys or the bitmap: a counter, and for the directed
// count the entry's direction bits.
template <int EXT>
__host__ __device__ constexpr uint32_t ext_entry_bytes() {
    return EXT == kExtDirected ? 5u : 4u;
}

template <int EXT>
__host__ __device__ inline uint32_t ext_bitmap_bytes(uint32_t words, int32_t dv) {
    return 8u * (words + 1u) + ext_entry_bytes<EXT>() * (uint32_t)dv;
}

template <int EXT>
__host__ __device__ inline uint32_t ext_sorted_bytes(int32_t dv) {
    return (4u + ext_entry_bytes<EXT>()) * (uint32_t)dv;
}

// v's table: mode 0 = rank bitmap, 1 = sorted list in LDS, 2 = sorted list in HBM.
struct ExtTable {
    int mode;
    const int32_t* keys;  // sorted list (LDS or HBM)
    uint32_t* bm;         // bitmap words and first indices
    uint32_t* cnt;        // per entry
    uint8_t* dirv;        // per entry (directed)
    int32_t dv;
    int32_t base;         // bitmap: rank v + 1 is bit 0
    uint32_t words;
};

// Entry index of candidate x in N+(v), or -1.
__device__ __forceinline__ int ext_find(const ExtTable& tb, int32_t x) {
    if (tb.mode == 0) {
        const uint32_t ii = (uint32_t)(x - tb.base);  // candidates are ranks above v
        const uint32_t wi = min(ii >> 5, tb.words);   // beyond the range: the zero guard word
        const uint2 e = *reinterpret_cast<const uint2*>(tb.bm + 2 * wi);
        if (!__builtin_amdgcn_ubfe(e.x, ii, 1u)) return -1;
        return (int)(e.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(e.x, 0u, ii)));
    }
    return sorted_find(tb.keys, tb.dv, x);
}

// The tails of the in-edges of v taken by this wave (wave wig of NWAVES takes in-edges
// i0 + wig, i0 + wig + NWAVES, ...), 64 candidates per window.
template <typename OffT, int EXT, int NWAVES>
__device__ void ext_walk(const ExtArgs<OffT>& a, OffT b0, OffT i0, OffT i1, const ExtTable& tb, int wig,
                         unsigned long long& local) {
    const int lane = lane_id();
    constexpr OffT kSpan = (OffT)kWave * NWAVES;
    for (OffT cb = i0 + wig; cb < i1; cb += kSpan) {
        const OffT k = cb + (OffT)lane * NWAVES;
        int32_t u = 0, len = 0;
        OffT st = 0;
        uint32_t duv = 0;
        if (k < i1) {
            u = a.in_u[k];
            st = a.in_start[k];
            len = a.in_len[k];
            if constexpr (EXT == kExtDirected) duv = a.dir[st - 1];  // the in-edge u -> v itself
        }
        const int nk = (int)__builtin_amdgcn_readfirstlane((int)min((OffT)kWave, (i1 - cb + NWAVES - 1) / NWAVES));
        for (int j = 0; j < nk; ++j) {
            const int32_t tu = __builtin_amdgcn_readlane(u, j);
            const int32_t tl = __builtin_amdgcn_readlane(len, j);
            const OffT ts = lane_value(st, j);
            const uint32_t tuv = (uint32_t)__builtin_amdgcn_readlane((int32_t)duv, j);
            const uint32_t f_uv = tuv & 1u, b_uv = tuv >> 1;
            uint32_t tail_sum = 0;  // wave-uniform: hits of this tail (edges) or u's share (directed)
            for (int32_t base = 0; base < tl; base += kWave) {
                const int32_t idx = base + lane;
                const bool valid = idx < tl;
                const OffT p = ts + (OffT)(valid ? idx : 0);
                const int32_t x = a.adj[p];
                int pos = valid ? ext_find(tb, x) : -1;
                const bool hit = pos >= 0;
                if constexpr (EXT == kExtEdges) {
                    if (hit) {
                        atomicAdd(&a.ce[p], 1u);  // edge u -> x: triangle (u, v, x) with v between
                        if (tb.mode == 2) {
                            atomicAdd(&a.t[x], 1ull);
                            atomicAdd(&a.ce[b0 + pos], 1u);
                        } else {
                            atomicAdd(&tb.cnt[pos], 1u);
                        }
                    }
                    tail_sum += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(hit));
                } else {
                    uint32_t wu = 0;
                    if (hit) {
                        const uint32_t duw = a.dir[p];
                        const uint32_t dvw = tb.mode == 2 ? (uint32_t)a.dir[b0 + pos] : (uint32_t)tb.dirv[pos];
                        const uint32_t f_uw = duw & 1u, b_uw = duw >> 1, f_vw = dvw & 1u, b_vw = dvw >> 1;
                        wu = f_uw * (f_vw + b_vw);
                        local += b_uv * f_vw * (f_uw + b_uw);
                        const uint32_t ww = b_uw * (f_uv + b_uv);
                        if (tb.mode == 2) {
                            if (ww * b_vw) atomicAdd(&a.t[x], (unsigned long long)(ww * b_vw));
                        } else if (ww) {
                            atomicAdd(&tb.cnt[pos], ww);
                        }
                    }
                    tail_sum += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((wu & 1u) != 0)) +
                                2u * (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((wu & 2u) != 0));
                }
            }
            if constexpr (EXT == kExtEdges) {
                if (lane == 0 && tail_sum) {
                    atomicAdd(&a.t[tu], (unsigned long long)tail_sum);
                    atomicAdd(&a.ce[ts - 1], tail_sum);  // edge u -> v: the triangles above v
                }
                if (lane == 0) local += tail_sum;
            } else {
                const uint32_t su = f_uv * tail_sum;
                if (lane == 0 && su) atomicAdd(&a.t[tu], (unsigned long long)su);
            }
        }
    }
}

// One vertex with a group of NWAVES waves and an LDS region (nullptr: search N+(v) in HBM).
template <typename OffT, int EXT, int NWAVES>
__device__ void ext_vertex(const ExtArgs<OffT>& a, int32_t v, uint8_t* region, uint32_t region_bytes, int gtid,
                           int wig, unsigned long long& local) {
    constexpr int gsize = NWAVES * kWave;
    const OffT b0 = a.out_off[v], b1 = a.out_off[v + 1];
    const int32_t dv = (int32_t)(b1 - b0);
    const int32_t* nv = a.adj + b0;
    const OffT i0 = a.in_off[v], i1 = a.in_off[v + 1];
    ExtTable tb;
    tb.dv = dv;
    tb.base = v + 1;
    tb.keys = nv;
    tb.bm = nullptr;
    tb.cnt = nullptr;
    tb.dirv = nullptr;
    tb.words = 0;
    if (region == nullptr) {
        tb.mode = 2;
    } else {
        const uint32_t span = dv > 0 ? (uint32_t)(nv[dv - 1] - v) : 0u;
        tb.words = (span + 31u) >> 5;
        // the schedule keeps every block and wave vertex within its region as a sorted list;
        // a list that did not fit would be searched in HBM rather than overrun the region
        tb.mode = ext_bitmap_bytes<EXT>(tb.words, dv) <= region_bytes ? 0
                  : ext_sorted_bytes<EXT>(dv) <= region_bytes          ? 1
                                                                       : 2;
    }
    if (tb.mode == 0) {
        tb.bm = (uint32_t*)region;
        tb.cnt = (uint32_t*)(region + 8u * (tb.words + 1u));
        tb.dirv = (uint8_t*)(tb.cnt + dv);
        for (uint32_t s = gtid; s <= tb.words; s += gsize) tb.bm[2 * s] = 0u;  // with the guard word
        for (int j = gtid; j < dv; j += gsize) tb.cnt[j] = 0u;
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t i = (uint32_t)(nv[j] - tb.base);
            atomicOr(&tb.bm[2 * (i >> 5)], 1u << (i & 31u));
            if (j == 0 || ((uint32_t)(nv[j - 1] - tb.base) >> 5) != (i >> 5)) tb.bm[2 * (i >> 5) + 1] = (uint32_t)j;
            if constexpr (EXT == kExtDirected) tb.dirv[j] = a.dir[b0 + j];
        }
    } else if (tb.mode == 1) {
        int32_t* keys = (int32_t*)region;
        tb.keys = keys;
        tb.cnt = (uint32_t*)(keys + dv);
        tb.dirv = (uint8_t*)(tb.cnt + dv);
        for (int j = gtid; j < dv; j += gsize) {
            keys[j] = nv[j];
            tb.cnt[j] = 0u;
            if constexpr (EXT == kExtDirected) tb.dirv[j] = a.dir[b0 + j];
        }
    }
    group_sync<NWAVES>();
    ext_walk<OffT, EXT, NWAVES>(a, b0, i0, i1, tb, wig, local);
    group_sync<NWAVES>();
    if (tb.mode != 2) {
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t c = tb.cnt[j];
            if (!c) continue;
            if constexpr (EXT == kExtEdges) {
                atomicAdd(&a.t[nv[j]], (unsigned long long)c);
                atomicAdd(&a.ce[b0 + j], c);  // edge v -> w: the triangles below v
            } else {
                const uint32_t cw = c * ((uint32_t)tb.dirv[j] >> 1);
                if (cw) atomicAdd(&a.t[nv[j]], (unsigned long long)cw);
            }
        }
    }
    group_sync<NWAVES>();
}

// Block items first (block vertices, then sorted-list vertices, then those beyond the table),
// one at a time from a queue; then light vertices, one wave each.
template <typename OffT, int EXT>
__global__ __launch_bounds__(kCountThreads) void k_count_ext(ExtArgs<OffT> a, uint32_t block_bytes) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int64_t s_item;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t nb = a.n_block + a.n_list + a.n_global;
    for (int64_t it = blockIdx.x;;) {
        if (it >= nb) break;
        int32_t v;
        bool global = false;
        if (it < a.n_block) {
            v = a.vlist[it];
        } else if (it < a.n_block + a.n_list) {
            v = a.vlist[a.n_block + a.n_wave + (it - a.n_block)];
        } else {
            v = a.vlist[a.n_block + a.n_wave + a.n_list + (it - a.n_block - a.n_list)];
            global = true;
        }
        unsigned long long local = 0;
        ext_vertex<OffT, EXT, kWavesPerBlock>(a, v, global ? nullptr : lds, block_bytes, threadIdx.x, w, local);
        const unsigned long long ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], ws);
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int64_t)gridDim.x + (int64_t)atomicAdd(&a.ctr[0], 1u);
        __syncthreads();
        it = s_item;
    }
    const uint32_t wave_bytes = block_bytes / kWavesPerBlock;
    uint8_t* wregion = lds + (size_t)w * wave_bytes;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t it = (int64_t)blockIdx.x * kWavesPerBlock + w;;) {
        if (it >= a.n_wave) break;
        unsigned long long local = 0;
        const int32_t v = a.vlist[a.n_block + it];
        ext_vertex<OffT, EXT, 1>(a, v, wregion, wave_bytes, lane, 0, local);
        const unsigned long long ws = wave_sum(local);
        if (lane == 0 && ws) atomicAdd(&a.t[v], ws);
        unsigned int q = 0;
        if (lane == 0) q = atomicAdd(&a.ctr[1], 1u);
        it = waves + (int64_t)__shfl(q, 0, kWave);
    }
}

template <typename OffT, int EXT>
static tc_lcc_status launch_ext_typed(tc_lcc_graph g, uint32_t* ce, hipStream_t st) {
    GraphDev& d = g->d;
    ExtArgs<OffT> a;
    a.out_off = (const OffT*)d.out_off;
    a.adj = d.adj;
    a.in_off = (const OffT*)d.in_off;
    a.in_u = d.in_u;
    a.in_start = (const OffT*)d.in_start;
    a.in_len = d.in_len;
    a.vlist = d.vlist;
    a.n_block = d.n_block;
    a.n_wave = d.n_wave;
    a.n_list = d.n_list;
    a.n_global = d.n_global;
    a.t = d.t_rank;
    a.ctr = d.counters + 8;
    a.ce = ce;
    a.dir = d.dir;
    const int64_t items = d.n_block + d.n_list + d.n_global + d.n_wave;
    if (items == 0) return TC_LCC_OK;
    // the table of d.hash_slots slots holds any vertex the schedule gives a block or a wave as a
    // sorted list with its counters (and direction bits): 9 bytes per slot, a quarter per wave
    const uint32_t block_bytes = (uint32_t)d.hash_slots * (4u + ext_entry_bytes<EXT>());
    auto kern = k_count_ext<OffT, EXT>;
    int per_cu = 0;
    TCL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kCountThreads, block_bytes));
    if (per_cu < 1) {
        set_error("count: the extended table of %u bytes does not fit a compute unit", block_bytes);
        return TC_LCC_DEVICE_ERROR;
    }
    int64_t grid = (int64_t)g->ctx->cu_count * per_cu;
    const int64_t want = d.n_block + d.n_list + d.n_global + (d.n_wave + kWavesPerBlock - 1) / kWavesPerBlock;
    if (grid > want) grid = want;
    if (grid < 1) grid = 1;
    kern<<<(unsigned)grid, kCountThreads, block_bytes, st>>>(a, block_bytes);
    TCL_HIP(hipGetLastError());
    return TC_LCC_OK;
}

tc_lcc_status launch_count_edges(tc_lcc_graph g, uint32_t* ce, hipStream_t st) {
    return g->d.off_bytes == 4 ? launch_ext_typed<int32_t, kExtEdges>(g, ce, st)
                               : launch_ext_typed<int64_t, kExtEdges>(g, ce, st);
}

tc_lcc_status launch_count_directed(tc_lcc_graph g, hipStream_t st) {
    return g->d.off_bytes == 4 ? launch_ext_typed<int32_t, kExtDirected>(g, nullptr, st)
                               : launch_ext_typed<int64_t, kExtDirected>(g, nullptr, st);
}

// ------------------------------------------------------------------ outputs

// Eq. 1 with exact integers: numerator num(v) and denominator deg+(v) (deg+(v) - 1), one IEEE
// division; deg+ < 2 gives +0.0.  Outputs in original vertex order.
__global__ void k_epilogue_directed(int64_t n, const int32_t* __restrict__ order, const int32_t* __restrict__ dout_r,
                                    const unsigned long long* __restrict__ t_rank, unsigned long long* __restrict__ tri,
                                    double* __restrict__ lcc) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = order[r];
        const unsigned long long num = t_rank[r];
        const int64_t d = dout_r[r];
        tri[v] = num;
        if (lcc) {
            double x = 0.0;
            if (d >= 2) x = (double)num / (double)((unsigned long long)d * (unsigned long long)(d - 1));
            lcc[v] = x;
        }
    }
}

tc_lcc_status launch_epilogue_directed(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st) {
    if (g->d.n == 0) return TC_LCC_OK;
    k_epilogue_directed<<<grid_for((size_t)g->d.n, 256, 8192), 256, 0, st>>>(
        g->d.n, g->d.order, g->d.dout_r, g->d.t_rank, (unsigned long long*)tri, lcc);
    TCL_HIP(hipGetLastError());
    return TC_LCC_OK;
}

// Per oriented edge e at position e of adj (source rank found by a search of out_off): the key
// (lower original id << bits | higher original id) for the sort into the output order.
template <typename OffT>
__global__ void k_edge_keys(const OffT* __restrict__ out_off, int64_t n, const int32_t* __restrict__ adj, size_t m,
                            const int32_t* __restrict__ order, int bits, uint64_t* __restrict__ keys) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < m; e += (size_t)gridDim.x * blockDim.x) {
        // source rank: the last r with out_off[r] <= e
        int64_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if ((size_t)out_off[mid] <= e) lo = mid;
            else hi = mid;
        }
        const uint32_t x = (uint32_t)order[lo], y = (uint32_t)order[adj[e]];
        const uint64_t a = x < y ? x : y, b = x < y ? y : x;
        keys[e] = (a << bits) | b;
    }
}

__global__ void k_rank_of(const int32_t* __restrict__ order, int64_t n, int32_t* __restrict__ rank) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        rank[order[r]] = (int32_t)r;
}

// Sorted key i = edge {x < y}: its oriented position (the higher rank's place in the lower
// rank's N+, a binary search) and its count.
template <typename OffT>
__global__ void k_edge_out(const uint64_t* __restrict__ keys, size_t m, int bits, const int32_t* __restrict__ rank,
                           const OffT* __restrict__ out_off, const int32_t* __restrict__ adj,
                           const uint32_t* __restrict__ ce, int32_t* __restrict__ es, int32_t* __restrict__ ed,
                           uint32_t* __restrict__ ec) {
    const uint64_t mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        const int32_t x = (int32_t)(k >> bits), y = (int32_t)(k & mask);
        if (es) es[i] = x;
        if (ed) ed[i] = y;
        if (ec) {
            const int32_t rx = rank[x], ry = rank[y];
            const int32_t lo = rx < ry ? rx : ry, hi = rx < ry ? ry : rx;
            OffT a = out_off[lo], b = out_off[lo + 1];
            while (a < b) {
                const OffT mid = a + ((b - a) >> 1);
                if (adj[mid] < hi) a = mid + 1;
                else b = mid;
            }
            ec[i] = ce[a];
        }
    }
}

template <typename OffT>
static hipError_t edge_output_typed(const GraphDev& d, uint64_t* keys, uint64_t* alt, void* scratch,
                                    unsigned int* err, int32_t* rank, const uint32_t* ce, int32_t* es, int32_t* ed,
                                    uint32_t* ec, hipStream_t st) {
    const size_t m = (size_t)d.m;
    const OffT* oo = (const OffT*)d.out_off;
    k_edge_keys<OffT><<<grid_for(m, 256, 16384), 256, 0, st>>>(oo, d.n, d.adj, m, d.order, d.bits, keys);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    uint64_t* sorted = keys;
    e = radix_sort_u64(keys, alt, m, 0, 2 * d.bits, scratch, err, st, &sorted);
    if (e != hipSuccess) return e;
    k_rank_of<<<grid_for((size_t)d.n, 256, 8192), 256, 0, st>>>(d.order, d.n, rank);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_edge_out<OffT><<<grid_for(m, 256, 16384), 256, 0, st>>>(sorted, m, d.bits, rank, oo, d.adj, ce, es, ed, ec);
    return hipGetLastError();
}

hipError_t edge_output(const GraphDev& d, uint64_t* keys, uint64_t* alt, void* scratch, unsigned int* err,
                       int32_t* rank, const uint32_t* ce, int32_t* es, int32_t* ed, uint32_t* ec, hipStream_t st) {
    return d.off_bytes == 4 ? edge_output_typed<int32_t>(d, keys, alt, scratch, err, rank, ce, es, ed, ec, st)
                            : edge_output_typed<int64_t>(d, keys, alt, scratch, err, rank, ce, es, ed, ec, st);
}

}  // namespace tcl
