// Batched path: many graphs counted by one persistent launch.
//
// A batch is a list of device-resident graphs.  Its work items are the active vertices of
// every graph (each graph's own work list, heaviest first), numbered consecutively across the
// batch: first the heavy vertices of all graphs, then the light ones.  A captured HIP graph runs,
// on one stream, a kernel for the heavy items (a block each), one for the light items (a wave
// each), the LCC epilogue over chunks of every
// graph's vertices, and a kernel that raises every graph's done flag.  Workers take items from
// device queues a few at a time, find an item's graph with a wave-wide search over the
// per-graph item offsets, and count the vertex as the single-graph kernel does (rank bitmap of
// N+(v) in LDS where it fits, bucket hash otherwise, HBM search beyond the LDS slice).  The
// grids are sized to the batch's items (a few grid classes), so a small batch does not start
// thousands of waves that only find an empty queue.  The epilogue resets each counter to zero
// after reading it, so the slot's counters are clean for the next batch without a clearing
// pass.  All sizes and pointers are read from device memory that each submission rewrites, so
// a capture does not depend on the batch.  Each context holds a few slots (own stream,
// descriptors, counters and HIP graphs), so batches can overlap on the GPU.
#include <cstring>
#include <set>

#include "batch_device.hpp"

namespace tcl {

constexpr int kBatchSlots = 4;
constexpr int kBatchThreads = 256;
constexpr int kEpiChunk = 4096;  // vertices per epilogue work item
constexpr int kQueueStride = 32;  // queue counters 128 bytes apart, one cache line each
constexpr int kMidGrab = 4;       // mid items per queue access

struct BatchGraph {
    const void* out_off;
    const int32_t* adj;
    const void* in_off;
    const int32_t* in_u;
    const void* in_start;
    const int32_t* in_len;
    const int32_t* vlist;
    const int32_t* order;
    const int32_t* deg_r;
    unsigned long long* t;  // this slot's counters for the graph (n entries)
    unsigned long long* tri;
    double* lcc;
    int64_t n;
    int64_t heavy;      // its heaviest vertices (>= 2^14 probes): vlist[0, heavy), heaviest first
    int64_t mid;        // its other vertices of the block classes: vlist[heavy, heavy + mid)
    int64_t light;      // its vertices of the wave class: vlist[heavy + mid, heavy + mid + light)
    int64_t heavy_base; // first heavy item of the graph in the batch
    int64_t mid_base;   // first mid item of the graph in the batch
    int64_t light_base; // first light item of the graph in the batch
    int64_t chunk_base; // first epilogue chunk of the graph in the batch
    int32_t index;      // position of the graph in the submission (its done flag)
    int32_t nchunks;    // epilogue chunks of the graph
    int32_t pad_chunks;
    uint32_t pad_;
};

struct BatchHeader {
    int32_t count;        // graphs in the batch
    int32_t count4;       // graphs [0, count4) use 4-byte offsets, the rest 8-byte ones
    int64_t heavy4, heavy;  // heavy items of the 4-byte graphs, of all graphs
    int64_t mid4, mid;      // mid items likewise
    int64_t light4, light;  // light items likewise
    uint32_t region;      // LDS bytes per wave
    uint32_t seq;         // submission number, written to the done flags
    unsigned int queue[4];  // [2 * which]: heavy items taken from the queue
    unsigned int mqueue[2][8 * kQueueStride];  // [which][x * kQueueStride]: mid grabs taken from segment x
    unsigned int lqueue[2][8 * kQueueStride];  // [which][x * kQueueStride]: light grabs taken from segment x
    int32_t xcds;         // queue segments of the mid and light items: the GPU's XCDs (at most 8)
    int32_t pad2_;
    int64_t chunks;       // epilogue chunks of all graphs
    int32_t grab;         // light vertices per queue access when there are plenty
    int32_t pad_;
};

template <typename OffT>
__device__ __forceinline__ CountArgs<OffT> batch_args(const BatchGraph& G) {
    CountArgs<OffT> a;
    a.out_off = (const OffT*)G.out_off;
    a.adj = G.adj;
    a.in_off = (const OffT*)G.in_off;
    a.in_u = G.in_u;
    a.in_start = (const OffT*)G.in_start;
    a.in_len = G.in_len;
    a.in_pos = nullptr;
    a.vlist = G.vlist;
    a.n_block = a.n_wave = a.n_global = 0;
    a.t = G.t;
    a.ctr = nullptr;
    a.slots = 0;
    a.merge_x100 = 100;
    return a;
}

// Last graph g in [g_lo, g_hi) whose items of `tier` (wave-uniform) start at or before `item`, found by the whole wave (all lanes active, `item` wave-uniform):
// each round the lanes test 64 evenly spaced graphs of the remaining range at once, so 4096
// graphs take two rounds of one load each instead of twelve dependent loads.  The bases grow
// with g and the first graph's base is at most `item`, so the lanes that pass form a prefix.
constexpr int kTierHeavy = 0, kTierMid = 1, kTierLight = 2;

__device__ __forceinline__ int64_t tier_base(const BatchGraph& G, int tier) {
    return tier == kTierHeavy ? G.heavy_base : tier == kTierMid ? G.mid_base : G.light_base;
}
__device__ __forceinline__ int64_t tier_count(const BatchGraph& G, int tier) {
    return tier == kTierHeavy ? G.heavy : tier == kTierMid ? G.mid : G.light;
}

__device__ __forceinline__ int batch_graph_of_wave(const BatchGraph* __restrict__ gs, int g_lo, int g_hi, int tier,
                                                   int64_t item) {
    const int lane = lane_id();
    int lo = g_lo, hi = g_hi;  // the answer lies in [lo, hi)
    while (hi - lo > 1) {
        const int step = (hi - lo + kWave - 1) / kWave;
        const int gi = lo + lane * step;
        const bool pass = gi < hi && tier_base(gs[gi], tier) <= item;
        const int k = (int)__popcll(__builtin_amdgcn_ballot_w64(pass));
        lo += (k - 1) * step;
        hi = min(hi, lo + step);
    }
    return lo;
}

// Two kernels, the two phases of the single-graph kernel, one after the other in the captured
// graph: the heavy vertices of all graphs (those with at least 2^14 probes), one block each (the
// block's whole LDS is the table), taken one at a time; then all others, one wave each in its
// slice of the LDS, taken several at a time (the tuning's batch_grab) when there are plenty.
// Apart, each kernel is compiled for its own phase only, so the light one keeps fewer registers
// per lane and more waves resident to hide latency.
template <typename OffT>
__global__ __launch_bounds__(kBatchThreads) void k_batch_heavy(const BatchGraph* __restrict__ gs, BatchHeader* h,
                                                               int which) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ int64_t s_item;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint32_t rb = h->region;
    const int g_lo = which ? h->count4 : 0, g_hi = which ? h->count : h->count4;
    // the first item of every block is fixed by its index; only later ones come from the queue
    // counter (atomics on one address serialize)
    const int64_t grid = gridDim.x;
    const int64_t hlo = which ? h->heavy4 : 0, hhi = which ? h->heavy : h->heavy4;
    for (int64_t item = hlo + blockIdx.x;;) {
        if (item >= hhi) break;
        int g = __builtin_amdgcn_readfirstlane(batch_graph_of_wave(gs, g_lo, g_hi, kTierHeavy, item));
        while (item >= gs[g].heavy_base + gs[g].heavy) ++g;  // graphs without heavy vertices
        const BatchGraph& G = gs[g];
        const CountArgs<OffT> a = batch_args<OffT>(G);
        const int32_t v = gld(G.vlist, item - G.heavy_base);
        unsigned long long local = 0;
        process_vertex<OffT, TC_LCC_PROBE_AUTO, kBatchThreads / kWave, true>(a, v, lds, rb * (kBatchThreads / kWave),
                                                                              threadIdx.x, w, local);
        const unsigned long long ws = wave_sum(local);
        if (lane == 0 && ws) gadd(G.t + v, ws);
        if (grid >= hhi - hlo) break;
        if (threadIdx.x == 0) s_item = hlo + grid + (int64_t)atomicAdd(&h->queue[2 * which], 1u);
        __syncthreads();
        item = s_item;
        __syncthreads();
    }

}

// One tier of the wave-per-vertex items (mid or light) of offset class `which`: items
// [lo, hi), taken `grab` at a time.  The items are cut into one contiguous segment per XCD
// (workgroups are dispatched to the XCDs in turn, so block b runs on XCD b mod nx), each with its
// own queue counter in its own cache line.  Consecutive items are vertices of the same few
// graphs, so a graph is mostly counted on one XCD and its lists stay in that XCD's L2 between
// the in-edges that read them; when a wave's own segment is used up it takes grabs from the
// other segments' queues in turn.  The first grab of every wave in its own segment is fixed by
// its index (atomics on one address serialize).  Which wave takes which item changes no count.
template <typename OffT>
__device__ __forceinline__ void wave_tier(const BatchGraph* __restrict__ gs, int g_lo, int g_hi, int tier, int64_t lo,
                                          int64_t hi,
                                          int grab, int nx, unsigned int* queues, uint8_t* region, uint32_t rb,
                                          uint32_t* tcnt) {
    constexpr int kWaves = kBatchThreads / kWave;
    const int w = threadIdx.x / kWave, lane = lane_id();
    const int64_t grid = gridDim.x;
    auto seg_lo = [&](int x) { return lo + (hi - lo) * x / nx; };
    // waves whose first grab lies in segment x: those of the blocks b with b mod nx = x
    auto seg_waves = [&](int x) { return (grid - x + nx - 1) / nx * kWaves; };
    // the next grab of segment x from its queue, or none when the fixed first grabs cover it
    auto from_queue = [&](int x) -> int64_t {
        const int64_t base = seg_lo(x) + seg_waves(x) * grab, end = seg_lo(x + 1);
        if (base >= end) return INT64_MAX;
        unsigned int q = 0;
        if (lane == 0) q = atomicAdd(&queues[x * kQueueStride], 1u);
        q = __shfl(q, 0, kWave);
        return base + (int64_t)q * grab;
    };
    const int x0 = (int)(blockIdx.x % nx);
    int xs = x0, visited = 1;
    int64_t item = seg_lo(x0) + ((int64_t)(blockIdx.x / nx) * kWaves + w) * grab;
    for (;;) {
        const int64_t shi = seg_lo(xs + 1);
        if (item >= shi) {
            // this segment is used up: the next one's queue
            if (visited == nx) break;
            ++visited;
            xs = xs + 1 == nx ? 0 : xs + 1;
            item = from_queue(xs);
            continue;
        }
        const int64_t end = min(item + (int64_t)grab, shi);
        // the grab's vertices with their graphs and list bounds, lane q holding item + q, all
        // loaded at once (a grab has at most 64 vertices)
        int gq = __builtin_amdgcn_readfirstlane(batch_graph_of_wave(gs, g_lo, g_hi, tier, item));
        int32_t hv = 0;
        OffT hb0 = 0, hb1 = 0, hi0 = 0, hi1 = 0;
        if (item + lane < end) {
            const int64_t it = item + lane;
            while (it >= tier_base(gs[gq], tier) + tier_count(gs[gq], tier)) ++gq;  // graphs without such items
            const BatchGraph& GL = gs[gq];
            const OffT* oo = (const OffT*)GL.out_off;
            const OffT* io = (const OffT*)GL.in_off;
            const int64_t first = tier == kTierMid ? GL.heavy : GL.heavy + GL.mid;
            hv = gld(GL.vlist, first + (it - tier_base(GL, tier)));
            hb0 = gld(oo, hv);
            hb1 = gld(oo, hv + 1);
            hi0 = gld(io, hv);
            hi1 = gld(io, hv + 1);
        }
        // a software pipeline over the grab: vertex q + 1's first entries of N+(v) and first
        // in-edges are loaded before vertex q is worked on
        const int nq = (int)(end - item);
        auto head = [&](int q) {
            return VertexHead<OffT>{__builtin_amdgcn_readlane(hv, q), lane_value(hb0, q), lane_value(hb1, q),
                                    lane_value(hi0, q), lane_value(hi1, q)};
        };
        LightPrefetch<OffT> pf = light_prefetch(batch_args<OffT>(gs[__builtin_amdgcn_readlane(gq, 0)]), head(0));
        for (int q = 0; q < nq; ++q) {
            LightPrefetch<OffT> next{0, 0, 0, 0};
            if (q + 1 < nq) next = light_prefetch(batch_args<OffT>(gs[__builtin_amdgcn_readlane(gq, q + 1)]), head(q + 1));
            const BatchGraph& G = gs[__builtin_amdgcn_readlane(gq, q)];
            const VertexHead<OffT> hd = head(q);
            unsigned long long local = 0;
            process_light<OffT>(batch_args<OffT>(G), hd, pf, region, rb, local, tcnt);
            const unsigned long long ws = wave_sum(local);
            if (lane == 0 && ws) gadd(G.t + hd.v, ws);
            pf = next;
        }
        item = from_queue(xs);
    }
}

// All vertices below the heavy threshold, one wave each in its slice of the LDS: first the mid
// items of every graph (the rest of the block classes: more probes than a wave-class vertex),
// a few per queue access, then the light items (the wave class), several per access when there
// are plenty.  Taking the larger items first keeps a grab of large items from ending the kernel
// late; grabs of 64 light items took 13.9 ms instead of 8.5 for the 4096-graph batch.  The
// kernel is bound by the latency of each vertex's few dependent steps, so resident waves matter
// more than registers: seven waves per SIMD (72 VGPRs, a few spilled) beat six (6.8 against 7.1
// ms for that batch) and four (8.3 ms).
template <typename OffT>
__global__ __launch_bounds__(kBatchThreads, 7) void k_batch_light(const BatchGraph* __restrict__ gs, BatchHeader* h,
                                                                  int which) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_tcnt[kBatchThreads];  // per wave: hits of the 64 tails of a chunk
    const int w = threadIdx.x / kWave;
    const uint32_t rb = h->region;
    const int g_lo = which ? h->count4 : 0, g_hi = which ? h->count : h->count4;
    const int64_t grid = gridDim.x;
    const int64_t waves = grid * (kBatchThreads / kWave);
    uint8_t* region = lds + (size_t)w * rb;
    uint32_t* tcnt = s_tcnt + w * kWave;
    const int nx = (int)min<int64_t>(max(h->xcds, 1), min<int64_t>(grid, 8));
    // one copy of the code for both tiers (the loop is not unrolled)
#pragma unroll 1
    for (int tier = kTierMid; tier <= kTierLight; ++tier) {
        const bool m = tier == kTierMid;
        const int64_t lo = m ? (which ? h->mid4 : 0) : (which ? h->light4 : 0);
        const int64_t hi = m ? (which ? h->mid : h->mid4) : (which ? h->light : h->light4);
        // several items per grab when there are plenty per wave (light: four grabs per wave; mid:
        // one), single ones when few (a small batch's latency is its longest wave)
        const int want = m ? kMidGrab : h->grab;
        const int grab = (hi - lo) >= waves * (int64_t)want * (m ? 1 : 4) ? want : 1;
        wave_tier<OffT>(gs, g_lo, g_hi, tier, lo, hi, grab, nx, m ? h->mqueue[which] : h->lqueue[which], region, rb,
                        tcnt);
    }
}

// Eq. 2 per vertex, as the single-graph epilogue, over chunks of kEpiChunk vertices of all
// graphs; each counter is reset to zero once read.
__global__ __launch_bounds__(256) void k_batch_epilogue(const BatchGraph* __restrict__ gs, const BatchHeader* h) {
    const int count = h->count;
    const int64_t chunks = h->chunks;
    for (int64_t c = blockIdx.x; c < chunks; c += gridDim.x) {
        int ga = 0, gb = count - 1;  // last graph with chunk_base <= c
        while (ga < gb) {
            const int mid = (ga + gb + 1) >> 1;
            if (gs[mid].chunk_base <= c) ga = mid;
            else gb = mid - 1;
        }
        const int g = __builtin_amdgcn_readfirstlane(ga);
        const BatchGraph& G = gs[g];
        const int64_t r0 = (c - G.chunk_base) * kEpiChunk;
        const int64_t r1 = min(r0 + (int64_t)kEpiChunk, G.n);
        for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
            const int32_t v = G.order[r];
            const unsigned long long tv = G.t[r];
            G.t[r] = 0ull;
            const int64_t d = G.deg_r[r];
            G.tri[v] = tv;
            if (G.lcc) {
                double x = 0.0;
                if (d >= 2) x = (double)(2ull * tv) / (double)((unsigned long long)d * (unsigned long long)(d - 1));
                G.lcc[v] = x;
            }
        }
    }
}

// The done flags of the batched graphs, after the epilogue kernel has finished (its results are
// then visible on the whole device): a system-wide fence, so that the host sees a flag only
// after what precedes it, then one flag per graph.  One fence per batch instead of one per graph.
__global__ __launch_bounds__(256) void k_batch_flags(const BatchGraph* __restrict__ gs, const BatchHeader* h,
                                                     unsigned int* __restrict__ done) {
    const int count = h->count;
    const unsigned int seq = h->seq;
    __threadfence_system();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        done[gs[i].index] = seq;
}

__global__ void k_batch_clear(unsigned long long* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// Done flag of a graph that ran through the single-graph launches on this stream.
__global__ void k_batch_mark(unsigned int* __restrict__ done, int index, unsigned int seq) {
    if (threadIdx.x == 0) {
        __threadfence_system();
        done[index] = seq;
    }
}

// ------------------------------------------------------------------ host side

namespace {

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    uint64_t ticket = 0;
    uint32_t seq = 0;
    std::vector<tc_lcc_graph> graphs;
    int count = 0;
    // device buffers (from the context pool)
    BatchGraph* d_graphs = nullptr;
    BatchHeader* d_hdr = nullptr;
    unsigned long long* d_scratch = nullptr;
    size_t cap_graphs = 0, cap_scratch = 0;
    // pinned host staging and done flags
    BatchGraph* h_graphs = nullptr;
    BatchHeader* h_hdr = nullptr;
    unsigned int* h_done = nullptr;
    unsigned int* d_done = nullptr;
    size_t cap_done = 0;
    // captured launches, keyed by (region class, which kernels)
    std::map<uint64_t, hipGraphExec_t> execs;
};

hipError_t slot_streams(Slot& s) {
    hipError_t e = hipSuccess;
    if (!s.stream && e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (!s.ev && e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
    return e;
}

struct Engine {
    Slot slots[kBatchSlots];
    uint64_t next_ticket = 1;
    uint32_t next_seq = 1;
    std::mutex mu;
    std::map<uint64_t, int> completed;  // tickets finished before their poll: graphs done
    int32_t xcds = 1;                   // the device's XCDs (light segments of the batched launch)
};

// created with the context (tc_lcc_ctx_create), so no two threads race to create it
Engine* engine(tc_lcc_ctx ctx) { return (Engine*)ctx->batch; }

void drop_execs(Slot& s) {
    for (auto& kv : s.execs) (void)hipGraphExecDestroy(kv.second);
    s.execs.clear();
}

// Device buffers of a free slot (no device work uses its buffers).  Each replacement is
// allocated before the buffer it replaces is released, so a failed allocation leaves the slot
// as it was; every change of a buffer drops the captured launches that point at it.  New
// counters are cleared here, on the slot's stream; after that every batch leaves the counters
// it used at zero (the epilogue resets them).
tc_lcc_status ensure_capacity(tc_lcc_ctx ctx, Slot& s, size_t graphs, size_t flags, size_t scratch) {
    Pool* pool = ctx->pool.get();
    if (flags > s.cap_done) {
        const size_t cap = std::max<size_t>(flags, 2 * s.cap_done);
        unsigned int* h = nullptr;
        unsigned int* dp = nullptr;
        if (hipHostMalloc((void**)&h, cap * sizeof(unsigned int), hipHostMallocMapped) != hipSuccess ||
            hipHostGetDevicePointer((void**)&dp, h, 0) != hipSuccess) {
            (void)hipGetLastError();
            if (h) (void)hipHostFree(h);
            set_error("batch: mapped host allocation failed");
            return TC_LCC_OUT_OF_MEMORY;
        }
        memset(h, 0, cap * sizeof(unsigned int));
        if (s.h_done) (void)hipHostFree(s.h_done);
        s.h_done = h;
        s.d_done = dp;
        s.cap_done = cap;
        drop_execs(s);
    }
    if (graphs > s.cap_graphs) {
        const size_t cap = std::max<size_t>(graphs, 2 * s.cap_graphs);
        void* p = nullptr;
        tc_lcc_status st = pool->alloc(cap * sizeof(BatchGraph), &p);
        if (st != TC_LCC_OK) return st;
        BatchGraph* h = nullptr;
        if (hipHostMalloc((void**)&h, cap * sizeof(BatchGraph), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            pool->release(p);
            set_error("batch: pinned host allocation failed");
            return TC_LCC_OUT_OF_MEMORY;
        }
        if (s.d_graphs) pool->release(s.d_graphs);
        if (s.h_graphs) (void)hipHostFree(s.h_graphs);
        s.d_graphs = (BatchGraph*)p;
        s.h_graphs = h;
        s.cap_graphs = cap;
        drop_execs(s);
    }
    if (!s.d_hdr) {
        void* p = nullptr;
        tc_lcc_status st = pool->alloc(sizeof(BatchHeader), &p);
        if (st != TC_LCC_OK) return st;
        BatchHeader* h = nullptr;
        if (hipHostMalloc((void**)&h, sizeof(BatchHeader), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            pool->release(p);
            set_error("batch: pinned host allocation failed");
            return TC_LCC_OUT_OF_MEMORY;
        }
        s.d_hdr = (BatchHeader*)p;
        s.h_hdr = h;
        drop_execs(s);
    }
    if (scratch > s.cap_scratch) {
        const size_t cap = std::max<size_t>(scratch, s.cap_scratch + s.cap_scratch / 2);
        void* p = nullptr;
        tc_lcc_status st = pool->alloc(cap * sizeof(unsigned long long), &p);
        if (st != TC_LCC_OK) return st;
        k_batch_clear<<<(unsigned)std::min<size_t>((cap + 255) / 256, 4096), 256, 0, s.stream>>>(
            (unsigned long long*)p, cap);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s.stream);
            pool->release(p);
            set_error("batch: clearing new counters failed: %s", hipGetErrorString(e));
            return TC_LCC_DEVICE_ERROR;
        }
        if (s.d_scratch) pool->release(s.d_scratch);
        s.d_scratch = (unsigned long long*)p;
        s.cap_scratch = cap;
        drop_execs(s);
    }
    return TC_LCC_OK;
}

// LDS bytes per wave that every vertex of g fits: the rank bitmap over all n ranks if it
// fits, else the bucket hash for the largest out-list.
uint32_t region_need(const GraphDev& d) {
    const uint32_t words = (uint32_t)((d.n + 31) / 32);
    const uint32_t bm = bitmap_bytes(words, d.max_dplus);
    const uint32_t hs = 8u * (uint32_t)hash_table_slots(d.max_dplus);
    return std::min(bm, hs);
}

// LDS bytes per wave of the batched launch: the smallest class that every batched graph's
// largest table fits, capped at the largest class.  Vertices whose tables do not fit (id
// ranges or out-lists too large for a slice) are searched in HBM by their wave or block.
constexpr uint32_t kRegionClasses[] = {2048, 4096};
constexpr int kNumRegionClasses = (int)(sizeof(kRegionClasses) / sizeof(kRegionClasses[0]));

// Count grids: a batch gets the smallest class with a block per heavy vertex plus a wave per
// light vertex, up to a full GPU of resident blocks.
constexpr unsigned kGridClasses[] = {64, 256, 1024};
constexpr int kNumGridClasses = (int)(sizeof(kGridClasses) / sizeof(kGridClasses[0]));

int grid_class(int64_t heavy, int64_t light) {
    constexpr int64_t per_block = kBatchThreads / kWave;
    const int64_t blocks = heavy + (light + per_block - 1) / per_block;
    for (int c = 0; c < kNumGridClasses; ++c)
        if (blocks <= (int64_t)kGridClasses[c]) return c;
    return kNumGridClasses;  // full GPU
}

tc_lcc_status capture(Slot& s, uint32_t region, bool has4, bool has8, int gclass, int cu_count,
                      hipGraphExec_t* out) {
    const uint64_t key = ((uint64_t)region << 8) | ((uint64_t)gclass << 2) | (has4 ? 1u : 0u) | (has8 ? 2u : 0u);
    auto it = s.execs.find(key);
    if (it != s.execs.end()) {
        *out = it->second;
        return TC_LCC_OK;
    }
    const size_t lds = (size_t)region * (kBatchThreads / kWave);
    // blocks of each kernel: what the GPU holds of it alone, or the grid class of a small batch
    auto grid = [&](const void* kern) -> unsigned {
        int per = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, kBatchThreads, lds) != hipSuccess) {
            (void)hipGetLastError();
            per = 1;
        }
        unsigned gsz = (unsigned)(cu_count * std::max(per, 1));
        if (gclass < kNumGridClasses) gsz = std::min(gsz, kGridClasses[gclass]);
        return gsz;
    };
    const unsigned h4 = grid((const void*)k_batch_heavy<int32_t>), l4 = grid((const void*)k_batch_light<int32_t>);
    const unsigned h8 = grid((const void*)k_batch_heavy<int64_t>), l8 = grid((const void*)k_batch_light<int64_t>);
    const unsigned ge = std::min(std::max(l4, l8), 1024u);
    hipGraph_t graph = nullptr;
    TCL_HIP(hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal));
    // heavy vertices first, each kernel with the whole GPU (heaviest first, so the heavy phase
    // ends on short items), then the light ones
    if (has4) k_batch_heavy<int32_t><<<h4, kBatchThreads, lds, s.stream>>>(s.d_graphs, s.d_hdr, 0);
    if (has8) k_batch_heavy<int64_t><<<h8, kBatchThreads, lds, s.stream>>>(s.d_graphs, s.d_hdr, 1);
    if (has4) k_batch_light<int32_t><<<l4, kBatchThreads, lds, s.stream>>>(s.d_graphs, s.d_hdr, 0);
    if (has8) k_batch_light<int64_t><<<l8, kBatchThreads, lds, s.stream>>>(s.d_graphs, s.d_hdr, 1);
    k_batch_epilogue<<<ge, 256, 0, s.stream>>>(s.d_graphs, s.d_hdr);
    k_batch_flags<<<1, 256, 0, s.stream>>>(s.d_graphs, s.d_hdr, s.d_done);
    hipError_t e = hipStreamEndCapture(s.stream, &graph);
    if (e != hipSuccess) {
        set_error("batch: stream capture failed: %s", hipGetErrorString(e));
        return TC_LCC_DEVICE_ERROR;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        set_error("batch: graph instantiation failed: %s", hipGetErrorString(e));
        return TC_LCC_DEVICE_ERROR;
    }
    s.execs[key] = exec;
    *out = exec;
    return TC_LCC_OK;
}

void finish_slot(Slot& s) {
    for (tc_lcc_graph g : s.graphs) g->inflight--;
    s.graphs.clear();
    s.busy = false;
}

}  // namespace

tc_lcc_status batch_engine_create(tc_lcc_ctx ctx) {
    Engine* e = new (std::nothrow) Engine();
    if (!e) {
        set_error("batch: engine allocation failed");
        return TC_LCC_OUT_OF_MEMORY;
    }
    int xcc = 1;
    if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, ctx->pool->device()) != hipSuccess) {
        (void)hipGetLastError();
        xcc = 1;
    }
    e->xcds = std::min(std::max(xcc, 1), 8);
    ctx->batch = e;
    return TC_LCC_OK;
}

std::mutex& batch_mutex(tc_lcc_ctx ctx) { return engine(ctx)->mu; }

tc_lcc_status batch_fence_graph(tc_lcc_ctx ctx, tc_lcc_graph g, hipStream_t st) {
    Engine* e = engine(ctx);
    for (Slot& s : e->slots) {
        if (!s.busy || s.stream == st) continue;
        for (tc_lcc_graph x : s.graphs)
            if (x == g) {
                TCL_HIP(hipStreamWaitEvent(st, s.ev, 0));
                break;
            }
    }
    return TC_LCC_OK;
}

void batch_engine_destroy(tc_lcc_ctx ctx) {
    if (!ctx->batch) return;
    Engine* e = (Engine*)ctx->batch;
    for (Slot& s : e->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        drop_execs(s);
        if (s.d_graphs) ctx->pool->release(s.d_graphs);
        if (s.d_hdr) ctx->pool->release(s.d_hdr);
        if (s.d_scratch) ctx->pool->release(s.d_scratch);
        if (s.h_graphs) (void)hipHostFree(s.h_graphs);
        if (s.h_hdr) (void)hipHostFree(s.h_hdr);
        if (s.h_done) (void)hipHostFree(s.h_done);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    delete e;
    ctx->batch = nullptr;
}

}  // namespace tcl

using namespace tcl;

namespace {

// What a submission needs of a graph's schedule, read under the graph's lock (a tc_lcc_run
// after a tuning change may rebuild the schedule; it first waits for the batches that hold
// the graph, and it cannot start while a submission holds the engine's lock).
struct Plan {
    int64_t heavy = 0, mid = 0, light = 0;
    bool solo = false;
};

}  // namespace

// A graph that takes the single-graph launches: directed, compact reverse lists, lists beyond a
// block's hash, or enough work to fill the GPU alone (the single-graph kernel's wave slices and
// block tables are larger than a batched slice, so fewer of its vertices search HBM; a batch
// pays only for graphs too small to fill the GPU).
constexpr uint64_t kSoloWedges = 1ull << 25;

static bool solo_graph(const GraphDev& d) {
    return d.directed || d.compact || d.n_global > 0 || d.n_list > 0 || d.wedges >= kSoloWedges;
}

bool tcl::batch_graph_solo(tc_lcc_graph g) {
    std::lock_guard<std::mutex> gl(g->mu);
    return solo_graph(g->d);
}

tc_lcc_status tcl::batch_reserve(tc_lcc_ctx ctx, size_t graphs) {
    TCL_HIP(hipSetDevice(ctx->device));
    Engine* e = engine(ctx);
    std::lock_guard<std::mutex> lk(e->mu);
    for (Slot& s : e->slots) {
        if (s.busy) continue;
        TCL_HIP(slot_streams(s));
        tc_lcc_status st = ensure_capacity(ctx, s, std::max<size_t>(graphs, 1), std::max<size_t>(graphs, 1), 1);
        if (st != TC_LCC_OK) return st;
    }
    return TC_LCC_OK;
}

tc_lcc_status tcl::batch_submit_with(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs, uint64_t* const* tri,
                                     double* const* lcc, unsigned long long* const* scratch, tc_lcc_ticket* out) {
    if (!ctx || count <= 0 || !graphs || !tri || !out) {
        set_error("tc_lcc_batch_submit: null argument or count <= 0");
        return TC_LCC_INVALID_ARGUMENT;
    }
    for (int i = 0; i < count; ++i) {
        if (!graphs[i] || graphs[i]->ctx != ctx || !tri[i]) {
            set_error("tc_lcc_batch_submit: graph %d is null, from another context, or has no output", i);
            return TC_LCC_INVALID_ARGUMENT;
        }
    }
    TCL_HIP(hipSetDevice(ctx->device));
    int grab = 16, heavy_bits = kBigWorkBits;
    {
        std::lock_guard<std::mutex> tl(ctx->mu);
        if (ctx->tuning.batch_grab > 0) grab = std::min(ctx->tuning.batch_grab, kWave);  // a lane per vertex of a grab
        if (ctx->tuning.batch_heavy_bits > 0) heavy_bits = ctx->tuning.batch_heavy_bits;
    }
    Engine* e = engine(ctx);
    // the engine's lock is held for the whole submission (lock order: engine, then graph)
    std::unique_lock<std::mutex> lk(e->mu);
    // a free slot; if all are busy, wait for the oldest submission
    Slot* s = nullptr;
    for (Slot& c : e->slots)
        if (!c.busy) {
            s = &c;
            break;
        }
    if (!s) {
        Slot* oldest = &e->slots[0];
        for (Slot& c : e->slots)
            if (c.ticket < oldest->ticket) oldest = &c;
        TCL_HIP(hipEventSynchronize(oldest->ev));
        e->completed[oldest->ticket] = oldest->count;
        finish_slot(*oldest);
        ctx->tickets_inflight--;
        s = oldest;
    }
    TCL_HIP(slot_streams(*s));

    // order: 4-byte-offset graphs first, then 8-byte ones; directed graphs and graphs with lists
    // longer than the single-graph launch's hash (which that launch takes as a sorted list in
    // its larger table) run through the single-graph launches instead.  Vertices of batched
    // graphs whose tables do not fit their slice are searched in HBM inside the batch.
    std::vector<Plan> plan((size_t)count);
    std::vector<int> ord4, ord8, solo;
    uint32_t need = 0;
    size_t need_scratch = 0;
    for (int i = 0; i < count; ++i) {
        tc_lcc_graph g = graphs[i];
        std::lock_guard<std::mutex> gl(g->mu);
        const GraphDev& d = g->d;
        const uint32_t r = region_need(d);
        Plan& p = plan[(size_t)i];
        if (solo_graph(d)) {
            p.solo = true;
            solo.push_back(i);
            continue;
        }
        // heavy: the leading work classes, those with >= 2^(heavy_bits - 1) probes
        int64_t big = 0;
        for (int c = 0; c <= 40 - heavy_bits && c < 48; ++c) big += d.class_count[c];
        p.heavy = big;
        p.mid = d.n_block - big;
        p.light = d.n_wave;
        need = std::max(need, std::min(r, kRegionClasses[kNumRegionClasses - 1]));
        need_scratch += (size_t)d.n;
        (d.off_bytes == 4 ? ord4 : ord8).push_back(i);
    }
    uint32_t region = kRegionClasses[kNumRegionClasses - 1];
    for (uint32_t c : kRegionClasses)
        if (need <= c) {
            region = c;
            break;
        }
    // the single-graph launches run after the batched kernel, smallest graph first, so
    // the earliest done flags come as soon as possible
    std::stable_sort(solo.begin(), solo.end(), [&](int a, int b) { return graphs[a]->d.wedges < graphs[b]->d.wedges; });
    const int nb = (int)(ord4.size() + ord8.size());
    // with counters given by the caller (each graph's own, all zero) the slot's are not used
    tc_lcc_status st = ensure_capacity(ctx, *s, (size_t)std::max(nb, 1), (size_t)count,
                                       scratch ? 1 : std::max<size_t>(need_scratch, 1));
    if (st != TC_LCC_OK) return st;

    // reserve the slot before anything is launched on it: from here on the graphs count as
    // in flight, and an error after a launch waits for the slot's stream before it returns
    const uint32_t seq = e->next_seq++;
    s->busy = true;
    s->seq = seq;
    s->count = count;
    s->ticket = e->next_ticket++;
    s->graphs.assign(graphs, graphs + count);
    for (int i = 0; i < count; ++i) graphs[i]->inflight++;
    ctx->tickets_inflight++;
    auto fail = [&](tc_lcc_status why) {
        (void)hipStreamSynchronize(s->stream);
        (void)hipGetLastError();
        finish_slot(*s);
        ctx->tickets_inflight--;
        return why;
    };

    int64_t heavy = 0, mid = 0, light = 0, heavy4 = 0, mid4 = 0, light4 = 0, chunk = 0;
    size_t soff = 0;
    int k = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i : (pass == 0 ? ord4 : ord8)) {
            const GraphDev& d = graphs[i]->d;
            const Plan& p = plan[(size_t)i];
            BatchGraph& b = s->h_graphs[k++];
            b.out_off = d.out_off;
            b.adj = d.adj;
            b.in_off = d.in_off;
            b.in_u = d.in_u;
            b.in_start = d.in_start;
            b.in_len = d.in_len;
            b.vlist = d.vlist;
            b.order = d.order;
            b.deg_r = d.deg_r;
            b.t = scratch ? scratch[i] : s->d_scratch + soff;
            b.tri = (unsigned long long*)tri[i];
            b.lcc = lcc ? lcc[i] : nullptr;
            b.n = d.n;
            b.heavy = p.heavy;
            b.mid = p.mid;
            b.light = p.light;
            b.heavy_base = heavy;
            b.mid_base = mid;
            b.light_base = light;
            b.chunk_base = chunk;
            b.index = i;
            b.nchunks = (int32_t)std::max<int64_t>(1, (d.n + kEpiChunk - 1) / kEpiChunk);  // an empty graph still gets its flag
            b.pad_chunks = 0;
            b.pad_ = 0;
            heavy += b.heavy;
            mid += b.mid;
            light += b.light;
            chunk += b.nchunks;
            soff += (size_t)d.n;
        }
        if (pass == 0) {
            heavy4 = heavy;
            mid4 = mid;
            light4 = light;
        }
    }
    s->h_hdr->count = nb;
    s->h_hdr->count4 = (int32_t)ord4.size();
    s->h_hdr->heavy4 = heavy4;
    s->h_hdr->heavy = heavy;
    s->h_hdr->mid4 = mid4;
    s->h_hdr->mid = mid;
    s->h_hdr->light4 = light4;
    s->h_hdr->light = light;
    s->h_hdr->region = region;
    s->h_hdr->seq = seq;
    for (unsigned int& q : s->h_hdr->queue) q = 0;
    for (auto& row : s->h_hdr->mqueue)
        for (unsigned int& q : row) q = 0;
    for (auto& row : s->h_hdr->lqueue)
        for (unsigned int& q : row) q = 0;
    s->h_hdr->xcds = e->xcds;
    s->h_hdr->pad2_ = 0;
    s->h_hdr->chunks = chunk;
    s->h_hdr->grab = grab;
    s->h_hdr->pad_ = 0;

    if (nb > 0) {
        hipGraphExec_t exec = nullptr;
        st = capture(*s, region, !ord4.empty(), !ord8.empty(), grid_class(heavy, mid + light), ctx->cu_count, &exec);
        if (st != TC_LCC_OK) return fail(st);
        if (hipMemcpyAsync(s->d_graphs, s->h_graphs, (size_t)nb * sizeof(BatchGraph), hipMemcpyHostToDevice,
                           s->stream) != hipSuccess ||
            hipMemcpyAsync(s->d_hdr, s->h_hdr, sizeof(BatchHeader), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
            hipGraphLaunch(exec, s->stream) != hipSuccess) {
            set_error("tc_lcc_batch_submit: launch failed: %s", hipGetErrorString(hipGetLastError()));
            return fail(TC_LCC_DEVICE_ERROR);
        }
    }
    // graphs beyond the batched launch's LDS slices: the single-graph launches, on this slot's
    // stream, leaving one block slot per CU free so that other slots' batches keep running
    for (int i : solo) {
        st = run_graph(graphs[i], tri[i], lcc ? lcc[i] : nullptr, s->stream, 1, true);
        if (st != TC_LCC_OK) return fail(st);
        k_batch_mark<<<1, 64, 0, s->stream>>>(s->d_done, i, seq);
        if (hipGetLastError() != hipSuccess) {
            set_error("tc_lcc_batch_submit: flag launch failed");
            return fail(TC_LCC_DEVICE_ERROR);
        }
    }
    if (hipEventRecord(s->ev, s->stream) != hipSuccess) {
        set_error("tc_lcc_batch_submit: event record failed");
        return fail(TC_LCC_DEVICE_ERROR);
    }
    *out = s->ticket;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_batch_submit(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs,
                                             uint64_t* const* tri, double* const* lcc, tc_lcc_ticket* out) {
    return batch_submit_with(ctx, count, graphs, tri, lcc, nullptr, out);
}

extern "C" tc_lcc_status tc_lcc_batch_poll(tc_lcc_ctx ctx, tc_lcc_ticket t, int block, int* graphs_done) {
    if (!ctx) {
        set_error("tc_lcc_batch_poll: null context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (!ctx->batch) {
        set_error("tc_lcc_batch_poll: unknown ticket %llu", (unsigned long long)t);
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(ctx->device));
    Engine* e = (Engine*)ctx->batch;
    std::lock_guard<std::mutex> lk(e->mu);
    auto done_it = e->completed.find(t);
    if (done_it != e->completed.end()) {
        if (graphs_done) *graphs_done = done_it->second;
        e->completed.erase(done_it);
        return TC_LCC_OK;
    }
    for (Slot& s : e->slots) {
        if (!s.busy || s.ticket != t) continue;
        hipError_t q = block ? hipEventSynchronize(s.ev) : hipEventQuery(s.ev);
        if (q == hipErrorNotReady) {
            if (graphs_done) {
                int c = 0;
                const int nb = (int)std::min<size_t>(s.cap_done, (size_t)s.count);
                for (int i = 0; i < nb; ++i) c += (__atomic_load_n(&s.h_done[i], __ATOMIC_ACQUIRE) == s.seq);
                *graphs_done = c;
            }
            return TC_LCC_NOT_READY;
        }
        if (q != hipSuccess) {
            set_error("tc_lcc_batch_poll: %s", hipGetErrorString(q));
            return TC_LCC_DEVICE_ERROR;
        }
        if (graphs_done) *graphs_done = s.count;
        finish_slot(s);
        ctx->tickets_inflight--;
        return TC_LCC_OK;
    }
    set_error("tc_lcc_batch_poll: unknown ticket %llu", (unsigned long long)t);
    return TC_LCC_INVALID_ARGUMENT;
}

extern "C" tc_lcc_status tc_lcc_batch_progress(tc_lcc_ctx ctx, tc_lcc_ticket t, int count, uint8_t* done) {
    if (!ctx || count < 0 || (count > 0 && !done)) {
        set_error("tc_lcc_batch_progress: null argument or negative count");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (!ctx->batch) {
        set_error("tc_lcc_batch_progress: unknown ticket %llu", (unsigned long long)t);
        return TC_LCC_INVALID_ARGUMENT;
    }
    Engine* e = (Engine*)ctx->batch;
    std::lock_guard<std::mutex> lk(e->mu);
    auto done_it = e->completed.find(t);
    if (done_it != e->completed.end()) {
        if (count != done_it->second) {
            set_error("tc_lcc_batch_progress: ticket has %d graphs, not %d", done_it->second, count);
            return TC_LCC_INVALID_ARGUMENT;
        }
        memset(done, 1, (size_t)count);
        return TC_LCC_OK;
    }
    for (Slot& s : e->slots) {
        if (!s.busy || s.ticket != t) continue;
        if (count != s.count) {
            set_error("tc_lcc_batch_progress: ticket has %d graphs, not %d", s.count, count);
            return TC_LCC_INVALID_ARGUMENT;
        }
        for (int i = 0; i < count; ++i) done[i] = __atomic_load_n(&s.h_done[i], __ATOMIC_ACQUIRE) == s.seq;
        return TC_LCC_OK;
    }
    set_error("tc_lcc_batch_progress: unknown ticket %llu", (unsigned long long)t);
    return TC_LCC_INVALID_ARGUMENT;
}
