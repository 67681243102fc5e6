// Graph builder (CSR with sorted, deduplicated, loop-free lists; Sec. II-A/II-B) and
// the degree-binned schedule of the count kernels.
//
//   raw pairs --(canonical 64-bit keys, loops marked)--> radix sort --> unique + degrees
//   --> rank vertices by (degree, id) --> relabel + orient every edge low rank -> high rank
//   --> radix sort --> oriented CSR N+(r) in rank space (lists ascending)
//   --> reverse lists: for every v, the in-edges (u -> v) whose tail N+(u) after v is nonempty
//   --> per-vertex probe counts ("work") --> bins for the count kernels.
//
// Ranking by (degree, id) orients each edge towards the higher-degree end, so
// |N+(r)| <= sqrt(2m), and relabelling by rank keeps every list sorted by rank: the
// entries of N+(u) after v are exactly the candidates w > v that close a triangle
// (u, v, w), the rank-space form of the upper-triangle offset of Sec. II-C.
#include "internal.hpp"
#include "scan.hpp"

namespace tcl {

constexpr int kB = 256;

__global__ void k_make_keys(const int32_t* __restrict__ src, const int32_t* __restrict__ dst, size_t m_in,
                            int64_t n, int bits, uint64_t* __restrict__ keys, int* __restrict__ bad) {
    const uint64_t loop = (1ull << (2 * bits)) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m_in; i += (size_t)gridDim.x * blockDim.x) {
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

__global__ void k_compact_unique(const uint64_t* __restrict__ k, size_t n, int bits,
                                 const uint32_t* __restrict__ pos, uint64_t* __restrict__ out,
                                 int32_t* __restrict__ deg) {
    const uint64_t loop = (1ull << (2 * bits)) - 1, mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t x = k[i];
        if (x != loop && (i == 0 || k[i - 1] != x)) {
            out[pos[i]] = x;
            atomicAdd(&deg[x >> bits], 1);
            atomicAdd(&deg[x & mask], 1);
        }
    }
}

__global__ void k_rank_keys(const int32_t* __restrict__ deg, int64_t n, int bits, uint64_t* __restrict__ rk) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        rk[v] = ((uint64_t)(uint32_t)deg[v] << bits) | (uint64_t)v;
}

__global__ void k_rank_scatter(const uint64_t* __restrict__ rk, int64_t n, int bits, int32_t* __restrict__ order,
                               int32_t* __restrict__ rank, int32_t* __restrict__ deg_r) {
    const uint64_t mask = (1ull << bits) - 1;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = rk[r];
        const int32_t v = (int32_t)(x & mask);
        order[r] = v;
        rank[v] = (int32_t)r;
        deg_r[r] = (int32_t)(x >> bits);
    }
}

__global__ void k_relabel(const uint64_t* __restrict__ uk, size_t m, int bits, const int32_t* __restrict__ rank,
                          uint64_t* __restrict__ ok, int32_t* __restrict__ dplus) {
    const uint64_t mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t x = uk[i];
        const uint32_t ra = (uint32_t)rank[x >> bits], rb = (uint32_t)rank[x & mask];
        const uint32_t lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
        ok[i] = ((uint64_t)lo << bits) | hi;
        atomicAdd(&dplus[lo], 1);
    }
}

template <typename OffT>
struct I32In {
    const int32_t* p;
    int64_t n;
    __device__ OffT operator()(size_t i) const { return (int64_t)i < n ? (OffT)p[i] : OffT(0); }
};

__global__ void k_split_adj(const uint64_t* __restrict__ ok, size_t m, int bits, int32_t* __restrict__ adj) {
    const uint64_t mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x)
        adj[i] = (int32_t)(ok[i] & mask);
}

// in-edge (u -> v) at position i of N+(u): its tail is adj[i+1 .. out_off[u+1]).  Keep it if
// the tail is nonempty and N+(v) is nonempty (otherwise no triangle can use it).
template <typename OffT>
__global__ void k_in_count(const uint64_t* __restrict__ ok, size_t m, int bits, const OffT* __restrict__ out_off,
                           const int32_t* __restrict__ dplus, int32_t* __restrict__ din,
                           unsigned long long* __restrict__ work) {
    const uint64_t mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t x = ok[i];
        const int64_t u = (int64_t)(x >> bits), v = (int64_t)(x & mask);
        const int64_t len = (int64_t)out_off[u + 1] - (int64_t)i - 1;
        if (len > 0 && dplus[v] > 0) {
            atomicAdd(&din[v], 1);
            atomicAdd(&work[v], (unsigned long long)len);
        }
    }
}

template <typename OffT>
__global__ void k_in_fill(const uint64_t* __restrict__ ok, size_t m, int bits, const OffT* __restrict__ out_off,
                          const int32_t* __restrict__ dplus, const OffT* __restrict__ in_off,
                          int32_t* __restrict__ cursor, int32_t* __restrict__ in_u, OffT* __restrict__ in_start,
                          int32_t* __restrict__ in_len) {
    const uint64_t mask = (1ull << bits) - 1;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < m; i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t x = ok[i];
        const int64_t u = (int64_t)(x >> bits), v = (int64_t)(x & mask);
        const int64_t len = (int64_t)out_off[u + 1] - (int64_t)i - 1;
        if (len > 0 && dplus[v] > 0) {
            const OffT p = in_off[v] + (OffT)atomicAdd(&cursor[v], 1);
            in_u[p] = (int32_t)u;
            in_start[p] = (OffT)(i + 1);
            in_len[p] = (int32_t)len;
        }
    }
}

// stats[0] = max |N+|, stats[1] = max degree, stats[2] = sum of work (wedges),
// stats[3] = sum of |N+(v)| over vertices with work (entries staged in LDS)
__global__ void k_stats(const int32_t* __restrict__ dplus, const int32_t* __restrict__ deg_r,
                        const unsigned long long* __restrict__ work, int64_t n, unsigned long long* stats) {
    __shared__ unsigned long long s[4][kB / kWave];
    unsigned long long a = 0, b = 0, c = 0, e = 0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long wr = work[r];
        a = max(a, (unsigned long long)dplus[r]);
        b = max(b, (unsigned long long)deg_r[r]);
        c += wr;
        if (wr) e += (unsigned long long)dplus[r];
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        a = max(a, (unsigned long long)__shfl_xor(a, d, kWave));
        b = max(b, (unsigned long long)__shfl_xor(b, d, kWave));
        c += __shfl_xor(c, d, kWave);
        e += __shfl_xor(e, d, kWave);
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
        s[0][w] = a;
        s[1][w] = b;
        s[2][w] = c;
        s[3][w] = e;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = 0;
        b = 0;
        c = 0;
        e = 0;
        for (int i = 0; i < kB / kWave; ++i) {
            a = max(a, s[0][i]);
            b = max(b, s[1][i]);
            c += s[2][i];
            e += s[3][i];
        }
        atomicMax(&stats[0], a);
        atomicMax(&stats[1], b);
        atomicAdd(&stats[2], c);
        atomicAdd(&stats[3], e);
    }
}

template <typename T>
__global__ void k_fill(T* p, size_t n, T v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, size_t n, T v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    k_fill<T><<<grid_for(n, kB, 4096), kB, 0, st>>>(p, n, v);
    return hipGetLastError();
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

template <typename OffT>
tc_lcc_status build_typed(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                          int on_device, hipStream_t st, tc_lcc_graph g) {
    GraphDev& d = g->d;
    Temps tmp{ctx->pool.get(), {}};
    const int bits = std::max(1, ceil_log2((uint64_t)n));
    d.n = n;
    d.bits = bits;
    const size_t M = (size_t)m_in;

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

    const size_t K = std::max<size_t>({M, (size_t)n, 1});
    uint64_t *ka, *kb;
    uint32_t* pos;
    void* sort_scratch;
    TCL_TRY(tmp.get(K, &ka));
    TCL_TRY(tmp.get(K, &kb));
    TCL_TRY(tmp.get(M + 1, &pos));
    TCL_TRY(tmp.get(radix_sort_scratch_bytes(K) + sizeof(uint32_t) * scan_scratch_elems(K + 1) * 2 + 1024,
                    (uint8_t**)&sort_scratch));
    int* bad;
    TCL_TRY(tmp.get(16, &bad));
    TCL_HIP(fill<int>(bad, 16, 0, st));

    int32_t* deg;
    TCL_TRY(tmp.get((size_t)n, &deg));
    TCL_HIP(fill<int32_t>(deg, (size_t)n, 0, st));

    mark(d, 0, st);
    // 1. canonical keys, sort, unique, degrees
    uint64_t* sorted = ka;
    uint64_t* ukeys = kb;
    uint32_t m32 = 0;
    if (M > 0) {
        k_make_keys<<<grid_for(M, kB, 8192), kB, 0, st>>>(s_dev, d_dev, M, n, bits, ka, bad);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(ka, kb, M, 2 * bits, sort_scratch, st, &sorted));
        ukeys = (sorted == ka) ? kb : ka;
        uint32_t* sscr = (uint32_t*)((uint8_t*)sort_scratch + radix_sort_scratch_bytes(K));
        TCL_HIP(exclusive_scan<uint32_t>(UniqueFlag{sorted, M, (1ull << (2 * bits)) - 1}, M + 1, pos, sscr, st));
        k_compact_unique<<<grid_for(M, kB, 8192), kB, 0, st>>>(sorted, M, bits, pos, ukeys, deg);
        TCL_HIP(hipGetLastError());
        int hb = 0;
        TCL_HIP(hipMemcpyAsync(&m32, pos + M, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
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

    mark(d, 1, st);
    // 2. rank by (degree, id)
    int32_t* rank;
    TCL_TRY(tmp.get((size_t)n, &rank));
    TCL_TRY(keep(g, (size_t)n, &d.order));
    TCL_TRY(keep(g, (size_t)n, &d.deg_r));
    {
        uint64_t *rk, *rk2, *rs;
        TCL_TRY(tmp.get((size_t)n, &rk));
        TCL_TRY(tmp.get((size_t)n, &rk2));
        k_rank_keys<<<grid_for(n, kB, 8192), kB, 0, st>>>(deg, n, bits, rk);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(rk, rk2, (size_t)n, 2 * bits, sort_scratch, st, &rs));
        k_rank_scatter<<<grid_for(n, kB, 8192), kB, 0, st>>>(rs, n, bits, d.order, rank, d.deg_r);
        TCL_HIP(hipGetLastError());
    }

    mark(d, 2, st);
    // 3. relabel + orient, sort, oriented CSR
    TCL_TRY(keep(g, (size_t)n, &d.dplus));
    TCL_HIP(fill<int32_t>(d.dplus, (size_t)n, 0, st));
    uint64_t* okeys = sorted;  // reuse the buffer that held the raw sorted keys
    uint64_t* osorted = okeys;
    OffT* out_off;
    TCL_TRY(keep(g, (size_t)n + 1, &out_off));
    d.out_off = out_off;
    TCL_TRY(keep(g, std::max<size_t>(m, 1), &d.adj));
    uint32_t* sscr = (uint32_t*)((uint8_t*)sort_scratch + radix_sort_scratch_bytes(K));
    OffT* scan_scr = (OffT*)sscr;
    if (m > 0) {
        k_relabel<<<grid_for(m, kB, 8192), kB, 0, st>>>(ukeys, m, bits, rank, okeys, d.dplus);
        TCL_HIP(hipGetLastError());
        TCL_HIP(radix_sort_u64(okeys, ukeys, m, 2 * bits, sort_scratch, st, &osorted));
    }
    TCL_HIP(exclusive_scan<OffT>(I32In<OffT>{d.dplus, n}, (size_t)n + 1, out_off, scan_scr, st));
    if (m > 0) {
        k_split_adj<<<grid_for(m, kB, 8192), kB, 0, st>>>(osorted, m, bits, d.adj);
        TCL_HIP(hipGetLastError());
    }

    mark(d, 3, st);
    // 4. reverse lists with nonempty tails, and per-vertex work
    int32_t* din;
    TCL_TRY(tmp.get((size_t)n, &din));
    TCL_HIP(fill<int32_t>(din, (size_t)n, 0, st));
    TCL_TRY(keep(g, (size_t)n, &d.work));
    TCL_HIP(fill<uint64_t>(d.work, (size_t)n, 0, st));
    if (m > 0) {
        k_in_count<OffT><<<grid_for(m, kB, 8192), kB, 0, st>>>(osorted, m, bits, out_off, d.dplus, din,
                                                               (unsigned long long*)d.work);
        TCL_HIP(hipGetLastError());
    }
    OffT* in_off;
    TCL_TRY(keep(g, (size_t)n + 1, &in_off));
    d.in_off = in_off;
    TCL_HIP(exclusive_scan<OffT>(I32In<OffT>{din, n}, (size_t)n + 1, in_off, scan_scr, st));
    OffT kept = 0;
    TCL_HIP(hipMemcpyAsync(&kept, in_off + n, sizeof(OffT), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    d.m_in_kept = (int64_t)kept;
    const size_t KE = std::max<size_t>((size_t)kept, 1);
    TCL_TRY(keep(g, KE, &d.in_u));
    OffT* in_start;
    TCL_TRY(keep(g, KE, &in_start));
    d.in_start = in_start;
    TCL_TRY(keep(g, KE, &d.in_len));
    if (m > 0) {
        TCL_HIP(fill<int32_t>(din, (size_t)n, 0, st));
        k_in_fill<OffT><<<grid_for(m, kB, 8192), kB, 0, st>>>(osorted, m, bits, out_off, d.dplus, in_off, din,
                                                              d.in_u, in_start, d.in_len);
        TCL_HIP(hipGetLastError());
    }

    mark(d, 4, st);
    // 5. run scratch and statistics
    TCL_TRY(keep(g, (size_t)n, &d.t_rank));
    TCL_TRY(keep(g, 64, &d.counters));
    TCL_TRY(keep(g, (size_t)n, &d.vlist));
    unsigned long long* stats;
    TCL_TRY(tmp.get(4, &stats));
    TCL_HIP(fill<unsigned long long>(stats, 4, 0ull, st));
    k_stats<<<grid_for(n, kB, 2048), kB, 0, st>>>(d.dplus, d.deg_r, (const unsigned long long*)d.work, n, stats);
    TCL_HIP(hipGetLastError());
    unsigned long long hs[4] = {0, 0, 0, 0};
    TCL_HIP(hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    d.max_dplus = (int32_t)hs[0];
    d.max_deg = (int64_t)hs[1];
    d.wedges = hs[2];
    d.staged = hs[3];
    return TC_LCC_OK;
}

}  // namespace

tc_lcc_status build_graph(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                          int on_device, int offset_bytes, hipStream_t st, tc_lcc_graph g) {
    // offsets index the m oriented edges; m <= m_in, so 4 bytes suffice when m_in < 2^31
    int ob = offset_bytes;
    if (ob == 0) ob = (m_in < (1ll << 31)) ? 4 : 8;
    g->d.off_bytes = ob;
    tc_lcc_status s = (ob == 4) ? build_typed<int32_t>(ctx, n, m_in, src, dst, on_device, st, g)
                                : build_typed<int64_t>(ctx, n, m_in, src, dst, on_device, st, g);
    if (s != TC_LCC_OK) return s;
    s = build_schedule(g, ctx->tuning, st);
    mark(g->d, 5, st);
    return s;
}

// ------------------------------------------------------------------ schedule (degree/work bins)

constexpr int kClassWave = 48, kClassGlobal = 50, kClassNone = 63;

__global__ void k_classify(const unsigned long long* __restrict__ work, const int32_t* __restrict__ dplus,
                           int64_t n, int bits, int64_t wave_work_max, int32_t wave_cap, int32_t block_cap,
                           int group, uint64_t* __restrict__ keys, unsigned long long* __restrict__ counts) {
    __shared__ unsigned int c[64];
    for (int i = threadIdx.x; i < 64; i += blockDim.x) c[i] = 0;
    __syncthreads();
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long w = work[v];
        const int32_t dp = dplus[v];
        int cls;
        if (w == 0) {
            cls = kClassNone;
        } else if (dp > block_cap) {
            cls = kClassGlobal;
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

// LDS slots of one block's table: hash tables get twice the list length (load <= 1/2).
int32_t table_slots(int probe, int32_t dplus_max) {
    int32_t need = probe == TC_LCC_PROBE_SORTED ? dplus_max : 2 * dplus_max;
    int32_t s = 256;
    while (s < need && s < kMaxTableSlots) s <<= 1;
    return s;
}

tc_lcc_status build_schedule(tc_lcc_graph g, const tc_lcc_tuning& tn, hipStream_t st) {
    GraphDev& d = g->d;
    const int probe = resolve_probe(tn.probe, d.n);
    d.hash_slots = table_slots(probe, d.max_dplus);
    const int32_t per_entry = probe == TC_LCC_PROBE_SORTED ? 1 : 2;
    const int32_t block_cap = d.hash_slots / per_entry;
    const int32_t wave_cap = (d.hash_slots / kWavesPerBlock) / per_entry;
    Temps tmp{g->ctx->pool.get(), {}};
    const size_t n = (size_t)d.n;
    uint64_t *ka, *kb, *res;
    unsigned long long* counts;
    void* scr;
    TCL_TRY(tmp.get(std::max<size_t>(n, 1), &ka));
    TCL_TRY(tmp.get(std::max<size_t>(n, 1), &kb));
    TCL_TRY(tmp.get(64, &counts));
    TCL_TRY(tmp.get(radix_sort_scratch_bytes(std::max<size_t>(n, 1)), (uint8_t**)&scr));
    TCL_HIP(fill<unsigned long long>(counts, 64, 0ull, st));
    const int group = tn.group;
    k_classify<<<grid_for(n, kB, 4096), kB, 0, st>>>((const unsigned long long*)d.work, d.dplus, d.n, d.bits,
                                                     tn.wave_work_max, wave_cap, block_cap, group, ka, counts);
    TCL_HIP(hipGetLastError());
    TCL_HIP(radix_sort_u64(ka, kb, n, d.bits + 6, scr, st, &res));
    unsigned long long hc[64];
    TCL_HIP(hipMemcpyAsync(hc, counts, sizeof(hc), hipMemcpyDeviceToHost, st));
    TCL_HIP(hipStreamSynchronize(st));
    int64_t nb = 0;
    for (int c = 0; c < kClassWave; ++c) nb += (int64_t)hc[c];
    d.n_block = nb;
    d.n_wave = (int64_t)hc[kClassWave];
    d.n_global = (int64_t)hc[kClassGlobal];
    const int64_t active = nb + d.n_wave + d.n_global;
    if (active > 0) {
        k_vlist<<<grid_for(active, kB, 4096), kB, 0, st>>>(res, active, d.bits, d.vlist);
        TCL_HIP(hipGetLastError());
    }
    TCL_HIP(hipStreamSynchronize(st));
    d.sched_probe = probe;
    return TC_LCC_OK;
}

}  // namespace tcl
