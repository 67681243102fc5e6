// C-ABI entry points, contexts, graphs and the device memory pool.
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "internal.hpp"

namespace tcl {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

const char* last_error() { return g_err; }

tc_lcc_tuning default_tuning() {
    tc_lcc_tuning t;
    memset(&t, 0, sizeof(t));
    t.probe = TC_LCC_PROBE_AUTO;
    t.group = 0;
    t.wave_work_max = 4096;
    t.wave_outdeg_max = 0;
    t.block_threads = 256;
    t.merge_ratio_x100 = 0;
    t.batch_grab = 16;
    t.batch_heavy_bits = kBigWorkBits;
    return t;
}

// ------------------------------------------------------------------ pool

size_t Pool::round(size_t bytes) {
    if (bytes <= 256) return 256;
    if (bytes <= (1u << 20)) {  // powers of two up to 1 MiB
        size_t s = 256;
        while (s < bytes) s <<= 1;
        return s;
    }
    const size_t g = 2u << 20;  // 2 MiB granules above
    return (bytes + g - 1) / g * g;
}

void Pool::fail_after(int64_t after) {
    std::lock_guard<std::mutex> lk(mu_);
    fail_after_ = after;
}

tc_lcc_status Pool::alloc(size_t bytes, void** out) {
    const size_t sz = round(bytes);
    std::lock_guard<std::mutex> lk(mu_);
    if (fail_after_ >= 0 && fail_after_-- == 0) {
        set_error("device allocation of %zu bytes refused (failure injection)", sz);
        return TC_LCC_OUT_OF_MEMORY;
    }
    auto it = free_.find(sz);
    if (it != free_.end()) {
        void* p = it->second;
        free_.erase(it);
        pooled_ -= sz;
        in_use_ += sz;
        live_[p] = sz;
        *out = p;
        return TC_LCC_OK;
    }
    if (budget_ && in_use_ + sz > budget_) {
        set_error("device budget of %llu bytes exceeded (%llu in use, %zu requested)",
                  (unsigned long long)budget_, (unsigned long long)in_use_, sz);
        return TC_LCC_OVER_BUDGET;
    }
    if (budget_ && in_use_ + pooled_ + sz > budget_) {
        // give cached blocks back before asking HIP for more
        for (auto& kv : free_) {
            (void)hipFree(kv.second);
        }
        free_.clear();
        pooled_ = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        pooled_ = 0;
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu bytes failed", sz);
            return TC_LCC_OUT_OF_MEMORY;
        }
    }
    in_use_ += sz;
    live_[p] = sz;
    *out = p;
    return TC_LCC_OK;
}

tc_lcc_status Pool::alloc_exact(size_t bytes, void** out) {
    std::lock_guard<std::mutex> lk(mu_);
    if (fail_after_ >= 0 && fail_after_-- == 0) {
        set_error("device allocation of %zu bytes refused (failure injection)", bytes);
        return TC_LCC_OUT_OF_MEMORY;
    }
    if (budget_ && in_use_ + bytes > budget_) {
        set_error("device budget of %llu bytes exceeded (%llu in use, %zu requested)",
                  (unsigned long long)budget_, (unsigned long long)in_use_, bytes);
        return TC_LCC_OVER_BUDGET;
    }
    if (budget_ && in_use_ + pooled_ + bytes > budget_) {
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        pooled_ = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        for (auto& kv : free_) (void)hipFree(kv.second);
        free_.clear();
        pooled_ = 0;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of %zu bytes failed", bytes);
            return TC_LCC_OUT_OF_MEMORY;
        }
    }
    in_use_ += bytes;
    live_[p] = bytes;
    *out = p;
    return TC_LCC_OK;
}

void Pool::free_exact(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    in_use_ -= it->second;
    live_.erase(it);
    (void)hipFree(p);
}

void Pool::release(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    const size_t sz = it->second;
    live_.erase(it);
    in_use_ -= sz;
    pooled_ += sz;
    free_.emplace(sz, p);
}

void Pool::trim() {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto& kv : free_) (void)hipFree(kv.second);
    free_.clear();
    pooled_ = 0;
}

Pool::~Pool() {
    trim();
    for (auto& kv : live_) (void)hipFree(kv.first);
}

}  // namespace tcl

using namespace tcl;

// ------------------------------------------------------------------ misc

extern "C" const char* tc_lcc_status_string(tc_lcc_status s) {
    switch (s) {
        case TC_LCC_OK: return "ok";
        case TC_LCC_INVALID_ARGUMENT: return "invalid argument";
        case TC_LCC_OUT_OF_MEMORY: return "out of memory";
        case TC_LCC_OVER_BUDGET: return "over budget";
        case TC_LCC_NOT_READY: return "not ready";
        case TC_LCC_BUSY: return "busy";
        case TC_LCC_DEVICE_ERROR: return "device error";
        case TC_LCC_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* tc_lcc_last_error(void) { return last_error(); }

// ------------------------------------------------------------------ context

extern "C" tc_lcc_status tc_lcc_ctx_create(int device, uint64_t hbm_budget_bytes, tc_lcc_ctx* out) {
    if (!out) {
        set_error("tc_lcc_ctx_create: null out");
        return TC_LCC_INVALID_ARGUMENT;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        set_error("tc_lcc_ctx_create: device %d not available (%d visible)", device, count);
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    TCL_HIP(hipGetDeviceProperties(&prop, device));
    tc_lcc_ctx c = new (std::nothrow) tc_lcc_ctx_s();
    if (!c) return TC_LCC_OUT_OF_MEMORY;
    c->device = device;
    c->pool.reset(new Pool(device, hbm_budget_bytes));
    c->tuning = default_tuning();
    c->cu_count = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    c->lds_per_block = prop.sharedMemPerBlock;
    tc_lcc_status bs = batch_engine_create(c);
    uint8_t* nb = nullptr;
    if (bs == TC_LCC_OK) bs = noalloc_base(device, &nb);  // this device's copy of the static scratch
    if (bs != TC_LCC_OK) {
        batch_engine_destroy(c);
        delete c;
        return bs;
    }
    *out = c;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_ctx_destroy(tc_lcc_ctx ctx) {
    if (!ctx) {
        set_error("tc_lcc_ctx_destroy: null context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (ctx->tickets_inflight.load() > 0 || ctx->graphs.load() > 0) {
        set_error("tc_lcc_ctx_destroy: %d graphs and %d batches still live", ctx->graphs.load(),
                  ctx->tickets_inflight.load());
        return TC_LCC_BUSY;
    }
    (void)hipSetDevice(ctx->device);
    batch_engine_destroy(ctx);
    delete ctx;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_ctx_memory(tc_lcc_ctx ctx, uint64_t* in_use, uint64_t* pooled) {
    if (!ctx) {
        set_error("tc_lcc_ctx_memory: null context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (in_use) *in_use = ctx->pool->in_use();
    if (pooled) *pooled = ctx->pool->pooled();
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_debug_fail_alloc(tc_lcc_ctx ctx, int64_t after) {
    if (!ctx) {
        set_error("tc_lcc_debug_fail_alloc: null context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    ctx->pool->fail_after(after);
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_get_tuning(tc_lcc_ctx ctx, tc_lcc_tuning* out) {
    if (!ctx || !out) {
        set_error("tc_lcc_get_tuning: null argument");
        return TC_LCC_INVALID_ARGUMENT;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    *out = ctx->tuning;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_set_tuning(tc_lcc_ctx ctx, const tc_lcc_tuning* in) {
    if (!ctx || !in) {
        set_error("tc_lcc_set_tuning: null argument");
        return TC_LCC_INVALID_ARGUMENT;
    }
    bool reserved_zero = true;
    for (int32_t r : in->reserved) reserved_zero = reserved_zero && r == 0;
    if (in->probe < 0 || in->probe > TC_LCC_PROBE_MERGE || in->group < 0 || in->group > 2 ||
        in->merge_ratio_x100 < 0 || in->merge_ratio_x100 > 100000 ||
        in->wave_work_max < 0 || in->wave_outdeg_max < 0 || (in->block_threads != 0 && in->block_threads != 256) ||
        in->batch_grab < 0 || in->batch_grab > 64 || in->batch_heavy_bits < 0 || in->batch_heavy_bits > 40 ||
        in->row_sort_max < 0 || in->row_sort_max > 4096 ||
        !reserved_zero) {
        set_error("tc_lcc_set_tuning: value out of range");
        return TC_LCC_INVALID_ARGUMENT;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuning = *in;
    ctx->tuning_gen++;
    return TC_LCC_OK;
}

// ------------------------------------------------------------------ graphs

static void graph_release(tc_lcc_graph g) {
    for (void* p : g->blocks) g->ctx->pool->release(p);
    g->blocks.clear();
    if (g->last_use) (void)hipEventDestroy(g->last_use);
    for (hipEvent_t& e : g->d.ev)
        if (e) (void)hipEventDestroy(e);
    delete g;
}

// A new graph built by `build(tuning, stream, graph)`, with its profiling events and last-use
// event; on failure the graph's memory is returned once the stream is idle.
template <typename Build>
static tc_lcc_status build_with(tc_lcc_ctx ctx, void* hip_stream, tc_lcc_graph* out, Build&& build) {
    TCL_HIP(hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)hip_stream;
    tc_lcc_graph g = new (std::nothrow) tc_lcc_graph_s();
    if (!g) return TC_LCC_OUT_OF_MEMORY;
    g->ctx = ctx;
    if (ctx->profiling) {
        g->d.prof = true;
        for (hipEvent_t& e : g->d.ev) {
            if (hipEventCreate(&e) != hipSuccess) {
                (void)hipGetLastError();
                graph_release(g);
                set_error("hipEventCreate failed");
                return TC_LCC_DEVICE_ERROR;
            }
        }
    }
    tc_lcc_tuning tn;
    uint64_t gen;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        tn = ctx->tuning;
        gen = ctx->tuning_gen;
    }
    tc_lcc_status s = build(tn, st, g);
    if (s == TC_LCC_OK) {
        g->d.sched_gen = gen;
        if (hipEventCreateWithFlags(&g->last_use, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(g->last_use, st) != hipSuccess) {
            (void)hipGetLastError();
            s = TC_LCC_DEVICE_ERROR;
            set_error("hipEventCreate/Record failed");
        }
    }
    if (s != TC_LCC_OK) {
        (void)hipStreamSynchronize(st);
        (void)hipGetLastError();
        graph_release(g);
        return s;
    }
    ctx->graphs++;
    *out = g;
    return TC_LCC_OK;
}

static tc_lcc_status build_common(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                                  int inputs_on_device, int offset_bytes, void* hip_stream, tc_lcc_graph* out,
                                  bool directed) {
    if (!ctx || !out) {
        set_error("tc_lcc_build_csr: null context or out");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (n < 1 || n > 2147483647ll || m_in < 0 || m_in >= (1ll << 32) || (m_in > 0 && (!src || !dst)) ||
        (offset_bytes != 0 && offset_bytes != 4 && offset_bytes != 8)) {
        set_error("tc_lcc_build_csr: bad size, pointer or offset width (n=%lld m_in=%lld offset_bytes=%d)",
                  (long long)n, (long long)m_in, offset_bytes);
        return TC_LCC_INVALID_ARGUMENT;
    }
    return build_with(ctx, hip_stream, out, [&](const tc_lcc_tuning& tn, hipStream_t st, tc_lcc_graph g) {
        return build_graph(ctx, n, m_in, src, dst, inputs_on_device, offset_bytes, tn, st, g, directed);
    });
}

extern "C" tc_lcc_status tc_lcc_build_streamed(tc_lcc_ctx ctx, int64_t n, uint64_t m_in, tc_lcc_pair_source source,
                                               void* user, uint64_t chunk_pairs, uint64_t partition_pairs,
                                               void* hip_stream, tc_lcc_graph* out) {
    if (!ctx || !out || !source) {
        set_error("tc_lcc_build_streamed: null context, source or out");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (n < 1 || n > 2147483647ll) {
        set_error("tc_lcc_build_streamed: n=%lld outside [1, 2^31-1]", (long long)n);
        return TC_LCC_INVALID_ARGUMENT;
    }
    const uint64_t chunk = chunk_pairs ? chunk_pairs : (1ull << 28);
    StreamSource src = [&](uint64_t first, uint64_t count, int32_t* s, int32_t* d, hipStream_t st) {
        const int rc = source(user, first, count, s, d, (void*)st);
        if (rc != 0) {
            set_error("tc_lcc_build_streamed: the pair source returned %d for pairs [%llu, %llu)", rc,
                      (unsigned long long)first, (unsigned long long)(first + count));
            return TC_LCC_INVALID_ARGUMENT;
        }
        return TC_LCC_OK;
    };
    return build_with(ctx, hip_stream, out, [&](const tc_lcc_tuning& tn, hipStream_t st, tc_lcc_graph g) {
        return build_streamed(ctx, n, m_in, src, chunk, partition_pairs, tn, st, g);
    });
}

extern "C" tc_lcc_status tc_lcc_build_csr(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src,
                                          const int32_t* dst, int inputs_on_device, int offset_bytes,
                                          void* hip_stream, tc_lcc_graph* out) {
    return build_common(ctx, n, m_in, src, dst, inputs_on_device, offset_bytes, hip_stream, out, false);
}

extern "C" tc_lcc_status tc_lcc_build_directed(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src,
                                               const int32_t* dst, int inputs_on_device, int offset_bytes,
                                               void* hip_stream, tc_lcc_graph* out) {
    return build_common(ctx, n, m_in, src, dst, inputs_on_device, offset_bytes, hip_stream, out, true);
}

extern "C" tc_lcc_status tc_lcc_graph_info(tc_lcc_graph g, tc_lcc_graph_stats* out) {
    if (!g || !out) {
        set_error("tc_lcc_graph_info: null argument");
        return TC_LCC_INVALID_ARGUMENT;
    }
    out->n = g->d.n;
    out->m = g->d.m;
    out->offset_bytes = g->d.off_bytes;
    out->max_out_degree = g->d.max_dplus;
    out->max_degree = g->d.max_deg;
    out->wedges = g->d.wedges;
    out->device_bytes = g->d.device_bytes;
    out->kept_in_edges = g->d.m_in_kept;
    out->active_vertices = g->d.n_block + g->d.n_wave + g->d.n_list + g->d.n_global;
    out->staged_entries = (int64_t)g->d.staged;
    out->block_vertices = g->d.n_block + g->d.n_list;
    out->count_grid = g->d.count_grid;
    out->count_lds_bytes = g->d.count_lds;
    out->count_blocks_per_cu = g->d.count_per_cu;
    out->table_slots = g->d.hash_slots;
    out->push_words = g->d.push_words;
    out->global_vertices = g->d.n_global;
    out->directed = g->d.directed ? 1 : 0;
    out->compact = g->d.compact ? 1 : 0;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_graph_export(tc_lcc_graph g, int64_t* degree, int32_t* order, int64_t* out_off,
                                             int32_t* out_adj) {
    if (!g) {
        set_error("tc_lcc_graph_export: null graph");
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(g->ctx->device));
    if (g->last_use) TCL_HIP(hipEventSynchronize(g->last_use));
    const size_t n = (size_t)g->d.n, m = (size_t)g->d.m;
    std::vector<int32_t> ord(n), dr(n);
    TCL_HIP(hipMemcpy(ord.data(), g->d.order, n * 4, hipMemcpyDeviceToHost));
    TCL_HIP(hipMemcpy(dr.data(), g->d.deg_r, n * 4, hipMemcpyDeviceToHost));
    if (order) memcpy(order, ord.data(), n * 4);
    if (degree)
        for (size_t r = 0; r < n; ++r) degree[ord[r]] = dr[r];
    if (out_off) {
        if (g->d.off_bytes == 8) {
            TCL_HIP(hipMemcpy(out_off, g->d.out_off, (n + 1) * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<int32_t> o(n + 1);
            TCL_HIP(hipMemcpy(o.data(), g->d.out_off, (n + 1) * 4, hipMemcpyDeviceToHost));
            for (size_t i = 0; i <= n; ++i) out_off[i] = o[i];
        }
    }
    if (out_adj && m) TCL_HIP(hipMemcpy(out_adj, g->d.adj, m * 4, hipMemcpyDeviceToHost));
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_graph_free(tc_lcc_graph g) {
    if (!g) {
        set_error("tc_lcc_graph_free: null graph");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (g->inflight.load() > 0) {
        set_error("tc_lcc_graph_free: graph used by %d unfinished batches", g->inflight.load());
        return TC_LCC_BUSY;
    }
    TCL_HIP(hipSetDevice(g->ctx->device));
    if (g->last_use) TCL_HIP(hipEventSynchronize(g->last_use));
    tc_lcc_ctx ctx = g->ctx;
    graph_release(g);
    ctx->graphs--;
    return TC_LCC_OK;
}

// ------------------------------------------------------------------ one graph

// The graph's lock held, its last use waited for, and its schedule made current for the
// context's tuning (a rebuild first waits for the batches that hold the graph).
static tc_lcc_status prepare_run(tc_lcc_graph g, hipStream_t st, bool engine_locked, tc_lcc_tuning& tn,
                                 std::unique_lock<std::mutex>& lk, bool allow_rebuild = true) {
    tc_lcc_ctx ctx = g->ctx;
    TCL_HIP(hipSetDevice(ctx->device));
    uint64_t gen;
    {
        std::lock_guard<std::mutex> cl(ctx->mu);
        tn = ctx->tuning;
        gen = ctx->tuning_gen;
    }
    std::unique_lock<std::mutex> el;
    lk = std::unique_lock<std::mutex>(g->mu);
    if (!allow_rebuild) gen = g->d.sched_gen;  // the schedule as it stands (results never depend on it)
    if (g->d.sched_gen != gen && !engine_locked) {
        // a schedule rebuild rewrites the vertex list that batches in flight read: take the
        // engine's lock (before the graph's) so that no batch starts meanwhile, and wait for
        // the batches that hold the graph
        lk.unlock();
        el = std::unique_lock<std::mutex>(batch_mutex(ctx));
        lk.lock();
    }
    TCL_HIP(hipStreamWaitEvent(st, g->last_use, 0));
    if (g->d.sched_gen != gen) {
        tc_lcc_status s = batch_fence_graph(ctx, g, st);
        if (s == TC_LCC_OK) s = build_schedule(g, tn, st);
        if (s != TC_LCC_OK) return s;
        g->d.sched_gen = gen;
    }
    return TC_LCC_OK;
}

tc_lcc_status tcl::run_graph(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st, int spare_per_cu,
                             bool engine_locked) {
    tc_lcc_tuning tn;
    std::unique_lock<std::mutex> lk;
    tc_lcc_status s = prepare_run(g, st, engine_locked, tn, lk);
    if (s != TC_LCC_OK) return s;
    mark(g->d, 6, st);
    s = launch_zero_counts(g, st);
    mark(g->d, 7, st);
    if (g->d.directed) {
        if (s == TC_LCC_OK) s = launch_count_directed(g, st);
        mark(g->d, 8, st);
        if (s == TC_LCC_OK) s = launch_epilogue_directed(g, tri, lcc, st);
    } else {
        if (s == TC_LCC_OK) s = launch_count(g, tn, spare_per_cu, st);
        mark(g->d, 8, st);
        if (s == TC_LCC_OK) s = launch_epilogue(g, tri, lcc, st);
    }
    mark(g->d, 9, st);
    if (s != TC_LCC_OK) return s;
    TCL_HIP(hipEventRecord(g->last_use, st));
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_run(tc_lcc_graph g, uint64_t* tri, double* lcc, void* hip_stream) {
    if (!g || !tri) {
        set_error("tc_lcc_run: null graph or output");
        return TC_LCC_INVALID_ARGUMENT;
    }
    return run_graph(g, tri, lcc, (hipStream_t)hip_stream, 0);
}

namespace {

__global__ void k_zero_u32(uint32_t* p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}

// Temporaries from the context's pool, given back when the call returns (it waits for its stream).
struct CallTemps {
    Pool* pool;
    std::vector<void*> held;
    ~CallTemps() {
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

}  // namespace

// Temporaries of the per-edge run: per-position counters, two key buffers for the sort into
// edge order, the sort's scratch, an error word and the rank of every id.
struct EdgeTemps {
    uint32_t* ce = nullptr;
    uint64_t* keys = nullptr;
    uint64_t* alt = nullptr;
    uint8_t* scratch = nullptr;
    unsigned int* err = nullptr;
    int32_t* rank = nullptr;
};

static tc_lcc_status edges_check(tc_lcc_graph g, uint64_t* tri, const char* who) {
    if (!g || !tri) {
        set_error("%s: null graph or output", who);
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (g->d.directed) {
        set_error("%s: per-edge counts are defined here for undirected graphs", who);
        return TC_LCC_UNSUPPORTED;
    }
    if (g->d.compact) {
        set_error("%s: not available for a graph with compact reverse lists (tc_lcc_build_streamed)", who);
        return TC_LCC_UNSUPPORTED;
    }
    return TC_LCC_OK;
}

// The per-edge run on given temporaries; waits for the stream before it returns.
static tc_lcc_status run_edges_on(tc_lcc_graph g, uint64_t* tri, double* lcc, int32_t* edge_src, int32_t* edge_dst,
                                  uint32_t* edge_tri, hipStream_t st, const EdgeTemps& t, bool allow_rebuild,
                                  const char* who) {
    const size_t m = (size_t)g->d.m;
    tc_lcc_tuning tn;
    tc_lcc_status s;
    {
        std::unique_lock<std::mutex> lk;
        s = prepare_run(g, st, false, tn, lk, allow_rebuild);
        if (s != TC_LCC_OK) return s;  // nothing of this call is on the stream yet
        // from the first launch on, every path waits for the stream before returning
        k_zero_u32<<<grid_for(std::max<size_t>(m, 64), 256, 8192), 256, 0, st>>>(t.ce, std::max<size_t>(m, 1));
        k_zero_u32<<<1, 64, 0, st>>>(t.err, 64);
        if (hipGetLastError() != hipSuccess) {
            set_error("%s: clearing the counters failed", who);
            s = TC_LCC_DEVICE_ERROR;
        }
        mark(g->d, 6, st);
        if (s == TC_LCC_OK) s = launch_zero_counts(g, st);
        mark(g->d, 7, st);
        if (s == TC_LCC_OK) s = launch_count_edges(g, t.ce, st);
        mark(g->d, 8, st);
        if (s == TC_LCC_OK) s = launch_epilogue(g, tri, lcc, st);
        if (s == TC_LCC_OK && m > 0 && (edge_src || edge_dst || edge_tri)) {
            const hipError_t e =
                edge_output(g->d, t.keys, t.alt, t.scratch, t.err, t.rank, t.ce, edge_src, edge_dst, edge_tri, st);
            if (e != hipSuccess) {
                set_error("%s: %s", who, hipGetErrorString(e));
                s = TC_LCC_DEVICE_ERROR;
            }
        }
        mark(g->d, 9, st);
        if (s == TC_LCC_OK && hipEventRecord(g->last_use, st) != hipSuccess) {
            set_error("%s: event record failed", who);
            s = TC_LCC_DEVICE_ERROR;
        }
    }
    unsigned int herr = 0;
    const hipError_t e1 = s == TC_LCC_OK ? hipMemcpyAsync(&herr, t.err, sizeof(herr), hipMemcpyDeviceToHost, st)
                                         : hipSuccess;
    const hipError_t e2 = hipStreamSynchronize(st);
    if (s != TC_LCC_OK) {
        (void)hipGetLastError();
        return s;
    }
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("%s: %s", who, hipGetErrorString(e1 != hipSuccess ? e1 : e2));
        return TC_LCC_DEVICE_ERROR;
    }
    if (herr) {
        set_error("%s: a radix sort pass gave up waiting for an earlier tile", who);
        return TC_LCC_DEVICE_ERROR;
    }
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_run_edges(tc_lcc_graph g, uint64_t* tri, double* lcc, int32_t* edge_src,
                                          int32_t* edge_dst, uint32_t* edge_tri, void* hip_stream) {
    tc_lcc_status s = edges_check(g, tri, "tc_lcc_run_edges");
    if (s != TC_LCC_OK) return s;
    const size_t m = (size_t)g->d.m, n = (size_t)g->d.n;
    CallTemps tmp{g->ctx->pool.get(), {}};  // given back after the call has waited for its stream
    EdgeTemps t;
    s = tmp.get(std::max<size_t>(m, 1), &t.ce);
    if (s == TC_LCC_OK) s = tmp.get(std::max<size_t>(m, 1), &t.keys);
    if (s == TC_LCC_OK) s = tmp.get(std::max<size_t>(m, 1), &t.alt);
    if (s == TC_LCC_OK) s = tmp.get(radix_sort_scratch_bytes(std::max<size_t>(m, 1)), &t.scratch);
    if (s == TC_LCC_OK) s = tmp.get(64, &t.err);
    if (s == TC_LCC_OK) s = tmp.get(std::max<size_t>(n, 1), &t.rank);
    if (s != TC_LCC_OK) return s;
    return run_edges_on(g, tri, lcc, edge_src, edge_dst, edge_tri, (hipStream_t)hip_stream, t, true,
                        "tc_lcc_run_edges");
}

// ------------------------------------------------------------------ per-edge run without allocation

// Every temporary of tc_lcc_run_edges_noalloc: one copy on each GPU the library runs on, held
// until the process ends.  In host code this name is not a device address; the address of
// each GPU's copy comes from hipGetSymbolAddress (noalloc_base) and only that is used.
static __device__ __align__(256) uint8_t scratch[TC_LCC_NOALLOC_BYTES];

namespace {

std::mutex g_noalloc_mu;
std::unordered_map<int, uint8_t*> g_noalloc_base;  // device -> its copy of `scratch`

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// The address of the current device's copy of the static buffer, looked up once per device
// (with that device current) and kept.
tc_lcc_status tcl::noalloc_base(int device, uint8_t** out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_base.find(device);
    if (it == g_noalloc_base.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            (void)hipGetLastError();
            set_error("static scratch of device %d: hipGetSymbolAddress failed: %s", device, hipGetErrorString(e));
            return TC_LCC_DEVICE_ERROR;
        }
        it = g_noalloc_base.emplace(device, (uint8_t*)p).first;
    }
    *out = it->second;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_run_edges_noalloc(tc_lcc_graph g, uint64_t* tri, double* lcc, int32_t* edge_src,
                                                  int32_t* edge_dst, uint32_t* edge_tri, void* hip_stream) {
    tc_lcc_status s = edges_check(g, tri, "tc_lcc_run_edges_noalloc");
    if (s != TC_LCC_OK) return s;
    const size_t m = std::max<size_t>((size_t)g->d.m, 1), n = std::max<size_t>((size_t)g->d.n, 1);
    // layout of the buffer: counters, keys, alternate keys, sort scratch, error word, ranks
    const size_t o_ce = 0, o_keys = o_ce + up256(4 * m), o_alt = o_keys + up256(8 * m);
    const size_t o_rs = o_alt + up256(8 * m), o_err = o_rs + up256(radix_sort_scratch_bytes(m));
    const size_t o_rank = o_err + 256, need = o_rank + up256(4 * n);
    if (need > (size_t)TC_LCC_NOALLOC_BYTES) {
        set_error("tc_lcc_run_edges_noalloc: the graph needs %zu bytes of temporaries (%zu edges, %zu vertices), "
                  "beyond the static buffer of %llu bytes",
                  need, (size_t)g->d.m, (size_t)g->d.n, (unsigned long long)TC_LCC_NOALLOC_BYTES);
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(g->ctx->device));
    uint8_t* base = nullptr;
    s = noalloc_base(g->ctx->device, &base);
    if (s != TC_LCC_OK) return s;
    EdgeTemps t;
    t.ce = (uint32_t*)(base + o_ce);
    t.keys = (uint64_t*)(base + o_keys);
    t.alt = (uint64_t*)(base + o_alt);
    t.scratch = base + o_rs;
    t.err = (unsigned int*)(base + o_err);
    t.rank = (int32_t*)(base + o_rank);
    return run_edges_on(g, tri, lcc, edge_src, edge_dst, edge_tri, (hipStream_t)hip_stream, t, false,
                        "tc_lcc_run_edges_noalloc");
}

// ------------------------------------------------------------------ profiling

extern "C" tc_lcc_status tc_lcc_set_profiling(tc_lcc_ctx ctx, int enable) {
    if (!ctx) {
        set_error("tc_lcc_set_profiling: null context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    ctx->profiling = enable != 0;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_graph_timings(tc_lcc_graph g, tc_lcc_timings* out) {
    if (!g || !out) {
        set_error("tc_lcc_graph_timings: null argument");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (!g->d.prof) {
        set_error("tc_lcc_graph_timings: the graph was built without profiling");
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(g->ctx->device));
    TCL_HIP(hipEventSynchronize(g->last_use));
    float ms[10] = {0};
    auto el = [&](int a, int b) -> float {
        float x = 0.f;
        if (hipEventElapsedTime(&x, g->d.ev[a], g->d.ev[b]) != hipSuccess) {
            (void)hipGetLastError();
            return -1.f;
        }
        return x;
    };
    ms[0] = el(0, 1);
    ms[1] = el(1, 2);
    ms[2] = el(2, 3);
    ms[3] = el(3, 4);
    ms[4] = el(4, 5);
    ms[5] = el(6, 7);
    ms[6] = el(7, 8);
    ms[7] = el(8, 9);
    out->build_sort_unique_ms = ms[0];
    out->build_rank_ms = ms[1];
    out->build_orient_ms = ms[2];
    out->build_reverse_ms = ms[3];
    out->build_schedule_ms = ms[4];
    out->run_zero_ms = ms[5];
    out->run_count_ms = ms[6];
    out->run_epilogue_ms = ms[7];
    return TC_LCC_OK;
}
