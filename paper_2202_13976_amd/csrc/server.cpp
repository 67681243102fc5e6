// Serving loop: continuous batching of triangle-count / LCC requests on device-resident graphs.
//
// Requests (graph, output buffers) arrive at any time through submit().  A dispatcher
// thread admits them in arrival order while their scratch fits the server's HBM budget,
// groups everything admitted at once into one batch of the persistent batched launch, and
// starts it as soon as one of the in-flight slots is free.
//
// The budget is memory actually held: with batching and a budget, the server takes one
// device arena of that size (rounded down to 8 bytes) when it is created (and the batch engine's descriptors
// for max_batch graphs), and nothing more while it serves.  A batched request needs its
// graph's counters, 8 bytes per vertex, carved first-fit from the arena at admission; they
// return to the arena when the request's graph is done, which is also when the epilogue has
// set them back to zero, so the next request finds them clean.  Requests for graphs that
// take the single-graph launches use their graph's own counters and need no arena space.
// Requests that arrive while earlier batches run join the next batch and overlap
// with them on the GPU.  Completion is observed per request from the per-graph done
// flags of its batch, so a small graph batched with a large one leaves as soon as it is
// counted; every request records its arrival, admission and completion times (steady
// clock, ns).
// With batching off the server runs one request at a time through tc_lcc_run, the
// plain one-graph-per-launch path, for comparison.
#include <chrono>
#include <cstring>
#include <iterator>

#include "internal.hpp"

namespace tcl {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t id = 0;
    tc_lcc_graph g = nullptr;
    uint64_t* tri = nullptr;
    double* lcc = nullptr;
    uint64_t bytes = 0;       // budget share: arena bytes (batching), or 8 B per vertex (plain path)
    uint64_t arena_off = ~0ull;  // its counters in the arena while it runs
    int64_t t_arrive = 0, t_admit = 0, t_done = 0;
    int batch_size = 0;
    tc_lcc_status status = TC_LCC_OK;
    bool done = false;
};

struct Flight {
    std::vector<Request*> reqs;
    std::vector<uint8_t> flags;  // per-request completion of a batch
    int open = 0;                // requests not yet retired
    uint64_t bytes = 0;
    tc_lcc_ticket ticket = 0;  // batching
    hipEvent_t ev = nullptr;   // plain path
};

}  // namespace
}  // namespace tcl

struct tc_lcc_server_s {
    tc_lcc_ctx ctx = nullptr;
    uint64_t budget = 0;
    int max_inflight = 2;
    int max_batch = 4096;
    bool batching = true;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<tcl::Request*> pending;
    std::unordered_map<uint64_t, tcl::Request*> reqs;
    std::vector<tcl::Flight> flights;
    uint64_t inflight_bytes = 0;
    uint64_t next_id = 1;
    // batching with a budget: the counters of running requests, first-fit in one device block
    uint8_t* arena = nullptr;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> bytes, coalesced
    bool stop = false;
    hipStream_t stream = nullptr;  // plain path
    std::thread worker;
    tc_lcc_status fatal = TC_LCC_OK;
};

namespace tcl {
namespace {

constexpr uint64_t kArenaAlign = 8;  // the counters are 8-byte words

uint64_t arena_need(const tc_lcc_graph g) {
    return (8ull * (uint64_t)g->d.n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// First fit of `bytes` in the arena's free ranges; ~0 if none is large enough.
uint64_t arena_take(tc_lcc_server s, uint64_t bytes) {
    for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
        if (it->second < bytes) continue;
        const uint64_t off = it->first, rest = it->second - bytes;
        s->free_ranges.erase(it);
        if (rest) s->free_ranges[off + bytes] = rest;
        return off;
    }
    return ~0ull;
}

void arena_give(tc_lcc_server s, uint64_t off, uint64_t bytes) {
    auto next = s->free_ranges.lower_bound(off);
    if (next != s->free_ranges.end() && off + bytes == next->first) {  // join the range after
        bytes += next->second;
        next = s->free_ranges.erase(next);
    }
    if (next != s->free_ranges.begin()) {  // join the range before
        auto prev = std::prev(next);
        if (prev->first + prev->second == off) {
            prev->second += bytes;
            return;
        }
    }
    s->free_ranges[off] = bytes;
}

// Completes one request of flight f: its budget share (its arena range, whose counters the
// epilogue has set back to zero by the time its done flag is seen) is returned and pollers
// wake up.
void retire(tc_lcc_server s, Flight& f, Request* r, int64_t t, tc_lcc_status st) {
    r->t_done = t;
    r->status = st;
    r->done = true;
    r->g->inflight--;
    s->inflight_bytes -= r->bytes;
    if (r->arena_off != ~0ull) {
        arena_give(s, r->arena_off, r->bytes);
        r->arena_off = ~0ull;
    }
    f.open--;
    s->cv_done.notify_all();
}

__global__ void k_arena_clear(unsigned long long* __restrict__ p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

void worker_loop(tc_lcc_server s) {
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. retire finished requests, and flights whose launch is over
        for (size_t i = 0; i < s->flights.size();) {
            Flight& f = s->flights[i];
            bool finished = false;
            tc_lcc_status st = TC_LCC_OK;
            if (s->batching) {
                // requests whose graph is done leave at once; the ticket is released
                // once the whole launch is over
                if (f.open > 0 &&
                    tc_lcc_batch_progress(s->ctx, f.ticket, (int)f.reqs.size(), f.flags.data()) == TC_LCC_OK) {
                    const int64_t t = now_ns();
                    for (size_t k = 0; k < f.reqs.size(); ++k) {
                        Request* r = f.reqs[k];
                        if (!f.flags[k] || r->done) continue;
                        retire(s, f, r, t, TC_LCC_OK);
                    }
                }
                st = tc_lcc_batch_poll(s->ctx, f.ticket, 0, nullptr);
                finished = st != TC_LCC_NOT_READY;
                if (st == TC_LCC_NOT_READY) st = TC_LCC_OK;
            } else {
                const hipError_t q = hipEventQuery(f.ev);
                finished = q != hipErrorNotReady;
                if (q != hipSuccess && q != hipErrorNotReady) st = TC_LCC_DEVICE_ERROR;
            }
            if (!finished) {
                ++i;
                continue;
            }
            const int64_t t = now_ns();
            for (Request* r : f.reqs)
                if (!r->done) retire(s, f, r, t, st);
            if (f.ev) (void)hipEventDestroy(f.ev);
            s->flights.erase(s->flights.begin() + (long)i);
        }
        // 2. admit and launch while a slot is free and the budget allows
        while ((int)s->flights.size() < s->max_inflight && !s->pending.empty()) {
            Flight f;
            while (!s->pending.empty() && (int)f.reqs.size() < s->max_batch) {
                Request* r = s->pending.front();
                if (s->arena) {
                    if (r->bytes) {
                        const uint64_t off = arena_take(s, r->bytes);
                        if (off == ~0ull) break;  // the head waits for counters to free up
                        r->arena_off = off;
                    }
                } else if (s->budget && s->inflight_bytes + f.bytes + r->bytes > s->budget) {
                    break;
                }
                s->pending.pop_front();
                f.reqs.push_back(r);
                f.bytes += r->bytes;
            }
            if (f.reqs.empty()) break;  // the head waits for memory to free up
            const int64_t t = now_ns();
            std::vector<tc_lcc_graph> gs;
            std::vector<uint64_t*> ts;
            std::vector<double*> ls;
            std::vector<unsigned long long*> cs;
            for (Request* r : f.reqs) {
                r->t_admit = t;
                r->batch_size = (int)f.reqs.size();
                r->g->inflight++;
                gs.push_back(r->g);
                ts.push_back(r->tri);
                ls.push_back(r->lcc);
                cs.push_back(r->arena_off != ~0ull ? (unsigned long long*)(s->arena + r->arena_off) : nullptr);
            }
            tc_lcc_status st;
            if (s->batching) {
                st = batch_submit_with(s->ctx, (int)gs.size(), gs.data(), ts.data(), ls.data(),
                                       s->arena ? cs.data() : nullptr, &f.ticket);
            } else {
                st = tc_lcc_run(gs[0], ts[0], ls[0], s->stream);
                if (st == TC_LCC_OK &&
                    (hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess ||
                     hipEventRecord(f.ev, s->stream) != hipSuccess)) {
                    (void)hipGetLastError();
                    st = TC_LCC_DEVICE_ERROR;
                }
            }
            if (st != TC_LCC_OK) {
                for (Request* r : f.reqs) {
                    r->status = st;
                    r->done = true;
                    r->t_done = now_ns();
                    r->g->inflight--;
                    if (r->arena_off != ~0ull) {  // nothing ran: the counters are still zero
                        arena_give(s, r->arena_off, r->bytes);
                        r->arena_off = ~0ull;
                    }
                }
                s->cv_done.notify_all();
                continue;
            }
            s->inflight_bytes += f.bytes;
            f.open = (int)f.reqs.size();
            f.flags.assign(f.reqs.size(), 0);
            s->flights.push_back(std::move(f));
        }
        if (s->stop && s->pending.empty() && s->flights.empty()) break;
        // 3. wait: poll quickly while work is on the GPU, otherwise sleep until a request arrives
        if (!s->flights.empty()) {
            lk.unlock();
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
        } else {
            s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

}  // namespace
}  // namespace tcl

using namespace tcl;

extern "C" tc_lcc_status tc_lcc_server_create(tc_lcc_ctx ctx, uint64_t hbm_budget_bytes, int max_inflight,
                                              int max_batch, tc_lcc_server* out) {
    if (!ctx || !out || max_inflight < 1 || max_batch < 1) {
        set_error("tc_lcc_server_create: null argument or non-positive limits");
        return TC_LCC_INVALID_ARGUMENT;
    }
    TCL_HIP(hipSetDevice(ctx->device));
    tc_lcc_server s = new (std::nothrow) tc_lcc_server_s();
    if (!s) return TC_LCC_OUT_OF_MEMORY;
    s->ctx = ctx;
    s->budget = hbm_budget_bytes;
    s->max_inflight = max_inflight < 4 ? max_inflight : 4;  // the batch engine has four slots
    s->max_batch = max_batch;
    s->batching = max_batch > 1 || max_inflight > 1;
    if (!s->batching && hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        set_error("tc_lcc_server_create: stream creation failed");
        return TC_LCC_DEVICE_ERROR;
    }
    if (s->batching && hbm_budget_bytes > 0) {
        // all the device memory the server will hold, taken now: the counters' arena, and the
        // batch engine's descriptors for max_batch graphs
        const uint64_t ab = hbm_budget_bytes / kArenaAlign * kArenaAlign;
        void* p = nullptr;
        tc_lcc_status st = ab ? ctx->pool->alloc_exact(ab, &p) : TC_LCC_OVER_BUDGET;
        if (st == TC_LCC_OK) {
            hipStream_t cs = nullptr;
            if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
                st = TC_LCC_DEVICE_ERROR;
            } else {
                k_arena_clear<<<(unsigned)std::min<uint64_t>((ab / 8 + 255) / 256, 4096), 256, 0, cs>>>(
                    (unsigned long long*)p, ab / 8);
                if (hipGetLastError() != hipSuccess || hipStreamSynchronize(cs) != hipSuccess) st = TC_LCC_DEVICE_ERROR;
                (void)hipStreamDestroy(cs);
            }
            if (st == TC_LCC_OK) st = batch_reserve(ctx, (size_t)std::min(max_batch, 1 << 16));
        }
        if (st != TC_LCC_OK) {
            (void)hipGetLastError();
            if (p) ctx->pool->free_exact(p);
            delete s;
            set_error("tc_lcc_server_create: the arena of the budget (%llu bytes) could not be set up",
                      (unsigned long long)hbm_budget_bytes);
            return st == TC_LCC_DEVICE_ERROR ? TC_LCC_DEVICE_ERROR : TC_LCC_OVER_BUDGET;
        }
        s->arena = (uint8_t*)p;
        s->free_ranges[0] = ab;
        s->budget = ab;
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_server_submit(tc_lcc_server s, tc_lcc_graph g, uint64_t* tri, double* lcc,
                                              uint64_t* request_id) {
    if (!s || !g || !tri || !request_id || g->ctx != s->ctx) {
        set_error("tc_lcc_server_submit: null argument or graph from another context");
        return TC_LCC_INVALID_ARGUMENT;
    }
    Request* r = new (std::nothrow) Request();
    if (!r) return TC_LCC_OUT_OF_MEMORY;
    r->g = g;
    r->tri = tri;
    r->lcc = lcc;
    if (s->arena) r->bytes = batch_graph_solo(g) ? 0 : arena_need(g);
    else r->bytes = 8ull * (uint64_t)g->d.n;
    if (s->budget && r->bytes > s->budget) {
        const unsigned long long need = r->bytes;
        delete r;
        set_error("tc_lcc_server_submit: request needs %llu bytes, budget is %llu", need,
                  (unsigned long long)s->budget);
        return TC_LCC_OVER_BUDGET;
    }
    r->t_arrive = now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            set_error("tc_lcc_server_submit: server is shutting down");
            return TC_LCC_BUSY;
        }
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->pending.push_back(r);
        *request_id = r->id;
    }
    s->cv_work.notify_one();
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_server_poll(tc_lcc_server s, uint64_t request_id, int block,
                                            tc_lcc_request_info* info) {
    if (!s) {
        set_error("tc_lcc_server_poll: null server");
        return TC_LCC_INVALID_ARGUMENT;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) {
        set_error("tc_lcc_server_poll: unknown request %llu", (unsigned long long)request_id);
        return TC_LCC_INVALID_ARGUMENT;
    }
    Request* r = it->second;
    if (!r->done) {
        if (!block) return TC_LCC_NOT_READY;
        s->cv_done.wait(lk, [&] { return r->done; });
    }
    if (info) {
        info->arrival_ns = r->t_arrive;
        info->admit_ns = r->t_admit;
        info->done_ns = r->t_done;
        info->batch_size = r->batch_size;
        info->status = r->status;
    }
    const tc_lcc_status st = r->status;
    s->reqs.erase(it);
    delete r;
    if (st != TC_LCC_OK) set_error("tc_lcc_server_poll: request failed (%s)", tc_lcc_status_string(st));
    return st;
}

extern "C" tc_lcc_status tc_lcc_server_destroy(tc_lcc_server s) {
    if (!s) {
        set_error("tc_lcc_server_destroy: null server");
        return TC_LCC_INVALID_ARGUMENT;
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->reqs) delete kv.second;
    if (s->stream) (void)hipStreamDestroy(s->stream);
    if (s->arena) s->ctx->pool->free_exact(s->arena);  // every batch has finished (the worker drained them)
    delete s;
    return TC_LCC_OK;
}
