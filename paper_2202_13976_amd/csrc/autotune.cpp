// Autotuner: picks the work-bin boundary, the probe strategy and the batched launch's
// grab size and heavy threshold by timing candidates on the caller's graphs.
//
// The search is coordinate-wise: first the single-graph settings (wave_work_max x probe,
// then the hybrid probe of Eq. 3 at the best wave_work_max), then, on top of the best of those, batch_grab, then batch_heavy_bits.  Every candidate's
// per-vertex counts are compared with those of the setting in force when the call began,
// so a tuning that changed results would be caught here (results must not depend on it).
// The chosen setting is installed in the context and can be saved as JSON keyed by the
// device's name, and installed again later with tc_lcc_tuning_load.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"

namespace tcl {
namespace {

struct Bench {
    tc_lcc_ctx ctx;
    std::vector<tc_lcc_graph> graphs;
    std::vector<uint64_t*> tri;                 // device outputs, one per graph
    std::vector<std::vector<uint64_t>> ref;     // counts under the starting setting
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

double median(std::vector<double> v) {
    std::sort(v.begin(), v.end());
    return v.empty() ? 0.0 : v[v.size() / 2];
}

tc_lcc_status install(tc_lcc_ctx ctx, const tc_lcc_tuning& t) { return tc_lcc_set_tuning(ctx, &t); }

// Counts of every graph equal the reference (or become it when the reference is empty).
tc_lcc_status check(Bench& b) {
    const bool take = b.ref.empty();
    if (take) b.ref.resize(b.graphs.size());
    std::vector<uint64_t> h;
    for (size_t i = 0; i < b.graphs.size(); ++i) {
        const size_t n = (size_t)b.graphs[i]->d.n;
        h.resize(n);
        TCL_HIP(hipMemcpyAsync(h.data(), b.tri[i], n * sizeof(uint64_t), hipMemcpyDeviceToHost, b.st));
        TCL_HIP(hipStreamSynchronize(b.st));
        if (take) {
            b.ref[i] = h;
        } else if (h != b.ref[i]) {
            set_error("tc_lcc_autotune: graph %zu gave different counts under a candidate setting", i);
            return TC_LCC_DEVICE_ERROR;
        }
    }
    return TC_LCC_OK;
}

// Sum over the graphs of the median single-graph run time (ms), after one warm run each
// (which also rebuilds the schedule for the installed setting).
tc_lcc_status time_single(Bench& b, int reps, double* score) {
    double total = 0.0;
    std::vector<double> ts;
    for (size_t i = 0; i < b.graphs.size(); ++i) {
        tc_lcc_status s = tc_lcc_run(b.graphs[i], b.tri[i], nullptr, b.st);
        if (s != TC_LCC_OK) return s;
        ts.clear();
        for (int r = 0; r < reps; ++r) {
            TCL_HIP(hipEventRecord(b.e0, b.st));
            s = tc_lcc_run(b.graphs[i], b.tri[i], nullptr, b.st);
            if (s != TC_LCC_OK) return s;
            TCL_HIP(hipEventRecord(b.e1, b.st));
            TCL_HIP(hipEventSynchronize(b.e1));
            float ms = 0.f;
            TCL_HIP(hipEventElapsedTime(&ms, b.e0, b.e1));
            ts.push_back(ms);
        }
        total += median(ts);
    }
    *score = total;
    return check(b);
}

// Median wall time (ms) of one batched submission of all the graphs, after a warm one.
tc_lcc_status time_batch(Bench& b, int reps, double* score) {
    const int count = (int)b.graphs.size();
    std::vector<double*> lcc(b.graphs.size(), nullptr);
    std::vector<double> ts;
    for (int r = -1; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        tc_lcc_ticket tk = 0;
        tc_lcc_status s = tc_lcc_batch_submit(b.ctx, count, b.graphs.data(), b.tri.data(), lcc.data(), &tk);
        if (s != TC_LCC_OK) return s;
        s = tc_lcc_batch_poll(b.ctx, tk, 1, nullptr);
        if (s != TC_LCC_OK) return s;
        const auto t1 = std::chrono::steady_clock::now();
        if (r >= 0) ts.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count());
    }
    *score = median(ts);
    return check(b);
}

std::string device_name(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string s = std::string(p.name) + " " + p.gcnArchName;
    for (char& c : s)
        if (c == '"' || c == '\\') c = '_';
    return s;
}

tc_lcc_status write_json(const char* path, const std::string& dev, const tc_lcc_tuning& t, double single_ms,
                         double batch_ms) {
    FILE* f = fopen(path, "w");
    if (!f) {
        set_error("tc_lcc_autotune: cannot write %s", path);
        return TC_LCC_INVALID_ARGUMENT;
    }
    fprintf(f,
            "{\n \"device\": \"%s\",\n \"tuning\": {\"probe\": %d, \"group\": %d, \"wave_work_max\": %lld, "
            "\"wave_outdeg_max\": %d, \"block_threads\": %d, \"batch_grab\": %d, \"batch_heavy_bits\": %d, "
            "\"merge_ratio_x100\": %d, \"row_sort_max\": %d},\n"
            " \"single_ms\": %.6f,\n \"batch_ms\": %.6f\n}\n",
            dev.c_str(), t.probe, t.group, (long long)t.wave_work_max, t.wave_outdeg_max, t.block_threads,
            t.batch_grab, t.batch_heavy_bits, t.merge_ratio_x100, t.row_sort_max, single_ms, batch_ms);
    const bool ok = fclose(f) == 0;
    if (!ok) {
        set_error("tc_lcc_autotune: cannot write %s", path);
        return TC_LCC_INVALID_ARGUMENT;
    }
    return TC_LCC_OK;
}

// Integer value of "key": in a JSON text written by write_json.
bool json_int(const std::string& text, const char* key, long long* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t p = text.find(k);
    if (p == std::string::npos) return false;
    const char* s = text.c_str() + p + k.size();
    char* end = nullptr;
    const long long v = strtoll(s, &end, 10);
    if (end == s) return false;
    *out = v;
    return true;
}

}  // namespace
}  // namespace tcl

using namespace tcl;

extern "C" tc_lcc_status tc_lcc_autotune(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs, int what, int reps,
                                         const char* json_path, tc_lcc_tuning* out) {
    if (!ctx || count <= 0 || !graphs || reps <= 0 || (what & ~3) != 0 || what == 0) {
        set_error("tc_lcc_autotune: null argument, count <= 0, reps <= 0 or what not in 1..3");
        return TC_LCC_INVALID_ARGUMENT;
    }
    for (int i = 0; i < count; ++i)
        if (!graphs[i] || graphs[i]->ctx != ctx) {
            set_error("tc_lcc_autotune: graph %d is null or from another context", i);
            return TC_LCC_INVALID_ARGUMENT;
        }
    TCL_HIP(hipSetDevice(ctx->device));
    Bench b;
    b.ctx = ctx;
    b.graphs.assign(graphs, graphs + count);
    tc_lcc_tuning start;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        start = ctx->tuning;
    }
    tc_lcc_status st = TC_LCC_OK;
    for (int i = 0; i < count && st == TC_LCC_OK; ++i) {
        void* p = nullptr;
        st = ctx->pool->alloc((size_t)std::max<int64_t>(graphs[i]->d.n, 1) * sizeof(uint64_t), &p);
        if (st == TC_LCC_OK) b.tri.push_back((uint64_t*)p);
    }
    if (st == TC_LCC_OK && (hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking) != hipSuccess ||
                            hipEventCreate(&b.e0) != hipSuccess || hipEventCreate(&b.e1) != hipSuccess)) {
        (void)hipGetLastError();
        set_error("tc_lcc_autotune: stream or event creation failed");
        st = TC_LCC_DEVICE_ERROR;
    }

    tc_lcc_tuning best = start;
    double best_single = 0.0, best_batch = 0.0;
    auto single_pass = [&]() -> tc_lcc_status {
        // reference counts under the starting setting, then the candidates
        tc_lcc_status s = time_single(b, reps, &best_single);
        if (s != TC_LCC_OK) return s;
        const int32_t probes[] = {TC_LCC_PROBE_AUTO, TC_LCC_PROBE_HASH};
        const int64_t works[] = {1024, 2048, 4096, 8192, 16384};
        for (int32_t pr : probes)
            for (int64_t w : works) {
                tc_lcc_tuning t = best;
                t.probe = pr;
                t.group = 0;
                t.wave_work_max = w;
                s = install(ctx, t);
                if (s != TC_LCC_OK) return s;
                double ms = 0.0;
                s = time_single(b, reps, &ms);
                if (s != TC_LCC_OK) return s;
                if (ms < best_single) {
                    best_single = ms;
                    best = t;
                }
            }
        // the hybrid of Eq. 3 (merge path or binary search per in-edge) at the best bin boundary
        {
            tc_lcc_tuning t = best;
            t.probe = TC_LCC_PROBE_MERGE;
            t.merge_ratio_x100 = 0;
            s = install(ctx, t);
            if (s != TC_LCC_OK) return s;
            double ms = 0.0;
            s = time_single(b, reps, &ms);
            if (s != TC_LCC_OK) return s;
            if (ms < best_single) {
                best_single = ms;
                best = t;
            }
        }
        return install(ctx, best);
    };
    auto batch_pass = [&]() -> tc_lcc_status {
        tc_lcc_status s = install(ctx, best);
        if (s != TC_LCC_OK) return s;
        if (!(what & 1)) {
            // the counts of the starting setting are the reference
            for (size_t i = 0; i < b.graphs.size(); ++i) {
                s = tc_lcc_run(b.graphs[i], b.tri[i], nullptr, b.st);
                if (s != TC_LCC_OK) return s;
            }
            s = check(b);
            if (s != TC_LCC_OK) return s;
        }
        s = time_batch(b, reps, &best_batch);
        if (s != TC_LCC_OK) return s;
        const int32_t grabs[] = {1, 4, 8, 16};
        const int32_t bits[] = {12, 13, 14, 15, 16, 18};
        tc_lcc_tuning base = best;
        for (int32_t gsz : grabs) {
            tc_lcc_tuning t = base;
            t.batch_grab = gsz;
            s = install(ctx, t);
            if (s != TC_LCC_OK) return s;
            double ms = 0.0;
            s = time_batch(b, reps, &ms);
            if (s != TC_LCC_OK) return s;
            if (ms < best_batch) {
                best_batch = ms;
                best = t;
            }
        }
        base = best;
        for (int32_t hb : bits) {
            tc_lcc_tuning t = base;
            t.batch_heavy_bits = hb;
            s = install(ctx, t);
            if (s != TC_LCC_OK) return s;
            double ms = 0.0;
            s = time_batch(b, reps, &ms);
            if (s != TC_LCC_OK) return s;
            if (ms < best_batch) {
                best_batch = ms;
                best = t;
            }
        }
        return install(ctx, best);
    };
    if (st == TC_LCC_OK && (what & 1)) st = single_pass();
    if (st == TC_LCC_OK && (what & 2)) st = batch_pass();
    if (st != TC_LCC_OK) (void)install(ctx, start);  // leave the context as it was

    if (b.st) (void)hipStreamSynchronize(b.st);
    for (uint64_t* p : b.tri) ctx->pool->release(p);
    if (b.e0) (void)hipEventDestroy(b.e0);
    if (b.e1) (void)hipEventDestroy(b.e1);
    if (b.st) (void)hipStreamDestroy(b.st);
    if (st != TC_LCC_OK) return st;
    if (json_path) {
        st = write_json(json_path, device_name(ctx->device), best, best_single, best_batch);
        if (st != TC_LCC_OK) return st;
    }
    if (out) *out = best;
    return TC_LCC_OK;
}

extern "C" tc_lcc_status tc_lcc_tuning_load(tc_lcc_ctx ctx, const char* json_path) {
    if (!ctx || !json_path) {
        set_error("tc_lcc_tuning_load: null argument");
        return TC_LCC_INVALID_ARGUMENT;
    }
    FILE* f = fopen(json_path, "r");
    if (!f) {
        set_error("tc_lcc_tuning_load: cannot read %s", json_path);
        return TC_LCC_INVALID_ARGUMENT;
    }
    std::string text;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    fclose(f);
    const std::string key = "\"device\": \"";
    const size_t p = text.find(key);
    const size_t q = p == std::string::npos ? p : text.find('"', p + key.size());
    if (p == std::string::npos || q == std::string::npos) {
        set_error("tc_lcc_tuning_load: no device name in %s", json_path);
        return TC_LCC_INVALID_ARGUMENT;
    }
    const std::string dev = text.substr(p + key.size(), q - p - key.size());
    if (dev != device_name(ctx->device)) {
        set_error("tc_lcc_tuning_load: %s was tuned on \"%s\", this is \"%s\"", json_path, dev.c_str(),
                  device_name(ctx->device).c_str());
        return TC_LCC_UNSUPPORTED;
    }
    tc_lcc_tuning t = default_tuning();
    long long v = 0;
    struct Field {
        const char* key;
        long long* dst64;
        int32_t* dst32;
    };
    long long wwm = t.wave_work_max;
    const Field fields[] = {{"probe", nullptr, &t.probe},
                            {"group", nullptr, &t.group},
                            {"wave_work_max", &wwm, nullptr},
                            {"wave_outdeg_max", nullptr, &t.wave_outdeg_max},
                            {"block_threads", nullptr, &t.block_threads},
                            {"batch_grab", nullptr, &t.batch_grab},
                            {"batch_heavy_bits", nullptr, &t.batch_heavy_bits}};
    for (const Field& fd : fields) {
        if (!json_int(text, fd.key, &v)) {
            set_error("tc_lcc_tuning_load: no \"%s\" in %s", fd.key, json_path);
            return TC_LCC_INVALID_ARGUMENT;
        }
        if (fd.dst64) *fd.dst64 = v;
        else *fd.dst32 = (int32_t)v;
    }
    t.wave_work_max = (int64_t)wwm;
    // optional: files written before these fields existed do not have them
    if (json_int(text, "merge_ratio_x100", &v)) t.merge_ratio_x100 = (int32_t)v;
    if (json_int(text, "row_sort_max", &v)) t.row_sort_max = (int32_t)v;
    return tc_lcc_set_tuning(ctx, &t);
}
