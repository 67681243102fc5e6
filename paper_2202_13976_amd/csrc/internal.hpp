// Internal host-side structures and cross-file launchers of the tc_lcc library.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/tc_lcc.h"
#include "common.hpp"

namespace tcl {

// 64-bit offsets of a graph whose reverse lists are compact (u and a 16-bit row position per
// in-edge instead of u, tail start and tail length): a type of its own, so that kernels
// instantiated for it read the compact form (kCompactOff) and those for int64_t do not.
using OffCompact = long long;
static_assert(sizeof(OffCompact) == 8, "64-bit offsets");
static_assert(!std::is_same<OffCompact, int64_t>::value, "OffCompact must differ from int64_t");
template <typename OffT>
constexpr bool kCompactOff = std::is_same<OffT, OffCompact>::value;

// count kernel geometry: 256-thread blocks (4 waves); one block per heavy vertex,
// one wave per light vertex, each with an LDS table of N+(v).
constexpr int kCountThreads = 256;
constexpr int kWavesPerBlock = kCountThreads / kWave;
constexpr int32_t kMaxTableSlots = 4096;  // 4096 x (4 B id + 4 B counter) = 32 KiB per block
constexpr int kBigWorkBits = 15;          // default: probes >= 2^14 get a block in the batched launch

int resolve_probe(int probe, int64_t n);
int32_t table_slots(int probe, int32_t dplus_max);

// Bucket hash of a list of dv keys: a power of two >= 2 dv slots (load <= 1/2), at least 64.
// capacity(T) is the longest list a table of T slots takes.  (A load of 2/3 halves the
// tables of the largest lists but was slower at R-MAT scale 23: more vertices leave the
// bitmap and the wave slices.)
__host__ __device__ inline int32_t hash_table_slots(int32_t dv) {
    int32_t T = 64;
    while (T < 2 * dv) T <<= 1;
    return T;
}
__host__ __device__ inline int32_t hash_capacity(int32_t T) { return T / 2; }

// LDS bytes of the rank bitmap of a list of dv entries spanning `words` 32-rank words: the words
// with their first indices (plus a zero guard word), dv counters and one spare word per lane.
// The count takes the bitmap for a vertex wherever this fits its region, and the schedule keeps
// a block vertex whose list exceeds the hash in the block bins when it fits the block's table.
__host__ __device__ inline uint32_t bitmap_bytes(uint32_t words, int32_t dv) {
    return 8u * (words + 1u) + 4u * (uint32_t)dv + 4u * kWave;
}

// ------------------------------------------------------------------ device memory pool
// Caching allocator per context.  Blocks are rounded to size classes and kept on
// free lists after release; the budget covers blocks in use plus cached blocks.
class Pool {
   public:
    Pool(int device, uint64_t budget) : device_(device), budget_(budget) {}
    int device() const { return device_; }
    ~Pool();
    tc_lcc_status alloc(size_t bytes, void** out);
    void release(void* p);  // caller guarantees no pending device work uses p
    void trim();            // hipFree every cached block
    uint64_t in_use() const { return in_use_; }
    uint64_t pooled() const { return pooled_; }
    uint64_t budget() const { return budget_; }
    static size_t round(size_t bytes);
    // failure injection: the next `after` allocations succeed, the one after fails (< 0: off)
    void fail_after(int64_t after);
    // a block of exactly `bytes` (no size class), counted in use until free_exact, which gives
    // it back to HIP at once instead of caching it
    tc_lcc_status alloc_exact(size_t bytes, void** out);
    void free_exact(void* p);

   private:
    int device_;
    uint64_t budget_;
    uint64_t in_use_ = 0, pooled_ = 0;
    int64_t fail_after_ = -1;
    std::mutex mu_;
    std::multimap<size_t, void*> free_;
    std::unordered_map<void*, size_t> live_;
};

// ------------------------------------------------------------------ graph on the device
struct GraphDev {
    int64_t n = 0, m = 0;
    int off_bytes = 8;   // width of out_off / in_off / in_start
    int bits = 1;        // ceil(log2 n), at least 1
    void* out_off = nullptr;    // [n+1] oriented CSR offsets (rank space)
    int32_t* adj = nullptr;     // [m]   oriented lists, ascending ranks
    void* in_off = nullptr;     // [n+1] reverse lists: in-edges (u -> v) with a nonempty tail
    int32_t* in_u = nullptr;    // [m_in_kept] u of each in-edge
    void* in_start = nullptr;   // [m_in_kept] position in adj right after v inside N+(u)
    int32_t* in_len = nullptr;  // [m_in_kept] length of that tail of N+(u)
    // compact reverse lists (streamed build): in_start and in_len are absent; in_pos holds
    // the position of v in N+(u), so the tail is out_off[u] + in_pos + 1 .. out_off[u + 1]
    bool compact = false;
    uint16_t* in_pos = nullptr;  // [m_in_kept]
    int64_t m_in_kept = 0;
    int32_t* order = nullptr;   // [n] original id of rank r
    int32_t* deg_r = nullptr;   // [n] degree of rank r
    int32_t* dplus = nullptr;   // [n] |N+(r)|
    uint64_t* work = nullptr;   // [n] probes of r's count = sum of its in-edge tails
    unsigned long long* t_rank = nullptr;  // [n] scratch counters (rank space)
    unsigned int* counters = nullptr;      // [8] work-queue counters of the count kernel
    int32_t* vlist = nullptr;   // [n] scheduled vertices: block bin, wave bin, global bin
    int64_t n_block = 0, n_wave = 0, n_global = 0;
    int64_t n_list = 0;         // block vertices too long for the hash: the table as a sorted list
    int64_t class_count[48] = {};  // block-class vertices per work class (class c: bit length 40 - c)

    int32_t hash_slots = 64;    // LDS hash slots of one block (power of two)
    int32_t max_dplus = 0;
    int64_t max_deg = 0;
    uint64_t wedges = 0;
    uint64_t staged = 0;        // sum of |N+(v)| over vertices with work
    uint64_t push_words = 0;    // sum over oriented edges (u -> v) of |N+(v)|
    uint64_t device_bytes = 0;
    // profiling events: 0..5 build phase boundaries, 6..9 run phase boundaries
    hipEvent_t ev[10] = {};
    bool prof = false;
    int32_t count_grid = 0, count_lds = 0, count_per_cu = 0;  // last count launch
    int sched_probe = -1;       // probe the schedule was built for
    uint64_t sched_gen = ~0ull; // tuning generation the schedule was built for
    // directed input (Eq. 1): the lists above are its undirected skeleton
    bool directed = false;
    uint8_t* dir = nullptr;     // [m] per oriented edge: bit 0 input held low rank -> high rank,
                                //     bit 1 high -> low
    int32_t* dout_r = nullptr;  // [n] out-degree of rank r in the directed input
};

}  // namespace tcl

struct tc_lcc_ctx_s {
    int device = 0;
    std::unique_ptr<tcl::Pool> pool;
    std::mutex mu;
    tc_lcc_tuning tuning{};
    uint64_t tuning_gen = 0;
    std::atomic<int> graphs{0};
    std::atomic<int> tickets_inflight{0};
    int cu_count = 256;
    size_t lds_per_block = 65536;
    bool profiling = false;
    void* batch = nullptr;  // batch engine state (batch.cpp)
};

struct tc_lcc_graph_s {
    tc_lcc_ctx ctx = nullptr;
    tcl::GraphDev d;
    std::vector<void*> blocks;  // pool blocks owned by the graph
    hipEvent_t last_use = nullptr;
    std::atomic<int> inflight{0};
    std::mutex mu;
};

namespace tcl {

inline void mark(GraphDev& d, int i, hipStream_t st) {
    if (d.prof && d.ev[i]) (void)hipEventRecord(d.ev[i], st);
}

// radix.hip
size_t radix_sort_scratch_bytes(size_t n);
hipError_t radix_sort_u64(uint64_t* keys, uint64_t* alt, size_t n, int lo_bit, int nbits, void* scratch,
                          unsigned int* err, hipStream_t st, uint64_t** result, bool counted = false);
hipError_t radix_sort_u32(uint32_t* keys, uint32_t* alt, size_t n, int lo_bit, int nbits, void* scratch,
                          unsigned int* err, hipStream_t st, uint32_t** result, bool counted = false);
// counted = true: the caller has cleared the digit counts of the scratch (radix_counts_clear)
// and a kernel writing the keys has added every key's digits to radix_counts(scratch)
uint32_t* radix_counts(void* scratch);
hipError_t radix_counts_clear(void* scratch, hipStream_t st);

// build.hip
tc_lcc_status build_graph(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src,
                          const int32_t* dst, int inputs_on_device, int offset_bytes,
                          const tc_lcc_tuning& tn, hipStream_t st, tc_lcc_graph g, bool directed = false);
tc_lcc_status build_schedule(tc_lcc_graph g, const tc_lcc_tuning& tn, hipStream_t st);
// the streamed, partitioned build (compact reverse lists); source(first, count, src, dst, st)
// writes pairs [first, first + count) into the device buffers, ordered before later work on st
using StreamSource = std::function<tc_lcc_status(uint64_t, uint64_t, int32_t*, int32_t*, hipStream_t)>;
tc_lcc_status build_streamed(tc_lcc_ctx ctx, int64_t n, uint64_t m_in, const StreamSource& source, uint64_t chunk,
                             uint64_t part_cap, const tc_lcc_tuning& tn, hipStream_t st, tc_lcc_graph g);

// count.hip
// spare_per_cu: resident blocks per CU left free for other streams' kernels (0 = fill the GPU)
tc_lcc_status launch_count(tc_lcc_graph g, const tc_lcc_tuning& tn, int spare_per_cu, hipStream_t st);
tc_lcc_status launch_epilogue(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st);
tc_lcc_status launch_zero_counts(tc_lcc_graph g, hipStream_t st);

// count_ext.hip: counts that carry more per triangle (see there)
tc_lcc_status launch_count_edges(tc_lcc_graph g, uint32_t* ce, hipStream_t st);  // ce: [m], zeroed
tc_lcc_status launch_count_directed(tc_lcc_graph g, hipStream_t st);
tc_lcc_status launch_epilogue_directed(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st);
// per-edge outputs in (lower id, higher id) order from the per-position counts ce; keys and alt
// hold m words, scratch radix_sort_scratch_bytes(m), rank n entries
hipError_t edge_output(const GraphDev& d, uint64_t* keys, uint64_t* alt, void* scratch, unsigned int* err,
                       int32_t* rank, const uint32_t* ce, int32_t* es, int32_t* ed, uint32_t* ec, hipStream_t st);

// batch.hip
tc_lcc_status batch_engine_create(tc_lcc_ctx ctx);
void batch_engine_destroy(tc_lcc_ctx ctx);
// the batch engine's lock; it is taken before any graph's lock
std::mutex& batch_mutex(tc_lcc_ctx ctx);
// make st wait for every batch in flight that holds g (caller holds batch_mutex)
tc_lcc_status batch_fence_graph(tc_lcc_ctx ctx, tc_lcc_graph g, hipStream_t st);
// the submission of tc_lcc_batch_submit; scratch (may be null): per graph, zeroed counters of
// n entries the batch uses instead of the slot's own (graphs that take the single-graph
// launches ignore theirs); they are zero again once the graph's done flag is up
tc_lcc_status batch_submit_with(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs, uint64_t* const* tri,
                                double* const* lcc, unsigned long long* const* scratch, tc_lcc_ticket* out);
// whether a batch runs g through the single-graph launches (directed, compact reverse lists, or
// lists longer than a block's hash)
bool batch_graph_solo(tc_lcc_graph g);
// grow every idle slot's descriptors and flags to `graphs` entries now, so that later
// submissions of up to that many graphs with caller-given counters allocate nothing
tc_lcc_status batch_reserve(tc_lcc_ctx ctx, size_t graphs);

// api.cpp: the single-graph run of tc_lcc_run, with launch_count's spare_per_cu;
// engine_locked: the caller holds batch_mutex (tc_lcc_batch_submit)
tc_lcc_status run_graph(tc_lcc_graph g, uint64_t* tri, double* lcc, hipStream_t st, int spare_per_cu,
                        bool engine_locked = false);

// tuning defaults
tc_lcc_tuning default_tuning();

// api.cpp: the address of `device`'s copy of the static scratch of tc_lcc_run_edges_noalloc
// (looked up with that device current, once, and kept)
tc_lcc_status noalloc_base(int device, uint8_t** out);

}  // namespace tcl
