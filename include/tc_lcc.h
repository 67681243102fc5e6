/*
 * tc_lcc — per-vertex triangle counts and local clustering coefficients on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Strausz, Vella, Di Girolamo, Besta, Hoefler, "Asynchronous
 * Distributed-Memory Triangle Counting and LCC with RMA Caching".
 *   - graph model: simple undirected graph, no multi-edges, no loops (Sec. II-A),
 *     stored as CSR with sorted adjacency lists (Sec. II-B);
 *   - t(v): triangles through v, found by intersecting sorted adjacency lists
 *     with each triangle counted once (Sec. II-C, upper-triangle offset);
 *   - LCC(v) = 2 t(v) / (d(v) (d(v) - 1)) (Eq. 2); the degree comes for free
 *     from the offsets (Sec. III-A), so the score follows the count at once;
 *   - the per-vertex loop of Alg. 3 runs over the whole graph on one GPU.
 *
 * Conventions of every call:
 *   - returns tc_lcc_status; TC_LCC_OK (0) on success.  No C++ exception
 *     crosses this interface.  On any error no output is written and
 *     tc_lcc_last_error() holds a message for the calling thread.
 *   - "device pointer" = memory of the context's GPU (hipMalloc, or a torch
 *     tensor on that device); "host pointer" = ordinary process memory.
 *   - hip_stream is a hipStream_t passed as void*; NULL means the default stream.
 *   - vertex ids are int32 in [0, n); n <= 2^31 - 1.
 *   - the caller owns every buffer it passes; the library owns contexts,
 *     graphs and tickets until the matching destroy/free/poll.
 */
#ifndef TC_LCC_H
#define TC_LCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TC_LCC_OK = 0,
    TC_LCC_INVALID_ARGUMENT = 1, /* null pointer, id outside [0, n), bad size or option */
    TC_LCC_OUT_OF_MEMORY = 2,    /* a device or host allocation failed */
    TC_LCC_OVER_BUDGET = 3,      /* the request alone exceeds the context's HBM budget */
    TC_LCC_NOT_READY = 4,        /* poll: the ticket's work has not finished yet */
    TC_LCC_BUSY = 5,             /* object still referenced by unfinished work */
    TC_LCC_DEVICE_ERROR = 6,     /* a HIP call failed */
    TC_LCC_UNSUPPORTED = 7       /* valid request this build cannot serve */
} tc_lcc_status;

typedef struct tc_lcc_ctx_s* tc_lcc_ctx;     /* one GPU: memory pool, budget, tuning, queues */
typedef struct tc_lcc_graph_s* tc_lcc_graph; /* immutable device-resident graph */
typedef uint64_t tc_lcc_ticket;              /* handle of one submitted batch */

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory the context may hold at once (graphs + scratch); 0 = no cap.
 * *out receives the context.  INVALID_ARGUMENT for a bad device or null out. */
tc_lcc_status tc_lcc_ctx_create(int device, uint64_t hbm_budget_bytes, tc_lcc_ctx* out);

/* Destroy a context.  BUSY while batches are still in flight.  Graphs built in
 * it must be freed first (BUSY otherwise). */
tc_lcc_status tc_lcc_ctx_destroy(tc_lcc_ctx ctx);

/* Device bytes the context currently holds: in_use = blocks owned by graphs, batch slots and
 * running builds; pooled = released blocks the context keeps for reuse. */
tc_lcc_status tc_lcc_ctx_memory(tc_lcc_ctx ctx, uint64_t* in_use, uint64_t* pooled);

/* Testing aid for the failure paths: the context's next `after` device allocations succeed
 * and the one after them fails with OUT_OF_MEMORY, as if HBM were exhausted (after < 0 turns
 * it off; it is off in a new context).  Every call that fails this way writes no output and
 * leaves the context usable. */
tc_lcc_status tc_lcc_debug_fail_alloc(tc_lcc_ctx ctx, int64_t after);

/* ------------------------------------------------------------------ graphs */

/* Build the device graph of n vertices from m_in raw pairs (src[e], dst[e]).
 *
 * Pairs may come in any order, repeat, be self-loops, and list an edge in one
 * or both directions; the graph is the simple undirected graph they describe
 * (Sec. II-A).  Steps, all on the GPU: drop loops, canonicalise and sort the
 * pairs, remove repeats, count degrees, rank vertices by (degree, id), relabel
 * and orient every edge from the lower to the higher rank, build the oriented
 * CSR with sorted lists (Sec. II-B) and its reverse lists, and record the
 * degrees used by Eq. 2.
 *
 * src, dst: m_in int32 each; device pointers if inputs_on_device != 0, host
 *   pointers otherwise.  They are only read, and may be freed once this returns
 *   (the call waits for its stream).
 * offset_bytes: width of the CSR offsets, 4 or 8, or 0 to pick 4 when the edge
 *   count fits int32.
 * Errors: INVALID_ARGUMENT for n outside [1, 2^31-1], m_in < 0 or >= 2^32,
 *   null pointers with m_in > 0, or any id outside [0, n); OVER_BUDGET if the
 *   graph would exceed the context budget.  */
tc_lcc_status tc_lcc_build_csr(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src,
                               const int32_t* dst, int inputs_on_device, int offset_bytes,
                               void* hip_stream, tc_lcc_graph* out);

typedef struct {
    int64_t n;                /* vertices */
    int64_t m;                /* undirected edges after cleanup */
    int32_t offset_bytes;     /* 4 or 8 */
    int32_t max_out_degree;   /* max |N+(v)| of the degree orientation */
    int64_t max_degree;       /* max d(v) */
    uint64_t wedges;          /* candidate probes of one count: oriented wedges that can close */
    uint64_t device_bytes;    /* device memory held by the graph */
    int64_t kept_in_edges;    /* in-edges (u -> v) with a nonempty tail and nonempty N+(v) */
    int64_t active_vertices;  /* vertices with at least one probe */
    int64_t staged_entries;   /* sum of |N+(v)| over active vertices (LDS staging) */
    int64_t block_vertices;   /* active vertices given a whole block (the rest get one wave) */
    int32_t count_grid;       /* blocks of the last count launch (0 before the first run) */
    int32_t count_lds_bytes;  /* LDS per block of that launch */
    int32_t count_blocks_per_cu; /* resident blocks per compute unit the occupancy query allowed */
    int32_t table_slots;      /* LDS table slots of one block */
    uint64_t push_words;      /* sum over oriented edges (u -> v) of |N+(v)| (whole-list streaming) */
    int64_t global_vertices;  /* active vertices whose N+(v) exceeds the LDS table (searched in HBM) */
    int32_t directed;         /* 1: built by tc_lcc_build_directed (m, max_degree: its undirected skeleton) */
    int32_t compact;          /* 1: built by tc_lcc_build_streamed (compact reverse lists) */
} tc_lcc_graph_stats;

tc_lcc_status tc_lcc_graph_info(tc_lcc_graph g, tc_lcc_graph_stats* out);

/* Build the device graph of a DIRECTED input for the directed clustering coefficient of Eq. 1
 * (Sec. II-D).  Pair e is the edge e_ij from v_i = src[e] to v_j = dst[e] (Sec. II-A);
 * adj(v_i) is the set of out-neighbours and deg+(v_i) its size.  Self-loops are dropped and
 * repeats of the same ordered pair count once; (i, j) and (j, i) are two different edges.
 * The graph stores the undirected skeleton (as tc_lcc_build_csr would build it from the same
 * pairs) plus, per skeleton edge, which of its two directions the input held, and every
 * vertex's out-degree.  tc_lcc_run on such a graph computes Eq. 1 (see there);
 * tc_lcc_run_edges refuses it (UNSUPPORTED); in a batch it takes the single-graph launches.
 * Arguments, ownership and errors as tc_lcc_build_csr. */
tc_lcc_status tc_lcc_build_directed(tc_lcc_ctx ctx, int64_t n, int64_t m_in, const int32_t* src,
                                    const int32_t* dst, int inputs_on_device, int offset_bytes,
                                    void* hip_stream, tc_lcc_graph* out);

/* Pair source of tc_lcc_build_streamed.  Writes pairs [first, first + count) of the input's
 * sequence of m_in pairs into src[0, count) and dst[0, count): device buffers of the library,
 * valid during the call.  Device work that writes them must be enqueued on hip_stream (or be
 * finished when the source returns).  The same (first, count) must give the same pairs on every
 * call.  Returns 0 on success; any other value ends the build with INVALID_ARGUMENT. */
typedef int (*tc_lcc_pair_source)(void* user, uint64_t first, uint64_t count, int32_t* src, int32_t* dst,
                                  void* hip_stream);

/* Build the graph of tc_lcc_build_csr from more raw pairs than device memory holds beside the
 * build (R-MAT scale 30 of Table II: 1.7e10 pairs, 137 GB as int32).  The pairs are pulled from
 * `source` in chunks of chunk_pairs (0: a default of 2^28), in several passes over the whole
 * sequence:
 *   1. a histogram of the pairs' lower ends splits the id range into partitions of about
 *      partition_pairs pairs each (0: all in one);
 *   2. one pass per partition keeps the pairs whose lower end lies in it, and sorts and
 *      deduplicates them on the GPU into the partition's rows of the upper lists (lower id to
 *      higher ids);
 *   3. the lists are ranked, oriented and sorted as by tc_lcc_build_csr, and the reverse lists
 *      are built in a compact form: u and a 16-bit position per in-edge.
 * The graph is the simple undirected graph the pairs describe (Sec. II-A), with the orientation,
 * ranks and sorted lists of tc_lcc_build_csr (Sec. II-B), so tc_lcc_run's results are the same.
 * Offsets are 8 bytes wide.  Peak device memory is about 14 bytes per pair in flight plus the
 * graph (about 13 bytes per undirected edge and 25 per vertex).
 * The in-edges of a vertex are not in rank order in this form; tc_lcc_run_edges refuses such a
 * graph (UNSUPPORTED) and a batch gives it the single-graph launches.
 * Errors: INVALID_ARGUMENT for n outside [1, 2^31-1], a null source, an id outside [0, n), a
 *   source that fails or gives more pairs in a partition on a later pass than the histogram
 *   counted; UNSUPPORTED when an oriented list is longer than 65537 entries or a partition holds
 *   2^32 pairs or more; OUT_OF_MEMORY / OVER_BUDGET as tc_lcc_build_csr.
 * Synchronous: waits for hip_stream before it returns. */
tc_lcc_status tc_lcc_build_streamed(tc_lcc_ctx ctx, int64_t n, uint64_t m_in, tc_lcc_pair_source source, void* user,
                                    uint64_t chunk_pairs, uint64_t partition_pairs, void* hip_stream,
                                    tc_lcc_graph* out);

/* Copy the built structure to host memory (for checking the builder).  Every
 * pointer may be NULL to skip that array.
 *   degree[n]     (int64) d(v) of original vertex v
 *   order[n]      (int32) original id of the vertex of rank r (rank = sort by (d, id))
 *   out_off[n+1]  (int64) oriented CSR offsets in rank space
 *   out_adj[m]    (int32) oriented lists: ranks above r, ascending
 * Synchronous. */
tc_lcc_status tc_lcc_graph_export(tc_lcc_graph g, int64_t* degree, int32_t* order, int64_t* out_off,
                                  int32_t* out_adj);

/* Free a graph.  BUSY while a batch that uses it is in flight. */
tc_lcc_status tc_lcc_graph_free(tc_lcc_graph g);

/* ------------------------------------------------------------------ one graph */

/* Per-vertex triangle counts and LCC of one graph (Alg. 3's loop over every
 * vertex; Eq. 2).
 * tri: device pointer, n uint64: tri[v] = t(v), triangles containing vertex v.
 * lcc: device pointer, n double: 2 t(v) / (d(v) (d(v)-1)) as one IEEE binary64
 *      division of exact integers; 0.0 when d(v) < 2.  May be NULL to skip.
 * For a graph from tc_lcc_build_directed, Eq. 1 instead: tri[v] = the numerator, the edges
 *      e_jk with v_j, v_k out-neighbours of v (ordered pairs: e_jk and e_kj count apart), and
 *      lcc[v] = tri[v] / (deg+(v) (deg+(v)-1)), one IEEE division; 0.0 when deg+(v) < 2.
 * Asynchronous and ordered on hip_stream; the outputs are complete when the
 * stream reaches this point.  Runs of one graph are serialised by the library
 * (they share the graph's scratch counters).  */
tc_lcc_status tc_lcc_run(tc_lcc_graph g, uint64_t* tri, double* lcc, void* hip_stream);

/* Per-edge triangle counts: the entries of C = A A o A (Sec. V-B), c_ij = the triangles that
 * contain the edge {i, j} = |adj(i) ∩ adj(j)|, together with the per-vertex results of
 * tc_lcc_run (tri required, lcc may be NULL; same meaning).
 * edge_src, edge_dst: device int32[m], edge_tri: device uint32[m], m = the graph's undirected
 *   edge count (tc_lcc_graph_info): edge e joins edge_src[e] < edge_dst[e] (original ids), the
 *   edges in ascending (edge_src, edge_dst) order, the upper triangle of A row by row; any of
 *   the three may be NULL to skip it.  c_ij < 2^31 always (it is below the smaller degree).
 * Temporaries (about 24 bytes per edge) come from the context's pool; the call waits for
 * hip_stream before it returns.  UNSUPPORTED for a directed graph; OUT_OF_MEMORY or
 * OVER_BUDGET if the temporaries cannot be had (no output is written then). */
tc_lcc_status tc_lcc_run_edges(tc_lcc_graph g, uint64_t* tri, double* lcc, int32_t* edge_src, int32_t* edge_dst,
                               uint32_t* edge_tri, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): tc_lcc_run_edges with every temporary in a static
 * device buffer of TC_LCC_NOALLOC_BYTES that the library holds on each GPU it runs on until
 * the process ends.  The call allocates nothing (no hipMalloc, no pool block, no host buffer).
 * Arguments, outputs and results are those of tc_lcc_run_edges.  Limits and behaviour:
 *   - the temporaries need 20 bytes per undirected edge, 4 per vertex and the sort's tile
 *     counts (about 2 KiB per 16384 edges), each part rounded to 256 bytes; a graph that needs
 *     more than TC_LCC_NOALLOC_BYTES gets INVALID_ARGUMENT, before any device work;
 *   - the graph's schedule is used as it stands: a tuning change since the graph's last run is
 *     not applied (applying it would allocate); results never depend on it;
 *   - every call on one GPU uses that GPU's one buffer, and each call clears what it needs,
 *     so results never depend on an earlier call; calls that overlap on one GPU (other
 *     threads, other streams) race on the buffer and must be serialised by the caller;
 *   - synchronous: the call waits for hip_stream before it returns. */
#define TC_LCC_NOALLOC_BYTES (64ull << 20)
tc_lcc_status tc_lcc_run_edges_noalloc(tc_lcc_graph g, uint64_t* tri, double* lcc, int32_t* edge_src,
                                       int32_t* edge_dst, uint32_t* edge_tri, void* hip_stream);

/* ------------------------------------------------------------------ batches */

/* Count many graphs in one persistent launch.  graphs[i] (built in ctx) writes
 * tri[i] and lcc[i] (device pointers, n_i entries; lcc[i] may be NULL).
 * Work items over (graph, vertex tile) are taken from a device queue by a grid
 * sized to the GPU; the launch is recorded once in a HIP graph and replayed.
 * *out receives a ticket for batch_poll.  Results equal tc_lcc_run's for
 * every graph.  Graphs and outputs must stay alive until the ticket is done.  A batch runs on
 * the library's own streams, not ordered after the caller's: any work of the caller that
 * writes or reads the output buffers must be complete before the submission. */
tc_lcc_status tc_lcc_batch_submit(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs,
                                  uint64_t* const* tri, double* const* lcc, tc_lcc_ticket* out);

/* NOT_READY while the batch runs (block == 0), or waits for it (block != 0).
 * *graphs_done (may be NULL) receives how many graphs of the ticket finished.
 * OK releases the ticket; INVALID_ARGUMENT for an unknown ticket. */
tc_lcc_status tc_lcc_batch_poll(tc_lcc_ctx ctx, tc_lcc_ticket t, int block, int* graphs_done);

/* Per-graph completion of a ticket that has not been released by batch_poll.
 * done: host array of count bytes (count = the graphs of the submission); done[i]
 * becomes 1 once graph i's outputs are written, which work issued afterwards on any
 * stream of the device observes.  Graphs counted together in the persistent launch
 * finish together; graphs that take the single-graph launches (directed graphs, compact
 * reverse lists, lists beyond a block's hash, or at least 2^25 probes: enough work to fill the
 * GPU alone, which the single-graph kernel with its larger tables does faster) run after it,
 * least work first, and each finishes on its own.  Does not wait and does not release the ticket.  INVALID_ARGUMENT for an
 * unknown ticket or a count that differs from the submission's. */
tc_lcc_status tc_lcc_batch_progress(tc_lcc_ctx ctx, tc_lcc_ticket t, int count, uint8_t* done);

/* ------------------------------------------------------------------ serving */

/* A request server over device-resident graphs with continuous batching.
 * A dispatcher thread admits submitted requests in arrival order while their scratch fits
 * hbm_budget_bytes (0 = no cap), gathers everything admitted at once into one batched
 * launch, and starts it as soon as fewer than max_inflight batches are running; so
 * requests that arrive while others run are batched together and overlap with them.
 * The budget is device memory actually held: a batching server with a budget takes, when
 * it is created, one zeroed arena of the budget rounded down to 8 bytes (and the context's
 * batch descriptors for max_batch graphs), and allocates nothing while it serves.
 * A batched request takes its graph's counters (8 bytes per vertex) first-fit
 * from the arena and returns them, zeroed again by the epilogue, as soon as its own graph
 * is done (tc_lcc_batch_progress), not when its whole batch is; a request whose graph takes
 * the single-graph launches (see tc_lcc_batch_progress) uses the graph's own counters.  OVER_BUDGET from create if the arena cannot be had within the context's budget.
 * max_inflight = max_batch = 1 gives the plain path: one request at a time through
 * tc_lcc_run (its budget then bounds 8 bytes per vertex of the request in flight).  Results
 * are identical to tc_lcc_run's for every request. */
typedef struct tc_lcc_server_s* tc_lcc_server;

typedef struct {
    int64_t arrival_ns; /* submit time, steady clock */
    int64_t admit_ns;   /* time the request joined a launch */
    int64_t done_ns;    /* time its outputs were seen complete */
    int32_t batch_size; /* requests in that launch */
    int32_t status;     /* tc_lcc_status of the request */
} tc_lcc_request_info;

tc_lcc_status tc_lcc_server_create(tc_lcc_ctx ctx, uint64_t hbm_budget_bytes, int max_inflight, int max_batch,
                                   tc_lcc_server* out);

/* Enqueue one request: graph g (built in the server's context), outputs tri/lcc as in
 * tc_lcc_run (device pointers, kept alive until the request is polled complete).
 * Returns at once with *request_id.  OVER_BUDGET if the request alone exceeds the budget
 * (the arena's size, for a batching server).  The request runs on the library's own streams,
 * not ordered after the caller's: any work of the caller on tri/lcc must be complete first. */
tc_lcc_status tc_lcc_server_submit(tc_lcc_server s, tc_lcc_graph g, uint64_t* tri, double* lcc,
                                   uint64_t* request_id);

/* NOT_READY while the request is queued or running (block == 0), else waits.  On
 * completion fills *info (may be NULL), releases the id and returns the request's status.
 * INVALID_ARGUMENT for an unknown id. */
tc_lcc_status tc_lcc_server_poll(tc_lcc_server s, uint64_t request_id, int block, tc_lcc_request_info* info);

/* Finish every queued and running request, then destroy the server. */
tc_lcc_status tc_lcc_server_destroy(tc_lcc_server s);

/* ------------------------------------------------------------------ tuning */

typedef enum {
    TC_LCC_PROBE_AUTO = 0,   /* per vertex: rank bitmap of N+(v) when it fits LDS, else bucket hash */
    TC_LCC_PROBE_HASH = 1,   /* bucket hash of N+(v) in LDS for every vertex */
    TC_LCC_PROBE_SORTED = 2, /* sorted N+(v) in LDS, binary search per candidate (Sec. II-C1) */
    TC_LCC_PROBE_BITMAP = 3, /* same as AUTO (the bitmap is taken wherever it fits) */
    TC_LCC_PROBE_MERGE = 4   /* sorted N+(v) in LDS; per in-edge, the rule of Eq. 3 (Sec. III-C)
                                picks a wave-wide merge path (Alg. 2, SSI) or a binary search
                                of the shorter list's keys in the longer one (Sec. II-C1) */
} tc_lcc_probe;

typedef struct {
    int32_t probe;            /* tc_lcc_probe */
    int32_t group;            /* 0 by work, 1 every vertex to one wave, 2 every vertex to one block */
    int64_t wave_work_max;    /* group 0: vertices with at most this many probes go to one wave */
    int32_t wave_outdeg_max;  /* ... and at most this |N+(v)| (0: what a wave's LDS slice holds) */
    int32_t block_threads;    /* threads per count block: 256 (the only value built; 0 = 256) */
    int32_t merge_ratio_x100; /* PROBE_MERGE: Eq. 3's right side is scaled by this / 100
                                 (0 = 100, the rule as printed; 0..100000) */
    int32_t batch_grab;       /* batched launch: light vertices a wave takes per queue access
                                 when there are plenty (1..64; 0 = 16) */
    int32_t batch_heavy_bits; /* batched launch: vertices with >= 2^(bits-1) probes get a block
                                 (1..40; 0 = 15) */
    int32_t row_sort_max;     /* builder: rows of N+ up to this long are sorted in registers after a
                                 sort by source rank (1..4096; 0 = 4096); if a longer row exists,
                                 the oriented edges get a full radix sort instead */
    int32_t reserved[4];      /* must be 0 */
} tc_lcc_tuning;

/* Read or replace the context's tuning.  Results never depend on it.  INVALID_ARGUMENT for
 * values out of range.  A graph keeps the builder settings it was built with. */
tc_lcc_status tc_lcc_get_tuning(tc_lcc_ctx ctx, tc_lcc_tuning* out);
tc_lcc_status tc_lcc_set_tuning(tc_lcc_ctx ctx, const tc_lcc_tuning* in);

/* Autotuner.  Times candidate settings on the given graphs (built in ctx) and installs the
 * fastest in ctx:
 *   what & 1: single-graph launches: wave_work_max in {1024 .. 16384} and probe in
 *             {AUTO, HASH} (the bin boundary and the probe strategy), scored by the sum
 *             over the graphs of the median tc_lcc_run time (HIP events, reps runs);
 *   what & 2: the batched launch over all the graphs: batch_grab in {1, 4, 8, 16}, then
 *             batch_heavy_bits in {12, 13, 14, 15, 16, 18}, scored by the median wall
 *             time of submit + poll (reps runs).
 * Every candidate's per-vertex counts are compared with those of the setting in force when
 * the call began; any difference returns DEVICE_ERROR (results must not depend on tuning).
 * *out (may be NULL) receives the installed setting.  If json_path is not NULL the setting
 * is written there as JSON with the device's name and the measured times.  The graphs
 * must not be in use by other work during the call.  Synchronous. */
tc_lcc_status tc_lcc_autotune(tc_lcc_ctx ctx, int count, const tc_lcc_graph* graphs, int what, int reps,
                              const char* json_path, tc_lcc_tuning* out);

/* Install a setting written by tc_lcc_autotune.  UNSUPPORTED if it was tuned on a device of
 * another name; INVALID_ARGUMENT if the file cannot be read or parsed. */
tc_lcc_status tc_lcc_tuning_load(tc_lcc_ctx ctx, const char* json_path);

/* ------------------------------------------------------------------ profiling */

/* When enabled, the builds and the runs (tc_lcc_run, tc_lcc_run_edges) record HIP events on
 * their stream around each phase; tc_lcc_graph_timings reads the durations of the graph's last
 * build and last run (waiting for the run to finish).  Milliseconds.  For tc_lcc_run_edges,
 * run_count_ms is the extended count kernel and run_epilogue_ms the LCC epilogue plus the
 * per-edge output (sort into edge order and gather). */
typedef struct {
    float build_sort_unique_ms; /* canonical keys, radix sort, unique, degrees */
    float build_rank_ms;        /* rank by (degree, id) */
    float build_orient_ms;      /* relabel, orient, radix sort, oriented CSR */
    float build_reverse_ms;     /* reverse lists and per-vertex probe counts */
    float build_schedule_ms;    /* statistics and degree/work bins */
    float run_zero_ms;          /* clear counters */
    float run_count_ms;         /* intersection + scatter kernels */
    float run_epilogue_ms;      /* LCC epilogue */
} tc_lcc_timings;

tc_lcc_status tc_lcc_set_profiling(tc_lcc_ctx ctx, int enable);
tc_lcc_status tc_lcc_graph_timings(tc_lcc_graph g, tc_lcc_timings* out);

/* ------------------------------------------------------------------ measurement */

/* Copy `bytes` from src to dst (device pointers of the current device, 16-byte aligned,
 * bytes a multiple of 16, not overlapping) with a plain streaming kernel: 16-byte vector loads
 * and stores through the shader cores.  Its rate is the achievable HBM bandwidth that the
 * count kernel's roofline fraction is also reported against, and its known size scales the
 * HBM traffic counters.  Asynchronous on hip_stream.  INVALID_ARGUMENT for a null pointer or
 * a misaligned size or address. */
tc_lcc_status tc_lcc_hbm_copy(const void* src, void* dst, uint64_t bytes, void* hip_stream);

/* ------------------------------------------------------------------ misc */

const char* tc_lcc_status_string(tc_lcc_status s);
const char* tc_lcc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TC_LCC_H */
