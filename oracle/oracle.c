/*
 * CPU oracle for per-vertex triangle counts and the local clustering coefficient.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's CPU
 * baseline leg may call it; the GPU library never does, and the two share no
 * code.  Plain, single-threaded, slow on purpose: every function follows its
 * definition in Strausz et al., "Asynchronous Distributed-Memory Triangle
 * Counting and LCC with RMA Caching" so that it can be checked by eye.
 *
 * What is computed (the definition the GPU path must reach exactly):
 *   G = (V, E) simple undirected, V = [0, n), {u, v} in E iff u != v and (u, v)
 *   or (v, u) is an input pair (Sec. II-A: no multi-edges, no loops).
 *   t(v)   = number of triangles containing v
 *          = |{ {j, k} : j, k in adj(v), {j, k} in E }|          (Sec. II-D)
 *   LCC(v) = 2 t(v) / (d(v) (d(v) - 1)) for d(v) >= 2, else 0.0  (Eq. 2)
 *
 * Readings of the paper used here (each listed in the design notes):
 *   - Eq. 2's numerator counts unordered neighbour pairs, so it is t(v).
 *   - The degree in Eq. 2 is the degree in the simple undirected graph.
 *   - Vertices of degree < 2 stay in the output with t = 0 and LCC = +0.0.
 *   - Alg. 3's Intersect uses the upper-triangle offset of Sec. II-C.
 *   - Alg. 1 is taken for what Sec. II-C1 says it does (|A| lookups of the
 *     keys in the sorted longer list, counting the keys found); the printed
 *     listing is not followed line by line.
 *   - Eq. 3 picks SSI when |B|/|A| <= log2|B| - 1 (ties go to SSI).
 *
 * Also here, for the two extensions of the same method:
 *   c(e)   = triangles containing edge e = {i, j}: |adj(i) ∩ adj(j)|, the entry
 *            c_ij of C = A A o A (Sec. V-B), one per undirected edge;
 *   directed graphs (Eq. 1): adj(v_i) = out-neighbours, numerator = edges e_jk
 *            with v_j, v_k in adj(v_i), denominator deg+(v_i) (deg+(v_i) - 1).
 *
 * Pins: the tests check every function here against brute force written in
 * the test itself, closed forms, dense and sparse linear algebra (the algebraic
 * form of Sec. V-B), networkx, and exact rational arithmetic for the LCC bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Graph format (Sec. II-B): CSR with sorted adjacency lists                  */
/* ------------------------------------------------------------------------- */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/*
 * Build the CSR of the simple undirected graph behind n and the raw pairs.
 * Self-loops are dropped, each pair is stored in both directions, every list is
 * sorted and duplicates are removed.  off has n + 1 entries; adj needs room for
 * 2 * m_in entries.  Returns the number of adjacency entries (2m), or -1 if an
 * endpoint is outside [0, n).
 *
 * Method: bucket every directed entry by its source (a counting pass), sort each
 * bucket with qsort, drop repeats, then close the gaps.
 */
int64_t oracle_csr(int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst,
                   int64_t* off, int32_t* adj) {
    for (int64_t e = 0; e < m_in; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m_in; ++e) {
        if (src[e] == dst[e]) continue;
        cnt[src[e] + 1]++;
        cnt[dst[e] + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m_in; ++e) {
        if (src[e] == dst[e]) continue;
        adj[fill[src[e]]++] = dst[e];
        adj[fill[dst[e]]++] = src[e];
    }
    free(fill);
    int64_t out = 0;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t b = cnt[v], e = cnt[v + 1];
        qsort(adj + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t start = out;
        for (int64_t i = b; i < e; ++i)
            if (out == start || adj[out - 1] != adj[i]) adj[out++] = adj[i];
        off[v + 1] = out;
    }
    free(cnt);
    return out;
}

/* ------------------------------------------------------------------------- */
/* Intersections of two sorted lists (Sec. II-C1, II-C2, Eq. 3)              */
/* ------------------------------------------------------------------------- */

/* Sorted set intersection (Alg. 2): walk both lists, advance the smaller head,
 * count equal heads and advance both. */
uint64_t oracle_ssi(const int32_t* A, int64_t na, const int32_t* B, int64_t nb) {
    uint64_t counter = 0;
    int64_t i = 0, j = 0;
    while (i < na && j < nb) {
        if (A[i] == B[j]) {
            counter++;
            i++;
            j++;
        } else if (A[i] < B[j]) {
            i++;
        } else {
            j++;
        }
    }
    return counter;
}

/* Binary-search intersection (Sec. II-C1): the shorter list supplies the keys,
 * each key is looked up in the longer list; the count of keys found is returned.
 * Each lookup is a plain lower-bound search over the whole longer list. */
uint64_t oracle_bs(const int32_t* A, int64_t na, const int32_t* B, int64_t nb) {
    if (na > nb) {
        const int32_t* T = A; A = B; B = T;
        int64_t tn = na; na = nb; nb = tn;
    }
    uint64_t counter = 0;
    for (int64_t i = 0; i < na; ++i) {
        int32_t x = A[i];
        int64_t lo = 0, hi = nb; /* first index with B[idx] >= x lies in [lo, hi] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (B[mid] < x) lo = mid + 1;
            else hi = mid;
        }
        if (lo < nb && B[lo] == x) counter++;
    }
    return counter;
}

/* Eq. 3 decision with |A| <= |B|: SSI iff |B| / |A| <= log2|B| - 1.  Returns 1 for SSI. */
int oracle_eq3_prefers_ssi(int64_t na, int64_t nb) {
    if (na > nb) { int64_t t = na; na = nb; nb = t; }
    if (na == 0) return 1; /* empty intersection; either method does no lookups */
    return (double)nb / (double)na <= log2((double)nb) - 1.0;
}

/* Hybrid intersection: the method Eq. 3 selects. */
uint64_t oracle_hybrid(const int32_t* A, int64_t na, const int32_t* B, int64_t nb) {
    return oracle_eq3_prefers_ssi(na, nb) ? oracle_ssi(A, na, B, nb) : oracle_bs(A, na, B, nb);
}

typedef uint64_t (*isect_fn)(const int32_t*, int64_t, const int32_t*, int64_t);

/* ------------------------------------------------------------------------- */
/* O-A: the paper's edge-centric count (Sec. II-C, Alg. 3 on one process)     */
/* ------------------------------------------------------------------------- */

/*
 * For every vertex i and every edge e_ij: add |adj(i) ∩ {k in adj(j) : k > j}|.
 * The offset restricts the count to the upper triangle, so each pair {j, k} of
 * adjacent neighbours of i is counted once and the sum over j is t(i).
 * method: 0 = SSI (Alg. 2), 1 = binary search (Sec. II-C1), 2 = hybrid (Eq. 3).
 */
void oracle_tc_edge_centric(int64_t n, const int64_t* off, const int32_t* adj, int method,
                            uint64_t* t) {
    isect_fn f = method == 0 ? oracle_ssi : method == 1 ? oracle_bs : oracle_hybrid;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ti = 0;
        const int32_t* Ai = adj + off[i];
        int64_t ni = off[i + 1] - off[i];
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            int32_t j = adj[p];
            /* upper part of adj(j): the entries greater than j */
            int64_t s = off[j];
            while (s < off[j + 1] && adj[s] <= j) ++s;
            ti += f(Ai, ni, adj + s, off[j + 1] - s);
        }
        t[i] = ti;
    }
}

/* ------------------------------------------------------------------------- */
/* O-B: forward algorithm on the degree-ordered orientation                   */
/* ------------------------------------------------------------------------- */

/* rank order (d(v), v): returns 1 if u is ranked below v */
static inline int below(const int64_t* off, int32_t u, int32_t v) {
    int64_t du = off[u + 1] - off[u], dv = off[v + 1] - off[v];
    return du < dv || (du == dv && u < v);
}

/*
 * Every triangle has a unique lowest-ranked vertex u under the order (d(v), v).
 * N+(u) = neighbours ranked above u, kept sorted by id.  For each u, each v in
 * N+(u), and each w in N+(u) ∩ N+(v) (found by the Alg. 2 walk), the triangle
 * {u, v, w} is seen exactly once and adds 1 to t(u), t(v) and t(w).
 */
/*
 * Restricting the outer loop to u in [u_begin, u_end) gives the bounded sample
 * the benchmark times; t then holds partial counts.  Returns the number of
 * oriented edges (u, v) processed.
 */
int64_t oracle_tc_forward_range(int64_t n, const int64_t* off, const int32_t* adj,
                                int64_t u_begin, int64_t u_end, uint64_t* t) {
    int64_t* po = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t* pa = (int32_t*)malloc(sizeof(int32_t) * (size_t)(off[n] / 2 + 1));
    po[0] = 0;
    for (int64_t u = 0; u < n; ++u) {
        int64_t k = po[u];
        for (int64_t p = off[u]; p < off[u + 1]; ++p)
            if (below(off, (int32_t)u, adj[p])) pa[k++] = adj[p];
        po[u + 1] = k;
    }
    memset(t, 0, sizeof(uint64_t) * (size_t)n);
    int64_t edges = 0;
    for (int64_t u = u_begin; u < u_end; ++u) {
        for (int64_t p = po[u]; p < po[u + 1]; ++p) {
            int32_t v = pa[p];
            ++edges;
            int64_t i = po[u], j = po[v];
            while (i < po[u + 1] && j < po[v + 1]) {
                if (pa[i] == pa[j]) {
                    t[u]++;
                    t[v]++;
                    t[pa[i]]++;
                    i++;
                    j++;
                } else if (pa[i] < pa[j]) {
                    i++;
                } else {
                    j++;
                }
            }
        }
    }
    free(po);
    free(pa);
    return edges;
}

void oracle_tc_forward(int64_t n, const int64_t* off, const int32_t* adj, uint64_t* t) {
    oracle_tc_forward_range(n, off, adj, 0, n, t);
}

/* ------------------------------------------------------------------------- */
/* O-C: brute force over vertex triples                                      */
/* ------------------------------------------------------------------------- */

/* For every i < j < k with all three edges present, add 1 to t(i), t(j), t(k).
 * Dense adjacency, so only for small n. */
void oracle_tc_brute(int64_t n, const int64_t* off, const int32_t* adj, uint64_t* t) {
    uint8_t* A = (uint8_t*)calloc((size_t)(n * n), 1);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = off[i]; p < off[i + 1]; ++p) A[i * n + adj[p]] = 1;
    memset(t, 0, sizeof(uint64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
            if (!A[i * n + j]) continue;
            for (int64_t k = j + 1; k < n; ++k)
                if (A[j * n + k] && A[i * n + k]) {
                    t[i]++;
                    t[j]++;
                    t[k]++;
                }
        }
    free(A);
}

/* ------------------------------------------------------------------------- */
/* One vertex at a time (for sampled checks on graphs too large for O-B)     */
/* ------------------------------------------------------------------------- */

/* t(v) = number of edges {j, k} with j, k in adj(v), j < k: mark adj(v), then
 * for each neighbour j count its marked neighbours k > j.  mark has n bytes,
 * all zero on entry and on return. */
uint64_t oracle_tc_vertex(const int64_t* off, const int32_t* adj, int32_t v, uint8_t* mark) {
    for (int64_t p = off[v]; p < off[v + 1]; ++p) mark[adj[p]] = 1;
    uint64_t c = 0;
    for (int64_t p = off[v]; p < off[v + 1]; ++p) {
        int32_t j = adj[p];
        for (int64_t q = off[j]; q < off[j + 1]; ++q)
            if (adj[q] > j && mark[adj[q]]) c++;
    }
    for (int64_t p = off[v]; p < off[v + 1]; ++p) mark[adj[p]] = 0;
    return c;
}

/* t(v) and d(v) straight from the raw pairs, for graphs whose CSR is too large to
 * build here (Sec. II-D's definition over the simple graph of Sec. II-A): one scan
 * marks adj(v) (loops dropped, repeats marked once), a second gathers every pair
 * with both ends marked as the key (lower << 32 | higher), and the distinct keys
 * are the edges {j, k} among the neighbours: t(v) is their number.  mark has n
 * bytes, all zero on entry and on return; *deg receives d(v). */
static int cmp_u64(const void* a, const void* b) {
    const uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

uint64_t oracle_tc_vertex_pairs(int64_t m, const int32_t* src, const int32_t* dst, int32_t v, uint8_t* mark,
                                int64_t* deg) {
    int64_t d = 0;
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a == b) continue;
        const int32_t w = a == v ? b : (b == v ? a : -1);
        if (w >= 0 && !mark[w]) {
            mark[w] = 1;
            d++;
        }
    }
    int64_t cap = 1024, cnt = 0;
    uint64_t* keys = (uint64_t*)malloc((size_t)cap * sizeof(uint64_t));
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a == b || !mark[a] || !mark[b]) continue;
        if (cnt == cap) {
            cap *= 2;
            keys = (uint64_t*)realloc(keys, (size_t)cap * sizeof(uint64_t));
        }
        const uint64_t lo = (uint64_t)(a < b ? a : b), hi = (uint64_t)(a < b ? b : a);
        keys[cnt++] = lo << 32 | hi;
    }
    qsort(keys, (size_t)cnt, sizeof(uint64_t), cmp_u64);
    uint64_t t = 0;
    for (int64_t i = 0; i < cnt; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) t++;
    free(keys);
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a == v) mark[b] = 0;
        if (b == v) mark[a] = 0;
    }
    *deg = d;
    return t;
}

/* ------------------------------------------------------------------------- */
/* LCC (Eq. 2)                                                               */
/* ------------------------------------------------------------------------- */

/* LCC(v) = (2 t(v)) / (d(v) (d(v) - 1)), both integers formed exactly in 64 bits,
 * then one IEEE binary64 division (round to nearest even).  d < 2 gives 0.0. */
double oracle_lcc_one(uint64_t t, int64_t d) {
    if (d < 2) return 0.0;
    uint64_t num = 2 * t;
    uint64_t den = (uint64_t)d * (uint64_t)(d - 1);
    return (double)num / (double)den;
}

void oracle_lcc(int64_t n, const int64_t* off, const uint64_t* t, double* lcc) {
    for (int64_t v = 0; v < n; ++v) lcc[v] = oracle_lcc_one(t[v], off[v + 1] - off[v]);
}

/* ------------------------------------------------------------------------- */
/* Per-edge triangle counts (Sec. V-B: C = A A o A)                          */
/* ------------------------------------------------------------------------- */

/*
 * Entry c_ij of C = A A o A is the number of triangles that contain the edge
 * e_ij: the common neighbours of i and j, |adj(i) ∩ adj(j)| (Alg. 2).  One
 * output per undirected edge {i, j}, i < j, in the order of the CSR's upper
 * triangle (i ascending, then j ascending).  eu, ev and c need m = off[n] / 2
 * entries.  Returns the number of edges written.
 */
int64_t oracle_edge_counts(int64_t n, const int64_t* off, const int32_t* adj, int32_t* eu, int32_t* ev,
                           uint64_t* c) {
    int64_t e = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            int32_t j = adj[p];
            if (j <= i) continue;
            eu[e] = (int32_t)i;
            ev[e] = j;
            c[e] = oracle_ssi(adj + off[i], off[i + 1] - off[i], adj + off[j], off[j + 1] - off[j]);
            ++e;
        }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Directed graphs: Eq. 1                                                    */
/* ------------------------------------------------------------------------- */

/*
 * CSR of the directed graph behind the raw pairs (Sec. II-A: e_ij is the edge
 * from v_i to v_j, adj(v_i) its out-neighbours): self-loops dropped, repeats of
 * the same ordered pair removed, each out-list sorted.  off has n + 1 entries,
 * adj room for m_in.  Returns the number of edges, or -1 for an endpoint
 * outside [0, n).
 */
int64_t oracle_csr_directed(int64_t n, int64_t m_in, const int32_t* src, const int32_t* dst, int64_t* off,
                            int32_t* adj) {
    for (int64_t e = 0; e < m_in; ++e)
        if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return -1;
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < m_in; ++e)
        if (src[e] != dst[e]) cnt[src[e] + 1]++;
    for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t e = 0; e < m_in; ++e)
        if (src[e] != dst[e]) adj[fill[src[e]]++] = dst[e];
    free(fill);
    int64_t out = 0;
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t b = cnt[v], e = cnt[v + 1];
        qsort(adj + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t start = out;
        for (int64_t i = b; i < e; ++i)
            if (out == start || adj[out - 1] != adj[i]) adj[out++] = adj[i];
        off[v + 1] = out;
    }
    free(cnt);
    return out;
}

/*
 * Numerator of Eq. 1 for every vertex i: the edges e_jk with v_j, v_k in
 * adj(v_i).  Edge-centric as in Sec. II-C: for every e_ij, the out-neighbours of
 * j that are also out-neighbours of i, |adj(i) ∩ adj(j)| (Alg. 2).  There is no
 * upper-triangle offset here: e_jk and e_kj are different edges of a directed
 * graph and each one present counts.
 */
void oracle_tc_directed(int64_t n, const int64_t* off, const int32_t* adj, uint64_t* num) {
    for (int64_t i = 0; i < n; ++i) {
        uint64_t s = 0;
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            int32_t j = adj[p];
            s += oracle_ssi(adj + off[i], off[i + 1] - off[i], adj + off[j], off[j + 1] - off[j]);
        }
        num[i] = s;
    }
}

/* Eq. 1: C(i) = num(i) / (deg+(i) (deg+(i) - 1)), both integers exact in 64 bits and one
 * IEEE binary64 division (round to nearest even); deg+ < 2 gives 0.0. */
double oracle_lcc_directed_one(uint64_t num, int64_t dout) {
    if (dout < 2) return 0.0;
    uint64_t den = (uint64_t)dout * (uint64_t)(dout - 1);
    return (double)num / (double)den;
}

void oracle_lcc_directed(int64_t n, const int64_t* off, const uint64_t* num, double* lcc) {
    for (int64_t v = 0; v < n; ++v) lcc[v] = oracle_lcc_directed_one(num[v], off[v + 1] - off[v]);
}
