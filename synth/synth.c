/*
 * Seeded synthetic graph generators (input generation only).
 *
 * This module produces raw edge lists (COO pairs) shaped like the workloads of
 * Strausz et al., "Asynchronous Distributed-Memory Triangle Counting and LCC
 * with RMA Caching" (Sec. IV-A: R-MAT graphs with a=0.57, b=c=0.19, d=0.05 and
 * edge factor EF, i.e. EF * 2^scale generated edges, Table II sizes).  It holds
 * none of the triangle-counting arithmetic: pairs may repeat, may be self-loops
 * and come in one direction only; removing those is the consumer's job.
 *
 * Randomness: counter-based SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Output k of the generator
 * with state s is mix(s + (k+1) * gamma), gamma = 0x9E3779B97F4A7C15, which is
 * the k-th value the sequential SplitMix64 produces from state s.  Being
 * counter-based, edge e's draws depend only on (seed, e), so generation is
 * parallel and identical for any thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* k-th output of SplitMix64 started from state s */
static inline uint64_t sm_at(uint64_t s, uint64_t k) { return sm_mix(s + (k + 1) * SM_GAMMA); }

/* independent sub-streams of one user seed */
static inline uint64_t sub_seed(uint64_t seed, uint64_t tag) { return sm_mix(seed ^ (tag * SM_GAMMA)); }

enum { TAG_RMAT = 1, TAG_PERM = 2, TAG_ER = 3, TAG_FEISTEL = 4 };

uint64_t synth_splitmix64_at(uint64_t state, uint64_t k) { return sm_at(state, k); }

/* outputs k0 .. k0 + count - 1 of the stream `state` */
void synth_splitmix64_fill(uint64_t state, uint64_t k0, int64_t count, uint64_t* out) {
    for (int64_t i = 0; i < count; ++i) out[i] = sm_at(state, k0 + (uint64_t)i);
}

/* uniform integer in [0, bound) from a 64-bit draw (multiply-high; bias < bound / 2^64) */
static inline uint64_t bounded(uint64_t r, uint64_t bound) {
    return (uint64_t)(((unsigned __int128)r * bound) >> 64);
}

/*
 * Seeded uniform permutation of [0, n) by Fisher-Yates (Knuth, TAOCP vol. 2,
 * Algorithm P): for i = n-1 .. 1 swap perm[i] with perm[j], j uniform in [0, i],
 * j drawn from output i of the permutation stream.
 */
void synth_permutation(int64_t n, uint64_t seed, int32_t* perm) {
    const uint64_t s = sub_seed(seed, TAG_PERM);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i >= 1; --i) {
        int64_t j = (int64_t)bounded(sm_at(s, (uint64_t)i), (uint64_t)i + 1);
        int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

/* R-MAT quadrant thresholds on 32-bit draws: P(q=0)=a, P(q=1)=b, P(q=2)=c, P(q=3)=1-a-b-c */
typedef struct { uint64_t t0, t1, t2; } quad_t;

static quad_t make_quad(double a, double b, double c) {
    const double two32 = 4294967296.0;
    quad_t q;
    q.t0 = (uint64_t)(a * two32 + 0.5);
    q.t1 = (uint64_t)((a + b) * two32 + 0.5);
    q.t2 = (uint64_t)((a + b + c) * two32 + 0.5);
    return q;
}

/* One R-MAT pair with `levels` quadrant descents for attempt number k.
 * Level l consumes 32 bits: the high half of draw l/2 for even l, the low half for odd l.
 * Quadrant 0 keeps both bits 0, 1 sets the column bit, 2 the row bit, 3 both. */
static inline void rmat_pair(uint64_t s, uint64_t k, int levels, quad_t q, int64_t* u, int64_t* v) {
    const uint64_t per = (uint64_t)(levels + 1) / 2;
    uint64_t r = 0, row = 0, col = 0;
    for (int l = 0; l < levels; ++l) {
        if ((l & 1) == 0) r = sm_at(s, k * per + (uint64_t)(l >> 1));
        uint64_t x = (l & 1) ? (r & 0xffffffffULL) : (r >> 32);
        uint64_t bit = 1ULL << (levels - 1 - l);
        if (x >= q.t0) {
            if (x < q.t1) col |= bit;
            else if (x < q.t2) row |= bit;
            else { row |= bit; col |= bit; }
        }
    }
    *u = (int64_t)row;
    *v = (int64_t)col;
}

/*
 * R-MAT edge list over [0, n) with m_gen pairs.
 * levels = ceil(log2 n).  When n is a power of two every attempt is accepted and
 * pair e comes from attempt e.  Otherwise attempts are taken in order and a pair
 * with an endpoint >= n is rejected, until m_gen pairs are accepted.  Finally both
 * endpoints are mapped through a seeded uniform permutation of [0, n), which
 * removes the hub-at-low-id layout of raw R-MAT.  Returns 0 on success.
 */
int synth_rmat(int64_t n, int64_t m_gen, double a, double b, double c, uint64_t seed,
               int32_t* src, int32_t* dst) {
    if (n <= 0 || n > 2147483647LL || m_gen < 0) return -1;
    int levels = 0;
    while ((1LL << levels) < n) ++levels;
    const quad_t q = make_quad(a, b, c);
    const uint64_t s = sub_seed(seed, TAG_RMAT);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!perm) return -2;
    synth_permutation(n, seed, perm);
    if ((1LL << levels) == n) {
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < m_gen; ++e) {
            int64_t u, v;
            rmat_pair(s, (uint64_t)e, levels, q, &u, &v);
            src[e] = perm[u];
            dst[e] = perm[v];
        }
    } else {
        uint64_t k = 0;
        for (int64_t e = 0; e < m_gen;) {
            int64_t u, v;
            rmat_pair(s, k++, levels, q, &u, &v);
            if (u < n && v < n) {
                src[e] = perm[u];
                dst[e] = perm[v];
                ++e;
            }
        }
    }
    free(perm);
    return 0;
}

/*
 * Erdos-Renyi style edge list: m_gen ordered pairs, each endpoint uniform in
 * [0, n) (high / low 32 bits of one draw, scaled by multiply-high).
 */
int synth_er(int64_t n, int64_t m_gen, uint64_t seed, int32_t* src, int32_t* dst) {
    if (n <= 0 || n > 2147483647LL || m_gen < 0) return -1;
    const uint64_t s = sub_seed(seed, TAG_ER);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m_gen; ++e) {
        uint64_t r = sm_at(s, (uint64_t)e);
        src[e] = (int32_t)(((r >> 32) * (uint64_t)n) >> 32);
        dst[e] = (int32_t)(((r & 0xffffffffULL) * (uint64_t)n) >> 32);
    }
    return 0;
}

/*
 * The R-MAT workload for very large scales, generated in any range of pair numbers.
 * Pair e is R-MAT attempt e at `scale` levels (n = 2^scale, no rejection), with both ends
 * relabelled by a seeded bijection of [0, n) instead of the Fisher-Yates permutation, so that
 * any range of pairs is produced without a whole-graph pass: a 4-round balanced Feistel
 * network on the scale/2 high and low bits (scale even), round r's function being
 * mix(right + key_r) masked to scale/2 bits, key_r = output r of the Feistel stream.
 * Writes pairs first .. first + count - 1.  Returns 0, or -1 for an odd or out-of-range scale.
 */
static inline uint64_t feistel(uint64_t x, int half, const uint64_t* key) {
    const uint64_t mask = (1ULL << half) - 1;
    uint64_t l = x >> half, r = x & mask;
    for (int i = 0; i < 4; ++i) {
        const uint64_t f = sm_mix(r + key[i]) & mask;
        const uint64_t nl = r;
        r = l ^ f;
        l = nl;
    }
    return (l << half) | r;
}

uint64_t synth_rmat_stream(uint64_t seed) { return sub_seed(seed, TAG_RMAT); }

void synth_feistel_keys(uint64_t seed, uint64_t* key) {
    const uint64_t s = sub_seed(seed, TAG_FEISTEL);
    for (int i = 0; i < 4; ++i) key[i] = sm_at(s, (uint64_t)i);
}

void synth_rmat_thresholds(double a, double b, double c, uint64_t* t) {
    const quad_t q = make_quad(a, b, c);
    t[0] = q.t0;
    t[1] = q.t1;
    t[2] = q.t2;
}

int synth_rmat_feistel(int scale, double a, double b, double c, uint64_t seed, uint64_t first, int64_t count,
                       int32_t* src, int32_t* dst) {
    if (scale < 2 || scale > 30 || (scale & 1) || count < 0) return -1;
    const quad_t q = make_quad(a, b, c);
    const uint64_t s = sub_seed(seed, TAG_RMAT);
    uint64_t key[4];
    synth_feistel_keys(seed, key);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        int64_t u, v;
        rmat_pair(s, first + (uint64_t)i, scale, q, &u, &v);
        src[i] = (int32_t)feistel((uint64_t)u, scale / 2, key);
        dst[i] = (int32_t)feistel((uint64_t)v, scale / 2, key);
    }
    return 0;
}
