// Device code shared by the single-graph and the batched count kernels: the staged
// N+(v) (rank bitmap, bucket hash or sorted list in LDS), the tail walk that probes
// every candidate, and the per-triangle scatter.  See count.hip for the method.
#pragma once

#include "internal.hpp"

namespace tcl {

constexpr int kUnroll = 4;  // prefetched windows of 64 candidates

// Global-memory accessors.  A pointer that a kernel reads from memory (the batched path's graph
// descriptors) is a generic address to the compiler, and generic (flat) loads and atomics count
// against the same wait counter as LDS operations, so every LDS synchronisation of a walk would
// also wait for the memory operations in flight.  Every array the count reads or adds to lies in
// global memory; accessing it through a pointer of the global address space says so (pointers
// from kernel arguments are known to be global already).
template <typename T, typename I>
__device__ __forceinline__ T gld(const T* p, I i) {
    return ((const __attribute__((address_space(1))) T*)p)[i];
}
__device__ __forceinline__ void gadd(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long*)p, v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename OffT>
struct CountArgs {
    const OffT* out_off;
    const int32_t* adj;
    const OffT* in_off;
    const int32_t* in_u;
    const OffT* in_start;
    const int32_t* in_len;
    const uint16_t* in_pos;  // compact reverse lists (OffT = OffCompact): position of v in N+(u)
    const int32_t* vlist;
    int64_t n_block, n_wave, n_global;
    unsigned long long* t;
    unsigned int* ctr;
    int32_t slots;       // table slots of a block (power of two, >= 256)
    int32_t merge_x100;  // hybrid probe: scale of Eq. 3's right side, in hundredths
};

// bucket hash: high bits of a 24x24-bit product (one full-rate multiply)
__device__ __forceinline__ uint32_t hash32(int32_t x) { return __umul24((uint32_t)x, 0x9E3779u); }

template <int NWAVES>
__device__ __forceinline__ void group_sync() {
    if constexpr (NWAVES > 1) __syncthreads();
    else wave_lds_sync();
}

// Bucketed open addressing: 4 slots per bucket read with one 16-byte LDS load; a key
// lives in the first bucket with room from its hash bucket on.  Returns slot or -1.
__device__ __forceinline__ int hash_find(const int32_t* keys, uint32_t nb_mask, int logNB, int32_t x) {
    uint32_t b = logNB ? (hash32(x) >> (32 - logNB)) : 0u;
    for (;;) {
        const int4 k = *reinterpret_cast<const int4*>(keys + 4 * b);
        if (k.x == x) return (int)(4 * b);
        if (k.y == x) return (int)(4 * b + 1);
        if (k.z == x) return (int)(4 * b + 2);
        if (k.w == x) return (int)(4 * b + 3);
        if ((k.x | k.y | k.z | k.w) < 0) return -1;  // a free slot: x is absent
        b = (b + 1) & nb_mask;
    }
}

// continue a lookup at bucket b (after the first bucket was full and did not hold x)
__device__ __forceinline__ int hash_find_from(const int32_t* keys, uint32_t nb_mask, uint32_t b, int32_t x) {
    for (;;) {
        const int4 k = *reinterpret_cast<const int4*>(keys + 4 * b);
        if (k.x == x) return (int)(4 * b);
        if (k.y == x) return (int)(4 * b + 1);
        if (k.z == x) return (int)(4 * b + 2);
        if (k.w == x) return (int)(4 * b + 3);
        if ((k.x | k.y | k.z | k.w) < 0) return -1;
        b = (b + 1) & nb_mask;
    }
}

__device__ __forceinline__ void hash_insert(int32_t* keys, uint32_t nb_mask, int logNB, int32_t x) {
    uint32_t b = logNB ? (hash32(x) >> (32 - logNB)) : 0u;
    for (;;) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (atomicCAS(&keys[4 * b + k], -1, x) == -1) return;
        b = (b + 1) & nb_mask;
    }
}

__device__ __forceinline__ int sorted_find(const int32_t* keys, int32_t T, int32_t x) {
    int lo = 0, hi = T;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (keys[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return (lo < T && keys[lo] == x) ? lo : -1;
}

// The same search in a list that lies in global memory: is x in it?
__device__ __forceinline__ bool sorted_find_global(const int32_t* keys, int32_t T, int32_t x) {
    int lo = 0, hi = T;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gld(keys, mid) < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < T && gld(keys, lo) == x;
}

// A window: 64 consecutive candidates of one tail (lane i takes candidate base + i).
template <typename OffT>
struct Win {
    OffT st;      // tail start in adj
    int32_t len;  // tail length
    int32_t base; // first candidate of the window within the tail
    int32_t j;    // tail index within the wave's chunk (-1: no window)
};

// LDS view of the staged N+(v) for one probe method.
//   hash:   keys[T] (-1 = empty) and cnt[T], 4-slot buckets
//   sorted: keys[dv] = N+(v) and cnt[dv], binary search (or the hybrid of Eq. 3)
//   bitmap: bm[2 (words + 1)]: per 32-rank word of the range (v, vmax] the bits and the
//           index in N+(v) of the word's first entry, plus one zero guard word; cnt[dv].
//           The entry index of a hit is first + popcount of the bits below it; candidates
//           outside the range clamp onto the guard word.  One 8-byte LDS read per probe.
// Probe mode of lists longer than any LDS table: binary search in N+(v) where it lies in HBM,
// each hit added to t(w) at once (not a value of the public probe enum).
constexpr int kProbeGlobal = 16;

struct Table {
    int32_t* keys;           // LDS: hash slots or the sorted list
    const int32_t* gkeys;    // global mode: N+(v) where it lies in HBM
    uint32_t* cnt;
    unsigned long long* tg;  // global mode: t
    uint32_t* bm;
    int32_t T;
    uint32_t nb_mask;
    int logNB;
    int32_t base;   // bitmap: rank v + 1 is bit 0
    uint32_t span;  // bitmap: ranks v + 1 .. vmax
    uint32_t words;
};

// One candidate x against the hash or sorted table (the bitmap probe is inlined in the
// tail walk); counts the hit at its entry.
template <int MODE>
__device__ __forceinline__ bool probe_one(const Table& tb, int32_t x, bool val) {
    bool hit = false;
    if constexpr (MODE == TC_LCC_PROBE_HASH) {
        // bucket chain from the home bucket; each matching key bumps its own counter (the
        // slot is the bucket address plus an immediate offset)
        uint32_t b = hash32(x) >> (32 - tb.logNB);
        bool pending = val;
        for (;;) {
            const int4 kk = *reinterpret_cast<const int4*>(tb.keys + 4 * b);
            uint32_t* cb = tb.cnt + 4 * b;
            if (pending) {
                if (kk.x == x) {
                    atomicAdd(cb, 1u);
                    hit = true;
                }
                if (kk.y == x) {
                    atomicAdd(cb + 1, 1u);
                    hit = true;
                }
                if (kk.z == x) {
                    atomicAdd(cb + 2, 1u);
                    hit = true;
                }
                if (kk.w == x) {
                    atomicAdd(cb + 3, 1u);
                    hit = true;
                }
            }
            // keep looking only past a full bucket that did not hold x
            pending = pending && !hit && min(min(kk.x, kk.y), min(kk.z, kk.w)) >= 0;
            if (!__ballot(pending)) break;
            b = pending ? ((b + 1) & tb.nb_mask) : b;
        }
    } else if constexpr (MODE == kProbeGlobal) {
        hit = val && sorted_find_global(tb.gkeys, tb.T, x);
        if (hit) gadd(tb.tg + x, 1ull);
    } else {
        const int sl = sorted_find(tb.keys, tb.T, x);
        hit = val && sl >= 0;
        if (hit) atomicAdd(&tb.cnt[sl], 1u);
    }
    return hit;
}

// v's in-edge range and this lane's in-edge of the wave's first chunk (u, tail start, tail
// length), loaded as soon as v is known so that they arrive while N+(v) is staged.  Wave wig of
// NWAVES takes in-edges i0 + wig, i0 + wig + NWAVES, ...: lane l of a chunk holds the l-th.
template <typename OffT>
struct InEdges {
    OffT i0, i1;
    int32_t u;
    OffT st;
    int32_t len;
};

// In-edge k: u, the start of its tail in adj and the tail's length.  Compact reverse lists
// hold u and the position p of v in N+(u); the tail is N+(u) after p.
template <typename OffT>
__device__ __forceinline__ void load_in_edge(const CountArgs<OffT>& a, OffT k, int32_t& u, OffT& st, int32_t& len) {
    u = gld(a.in_u, k);
    if constexpr (kCompactOff<OffT>) {
        const OffT o0 = gld(a.out_off, u), o1 = gld(a.out_off, u + 1);
        st = o0 + (OffT)gld(a.in_pos, k) + 1;
        len = (int32_t)(o1 - st);
    } else {
        st = gld(a.in_start, k);
        len = gld(a.in_len, k);
    }
}

template <int NWAVES, typename OffT>
__device__ __forceinline__ InEdges<OffT> first_in_edges(const CountArgs<OffT>& a, OffT i0, OffT i1, int wig) {
    InEdges<OffT> e;
    e.i0 = i0;
    e.i1 = i1;
    e.u = 0;
    e.st = 0;
    e.len = 0;
    const OffT k = e.i0 + (OffT)lane_id() * NWAVES + wig;
    if (k < e.i1) load_in_edge(a, k, e.u, e.st, e.len);
    return e;
}

template <int NWAVES, typename OffT>
__device__ __forceinline__ InEdges<OffT> first_in_edges(const CountArgs<OffT>& a, int32_t v, int wig) {
    return first_in_edges<NWAVES>(a, gld(a.in_off, v), gld(a.in_off, v + 1), wig);
}

// The waves of a group walk the tails of v's in-edges, 64 in-edges (a chunk) at a time,
// and probe every candidate in windows of 64 consecutive candidates of one tail.  Wave
// wig of NWAVES takes in-edges wig, wig + NWAVES, ... (its chunks hold every NWAVES-th
// in-edge), so the waves of a block share each vertex evenly whatever its in-degree, and
// every tail stays with one wave.
//
// The window generator's state is wave-uniform (tail j is owned by lane j; the tail's
// start pointer is formed once per tail), so a window costs a few scalar operations.  A
// ring of 2 * kUnroll windows is kept in flight: the loads of one half arrive while the
// other half is probed.  For the rank bitmap the LDS reads of all windows of a half are
// issued before any is used, so one LDS round trip serves kUnroll windows.  Every hit
// found here is a triangle with v as its middle vertex, so the hits are also v's share
// (`local`).
template <typename OffT, int MODE, int NWAVES>
__device__ __forceinline__ void walk_tails(const CountArgs<OffT>& a, const InEdges<OffT>& ie, const Table& tb, int wig,
                           unsigned long long& local) {
    constexpr int kRing = 2 * kUnroll;
    const int lane = lane_id();
    const uint32_t lane4 = (uint32_t)lane * 4u;
    wig = __builtin_amdgcn_readfirstlane(wig);  // wave-uniform: keeps the generator scalar
    const OffT i0 = ie.i0, i1 = ie.i1;
    // the in-edges of the next chunk are loaded while this one is walked
    int32_t nu = ie.u;
    OffT nst = ie.st;
    int32_t nlen = ie.len;
    constexpr OffT kSpan = (OffT)kWave * NWAVES;  // in-edges a chunk of the group covers
    for (OffT cb = i0; cb < i1; cb += kSpan) {
        const OffT k = cb + (OffT)lane * NWAVES + wig;
        const bool ok = k < i1;
        const int32_t u = nu;
        const OffT st = nst;
        const int32_t len = nlen;
        if (k + kSpan < i1) load_in_edge(a, k + kSpan, nu, nst, nlen);
        // lanes of this wave holding an in-edge of the chunk
        const OffT rest = i1 - cb - wig;
        const int nk = (int)__builtin_amdgcn_readfirstlane(
            rest <= 0 ? 0 : (int)min((OffT)kWave, (rest + NWAVES - 1) / NWAVES));
        uint32_t mine = 0;  // hits of the tail this lane owns (tail index == lane)
        // this lane's tail as an address and a byte length, formed once per chunk, so that a
        // tail switch only reads them out of the owner lane (the loads cast the address to the
        // global address space)
        const uint64_t taddr = (uint64_t)(uintptr_t)a.adj + (uint64_t)st * 4u;
        const uint32_t tbytes = (uint32_t)len * 4u;

        // generator (wave-uniform): tail gj (gjv = gj while gj < nk, else -1), next window at
        // byte gbase4 of the tail, the tail's last candidate at byte glast4; a spent generator
        // yields windows of tail -1 that read adj[0]
        const char* tptr = (const char*)a.adj;
        int gj = 0, gjv = -1;
        int32_t gbase4 = 0, gend4 = 4;
        uint32_t glast4 = 0;
        auto fetch_tail = [&]() {
            if (gj < nk) {
                tptr = (const char*)(uintptr_t)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)taddr, gj) |
                                                 ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(taddr >> 32), gj)
                                                  << 32));
                gend4 = (int32_t)__builtin_amdgcn_readlane(tbytes, gj);
                gjv = gj;
            } else {
                tptr = (const char*)a.adj;
                gend4 = 4;
                gjv = -1;
            }
            glast4 = (uint32_t)gend4 - 4u;
        };
        // next window: the next 64 candidates of this tail, else the start of this wave's
        // next tail
        auto advance = [&]() {
            gbase4 += kWave * 4;
            if (__builtin_expect(gbase4 >= gend4, 0)) {
                gbase4 = 0;
                gj += 1;
                fetch_tail();
            }
        };
        gj = 0;
        fetch_tail();
        // next window of this wave: its tail j, the bytes of candidates from the window on
        // (lanes with lane4 >= lim hold none), and this lane's candidate (lanes past the tail
        // re-read its last one); a spent generator yields tail -1
        auto gen = [&](int& j, int& lim) -> int32_t {
            j = gjv;
            lim = gend4 - gbase4;
            const uint32_t off4 = min((uint32_t)gbase4 + lane4, glast4);
            const int32_t x = gld((const int32_t*)(tptr + off4), 0);
            advance();
            return x;
        };

        int js[kRing], lims[kRing];
        int32_t xs[kRing];
#pragma unroll
        for (int q = 0; q < kRing; ++q) xs[q] = gen(js[q], lims[q]);
        // a window's hits go to the lane that owns its tail: one vector add with only that lane
        // in the exec mask (saved and restored around it), no tail-switch branch
        auto account = [&](int j, unsigned long long H) {
            const uint32_t c = (uint32_t)__popcll(H);
            const unsigned long long m = 1ull << (j & 63);
            unsigned long long saved;
            asm volatile("s_and_saveexec_b64 %1, %2\n\tv_add_u32 %0, %3, %0\n\ts_mov_b64 exec, %1"
                         : "+v"(mine), "=&s"(saved)
                         : "s"(m), "s"(c));
        };
        while (js[0] >= 0) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if constexpr (MODE == TC_LCC_PROBE_BITMAP) {
                    uint32_t ii[kUnroll], wd[kUnroll], fs[kUnroll];
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q) {
                        ii[q] = (uint32_t)(xs[h * kUnroll + q] - tb.base);  // candidates are ranks above v
                        const uint32_t wi = min(ii[q] >> 5, tb.words);      // beyond the range: guard word
                        const uint2 e = *reinterpret_cast<const uint2*>(tb.bm + 2 * wi);  // word, first index
                        wd[q] = e.x;
                        fs[q] = e.y;
                    }
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q) {
                        const int sl = h * kUnroll + q;
                        asm volatile("" : "+v"(fs[q]));  // keep the read ahead of the hit branch
                        if (js[sl] >= 0) {
                            // v_bfe takes offset and width modulo 32: bit ii % 32 of the word,
                            // and the bits below it
                            const bool in_tail = (int32_t)lane4 < lims[sl];
                            const bool set = __builtin_amdgcn_ubfe(wd[q], ii[q], 1u) != 0u;
                            // two ballots of plain compares, combined in scalar registers
                            const unsigned long long H =
                                __builtin_amdgcn_ballot_w64(in_tail) & __builtin_amdgcn_ballot_w64(set);
                            // every lane adds 1: a hit to its entry's counter, any other lane to
                            // a spare word of its own after the counters (no exec-mask change)
                            const uint32_t pos = (in_tail && set)
                                                     ? (uint32_t)__popc(__builtin_amdgcn_ubfe(wd[q], 0u, ii[q])) + fs[q]
                                                     : (uint32_t)tb.T + (uint32_t)lane;
                            atomicAdd((uint32_t*)((char*)tb.cnt + (pos << 2)), 1u);
                            account(js[sl], H);
                        }
                        xs[sl] = gen(js[sl], lims[sl]);
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < kUnroll; ++q) {
                        const int sl = h * kUnroll + q;
                        const int32_t x = xs[sl];
                        const int j = js[sl], lim = lims[sl];
                        xs[sl] = gen(js[sl], lims[sl]);
                        if (j >= 0) {
                            const bool hit = probe_one<MODE>(tb, x, (int32_t)lane4 < lim);
                            account(j, __builtin_amdgcn_ballot_w64(hit));
                        }
                    }
                }
            }
        }
        local += mine;
        if (ok && mine) gadd(a.t + u, (unsigned long long)mine);
    }
}

// The paper's hybrid intersection on the sorted N+(v) (keys[dv] in LDS): per in-edge, the
// tail A of N+(u) after v and B = N+(v) go to the sorted set intersection (Alg. 2) when the
// rule of Eq. 3 says it is the cheaper one (with s <= l the two lengths, l / s <= log2(l) - 1,
// its right side scaled by merge_x100 / 100), else to a binary search (Sec. II-C1).
//   merge: a merge path over the whole wave.  The merged order of A and B (ties: A first) is
//          cut into 64 equal pieces; lane i finds where its piece starts by a binary search
//          along its diagonal and merges it.  A pair is counted when its A entry is taken
//          while the B cursor rests on an equal key, so every common key once.
//   search: 64 keys of the shorter list at a time, each looked up in the longer one (the
//          tail is searched in global memory, N+(v) in LDS).
// Waves of a group take interleaved tails, as in the probe walk.
template <typename OffT, int NWAVES>
__device__ void walk_tails_hybrid(const CountArgs<OffT>& a, int32_t v, const Table& tb, int wig,
                                  unsigned long long& local) {
    const int lane = lane_id();
    wig = __builtin_amdgcn_readfirstlane(wig);
    const int32_t lb = tb.T;
    const int32_t* B = tb.keys;
    const float scale = (float)a.merge_x100 * 0.01f;
    const OffT i0 = gld(a.in_off, v), i1 = gld(a.in_off, v + 1);
    for (OffT cb = i0; cb < i1; cb += (OffT)kWave) {
        const OffT k = cb + lane;
        int32_t u = 0;
        OffT st = 0;
        int32_t len = 0;
        if (k < i1) load_in_edge(a, k, u, st, len);
        const int nk = (int)__builtin_amdgcn_readfirstlane((int)min((OffT)kWave, i1 - cb));
        for (int j = wig; j < nk; j += NWAVES) {
            const int32_t tu = lane_value(u, j);
            const int32_t la = lane_value(len, j);
            const int32_t* A = a.adj + lane_value(st, j);
            const int32_t sh = min(la, lb), lg = max(la, lb);
            const bool merge = sh > 0 && (float)lg <= (float)sh * (__log2f((float)lg) - 1.0f) * scale;
            uint32_t c = 0;
            if (merge) {
                const int32_t L = la + lb;
                const int32_t per = (L + kWave - 1) / kWave;
                const int32_t d0 = min(lane * per, L), d1 = min(d0 + per, L);
                // i = number of A entries among the first d0 of the merged order
                int32_t lo = max(0, d0 - lb), hi = min(d0, la);
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (A[mid] <= B[d0 - 1 - mid]) lo = mid + 1;
                    else hi = mid;
                }
                int32_t i = lo, jb = d0 - lo;
                int32_t x = i < la ? A[i] : 0;
                int32_t y = jb < lb ? B[jb] : 0;
                for (int32_t s = d0; s < d1; ++s) {
                    if (i < la && (jb >= lb || x <= y)) {
                        if (jb < lb && x == y) {
                            atomicAdd(&tb.cnt[jb], 1u);
                            ++c;
                        }
                        ++i;
                        if (i < la) x = A[i];
                    } else {
                        ++jb;
                        if (jb < lb) y = B[jb];
                    }
                }
            } else if (la <= lb) {
                for (int32_t b = 0; b < la; b += kWave) {
                    const int32_t i = b + lane;
                    if (i < la) {
                        const int sl = sorted_find(B, lb, A[i]);
                        if (sl >= 0) {
                            atomicAdd(&tb.cnt[sl], 1u);
                            ++c;
                        }
                    }
                }
            } else {
                for (int32_t b = 0; b < lb; b += kWave) {
                    const int32_t jb = b + lane;
                    if (jb < lb) {
                        const int32_t y = B[jb];
                        int32_t lo = 0, hi = la;
                        while (lo < hi) {
                            const int32_t mid = (lo + hi) >> 1;
                            if (A[mid] < y) lo = mid + 1;
                            else hi = mid;
                        }
                        if (lo < la && A[lo] == y) {
                            atomicAdd(&tb.cnt[jb], 1u);
                            ++c;
                        }
                    }
                }
            }
            const uint32_t ct = wave_sum(c);
            if (lane == 0 && ct) gadd(a.t + tu, (unsigned long long)ct);
            local += c;
        }
    }
}

// One vertex v, processed by a group of NWAVES waves (gtid = thread index in the group,
// wig = wave index in the group) with an LDS region of region_bytes.  The probe method is
// chosen per vertex: the rank bitmap when it fits (AUTO or BITMAP), else the hash; or the
// sorted list (binary search per candidate, or the hybrid of Eq. 3) when asked for.  Returns this lane's share of t(v) in `local`.
// A vertex with the bounds of its out-list and in-edge list.
template <typename OffT>
struct VertexHead {
    int32_t v;
    OffT b0, b1, i0, i1;
};

template <typename OffT>
__device__ __forceinline__ VertexHead<OffT> vertex_head(const CountArgs<OffT>& a, int32_t v) {
    return VertexHead<OffT>{v, gld(a.out_off, v), gld(a.out_off, v + 1), gld(a.in_off, v), gld(a.in_off, v + 1)};
}

// FALLBACK (the batched kernel of the heavy vertices): a vertex whose bucket hash does not fit
// the region either is searched in N+(v) where it lies in HBM (each hit added to t(w) at once),
// so a graph whose largest lists exceed a batched slice still runs in the batch.  (The batched
// light vertices have their own routine, with windows across tail boundaries.)
template <typename OffT, int PROBE, int NWAVES, bool FALLBACK = false>
__device__ __forceinline__ void process_vertex(const CountArgs<OffT>& a, const VertexHead<OffT>& hd, uint8_t* region,
                               uint32_t region_bytes, int gtid, int wig, unsigned long long& local) {
    static_assert(!FALLBACK || NWAVES > 1, "batched light vertices take process_light");
    constexpr int gsize = NWAVES * kWave;
    const int32_t v = hd.v;
    const OffT b0 = hd.b0;
    const int32_t dv = (int32_t)(hd.b1 - b0);
    const int32_t* nv = a.adj + b0;
    const InEdges<OffT> ie = first_in_edges<NWAVES>(a, hd.i0, hd.i1, __builtin_amdgcn_readfirstlane(wig));

    Table tb;
    tb.base = v + 1;
    int mode;
    if constexpr (PROBE == TC_LCC_PROBE_SORTED || PROBE == TC_LCC_PROBE_MERGE) {
        mode = PROBE;
    } else {
        tb.span = (uint32_t)(gld(nv, dv - 1) - v);
        tb.words = (tb.span + 31u) >> 5;
        mode = (PROBE != TC_LCC_PROBE_HASH && bitmap_bytes(tb.words, dv) <= region_bytes) ? TC_LCC_PROBE_BITMAP
                                                                                           : TC_LCC_PROBE_HASH;
        if constexpr (FALLBACK) {
            if (mode == TC_LCC_PROBE_HASH && 8u * (uint32_t)hash_table_slots(dv) > region_bytes) {
                mode = kProbeGlobal;
                tb.gkeys = nv;
                tb.T = dv;
                tb.tg = a.t;
            }
        }
    }
    if constexpr (FALLBACK) {
        if (mode == kProbeGlobal) {
            walk_tails<OffT, kProbeGlobal, NWAVES>(a, ie, tb, wig, local);
            group_sync<NWAVES>();
            return;
        }
    }

    // ---- stage N+(v)
    if (mode == TC_LCC_PROBE_BITMAP) {
        tb.bm = (uint32_t*)region;
        tb.cnt = (uint32_t*)(region + 8u * (tb.words + 1u));  // dv counters, then 64 spare words
        tb.T = dv;
        for (uint32_t s = gtid; s <= tb.words; s += gsize) tb.bm[2 * s] = 0u;  // with the guard word
        for (int j = gtid; j < dv; j += gsize) tb.cnt[j] = 0u;
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t i = (uint32_t)(gld(nv, j) - tb.base);
            atomicOr(&tb.bm[2 * (i >> 5)], 1u << (i & 31u));
            if (j == 0 || ((uint32_t)(gld(nv, j - 1) - tb.base) >> 5) != (i >> 5)) tb.bm[2 * (i >> 5) + 1] = (uint32_t)j;
        }
    } else if (mode == TC_LCC_PROBE_HASH) {
        const int32_t T = hash_table_slots(dv);
        const uint32_t nb = (uint32_t)T >> 2;
        tb.T = T;
        tb.nb_mask = nb - 1;
        tb.logNB = 31 - __clz(nb);
        tb.keys = (int32_t*)region;
        tb.cnt = (uint32_t*)(tb.keys + T);
        for (int s = gtid; s < T; s += gsize) {
            tb.keys[s] = -1;
            tb.cnt[s] = 0;
        }
        group_sync<NWAVES>();
        for (int j = gtid; j < dv; j += gsize) hash_insert(tb.keys, tb.nb_mask, tb.logNB, gld(nv, j));
    } else {
        tb.T = dv;
        tb.keys = (int32_t*)region;
        tb.cnt = (uint32_t*)(tb.keys + dv);
        for (int j = gtid; j < dv; j += gsize) {
            tb.keys[j] = gld(nv, j);
            tb.cnt[j] = 0;
        }
    }
    group_sync<NWAVES>();

    // ---- probe the tails of the in-edges
    if (mode == TC_LCC_PROBE_BITMAP) walk_tails<OffT, TC_LCC_PROBE_BITMAP, NWAVES>(a, ie, tb, wig, local);
    else if (mode == TC_LCC_PROBE_HASH) walk_tails<OffT, TC_LCC_PROBE_HASH, NWAVES>(a, ie, tb, wig, local);
    else if (mode == TC_LCC_PROBE_MERGE) walk_tails_hybrid<OffT, NWAVES>(a, v, tb, wig, local);
    else walk_tails<OffT, TC_LCC_PROBE_SORTED, NWAVES>(a, ie, tb, wig, local);
    group_sync<NWAVES>();

    // ---- flush the per-entry counters of N+(v)
    if (mode == TC_LCC_PROBE_HASH) {
        for (int s = gtid; s < tb.T; s += gsize) {
            // an empty slot (key -1) never matches a candidate, so its counter is 0; the key
            // test keeps the flush in bounds without resting on that
            const uint32_t c = tb.cnt[s];
            const int32_t key = tb.keys[s];
            if (c && key >= 0) gadd(a.t + key, (unsigned long long)c);
        }
    } else {
        for (int j = gtid; j < dv; j += gsize) {
            const uint32_t c = tb.cnt[j];
            if (c) gadd(a.t + gld(nv, j), (unsigned long long)c);
        }
    }
    group_sync<NWAVES>();
}

template <typename OffT, int PROBE, int NWAVES, bool FALLBACK = false>
__device__ __forceinline__ void process_vertex(const CountArgs<OffT>& a, int32_t v, uint8_t* region,
                                               uint32_t region_bytes, int gtid, int wig, unsigned long long& local) {
    process_vertex<OffT, PROBE, NWAVES, FALLBACK>(a, vertex_head(a, v), region, region_bytes, gtid, wig, local);
}

}  // namespace tcl
