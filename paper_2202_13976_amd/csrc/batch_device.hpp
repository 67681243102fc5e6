// Device code of the batched path's light vertices (one wave each): windows across tail
// boundaries for the short tails of small graphs, and a vertex routine whose first loads are
// issued while the previous vertex is counted.  Built on the shared count code (count_device.hpp).
#pragma once

#include "count_device.hpp"

namespace tcl {

// The waves of a group over the tails of v's in-edges with windows that cross tail boundaries:
// for graphs whose tails are short (the many-small-graphs batch: a dozen candidates per tail),
// a window of one tail would leave most of the 64 lanes idle.  Wave wig takes every NWAVES-th
// in-edge, 64 at a time (a chunk: lane k holds its k-th in-edge, as first_in_edges loads it);
// the chunk's tails are laid end to end (exclusive prefix sums of their lengths) and every
// window takes the next 64 candidates of that sequence.  Lane i finds the tail of its
// candidate by a binary search over the lanes' prefix sums (lane shuffles); kFlatRound windows
// are formed and their candidates loaded before any is probed, so that many loads are in flight
// per wave.  A hit is counted at its entry of N+(v) (or, searching N+(v) in HBM, added to t(w)
// at once); the hits of one tail in one window are summed by a popcount over that tail's lanes
// and added to the tail's LDS counter (tcnt: 64 words of this wave) by its last lane; the
// tails' counts go to t(u) once the chunk is done.
constexpr int kFlatRound = 3;

template <typename OffT, int MODE, int NWAVES = 1>
__device__ __forceinline__ void walk_flat(const CountArgs<OffT>& a, const InEdges<OffT>& ie, const Table& tb,
                                          uint32_t* tcnt, int wig, unsigned long long& local) {
    const int lane = lane_id();
    wig = __builtin_amdgcn_readfirstlane(wig);
    const OffT i0 = ie.i0, i1 = ie.i1;
    constexpr OffT kSpan = (OffT)kWave * NWAVES;
    int32_t u = ie.u, len = ie.len;
    OffT st = ie.st;
    const unsigned long long le = lanemask_lt() | (1ull << lane);
    for (OffT cb = i0; cb < i1; cb += kSpan) {
        if (cb != i0) {
            const OffT k = cb + (OffT)lane * NWAVES + wig;
            u = 0;
            st = 0;
            len = 0;
            if (k < i1) load_in_edge(a, k, u, st, len);
        }
        const int32_t incl = wave_inclusive_scan(len);
        const int32_t excl = incl - len;
        const int32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
        // candidate c of tail k lies at adj[st_k + (c - excl_k)] = adj[dk + c]
        const OffT dk = st - (OffT)excl;
        tcnt[lane] = 0u;
        wave_lds_sync();
        for (int32_t base = 0; base < total; base += kWave * kFlatRound) {
            int32_t xs[kFlatRound], ks[kFlatRound];
            bool vs[kFlatRound];
#pragma unroll
            for (int r = 0; r < kFlatRound; ++r) {
                const int32_t c = base + r * kWave + lane;
                vs[r] = c < total;
                ks[r] = 0;
                xs[r] = 0;
                if (base + r * kWave < total) {  // wave-uniform
                    // last tail k whose first candidate is at or before c (tails are nonempty)
                    int k = 0;
#pragma unroll
                    for (int step = kWave / 2; step >= 1; step >>= 1) {
                        const int probe = k + step;
                        const int32_t e = __shfl(excl, probe < kWave ? probe : kWave - 1, kWave);
                        if (probe < kWave && e <= c) k = probe;
                    }
                    ks[r] = k;
                    OffT d;
                    if constexpr (sizeof(OffT) == 8) {
                        const uint64_t d64 = (uint64_t)dk;
                        d = (OffT)((uint64_t)(uint32_t)__shfl((int32_t)(uint32_t)d64, k, kWave) |
                                   ((uint64_t)(uint32_t)__shfl((int32_t)(uint32_t)(d64 >> 32), k, kWave) << 32));
                    } else {
                        d = (OffT)__shfl((int32_t)dk, k, kWave);
                    }
                    if (vs[r]) xs[r] = gld(a.adj, d + (OffT)c);
                }
            }
#pragma unroll
            for (int r = 0; r < kFlatRound; ++r) {
                if (base + r * kWave >= total) break;  // wave-uniform
                const int32_t x = xs[r];
                const int k = ks[r];
                bool hit;
                if constexpr (MODE == TC_LCC_PROBE_BITMAP) {
                    const uint32_t ii = (uint32_t)(x - tb.base);  // candidates are ranks above v
                    const uint32_t wi = min(ii >> 5, tb.words);   // beyond the range: the zero guard word
                    const uint2 e = *reinterpret_cast<const uint2*>(tb.bm + 2 * wi);
                    hit = vs[r] && __builtin_amdgcn_ubfe(e.x, ii, 1u) != 0u;
                    if (hit) atomicAdd(&tb.cnt[e.y + (uint32_t)__popc(__builtin_amdgcn_ubfe(e.x, 0u, ii))], 1u);
                } else {
                    hit = probe_one<MODE>(tb, x, vs[r]);
                }
                local += hit ? 1ull : 0ull;
                // hits per tail: the lanes of one tail are contiguous; the last lane of each run
                // adds the run's hits (one LDS add per tail and window)
                const unsigned long long H = __builtin_amdgcn_ballot_w64(hit);
                const int kp = __shfl_up(k, 1, kWave);
                const int kn = __shfl_down(k, 1, kWave);
                const unsigned long long heads = __builtin_amdgcn_ballot_w64(lane == 0 || kp != k);
                const bool last = vs[r] && (lane == kWave - 1 || kn != k || base + r * kWave + lane + 1 >= total);
                if (last) {
                    const int start = 63 - __clzll(heads & le);
                    const uint32_t cnt = (uint32_t)__popcll(H & le & ~((1ull << start) - 1ull));
                    if (cnt) atomicAdd(&tcnt[k], cnt);
                }
            }
        }
        wave_lds_sync();
        const uint32_t mine = tcnt[lane];
        if (mine) gadd(a.t + u, (unsigned long long)mine);
        wave_lds_sync();
    }
}

// What a light vertex of the batched launch needs first, loaded while the previous vertex is
// worked on: this lane's entry of N+(v) (entry `lane`, for the first 64) and this lane's in-edge
// of v's first chunk (u, tail start, tail length).
template <typename OffT>
struct LightPrefetch {
    int32_t x;
    int32_t u;
    OffT st;
    int32_t len;
};

template <typename OffT>
__device__ __forceinline__ LightPrefetch<OffT> light_prefetch(const CountArgs<OffT>& a, const VertexHead<OffT>& hd) {
    LightPrefetch<OffT> p{0, 0, 0, 0};
    const int lane = lane_id();
    if ((OffT)lane < hd.b1 - hd.b0) p.x = gld(a.adj, hd.b0 + (OffT)lane);
    const OffT k = hd.i0 + (OffT)lane;
    if (k < hd.i1) load_in_edge(a, k, p.u, p.st, p.len);
    return p;
}

// A light vertex of the batched launch, one wave, as process_vertex with NWAVES = 1 and
// FALLBACK, but with its first loads already done (pf): N+(v) is staged from registers (the
// previous entry of each lane's from its neighbour lane), its last entry read from the lane that
// holds it, and the flush adds to t(w) by the entry each lane still holds, so the vertex waits on
// global memory only for its candidates (and for entries beyond the first 64).
template <typename OffT>
__device__ __forceinline__ void process_light(const CountArgs<OffT>& a, const VertexHead<OffT>& hd,
                                              const LightPrefetch<OffT>& pf, uint8_t* region, uint32_t region_bytes,
                                              unsigned long long& local, uint32_t* tcnt) {
    const int lane = lane_id();
    const int32_t v = hd.v;
    const int32_t dv = (int32_t)(hd.b1 - hd.b0);
    const int32_t* nv = a.adj + hd.b0;
    const InEdges<OffT> ie{hd.i0, hd.i1, pf.u, pf.st, pf.len};
    // entry j of N+(v) (j wave-uniform below 64: the lane that holds it)
    const int32_t last = dv <= kWave ? __builtin_amdgcn_readlane(pf.x, dv - 1) : gld(nv, dv - 1);

    Table tb;
    tb.base = v + 1;
    tb.span = (uint32_t)(last - v);
    tb.words = (tb.span + 31u) >> 5;
    int mode = bitmap_bytes(tb.words, dv) <= region_bytes ? TC_LCC_PROBE_BITMAP : TC_LCC_PROBE_HASH;
    if (mode == TC_LCC_PROBE_HASH && 8u * (uint32_t)hash_table_slots(dv) > region_bytes) {
        tb.gkeys = nv;
        tb.T = dv;
        tb.tg = a.t;
        walk_flat<OffT, kProbeGlobal, 1>(a, ie, tb, tcnt, 0, local);
        wave_lds_sync();
        return;
    }

    // ---- stage N+(v): lane l holds entry j0 + l of each round of 64
    if (mode == TC_LCC_PROBE_BITMAP) {
        tb.bm = (uint32_t*)region;
        tb.cnt = (uint32_t*)(region + 8u * (tb.words + 1u));  // dv counters, then 64 spare words
        tb.T = dv;
        for (uint32_t s = lane; s <= tb.words; s += kWave) tb.bm[2 * s] = 0u;  // with the guard word
        for (int j = lane; j < dv; j += kWave) tb.cnt[j] = 0u;
        wave_lds_sync();
        int32_t carry = 0;  // entry j0 - 1
        for (int j0 = 0; j0 < dv; j0 += kWave) {
            const int j = j0 + lane;
            const int32_t x = j0 == 0 ? pf.x : (j < dv ? gld(nv, j) : 0);
            int32_t xp = __shfl_up(x, 1, kWave);
            if (lane == 0) xp = carry;
            carry = __builtin_amdgcn_readlane(x, kWave - 1);
            if (j < dv) {
                const uint32_t i = (uint32_t)(x - tb.base);
                atomicOr(&tb.bm[2 * (i >> 5)], 1u << (i & 31u));
                if (j == 0 || ((uint32_t)(xp - tb.base) >> 5) != (i >> 5)) tb.bm[2 * (i >> 5) + 1] = (uint32_t)j;
            }
        }
    } else {
        const int32_t T = hash_table_slots(dv);
        const uint32_t nb = (uint32_t)T >> 2;
        tb.T = T;
        tb.nb_mask = nb - 1;
        tb.logNB = 31 - __clz(nb);
        tb.keys = (int32_t*)region;
        tb.cnt = (uint32_t*)(tb.keys + T);
        for (int s = lane; s < T; s += kWave) {
            tb.keys[s] = -1;
            tb.cnt[s] = 0;
        }
        wave_lds_sync();
        for (int j = lane; j < dv; j += kWave) hash_insert(tb.keys, tb.nb_mask, tb.logNB, j < kWave ? pf.x : gld(nv, j));
    }
    wave_lds_sync();

    // ---- probe the tails of the in-edges
    if (mode == TC_LCC_PROBE_BITMAP) walk_flat<OffT, TC_LCC_PROBE_BITMAP, 1>(a, ie, tb, tcnt, 0, local);
    else walk_flat<OffT, TC_LCC_PROBE_HASH, 1>(a, ie, tb, tcnt, 0, local);
    wave_lds_sync();

    // ---- flush the per-entry counters of N+(v)
    if (mode == TC_LCC_PROBE_HASH) {
        for (int s = lane; s < tb.T; s += kWave) {
            const uint32_t c = tb.cnt[s];
            const int32_t key = tb.keys[s];
            if (c && key >= 0) gadd(a.t + key, (unsigned long long)c);
        }
    } else {
        for (int j = lane; j < dv; j += kWave) {
            const uint32_t c = tb.cnt[j];
            if (c) gadd(a.t + (j < kWave ? pf.x : gld(nv, j)), (unsigned long long)c);
        }
    }
    wave_lds_sync();
}

}  // namespace tcl
