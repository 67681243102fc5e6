// Per-block digit counts for the LSD radix sort (8-bit digits), kept in LDS and added to the
// sort's global counts once per block.  Used by the sort's own counting kernel and by the
// kernels that write keys the sort takes next, so that those keys need not be read twice.
// Each block keeps kCountCopies copies of its counters and lane l adds to copy
// l % kCountCopies, so lanes with equal digits (common in the high digits of skewed keys)
// contend on fewer addresses; the copies of one counter are adjacent words, in different banks.
#pragma once

#include "common.hpp"

namespace tcl {

constexpr int kMaxPasses = 8;
constexpr int kCountCopies = 4;

struct DigitCounts {
    uint32_t h[kMaxPasses * 256 * kCountCopies];

    // all threads of the block
    __device__ __forceinline__ void clear(int passes) {
        for (int i = threadIdx.x; i < passes * 256 * kCountCopies; i += blockDim.x) h[i] = 0;
        __syncthreads();
    }
    template <typename K>
    __device__ __forceinline__ void add(K key, int lo_bit, int passes) {
        const uint32_t copy = (uint32_t)lane_id() % kCountCopies;
        key >>= lo_bit;
        for (int p = 0; p < passes; ++p)
            atomicAdd(&h[((p * 256 + (uint32_t)((key >> (8 * p)) & 255u)) * kCountCopies) + copy], 1u);
    }
    // all threads of the block, after their last add
    __device__ __forceinline__ void flush(uint32_t* __restrict__ hist, int passes) {
        __syncthreads();
        for (int i = threadIdx.x; i < passes * 256; i += blockDim.x) {
            uint32_t c = 0;
#pragma unroll
            for (int r = 0; r < kCountCopies; ++r) c += h[i * kCountCopies + r];
            if (c) atomicAdd(&hist[i], c);
        }
    }
};

// passes of 8 bits that cover nbits
__host__ __device__ inline int digit_passes(int nbits) { return (nbits + 7) / 8; }

}  // namespace tcl
