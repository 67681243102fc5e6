// Shared device helpers and internal declarations of the tc_lcc HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace tcl {

constexpr int kWave = 64;

// ---------------------------------------------------------------- error plumbing
// Host-side status propagation: every HIP call is checked and turned into a
// library status; the message is kept per thread for tc_lcc_last_error().
void set_error(const char* fmt, ...);
const char* last_error();

#define TCL_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) {                                                        \
            ::tcl::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),    \
                             __FILE__, __LINE__);                                      \
            return TC_LCC_DEVICE_ERROR;                                                \
        }                                                                              \
    } while (0)

// ---------------------------------------------------------------- wave primitives
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// inclusive scan over the 64 lanes of a wave (Hillis-Steele with cross-lane shuffles)
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Make LDS writes of this wave visible to the other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One entry of a per-lane value as seen from lane j (j wave-uniform).
template <typename OffT>
__device__ __forceinline__ OffT lane_value(OffT x, int j) {
    if constexpr (sizeof(OffT) == 8) {
        const uint64_t y = (uint64_t)x;
        return (OffT)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)y, j) |
                      ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(y >> 32), j) << 32));
    } else {
        return (OffT)__builtin_amdgcn_readlane((int32_t)x, j);
    }
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    const int lane = lane_id();
    return lane == 0 ? 0ull : (~0ull >> (kWave - lane));
}

inline int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

inline unsigned grid_for(size_t n, int block, size_t cap = 1u << 20) {
    size_t g = (n + block - 1) / block;
    if (g == 0) g = 1;
    return (unsigned)(g < cap ? g : cap);
}

}  // namespace tcl
