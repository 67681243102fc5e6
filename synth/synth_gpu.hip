/*
 * The large-scale R-MAT recipe of synth.c (synth_rmat_feistel) on the GPU: the same
 * counter-based SplitMix64 draws, quadrant thresholds and Feistel relabelling, one pair per
 * thread, so that a range of pairs is written straight into device memory.  Input generation
 * only; the tests check it against the C version pair for pair.  Also a plain copy of int32
 * ranges between device arrays, for pair sources that serve stored pairs in chunks.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t feistel(uint64_t x, int half, uint64_t k0, uint64_t k1, uint64_t k2, uint64_t k3) {
    const uint64_t mask = (1ULL << half) - 1;
    uint64_t l = x >> half, r = x & mask;
    const uint64_t key[4] = {k0, k1, k2, k3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t f = sm_mix(r + key[i]) & mask;
        const uint64_t nl = r;
        r = l ^ f;
        l = nl;
    }
    return (l << half) | r;
}

__global__ void k_rmat_feistel(int scale, uint64_t s, uint64_t t0, uint64_t t1, uint64_t t2, uint64_t k0, uint64_t k1,
                               uint64_t k2, uint64_t k3, uint64_t first, int64_t count, int32_t* __restrict__ src,
                               int32_t* __restrict__ dst) {
    const uint64_t per = (uint64_t)(scale + 1) / 2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = first + (uint64_t)i;
        uint64_t r = 0, row = 0, col = 0;
        for (int l = 0; l < scale; ++l) {
            if ((l & 1) == 0) r = sm_mix(s + (k * per + (uint64_t)(l >> 1) + 1) * SM_GAMMA);
            const uint64_t x = (l & 1) ? (r & 0xffffffffULL) : (r >> 32);
            const uint64_t bit = 1ULL << (scale - 1 - l);
            if (x >= t0) {
                if (x < t1) col |= bit;
                else if (x < t2) row |= bit;
                else {
                    row |= bit;
                    col |= bit;
                }
            }
        }
        src[i] = (int32_t)feistel(row, scale / 2, k0, k1, k2, k3);
        dst[i] = (int32_t)feistel(col, scale / 2, k0, k1, k2, k3);
    }
}

/* stream_state: the R-MAT stream (sub-seed of TAG_RMAT), thresholds and keys as computed by
 * synth.c for the same seed (passed in by the Python wrapper). */
extern "C" int synth_gpu_rmat_feistel(int scale, uint64_t stream_state, const uint64_t* thresholds,
                                      const uint64_t* keys, uint64_t first, int64_t count, int32_t* src, int32_t* dst,
                                      void* hip_stream) {
    if (scale < 2 || scale > 30 || (scale & 1) || count < 0) return -1;
    if (count == 0) return 0;
    const int64_t blocks = (count + 255) / 256;
    k_rmat_feistel<<<(unsigned)(blocks < 65536 ? blocks : 65536), 256, 0, (hipStream_t)hip_stream>>>(
        scale, stream_state, thresholds[0], thresholds[1], thresholds[2], keys[0], keys[1], keys[2], keys[3], first,
        count, src, dst);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

__global__ void k_copy_i32(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t count) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

/* b[0, count) = a[0, count), both device arrays, enqueued on hip_stream. */
extern "C" int synth_gpu_copy_i32(const int32_t* a, int32_t* b, int64_t count, void* hip_stream) {
    if (count < 0 || (count > 0 && (!a || !b))) return -1;
    if (count == 0) return 0;
    const int64_t blocks = (count + 255) / 256;
    k_copy_i32<<<(unsigned)(blocks < 16384 ? blocks : 16384), 256, 0, (hipStream_t)hip_stream>>>(a, b, count);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
