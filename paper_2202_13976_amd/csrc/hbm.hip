// A streaming copy through the shader cores: the achievable HBM bandwidth of this GPU, which
// the count kernel's roofline fraction is reported against beside the datasheet peak, and a
// transfer of known size for scaling the HBM traffic counters (a DMA copy would not pass
// through the counters' path).
#include "internal.hpp"

namespace tcl {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte access

constexpr int kCopyThreads = 256;
constexpr int kCopyVec = 1;  // 16-byte vectors per thread and step, all loaded before any store
constexpr int kCopyBlocksPerCu = 4;

__global__ __launch_bounds__(kCopyThreads) void k_hbm_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                           size_t n16) {
    const size_t stride = (size_t)gridDim.x * kCopyThreads;
    size_t i = (size_t)blockIdx.x * kCopyThreads + threadIdx.x;
    for (; i + (kCopyVec - 1) * stride < n16; i += kCopyVec * stride) {
        u32x4 v[kCopyVec];
#pragma unroll
        for (int q = 0; q < kCopyVec; ++q) v[q] = __builtin_nontemporal_load(src + i + q * stride);
#pragma unroll
        for (int q = 0; q < kCopyVec; ++q) __builtin_nontemporal_store(v[q], dst + i + q * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace tcl

using namespace tcl;

extern "C" tc_lcc_status tc_lcc_hbm_copy(const void* src, void* dst, uint64_t bytes, void* hip_stream) {
    if (!src || !dst || (bytes & 15u) || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u)) {
        set_error("tc_lcc_hbm_copy: null pointer, or a size or address not a multiple of 16");
        return TC_LCC_INVALID_ARGUMENT;
    }
    if (bytes == 0) return TC_LCC_OK;
    int dev = 0, cus = 256;
    TCL_HIP(hipGetDevice(&dev));
    TCL_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const size_t n16 = bytes / 16;
    // 4 blocks of one 16-byte vector per thread and step per compute unit: the fastest of the
    // shapes tried (1-8 vectors per step, 2-32 blocks per compute unit, with and without the
    // nontemporal hint), at the bandwidth of the runtime's own device-to-device copy
    const size_t want = (n16 + kCopyThreads - 1) / kCopyThreads;
    const unsigned grid = (unsigned)std::min<size_t>(std::max<size_t>(want, 1), (size_t)cus * kCopyBlocksPerCu);
    k_hbm_copy<<<grid, kCopyThreads, 0, (hipStream_t)hip_stream>>>((const u32x4*)src, (u32x4*)dst, n16);
    TCL_HIP(hipGetLastError());
    return TC_LCC_OK;
}
