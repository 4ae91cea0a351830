// Device-to-device copy used as the measured bandwidth reference of the
// roofline reports: the HBM rate a plain streaming kernel reaches on this
// GPU (16-byte loads and stores, four in flight per lane, no reuse).
#include <hip/hip_runtime.h>

#include "ebs_internal.h"

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int COPY_BLOCK = 256;
constexpr int COPY_UNROLL = 4;

__global__ void __launch_bounds__(COPY_BLOCK) k_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                      size_t n) {
    const size_t base = (size_t)blockIdx.x * COPY_BLOCK * COPY_UNROLL + threadIdx.x;
    u32x4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const size_t i = base + (size_t)u * COPY_BLOCK;
        if (i < n) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) {
        const size_t i = base + (size_t)u * COPY_BLOCK;
        if (i < n) __builtin_nontemporal_store(v[u], dst + i);
    }
}

}  // namespace

extern "C" ebs_status ebs_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream) {
    if (!dst || !src) return EBS_E_ARG;
    if (((uintptr_t)dst | (uintptr_t)src | bytes) & 15) return EBS_E_ARG;
    const uintptr_t d = (uintptr_t)dst, s = (uintptr_t)src;
    if (d < s + bytes && s < d + bytes) return EBS_E_ARG;
    const size_t n = bytes / 16;
    if (n == 0) return EBS_OK;
    const size_t per = (size_t)COPY_BLOCK * COPY_UNROLL;
    const size_t blocks = (n + per - 1) / per;
    if (blocks > 0x7FFFFFFFu) return EBS_E_UNSUPPORTED;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(COPY_BLOCK), 0, (hipStream_t)hip_stream,
                       (const u32x4*)src, (u32x4*)dst, n);
    return hipGetLastError() == hipSuccess ? EBS_OK : EBS_E_HIP;
}
