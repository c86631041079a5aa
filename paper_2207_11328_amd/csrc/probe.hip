// Stream copy: the achievable HBM bandwidth against which the derivative
// call's traffic is reported (a measurement aid; no part of the method).
// Each thread moves 16-byte vectors in a grid-stride loop, U of them loaded
// before any is stored so that several loads per lane are in flight; the
// grid is a fixed number of workgroups per CU.
#include <hip/hip_runtime.h>

#include "sph_device.h"

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void k_stream_copy(const v4u *__restrict__ src, v4u *__restrict__ dst,
                                                          size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
    for (; i + (kUnroll - 1) * stride < n; i += kUnroll * stride) {
        v4u v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = __builtin_nontemporal_load(&src[i + u * stride]);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) __builtin_nontemporal_store(v[u], &dst[i + u * stride]);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" sph_status sph_stream_copy(const void *src, void *dst, size_t bytes, int32_t blocks_per_cu, void *stream)
{
    if ((bytes > 0 && (!src || !dst)) || (bytes & 15u) || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
        return SPH_ERR_ARG;
    if (blocks_per_cu < 1 || blocks_per_cu > 64) return SPH_ERR_ARG;
    if (bytes == 0) return SPH_OK;
    const size_t n = bytes / 16;
    const unsigned blocks = (unsigned)sph_device_cus() * (unsigned)blocks_per_cu;
    k_stream_copy<<<blocks, kThreads, 0, (hipStream_t)stream>>>((const v4u *)src, (v4u *)dst, n);
    SPH_CHECK_LAUNCH();
    return SPH_OK;
}
