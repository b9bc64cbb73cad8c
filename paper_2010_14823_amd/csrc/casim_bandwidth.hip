// Streaming ceiling of the device: hand-written copy, read and write kernels
// over a flat buffer with 16-byte non-temporal accesses (global_load_dwordx4
// and global_store_dwordx4 with the nt bit), four independent accesses in
// flight per lane and a grid-stride loop.  A diagnostic beside the step: the
// bandwidth a kernel that only moves bytes reaches on this GPU, against
// which the step's own streaming floor (casim_debug_stream) and the step
// itself are compared.
#include "casim_internal.h"
#include "casim_mlp_internal.h"

namespace casim {
namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
constexpr int kBwThreads = 256;
constexpr int kBwUnroll = 4;
constexpr int64_t kBwMaxBlocks = 4096;

__device__ __forceinline__ u32x4 xor_wave(u32x4 v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        v.x ^= __shfl_xor(v.x, m);
        v.y ^= __shfl_xor(v.y, m);
        v.z ^= __shfl_xor(v.z, m);
        v.w ^= __shfl_xor(v.w, m);
    }
    return v;
}

// KIND 0: dst = src; 1: read src, one XOR of the block's words into
// dst[blockIdx.x]; 2: dst = 0.  n counts 16-byte words.
template <int KIND>
__global__ __launch_bounds__(kBwThreads) void bandwidth_kernel(const u32x4 *__restrict__ src,
                                                               u32x4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBwThreads;
    int64_t i = (int64_t)blockIdx.x * kBwThreads + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    const u32x4 zero = {0u, 0u, 0u, 0u};
    for (; i + (kBwUnroll - 1) * stride < n; i += kBwUnroll * stride) {
        u32x4 v[kBwUnroll];
        if (KIND != 2) {
#pragma unroll
            for (int u = 0; u < kBwUnroll; ++u) v[u] = __builtin_nontemporal_load(src + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < kBwUnroll; ++u) {
            if (KIND == 0) __builtin_nontemporal_store(v[u], dst + i + u * stride);
            if (KIND == 1) acc ^= v[u];
            if (KIND == 2) __builtin_nontemporal_store(zero, dst + i + u * stride);
        }
    }
    for (; i < n; i += stride) {
        if (KIND == 0) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
        if (KIND == 1) acc ^= __builtin_nontemporal_load(src + i);
        if (KIND == 2) __builtin_nontemporal_store(zero, dst + i);
    }
    if (KIND == 1) {
        __shared__ u32x4 part[kBwThreads / 64];
        acc = xor_wave(acc);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            u32x4 b = part[0];
#pragma unroll
            for (int w = 1; w < kBwThreads / 64; ++w) b ^= part[w];
            dst[blockIdx.x] = b;
        }
    }
}

}  // namespace
}  // namespace casim

using namespace casim;

extern "C" int casim_debug_bandwidth(const void *src, void *dst, int64_t bytes, int32_t kind, void *stream) {
    if (kind < 0 || kind > 2 || bytes < 0 || (bytes & 15)) return CASIM_EINVAL;
    if (!dst || (kind != 2 && !src)) return CASIM_EINVAL;
    if ((((uintptr_t)dst) | (kind != 2 ? (uintptr_t)src : 0u)) & 15u) return CASIM_EINVAL;
    if (bytes == 0) return CASIM_OK;
    const int64_t n = bytes / 16;
    int64_t blocks = (n + (int64_t)kBwThreads * kBwUnroll - 1) / ((int64_t)kBwThreads * kBwUnroll);
    if (blocks > kBwMaxBlocks) blocks = kBwMaxBlocks;
    const u32x4 *s = static_cast<const u32x4 *>(src);
    u32x4 *d = static_cast<u32x4 *>(dst);
    const hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)blocks), block(kBwThreads);
    if (kind == 0) hipLaunchKernelGGL(bandwidth_kernel<0>, grid, block, 0, st, s, d, n);
    else if (kind == 1) hipLaunchKernelGGL(bandwidth_kernel<1>, grid, block, 0, st, s, d, n);
    else hipLaunchKernelGGL(bandwidth_kernel<2>, grid, block, 0, st, s, d, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CASIM_OK : casim_record_hip_error((int)e, hipGetErrorString(e));
}
