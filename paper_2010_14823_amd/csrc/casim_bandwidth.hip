// Streaming ceiling of the device: hand-written copy, read and write kernels
// over a flat buffer with non-temporal accesses of 8 or 16 bytes per lane
// (global_load/store_dwordx2 or _dwordx4 with the nt bit) and a grid-stride
// loop over a caller-chosen number of 256-thread blocks.  Which width and
// grid stream fastest differs between reading and writing, so the ceiling
// is the best of a small sweep.  A diagnostic beside the step: the bandwidth
// a kernel that only moves bytes reaches on this GPU, against which the
// step's own streaming floor (casim_debug_stream) and the step itself are
// compared.
#include "casim_internal.h"
#include "casim_mlp_internal.h"

namespace casim {
namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBwThreads = 256;

template <typename T>
__device__ __forceinline__ T xor_wave(T v) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
#pragma unroll
        for (int j = 0; j < (int)(sizeof(T) / 4); ++j) v[j] ^= __shfl_xor(v[j], m);
    }
    return v;
}

// KIND 0: dst = src; 1: read src, one XOR of the block's words into
// dst[blockIdx.x]; 2: dst = 0.  T is the per-lane word (8 or 16 bytes), n
// counts words.
template <int KIND, typename T>
__global__ __launch_bounds__(kBwThreads) void bandwidth_kernel(const T *__restrict__ src, T *__restrict__ dst,
                                                               int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBwThreads;
    T acc = T(0u);
    const T zero = T(0u);
    for (int64_t i = (int64_t)blockIdx.x * kBwThreads + threadIdx.x; i < n; i += stride) {
        if (KIND == 0) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
        if (KIND == 1) acc ^= __builtin_nontemporal_load(src + i);
        if (KIND == 2) __builtin_nontemporal_store(zero, dst + i);
    }
    if (KIND == 1) {
        __shared__ T part[kBwThreads / 64];
        acc = xor_wave(acc);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            T b = part[0];
#pragma unroll
            for (int w = 1; w < kBwThreads / 64; ++w) b ^= part[w];
            dst[blockIdx.x] = b;
        }
    }
}

template <typename T>
hipError_t launch_bandwidth(const void *src, void *dst, int64_t n, int kind, int64_t blocks, hipStream_t st) {
    const T *s = static_cast<const T *>(src);
    T *d = static_cast<T *>(dst);
    const dim3 grid((unsigned)blocks), block(kBwThreads);
    if (kind == 0) hipLaunchKernelGGL((bandwidth_kernel<0, T>), grid, block, 0, st, s, d, n);
    else if (kind == 1) hipLaunchKernelGGL((bandwidth_kernel<1, T>), grid, block, 0, st, s, d, n);
    else hipLaunchKernelGGL((bandwidth_kernel<2, T>), grid, block, 0, st, s, d, n);
    return hipGetLastError();
}

}  // namespace
}  // namespace casim

using namespace casim;

extern "C" int casim_debug_bandwidth(const void *src, void *dst, int64_t bytes, int32_t kind, int32_t width,
                                     int32_t blocks, void *stream) {
    if (kind < 0 || kind > 2 || bytes < 0 || (width != 8 && width != 16) || (bytes % width)) return CASIM_EINVAL;
    if (blocks < 1 || blocks > (1 << 20)) return CASIM_EINVAL;
    if (!dst || (kind != 2 && !src)) return CASIM_EINVAL;
    if ((((uintptr_t)dst) | (kind != 2 ? (uintptr_t)src : 0u)) & (uintptr_t)(width - 1)) return CASIM_EINVAL;
    const int64_t n = bytes / width;
    if (n == 0) return CASIM_OK;
    // the read kernel stores one word per block: never more blocks than words
    const int64_t nb = blocks < n ? blocks : n;
    const hipError_t e = width == 8 ? launch_bandwidth<u32x2>(src, dst, n, kind, nb, (hipStream_t)stream)
                                    : launch_bandwidth<u32x4>(src, dst, n, kind, nb, (hipStream_t)stream);
    return e == hipSuccess ? CASIM_OK : casim_record_hip_error((int)e, hipGetErrorString(e));
}
