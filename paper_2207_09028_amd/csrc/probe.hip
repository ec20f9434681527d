// HBM bandwidth probes: plain streaming kernels of a known size.  Their times
// give the achievable read-only, write-only, copy and mixed rates of the device, the
// denominators beside the 8 TB/s spec figure that the pair passes (pass 1
// mostly writes, pass 3 mostly reads, pass 2 reads and writes in equal parts)
// are measured against, and their FETCH_SIZE / WRITE_SIZE counters calibrate
// the counter-measured traffic of the library kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "internal.hpp"

namespace {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int W> struct VecT;
template <> struct VecT<8> { using type = u32x2; };
template <> struct VecT<16> { using type = u32x4; };

constexpr int kProbeThreads = 256;
constexpr int kProbeUnroll = 4;

template <typename V, bool NT>
__device__ __forceinline__ V ld(const V* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <typename V, bool NT>
__device__ __forceinline__ void st(V* p, V v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <typename V>
__device__ __forceinline__ uint32_t fold(V v) {
    uint32_t r = v.x ^ v.y;
    if constexpr (sizeof(V) == 16) r ^= v.z ^ v.w;
    return r;
}

// kind 0: read n vectors; the xor of everything read is stored only if it equals
// `sentinel`, so the loads stay live but (almost) nothing is written
template <typename V, bool NT>
__global__ void __launch_bounds__(kProbeThreads) probe_read(const V* __restrict__ src, size_t n, uint32_t sentinel,
                                                            uint32_t* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
        V v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = ld<V, NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) acc ^= fold(v[u]);
    }
    for (; i < n; i += stride) acc ^= fold(ld<V, NT>(src + i));
    if (acc == sentinel) sink[0] = acc;
}

// kind 1: write n vectors of a value that depends on the index
template <typename V, bool NT>
__global__ void __launch_bounds__(kProbeThreads) probe_write(V* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    for (size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride) {
        V v;
        v.x = (uint32_t)i;
        v.y = (uint32_t)(i >> 32);
        if constexpr (sizeof(V) == 16) {
            v.z = v.x;
            v.w = v.y;
        }
        st<V, NT>(dst + i, v);
    }
}

// kind 2: copy n vectors
template <typename V, bool NT>
__global__ void __launch_bounds__(kProbeThreads) probe_copy(const V* __restrict__ src, V* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x;
    for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
        V v[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) v[u] = ld<V, NT>(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) st<V, NT>(dst + i + u * stride, v[u]);
    }
    for (; i < n; i += stride) st<V, NT>(dst + i, ld<V, NT>(src + i));
}

// kind 3: write n vectors and read one vector of src for every `every` written (src
// holds n / every vectors): a write stream with a share of reads, like pass 1
template <typename V, bool NT>
__global__ void __launch_bounds__(kProbeThreads) probe_mixed(const V* __restrict__ src, V* __restrict__ dst,
                                                             size_t n, int every, uint32_t sentinel,
                                                             uint32_t* __restrict__ sink) {
    const size_t stride = (size_t)gridDim.x * kProbeThreads;
    uint32_t acc = 0;
    size_t k = 0;
    for (size_t i = (size_t)blockIdx.x * kProbeThreads + threadIdx.x; i < n; i += stride, ++k) {
        V v;
        v.x = (uint32_t)i;
        v.y = (uint32_t)(i >> 32);
        if constexpr (sizeof(V) == 16) {
            v.z = v.x;
            v.w = v.y;
        }
        st<V, NT>(dst + i, v);
        if (k % every == 0) acc ^= fold(ld<V, NT>(src + i / every));
    }
    if (acc == sentinel) sink[0] = acc;
}

template <typename V, bool NT>
hipError_t launch_probe(int kind, int every, void* dst, const void* src, size_t n, int grid, hipStream_t s) {
    if (kind == 3) {
        hipLaunchKernelGGL((probe_mixed<V, NT>), dim3(grid), dim3(kProbeThreads), 0, s, static_cast<const V*>(src),
                           static_cast<V*>(dst), n, every, 0x9e3779b9u, static_cast<uint32_t*>(dst));
    } else if (kind == 0) {
        hipLaunchKernelGGL((probe_read<V, NT>), dim3(grid), dim3(kProbeThreads), 0, s, static_cast<const V*>(src), n,
                           0x9e3779b9u, static_cast<uint32_t*>(dst));
    } else if (kind == 1) {
        hipLaunchKernelGGL((probe_write<V, NT>), dim3(grid), dim3(kProbeThreads), 0, s, static_cast<V*>(dst), n);
    } else {
        hipLaunchKernelGGL((probe_copy<V, NT>), dim3(grid), dim3(kProbeThreads), 0, s, static_cast<const V*>(src),
                           static_cast<V*>(dst), n);
    }
    return hipGetLastError();
}

}  // namespace

extern "C" occrik_status occrik_hbm_probe(int32_t kind, int32_t width, int32_t nontemporal, int32_t read_every,
                                          void* dst, const void* src, size_t bytes, int32_t reps, void* stream,
                                          double* ms_per_rep) {
    if (kind < 0 || kind > 3 || (width != 8 && width != 16) || reps < 1 || !ms_per_rep || bytes == 0 ||
        bytes % (size_t)width != 0 || (kind == 3 && read_every < 1))
        return OCCRIK_ERR_INVALID_ARG;
    if ((kind != 1 && !src) || !dst) return OCCRIK_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(dst) | (kind != 1 ? reinterpret_cast<uintptr_t>(src) : 0)) % width != 0)
        return OCCRIK_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return OCCRIK_ERR_DEVICE;
    const size_t n = bytes / (size_t)width;
    const int grid = ncu * 8;
    auto run = [&]() -> hipError_t {
        if (width == 8)
            return nontemporal ? launch_probe<u32x2, true>(kind, read_every, dst, src, n, grid, s)
                               : launch_probe<u32x2, false>(kind, read_every, dst, src, n, grid, s);
        return nontemporal ? launch_probe<u32x4, true>(kind, read_every, dst, src, n, grid, s)
                           : launch_probe<u32x4, false>(kind, read_every, dst, src, n, grid, s);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = run();  // untimed first pass
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = run();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return OCCRIK_ERR_DEVICE;
    *ms_per_rep = double(ms) / reps;
    return OCCRIK_OK;
}
