// Measurement probes: the two ceilings the sampling kernels are held against.
//
//   k_probe_philox  Philox4x32-10 blocks with the coin layout of the world
//                   kernels (counter (slot group, world, 0, 0), key from the
//                   query seed) and nothing else: the rate at which the chip
//                   can draw coins when no memory is touched.
//   k_probe_copy    a plain device-to-device copy with 16-byte accesses: the
//                   HBM bandwidth a streaming kernel can reach.
//
// Each runs once per call and reports its own duration from events recorded
// by its launch.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "imin.h"
#include "imin_device.hpp"

namespace {

constexpr int kProbeNT = 256;

__global__ __launch_bounds__(kProbeNT) void k_probe_philox(uint32_t worlds, uint32_t groups_per_world, uint32_t key0,
                                                           uint32_t key1, uint32_t* out) {
    uint32_t acc = 0u;
    for (uint32_t w = blockIdx.x; w < worlds; w += gridDim.x)
        for (uint32_t b = threadIdx.x; b < groups_per_world; b += kProbeNT) {
            const uint4 c = imin::philox_block(b, w, key0, key1);
            acc ^= c.x ^ c.y ^ c.z ^ c.w;
        }
    out[(size_t)blockIdx.x * kProbeNT + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kProbeNT) void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                         size_t n) {
    const size_t stride = (size_t)gridDim.x * kProbeNT;
    size_t i = (size_t)blockIdx.x * kProbeNT + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// Launch with events around exactly the kernel, wait, and report its time.
template <class... P, class... A>
imin_status_t timed_launch(void (*k)(P...), int grid, hipStream_t s, float* ms, A... a) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return IMIN_ERR_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return IMIN_ERR_DEVICE;
    }
    hipExtLaunchKernelGGL(k, dim3((unsigned)grid), dim3(kProbeNT), 0, s, e0, e1, 0, a...);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return IMIN_ERR_DEVICE;
    *ms = t;
    return IMIN_OK;
}

}  // namespace

extern "C" {

imin_status_t imin_probe_philox(int64_t worlds, int32_t groups_per_world, uint64_t key, uint32_t* out,
                                int64_t out_count, int32_t grid, void* stream, float* ms) {
    if (worlds < 1 || worlds > (int64_t)0xFFFFFFFFll || groups_per_world < 1 || !out || !ms || grid < 1 ||
        out_count < (int64_t)grid * kProbeNT)
        return IMIN_ERR_INVALID;
    return timed_launch(k_probe_philox, grid, (hipStream_t)stream, ms, (uint32_t)worlds, (uint32_t)groups_per_world,
                        (uint32_t)key, (uint32_t)(key >> 32), out);
}

imin_status_t imin_probe_copy(void* dst, const void* src, size_t bytes, int32_t grid, void* stream, float* ms) {
    if (!dst || !src || !ms || grid < 1 || bytes == 0 || bytes % 16 != 0 || ((uintptr_t)dst | (uintptr_t)src) % 16 != 0)
        return IMIN_ERR_INVALID;
    return timed_launch(k_probe_copy, grid, (hipStream_t)stream, ms, (const uint4*)src, (uint4*)dst, bytes / 16);
}

}  // extern "C"
