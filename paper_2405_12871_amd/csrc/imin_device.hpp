// Device helpers shared by the kernels: the coin generator, bit tests and
// block-wide scans for wave64 workgroups.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace imin {

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0, c1, c2, c3),
// key (k0, k1).  Ten rounds of two 32x32->64 products; the key advances by the
// Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                               uint32_t k1) {
    uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)x0 * 0xD2511F53ull;
        const uint64_t b = (uint64_t)x2 * 0xCD9E8D57ull;
        const uint32_t n0 = (uint32_t)(b >> 32) ^ x1 ^ k0;
        const uint32_t n2 = (uint32_t)(a >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)b;
        x3 = (uint32_t)a;
        x0 = n0;
        x2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(x0, x1, x2, x3);
}

// The coin blocks: counter words 2 and 3 are zero, counter (c0, c1, 0, 0).
__device__ __forceinline__ uint4 philox_block(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
    return philox4x32_10(c0, c1, 0u, 0u, k0, k1);
}

__device__ __forceinline__ bool bit_set(const uint32_t* bits, int32_t v) {
    return (bits[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u;
}

// Exclusive prefix sum over a workgroup of NT threads (NT a multiple of 64)
// of int, or of uint32_t where sums may pass 2^31 (they wrap modulo 2^32);
// `tmp` holds NT/64 values of LDS.  All threads must call it.
template <int NT, class T = int>
__device__ __forceinline__ T block_excl_scan(T x, T* tmp, T& total) {
    static_assert(sizeof(T) == 4, "32-bit sums");
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    T inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if constexpr (NT == 64) {
        total = __shfl(inc, 63, 64);
        return inc - x;
    } else {
        if (lane == 63) tmp[wid] = inc;
        __syncthreads();
        T pre = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            const T v = tmp[i];
            pre += (i < wid) ? v : T(0);
            tot += v;
        }
        __syncthreads();
        total = tot;
        return pre + inc - x;
    }
}

// 64-bit exclusive prefix sum over a workgroup of NT threads; `tmp` holds
// NT/64 long longs of LDS.  All threads must call it.
template <int NT>
__device__ __forceinline__ long long block_excl_scan_ll(long long x, long long* tmp, long long& total) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    long long inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const long long y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) tmp[wid] = inc;
    __syncthreads();
    long long pre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const long long v = tmp[i];
        pre += (i < wid) ? v : 0;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return pre + inc - x;
}

// Sum over a workgroup of NT threads; `tmp` holds NT/64 values of LDS.
template <int NT>
__device__ __forceinline__ long long block_sum_ll(long long x, long long* tmp) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    if constexpr (NT == 64) {
        return x;
    } else {
        if (lane == 0) tmp[wid] = x;
        __syncthreads();
        long long s = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += tmp[i];
        __syncthreads();
        return s;
    }
}

// Per-workgroup sums keyed by node id in LDS: open addressing with linear
// probing over 2^LOG slots (key -1 = empty).  A sum that finds no slot goes
// straight to `spill[u]`.  Integer sums, so the order of additions does not
// matter.
template <int LOG>
struct LdsSums {
    static constexpr int kSlots = 1 << LOG;
    static constexpr int kProbes = 32;
    int32_t keys[kSlots];
    unsigned long long vals[kSlots];

    template <int NT>
    __device__ void clear() {
        for (int i = threadIdx.x; i < kSlots; i += NT) {
            keys[i] = -1;
            vals[i] = 0;
        }
    }
    __device__ void add(int32_t u, long long d, int64_t* spill) {
        const uint32_t h = ((uint32_t)u * 0x9E3779B1u) >> (32 - LOG);
        for (int p = 0; p < kProbes; ++p) {
            const uint32_t sl = (h + (uint32_t)p) & (kSlots - 1);
            int32_t k = keys[sl];
            if (k == -1) {
                k = atomicCAS(&keys[sl], -1, u);
                if (k == -1) k = u;
            }
            if (k == u) {
                atomicAdd(&vals[sl], (unsigned long long)d);
                return;
            }
        }
        atomicAdd((unsigned long long*)&spill[u], (unsigned long long)d);
    }
    // add every nonzero sum to out[key]; after a workgroup barrier
    template <int NT>
    __device__ void flush(int64_t* out) {
        for (int i = threadIdx.x; i < kSlots; i += NT) {
            const int32_t k = keys[i];
            const unsigned long long v = vals[i];
            if (k >= 0 && v != 0) atomicAdd((unsigned long long*)&out[k], v);
        }
    }
};

}  // namespace imin
