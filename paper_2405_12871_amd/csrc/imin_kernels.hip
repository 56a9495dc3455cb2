// Device code around the world evaluation: graph ingest (offsets, coin
// thresholds, validation), query set-up, the per-node gain reduction of a
// from-scratch pass and the greedy selection.
//
// A from-scratch pass sums the per-world counts by node bucket: the entries
// are partitioned into node buckets and each bucket's sums are formed in LDS,
// so no per-node counter in global memory is updated by more than one
// workgroup per slice of a bucket.  (Incremental rounds add their count
// changes to the gains with integer atomics in the world kernels.)
#include <algorithm>

#include "imin.h"
#include "imin_device.hpp"
#include "imin_internal.hpp"
#include "imin_select.hpp"

namespace imin {

// ------------------------------------------------------ graph ingest
// Offsets to int32, thresholds from probabilities (p == 1: always live;
// otherwise floor(p * 2^32), exact in double), validation of everything.
__global__ void k_graph_ingest(GraphDev g, const int64_t* row_ptr, const int32_t* col_in,
                               const float* p, RoundCtl* ctl) {
    const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t flags = 0;
    for (size_t u = tid; u <= (size_t)g.n; u += stride) {
        const int64_t r = row_ptr[u];
        if (r < 0 || r > g.m) flags |= kFlagBadOffsets;
        if (u == 0 && r != 0) flags |= kFlagBadOffsets;
        if (u == (size_t)g.n && r != g.m) flags |= kFlagBadOffsets;
        if (u < (size_t)g.n && row_ptr[u + 1] < r) flags |= kFlagBadOffsets;
        g.off[u] = (int32_t)r;
    }
    for (size_t e = tid; e < (size_t)g.m_pad; e += stride) {
        if (e < (size_t)g.m) {
            const int32_t v = col_in[e];
            const float pe = p[e];
            if (v < 0 || v >= g.n) flags |= kFlagBadCol;
            uint32_t th = 0;
            if (!(pe >= 0.0f && pe <= 1.0f)) {
                flags |= kFlagBadProb;
            } else if (pe == 1.0f) {
                th = kAlwaysLive;
            } else {
                th = (uint32_t)((double)pe * 4294967296.0);
            }
            g.col[e] = v;
            g.thr[e] = th;
        } else {
            g.col[e] = 0;
            g.thr[e] = 0u;
        }
    }
    if (flags) atomicOr(&ctl->flags, flags);
}

hipError_t launch_graph_ingest(const GraphDev& g, const int64_t* row_ptr, const int32_t* col_in,
                               const float* p, RoundCtl* ctl, hipStream_t s) {
    k_graph_ingest<<<2048, 256, 0, s>>>(g, row_ptr, col_in, p, ctl);
    return hipGetLastError();
}

// p[0 .. count) = v; with ctl given, nothing once the solve has stopped
template <class T>
__global__ void k_fill(T* p, T v, size_t count, const RoundCtl* ctl) {
    if (ctl && ctl->stop) return;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

template <class T>
static hipError_t fill(T* p, T v, size_t count, hipStream_t s, const RoundCtl* ctl = nullptr) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill<T><<<(unsigned)blocks, 256, 0, s>>>(p, v, count, ctl);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }
hipError_t launch_fill_i64(int64_t* p, int64_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }
hipError_t launch_fill_i64_live(int64_t* p, int64_t v, size_t c, const RoundCtl* ctl, hipStream_t s) {
    return fill(p, v, c, s, ctl);
}
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }

// ------------------------------------------------------- query set-up
// excl must be zero on entry.  Seeds are checked for range and repeats (the
// first pass marks them, the second finds duplicates by counting), blocked
// nodes for range and for being seeds.
__global__ void k_query_seeds(int32_t n, const int32_t* seeds, int32_t n_seeds, uint32_t* excl,
                              RoundCtl* ctl) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_seeds; i += gridDim.x * blockDim.x) {
        const int32_t v = seeds[i];
        if (v < 0 || v >= n) {
            atomicOr(&ctl->flags, (uint32_t)kFlagBadSeed);
            continue;
        }
        const uint32_t bit = 1u << (v & 31);
        const uint32_t old = atomicOr(&excl[v >> 5], bit);
        if (old & bit) atomicOr(&ctl->flags, (uint32_t)kFlagDupSeed);
    }
}

__global__ void k_query_blocked(int32_t n, const int32_t* blocked, int32_t n_blocked, uint32_t* excl,
                                RoundCtl* ctl) {
    // runs after all seeds are marked: a blocked id whose bit is already set
    // by a seed is an error; repeated blocked ids are fine
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_blocked; i += gridDim.x * blockDim.x) {
        const int32_t v = blocked[i];
        if (v < 0 || v >= n) {
            atomicOr(&ctl->flags, (uint32_t)kFlagBadBlocked);
            continue;
        }
        if (bit_set(excl, v)) {
            atomicOr(&ctl->flags, (uint32_t)kFlagBlockedSeed);
        }
    }
}

__global__ void k_query_blocked_mark(int32_t n, const int32_t* blocked, int32_t n_blocked,
                                     uint32_t* excl) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_blocked; i += gridDim.x * blockDim.x) {
        const int32_t v = blocked[i];
        if (v >= 0 && v < n) atomicOr(&excl[v >> 5], 1u << (v & 31));
    }
}

hipError_t launch_query_setup(const GraphDev& g, const int32_t* seeds, int32_t n_seeds,
                              const int32_t* blocked, int32_t n_blocked, uint32_t* excl,
                              RoundCtl* ctl, hipStream_t s) {
    const int words = (g.n + 31) >> 5;
    hipError_t e = fill<uint32_t>(excl, 0u, (size_t)words, s);
    if (e != hipSuccess) return e;
    k_query_seeds<<<(n_seeds + 255) / 256, 256, 0, s>>>(g.n, seeds, n_seeds, excl, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_blocked > 0) {
        k_query_blocked<<<(n_blocked + 255) / 256, 256, 0, s>>>(g.n, blocked, n_blocked, excl, ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_query_blocked_mark<<<(n_blocked + 255) / 256, 256, 0, s>>>(g.n, blocked, n_blocked, excl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------- counters
__global__ void k_ctl_reset_round(RoundCtl* ctl) {
    if (ctl->stop) return;
    ctl->total = 0;
    ctl->best_gain = 0;
}
__global__ void k_ctl_reset_tile(RoundCtl* ctl) {
    if (ctl->stop) return;
    for (int i = 0; i < 3; ++i) ctl->next[i] = 0;
    for (int i = 0; i < 5; ++i) {
        ctl->list_n[i] = 0;
    }
    ctl->pair_count = 0;
    ctl->big_count = 0;
    ctl->tile_total = 0;
    ctl->xbig_count = 0;
    ctl->xtile_total = 0;
}
__global__ void k_ctl_init(RoundCtl* ctl) {
    RoundCtl c{};
    c.expect_total = -1;
    *ctl = c;
}

__global__ void k_guard(RoundCtl* ctl, uint32_t mask, uint64_t theta, unsigned long long* hints) {
    if (ctl->flags & mask) ctl->stop = 1;
    if (hints && theta) {  // shares of the worlds handed on to tier 1 and tier 2 (1/1024 units)
        atomicMax(&hints[2], ((unsigned long long)ctl->list_n[1] << 10) / theta);
        atomicMax(&hints[3], ((unsigned long long)ctl->list_n[2] << 10) / theta);
    }
}

__global__ void k_solve_status(RoundCtl* ctl, int32_t* status, int32_t* n_selected, uint64_t theta,
                               unsigned long long* hints) {
    const uint32_t f = ctl->flags;
    int32_t st = IMIN_OK;
    if (f & kFlagDataMask) st = IMIN_ERR_DATA;
    else if (f & kFlagCapacityMask) st = IMIN_ERR_WORKSPACE;
    else if (f & kFlagFatalMask) st = IMIN_ERR_INTERNAL;
    if (status) *status = st;
    if (st != IMIN_OK && n_selected) *n_selected = 0;
    if (hints && theta) {
        atomicMax(&hints[0], (ctl->big_count << 10) / theta);
        atomicMax(&hints[1], (ctl->xbig_count << 10) / theta);
    }
}

__global__ void k_max_degree(GraphDev g, int32_t* out) {
    int d = 0;
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < g.n; u += gridDim.x * blockDim.x)
        d = max(d, g.off[u + 1] - g.off[u]);
    if (d > 0) atomicMax(out, d);
}

hipError_t launch_ctl_init(RoundCtl* ctl, hipStream_t s) {
    k_ctl_init<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}

hipError_t launch_guard(RoundCtl* ctl, uint32_t mask, hipStream_t s, uint64_t theta, unsigned long long* hints) {
    k_guard<<<1, 1, 0, s>>>(ctl, mask, theta, hints);
    return hipGetLastError();
}

hipError_t launch_solve_status(RoundCtl* ctl, int32_t* device_status, int32_t* n_selected, uint64_t theta,
                               unsigned long long* hints, hipStream_t s) {
    k_solve_status<<<1, 1, 0, s>>>(ctl, device_status, n_selected, theta, hints);
    return hipGetLastError();
}

hipError_t launch_max_degree(const GraphDev& g, int32_t* out, hipStream_t s) {
    k_max_degree<<<256, 256, 0, s>>>(g, out);
    return hipGetLastError();
}

hipError_t launch_ctl_reset_round(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_round<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}
hipError_t launch_ctl_reset_tile(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_tile<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}

// ------------------------------------------------------- gain reduction
// gain[u] += the counts of every (node u, count) entry of a tile's worlds
// (Section 2.2: the estimate of D(u) is the average of u's dominator-subtree
// sizes over the worlds; the sum is that average times the world count),
// read where the world kernels left them.  Nodes are cut into nb buckets of
// 2^shift consecutive ids:
//   k_gain_count      entries per bucket: an LDS histogram per workgroup of
//                     worlds, one counter update per bucket and workgroup;
//   k_gain_scan       64-bit bucket bases and partition cursors;
//   k_gain_partition  every entry as an 8-byte record (node, count) into its
//                     bucket's range: a batch of entries is counted per
//                     bucket in LDS, the batch's share of each bucket
//                     reserved with one counter update, the records staged
//                     bucket by bucket and each bucket's run written to
//                     consecutive addresses;
//   k_gain_own        one workgroup per (bucket, slice) sums its records'
//                     counts per node in LDS and adds the sums to gain: with
//                     one slice per bucket no two workgroups touch a node,
//                     with several each node gets one atomic add per slice.
// Integer sums: the result does not depend on any order.
constexpr int kGainNT = 512;
constexpr int kGainWorlds = 128;     // worlds per counting / partition workgroup
constexpr int kGainStage = 8192;     // records per partition batch
constexpr int kGainOwnNT = 1024;
static_assert(kGainWorlds <= kGainNT, "one world per thread when loading the ranges");
static_assert(kGainStage % kGainNT == 0, "whole batches per thread");

// Per-workgroup ranges of the worlds [w0, w0 + nw): woff / wpre (the flat
// numbering of their entries) in LDS; returns the workgroup's entry count.
// A range outside the entry arrays counts as empty and raises kFlagBounds.
__device__ __forceinline__ int gain_ranges(const GainSrc& src, uint32_t w0, int nw, long long* woff, int32_t* wpre,
                                           int* tmp, RoundCtl* ctl) {
    const int t = threadIdx.x;
    int len = 0;
    if (t < nw) {
        const long long o = src.off[w0 + t];
        len = src.len[w0 + t];
        if (o < 0 || len < 0 || (unsigned long long)o + (unsigned long long)len > src.cap) {
            atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            len = 0;
        }
        woff[t] = o;
    }
    int total;
    const int ex = block_excl_scan<kGainNT>(len, tmp, total);
    if (t <= nw) wpre[t] = ex;  // wpre[nw] = total
    __syncthreads();
    return total;
}

// the world of flat entry k: wpre[lo] <= k < wpre[lo + 1]
__device__ __forceinline__ int gain_world_of(const int32_t* wpre, int nw, int k) {
    int lo = 0, hi = nw;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wpre[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kGainNT) void k_gain_count(GainSrc src, GainBufs gb, RoundCtl* ctl) {
    __shared__ int32_t h[kGainMaxBuckets];
    __shared__ long long woff[kGainWorlds];
    __shared__ int32_t wpre[kGainWorlds + 1];
    __shared__ int tmp[kGainNT / 64];
    if (ctl->stop) return;
    const uint32_t w0 = blockIdx.x * (uint32_t)kGainWorlds;
    const int nw = (int)min((uint32_t)kGainWorlds, src.count - w0);
    for (int i = threadIdx.x; i < gb.nb; i += kGainNT) h[i] = 0;
    const int total = gain_ranges(src, w0, nw, woff, wpre, tmp, ctl);
    bool bad = false;
    for (int k0 = 0; k0 < total; k0 += 4 * kGainNT) {
        int32_t u[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + threadIdx.x + j * kGainNT;
            u[j] = -1;
            if (k < total) {
                const int lo = gain_world_of(wpre, nw, k);
                u[j] = src.node[woff[lo] + (k - wpre[lo])];
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (u[j] < 0) continue;
            const uint32_t bk = (uint32_t)u[j] >> gb.shift;
            if (bk < (uint32_t)gb.nb) atomicAdd(&h[bk], 1);
            else bad = true;
        }
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    __syncthreads();
    for (int i = threadIdx.x; i < gb.nb; i += kGainNT)
        if (h[i]) atomicAdd((unsigned long long*)&gb.bcnt[i], (unsigned long long)h[i]);
}

__global__ __launch_bounds__(1024) void k_gain_scan(GainBufs gb, RoundCtl* ctl) {
    __shared__ long long tmp[16];
    if (ctl->stop) return;
    long long run = 0;
    for (int c0 = 0; c0 < gb.nb; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const long long v = i < gb.nb ? gb.bcnt[i] : 0;
        long long tot;
        const long long ex = block_excl_scan_ll<1024>(v, tmp, tot);
        if (i < gb.nb) {
            gb.bbase[i] = run + ex;
            gb.bcur[i] = run + ex;
        }
        run += tot;
    }
    if (threadIdx.x == 0) {
        gb.bbase[gb.nb] = run;
        if ((unsigned long long)run > gb.rec_cap) atomicOr(&ctl->flags, (uint32_t)kFlagReduceCapacity);
    }
}

size_t gain_partition_lds(int nb) {
    return (size_t)kGainStage * sizeof(int2) + (size_t)nb * (sizeof(int32_t) + sizeof(long long));
}

__global__ __launch_bounds__(kGainNT) void k_gain_partition(GainSrc src, GainBufs gb, RoundCtl* ctl) {
    extern __shared__ int2 gpart_lds[];
    int2* stage = gpart_lds;                                                        // [kGainStage]
    long long* bdel = reinterpret_cast<long long*>(stage + kGainStage);             // [nb] global - local
    int32_t* bnum = reinterpret_cast<int32_t*>(bdel + gb.nb);                       // [nb] count, then base
    __shared__ long long woff[kGainWorlds];
    __shared__ int32_t wpre[kGainWorlds + 1];
    __shared__ int tmp[kGainNT / 64];
    constexpr int kPer = kGainStage / kGainNT;
    if (ctl->stop) return;
    const int t = threadIdx.x;
    const uint32_t w0 = blockIdx.x * (uint32_t)kGainWorlds;
    const int nw = (int)min((uint32_t)kGainWorlds, src.count - w0);
    const int total = gain_ranges(src, w0, nw, woff, wpre, tmp, ctl);
    const int nb = gb.nb;
    bool bad = false;
    for (int k0 = 0; k0 < total; k0 += kGainStage) {
        const int k1 = min(total, k0 + kGainStage);
        for (int i = t; i < nb; i += kGainNT) bnum[i] = 0;
        __syncthreads();
        int32_t ru[kPer], rc[kPer], rr[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = k0 + t + j * kGainNT;
            ru[j] = -1;
            rc[j] = rr[j] = 0;
            if (k < k1) {
                const int lo = gain_world_of(wpre, nw, k);
                const long long pos = woff[lo] + (k - wpre[lo]);
                ru[j] = src.node[pos];
                rc[j] = src.cnt[pos];
            }
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (ru[j] < 0) continue;
            const uint32_t bk = (uint32_t)ru[j] >> gb.shift;
            if (bk < (uint32_t)nb) rr[j] = atomicAdd(&bnum[bk], 1);
            else ru[j] = -1;
        }
        __syncthreads();
        // local bases, and the batch's share of each bucket
        const int per = (nb + kGainNT - 1) / kGainNT;
        const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
        int sum = 0;
        for (int bk = b0; bk < b1; ++bk) sum += bnum[bk];
        int staged;
        int base = block_excl_scan<kGainNT>(sum, tmp, staged);
        for (int bk = b0; bk < b1; ++bk) {
            const int c = bnum[bk];
            bnum[bk] = base;
            if (c)
                bdel[bk] = (long long)atomicAdd((unsigned long long*)&gb.bcur[bk], (unsigned long long)c) -
                           (long long)base;
            base += c;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (ru[j] >= 0) stage[bnum[(uint32_t)ru[j] >> gb.shift] + rr[j]] = make_int2(ru[j], rc[j]);
        __syncthreads();
        for (int i = t; i < staged; i += kGainNT) {
            const int2 r = stage[i];
            const unsigned long long g = (unsigned long long)(bdel[(uint32_t)r.x >> gb.shift] + i);
            if (g < gb.rec_cap) gb.rec[g] = r;
            else bad = true;
        }
        __syncthreads();
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
}

__global__ __launch_bounds__(kGainOwnNT) void k_gain_own(GainBufs gb, int32_t n, int64_t* gain, RoundCtl* ctl) {
    extern __shared__ unsigned long long gacc[];  // [1 << shift]
    if (ctl->stop) return;
    const int b = blockIdx.x / gb.slices;
    const int sl = blockIdx.x % gb.slices;
    const int width = 1 << gb.shift;
    for (int i = threadIdx.x; i < width; i += kGainOwnNT) gacc[i] = 0ull;
    __syncthreads();
    const unsigned long long cap = gb.rec_cap;
    const unsigned long long bs = min((unsigned long long)gb.bbase[b], cap);
    const unsigned long long be = min((unsigned long long)gb.bbase[b + 1], cap);
    const unsigned long long len = be - bs;
    const unsigned long long r0 = bs + len * (unsigned long long)sl / (unsigned long long)gb.slices;
    const unsigned long long r1 = bs + len * (unsigned long long)(sl + 1) / (unsigned long long)gb.slices;
    const int32_t node0 = b << gb.shift;
    for (unsigned long long q = r0; q < r1; q += 4ull * kGainOwnNT) {
        int2 e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned long long r = q + threadIdx.x + (unsigned long long)j * kGainOwnNT;
            e[j] = r < r1 ? gb.rec[r] : make_int2(-1, 0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t d = (uint32_t)(e[j].x - node0);
            if (d < (uint32_t)width) atomicAdd(&gacc[d], (unsigned long long)(uint32_t)e[j].y);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < width; i += kGainOwnNT) {
        const unsigned long long v = gacc[i];
        const int32_t u = node0 + i;
        if (v == 0ull || u >= n) continue;
        if (gb.slices == 1) gain[u] += (int64_t)v;
        else atomicAdd((unsigned long long*)&gain[u], v);
    }
}

GainBufs gain_buckets(int32_t n) {
    GainBufs gb{};
    int shift = 5;
    while (shift < 15 && (((long long)n + (1ll << shift) - 1) >> shift) > kGainMaxBuckets) ++shift;
    gb.shift = shift;
    gb.nb = (int)(((long long)n + (1ll << shift) - 1) >> shift);
    gb.slices = 1;
    return gb;
}

int gain_slices(const GainBufs& gb, unsigned long long entries, int cus) {
    // enough (bucket, slice) workgroups to cover the chip; more when the
    // buckets are long
    const long long want = (long long)cus * (entries > (64ull << 20) ? 4 : 1);
    return (int)std::max(1ll, std::min(64ll, (want + gb.nb - 1) / gb.nb));
}

hipError_t launch_gain_reduce(const GainSrc& src, const GainBufs& gb, int32_t n, int64_t* gain, RoundCtl* ctl,
                              hipStream_t s) {
    if (gb.nb < 1 || gb.nb > kGainMaxBuckets || ((long long)gb.nb << gb.shift) < (long long)n || gb.slices < 1)
        return hipErrorInvalidValue;
    if (src.count == 0) return hipSuccess;
    hipError_t e = fill<long long>(gb.bcnt, 0ll, (size_t)gb.nb, s);
    if (e != hipSuccess) return e;
    const unsigned groups = (src.count + kGainWorlds - 1) / kGainWorlds;
    k_gain_count<<<groups, kGainNT, 0, s>>>(src, gb, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_gain_scan<<<1, 1024, 0, s>>>(gb, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t lds = gain_partition_lds(gb.nb);
    if ((e = hipFuncSetAttribute((const void*)k_gain_partition, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return e;
    k_gain_partition<<<groups, kGainNT, lds, s>>>(src, gb, ctl);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const size_t olds = sizeof(unsigned long long) << gb.shift;
    if ((e = hipFuncSetAttribute((const void*)k_gain_own, hipFuncAttributeMaxDynamicSharedMemorySize, (int)olds)) !=
        hipSuccess)
        return e;
    k_gain_own<<<(unsigned)(gb.nb * gb.slices), kGainOwnNT, olds, s>>>(gb, n, gain, ctl);
    return hipGetLastError();
}

__global__ void k_sum_sizes(const int32_t* ws, uint32_t count, RoundCtl* ctl) {
    __shared__ long long tmp[4];
    if (ctl->stop) return;
    long long s = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        s += ws[i];
    s = block_sum_ll<256>(s, tmp);
    if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)&ctl->total, (unsigned long long)s);
}

hipError_t launch_sum_sizes(const int32_t* ws, uint32_t count, RoundCtl* ctl, hipStream_t s) {
    unsigned blocks = (count + 255) / 256;
    if (blocks > 64) blocks = 64;  // one counter update per block
    if (blocks == 0) return hipSuccess;
    k_sum_sizes<<<blocks, 256, 0, s>>>(ws, count, ctl);
    return hipGetLastError();
}

// ------------------------------------------------ generic exclusive scan
// ----------------------------------------------------------- selection
// argmax over candidates (not seeds, not blocked) of (gain desc, id asc).
// Two launches: every workgroup of the first reduces a slice of the
// candidates (and of the dsz slots) to a part; then one workgroup, or in an
// incremental round the search for the next round's changed worlds,
// combines the parts and applies the round's selection.  (A single launch
// whose last workgroup combines the parts needs a counter that every
// workgroup updates, and same-address atomics serialise.)
__global__ __launch_bounds__(256) void k_select_partial(RoundCtl* ctl, int32_t n, const int64_t* gain,
                                                        const uint32_t* excl, int64_t* pg, int32_t* pu,
                                                        long long* dsz, int32_t dsz_n, long long* pd) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    __shared__ long long sd[4];
    // the stop flag is read with the first gains rather than before them
    const int32_t stop = ctl->stop;
    // nodes lost by the changed worlds of the round: this part's slots,
    // loaded with the gains
    long long dl = 0;
    if (dsz) {
        const int per = (dsz_n + (int)gridDim.x - 1) / (int)gridDim.x;
        const int s0 = (int)blockIdx.x * per;
        const int s1 = min(s0 + per, dsz_n);
        for (int i = s0 + (int)threadIdx.x; i < s1; i += 256) dl += dsz[i];
    }
    int64_t bg = 0;
    int32_t bu = -1;
    // eight candidates per thread in flight at a time (all of a 2^20-node
    // graph's in one pass with 512 parts)
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t u0 = (int64_t)blockIdx.x * 256 + threadIdx.x; u0 < n; u0 += 8 * stride) {
        int64_t gv[8];
        uint32_t ex[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t v = u0 + j * stride;
            gv[j] = v < n ? gain[v] : 0;
            ex[j] = v < n ? excl[(uint32_t)v >> 5] : ~0u;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int32_t v = (int32_t)(u0 + j * stride);
            if (!((ex[j] >> ((uint32_t)v & 31u)) & 1u) && better(gv[j], v, bg, bu)) {
                bg = gv[j];
                bu = v;
            }
        }
    }
    if (dsz && !stop) {
        const int per = (dsz_n + (int)gridDim.x - 1) / (int)gridDim.x;
        const int s0 = (int)blockIdx.x * per;
        const int s1 = min(s0 + per, dsz_n);
        for (int i = s0 + (int)threadIdx.x; i < s1; i += 256) dsz[i] = 0;
    }
    select_block_best(bg, bu, dl, sg, su, sd);
    if (stop) return;  // uniform
    if (threadIdx.x == 0) {
        pg[blockIdx.x] = bg;
        pu[blockIdx.x] = bu;
        pd[blockIdx.x] = dl;
        if (blockIdx.x == 0) {
            // a solve that met a fatal condition (bad data, scratch too
            // small, a failed check) commits nothing more
            if (ctl->flags & kFlagFatalMask) ctl->stop = 1;
            // for the combining launch: the round, and the next round's counters cleared
            ctl->round_snap = ctl->round;
            for (int i = 0; i < 3; ++i) ctl->next[i] = 0;
            for (int i = 0; i < 5; ++i) {
                ctl->list_n[i] = 0;
            }
            ctl->pair_count = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_select_final(SelectOut so, RoundCtl* ctl) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    __shared__ long long sd[4];
    int64_t bg;
    int32_t bu;
    long long dl;
    select_combine(so, bg, bu, dl, sg, su, sd);
    if (threadIdx.x != 0 || ctl->stop) return;
    select_commit(ctl, so, ctl->round, bg, bu, dl);
}

hipError_t launch_select(const GraphDev& g, const int64_t* gain, RoundCtl* ctl, const SelectOut& so, long long* dsz,
                         int32_t dsz_n, bool combine, hipStream_t s) {
    k_select_partial<<<so.parts, 256, 0, s>>>(ctl, g.n, gain, so.excl, so.pg, so.pu, dsz, dsz_n, so.pd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !combine) return e;
    k_select_final<<<1, 256, 0, s>>>(so, ctl);
    return hipGetLastError();
}

} // namespace imin
