// Device code around the world evaluation: graph ingest (offsets, coin
// thresholds, validation), query set-up, the atomic-free per-node gain
// reduction and the greedy selection.
//
// The per-node sums over worlds are formed without global atomics: a tile's
// (node, count) pairs are counting-sorted into node buckets of 8192 nodes,
// each (bucket, slice) is accumulated in LDS, and the slices' partial vectors
// are added in a fixed order.
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

template <class T>
__global__ void k_fill(T* p, T v, size_t count) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

template <class T>
static hipError_t fill(T* p, T v, size_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    k_fill<T><<<(unsigned)blocks, 256, 0, s>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }
hipError_t launch_fill_i64(int64_t* p, int64_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }

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
    for (int i = 0; i < 4; ++i) {
        ctl->list_n[i] = 0;
    }
    ctl->pair_count = 0;
    ctl->big_count = 0;
    ctl->tile_total = 0;
    ctl->xbig_count = 0;
    ctl->xtile_total = 0;
}
hipError_t launch_ctl_reset_round(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_round<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}
hipError_t launch_ctl_reset_tile(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_tile<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}

// ------------------------------------------------------- pair reduction
// Counting sort of the tile's pairs by node bucket (8192 nodes), then one
// LDS accumulation per (bucket, slice), then a fixed-order sum of slices.
constexpr int kRedNT = 256;
constexpr int kMaxBuckets = 2048;  // n < 2^24

__device__ __forceinline__ void chunk_range(unsigned long long P, int g1, int c, unsigned long long& a,
                                            unsigned long long& b) {
    a = P * (unsigned long long)c / (unsigned long long)g1;
    b = P * (unsigned long long)(c + 1) / (unsigned long long)g1;
}

__global__ __launch_bounds__(kRedNT) void k_hist(RoundCtl* ctl, const int32_t* pair_node,
                                                 unsigned long long cap, ReduceBufs rb) {
    __shared__ int h[kMaxBuckets];
    if (ctl->stop) return;
    unsigned long long P = ctl->pair_count;
    if (P > cap || P > rb.sorted_cap || (ctl->flags & kFlagPairOverflow)) {
        // never sort more entries than both buffers hold; flag it instead
        if (P && blockIdx.x == 0 && threadIdx.x == 0 && !(ctl->flags & kFlagPairOverflow))
            atomicOr(&ctl->flags, (uint32_t)kFlagReduceCapacity);
        P = 0;
    }
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT) h[i] = 0;
    __syncthreads();
    unsigned long long a, b;
    chunk_range(P, rb.g1, blockIdx.x, a, b);
    for (unsigned long long i = a + threadIdx.x; i < b; i += kRedNT)
        atomicAdd(&h[pair_node[i] >> kBucketShift], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT) rb.hist[(size_t)i * rb.g1 + blockIdx.x] = h[i];
}

// single-workgroup exclusive scan of hist[0 .. nb*g1) in place; hist[nb*g1] =
// total.  64-bit: a tile's pairs may exceed 2^31.
__global__ __launch_bounds__(1024) void k_scan(const RoundCtl* ctl, ReduceBufs rb) {
    __shared__ long long tmp[16];
    __shared__ long long carry;
    if (ctl->stop) return;
    const int total = rb.nb * rb.g1;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < total; base += 1024 * 4) {
        long long v[4];
        long long loc = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            v[k] = (i < total) ? rb.hist[i] : 0;
            loc += v[k];
        }
        long long tot;
        const long long ex = block_excl_scan_ll<1024>(loc, tmp, tot);
        long long run = carry + ex;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            if (i < total) rb.hist[i] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) rb.hist[total] = carry;
}

__global__ __launch_bounds__(kRedNT) void k_scatter(const RoundCtl* ctl, const int32_t* pair_node,
                                                    const int32_t* pair_cnt, unsigned long long cap,
                                                    ReduceBufs rb) {
    __shared__ unsigned long long cur[kMaxBuckets];
    if (ctl->stop) return;
    unsigned long long P = ctl->pair_count;
    if (P > cap || P > rb.sorted_cap || (ctl->flags & kFlagPairOverflow)) P = 0;
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT)
        cur[i] = (unsigned long long)rb.hist[(size_t)i * rb.g1 + blockIdx.x];
    __syncthreads();
    unsigned long long a, b;
    chunk_range(P, rb.g1, blockIdx.x, a, b);
    for (unsigned long long i = a + threadIdx.x; i < b; i += kRedNT) {
        const int32_t v = pair_node[i];
        const unsigned long long pos = atomicAdd(&cur[v >> kBucketShift], 1ull);
        rb.sorted_node[pos] = v;
        rb.sorted_cnt[pos] = pair_cnt[i];
    }
}

// One workgroup per (bucket, slice): LDS accumulation of the slice's pairs.
// With one slice the workgroup owns its bucket's nodes and adds the sums
// straight into gain; otherwise it writes a partial vector for k_sum_slices.
__global__ __launch_bounds__(kRedNT) void k_accum(const RoundCtl* ctl, int32_t n, ReduceBufs rb, int64_t* gain) {
    __shared__ unsigned long long acc[1 << kBucketShift];
    if (ctl->stop) return;
    const int bucket = blockIdx.x / rb.slices;
    const int slice = blockIdx.x % rb.slices;
    const long long bs = rb.hist[(size_t)bucket * rb.g1];
    const long long be = (bucket + 1 < rb.nb) ? rb.hist[(size_t)(bucket + 1) * rb.g1] : rb.hist[(size_t)rb.nb * rb.g1];
    const long long len = be - bs;
    if (rb.slices == 1 && len == 0) return;  // nothing to add to this bucket
    for (int i = threadIdx.x; i < (1 << kBucketShift); i += kRedNT) acc[i] = 0ull;
    __syncthreads();
    const long long a = bs + len * slice / rb.slices;
    const long long b = bs + len * (slice + 1) / rb.slices;
    const int32_t node0 = bucket << kBucketShift;
    for (long long i = a + threadIdx.x; i < b; i += kRedNT)
        atomicAdd(&acc[rb.sorted_node[i] - node0], (unsigned long long)(long long)rb.sorted_cnt[i]);
    __syncthreads();
    if (rb.slices == 1) {
        for (int i = threadIdx.x; i < (1 << kBucketShift); i += kRedNT) {
            const long long v = (long long)acc[i];
            if (v != 0 && node0 + i < n) gain[node0 + i] += v;
        }
        return;
    }
    int64_t* out = rb.part + (size_t)slice * ((size_t)rb.nb << kBucketShift) + ((size_t)bucket << kBucketShift);
    for (int i = threadIdx.x; i < (1 << kBucketShift); i += kRedNT) out[i] = (int64_t)acc[i];
}

__global__ void k_sum_slices(const RoundCtl* ctl, int32_t n, ReduceBufs rb, int64_t* gain) {
    if (ctl->stop) return;
    const size_t stride_s = (size_t)rb.nb << kBucketShift;
    for (size_t u = blockIdx.x * (size_t)blockDim.x + threadIdx.x; u < (size_t)n;
         u += (size_t)gridDim.x * blockDim.x) {
        int64_t s = gain[u];
        for (int k = 0; k < rb.slices; ++k) s += rb.part[k * stride_s + u];
        gain[u] = s;
    }
}

hipError_t launch_reduce_pairs(const GraphDev& g, const TileOut& out, const ReduceBufs& rb,
                               RoundCtl* ctl, int64_t* gain, hipStream_t s) {
    k_hist<<<rb.g1, kRedNT, 0, s>>>(ctl, out.pair_node, out.pair_cap, rb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_scan<<<1, 1024, 0, s>>>(ctl, rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scatter<<<rb.g1, kRedNT, 0, s>>>(ctl, out.pair_node, out.pair_cnt, out.pair_cap, rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_accum<<<rb.nb * rb.slices, kRedNT, 0, s>>>(ctl, g.n, rb, gain);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (rb.slices > 1) {
        k_sum_slices<<<1024, 256, 0, s>>>(ctl, g.n, rb, gain);
        e = hipGetLastError();
    }
    return e;
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
            // for the combining launch: the round, and the next round's counters cleared
            ctl->round_snap = ctl->round;
            for (int i = 0; i < 3; ++i) ctl->next[i] = 0;
            for (int i = 0; i < 4; ++i) {
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
