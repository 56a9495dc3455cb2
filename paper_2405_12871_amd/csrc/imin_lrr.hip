// Global Sampling (Section 4.2, Algorithm 3; Definition 4.3): one LRR set per
// sample.
//
// Sample i of a pool is world w = w_begin + i of the pool's key.  Its target
// v is V'_s[(r * |V'_s|) >> 32], r the first word of the Philox block at
// counter (0, w, 1, 0) (edge coins use counter word 2 = 0, so the two never
// share a block).  The LRR set is empty when no seed reaches v in the world,
// else the nodes that reach v in phi^s, the live subgraph induced by the
// reached non-seeds.
//
// The forward reach of S is never built.  A reverse search from v over live
// in-edges, never entering a seed, collects v's cone C: the non-seeds with a
// live path to v that avoids every seed.  A cone node is reached from S
// exactly when some seed has a live edge into C followed by a live path
// inside C (the part of any seed-to-node path after its last seed stays in
// C), so a forward closure inside C from those entry edges gives the LRR set
// (the entry nodes and everything they reach in C); it is empty exactly when
// no entry edge exists.  Under weighted cascade probabilities the cone is
// small, as a reverse random walk.
//
// One wave per sample.  Each level of either search spreads the edges of all
// its frontier nodes over the wave's lanes, so a sample costs a few dependent
// round trips per level whatever its cone's degrees; the in-edges are
// records of 16 bytes (tail, slot, threshold), one load each.
//
// Each slot (workgroup) owns a stamp per node and a
// list sized for the whole graph, so any cone fits; a stamp of 2t+1 marks
// the cone of the slot's t-th sample and 2t+2 its LRR set, so stamps are
// never cleared between samples (nor between calls: a slot's epoch only
// grows).  The list holds the cone during the reverse search; the entry
// nodes are then moved to its front, and the forward closure appends the
// rest of the set behind them (the set is part of the cone, so it fits).
#include <hip/hip_runtime.h>

#include "imin_device.hpp"
#include "imin_internal.hpp"

namespace imin {
namespace {

constexpr int kLrrNT = 64;  // one wave per sample: most cones are small
static_assert(kLrrNT == 64, "the sampling workgroup is one wave");

// Edge e's coin in world w against threshold thr (thresholds 0 and 2^32 - 1
// need no draw).
__device__ __forceinline__ bool live_edge(const QueryDev& q, uint32_t w, int32_t e, uint32_t thr) {
    if (thr == kAlwaysLive) return true;
    if (thr == 0u) return false;
    const uint4 c = philox_block((uint32_t)e >> 2, w, q.key0, q.key1);
    const uint32_t x = ((e & 3) == 0) ? c.x : ((e & 3) == 1) ? c.y : ((e & 3) == 2) ? c.z : c.w;
    return x < thr;
}

struct LrrRows {
    int32_t x[kLrrNT];
    int32_t e0[kLrrNT];
    int32_t start[kLrrNT];
};

// The edges of the rows list[lo, hi) spread over the wave, up to 64 rows at
// a time: the rows' edge counts are scanned across the lanes, and lane t
// takes edges t, t + 64, ... of their concatenation, finding its row by a
// binary search over the rows' starts.  range(x) gives row x's edge range;
// edge(x, j) is called for each edge j of row x.  Ends with a barrier.
template <class Range, class Edge>
__device__ __forceinline__ void lrr_expand(const int32_t* list, int lo, int hi, LrrRows& rows, Range range,
                                           Edge edge) {
    const int t = threadIdx.x;
    for (int base = lo; base < hi; base += kLrrNT) {
        const int c = base + t;
        int32_t x = 0, e0 = 0, d = 0;
        if (c < hi) {
            x = list[c];
            const int2 r = range(x);
            e0 = r.x;
            d = r.y - r.x;
        }
        int incl = d;
#pragma unroll
        for (int o = 1; o < kLrrNT; o <<= 1) {
            const int y = __shfl_up(incl, o, kLrrNT);
            if (t >= o) incl += y;
        }
        const int total = __shfl(incl, kLrrNT - 1, kLrrNT);
        rows.x[t] = x;
        rows.e0[t] = e0;
        rows.start[t] = incl - d;
        __syncthreads();
        const int nrows = min(hi - base, kLrrNT);
        for (int j = t; j < total; j += kLrrNT) {
            int a = 0, b = nrows - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (rows.start[mid] <= j) a = mid;
                else b = mid - 1;
            }
            edge(rows.x[a], rows.e0[a] + (j - rows.start[a]));
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kLrrNT) void k_lrr(GraphDev g, QueryDev q, RoundCtl* ctl, uint32_t w_begin,
                                                uint32_t count, LrrDev L, TileOut out) {
    __shared__ int s_n;
    __shared__ unsigned long long s_base;
    __shared__ LrrRows rows;
    if (ctl->stop) return;
    const int t = threadIdx.x;
    const size_t n = (size_t)g.n;
    const size_t slot = blockIdx.x;
    int32_t* stamp = L.stamp + slot * n;
    int32_t* list = L.list + slot * n;
    int ep = L.epoch[slot];
    bool bad = false;
    for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
        ++ep;
        const int e1 = 2 * ep + 1, e2 = 2 * ep + 2;
        const uint32_t w = w_begin + i;
        const uint4 r = philox4x32_10(0u, w, 1u, 0u, q.key0, q.key1);
        const int32_t v = L.vprime[(uint32_t)(((uint64_t)r.x * (uint64_t)L.nvp) >> 32)];
        if (t == 0) {
            stamp[v] = e1;
            list[0] = v;
            s_n = 1;
        }
        __syncthreads();
        // reverse search, a level at a time: v's cone, with the cone nodes
        // that have a live edge from a seed stamped as set members
        int lo = 0, hi = 1;
        while (lo < hi) {
            lrr_expand(
                list, lo, hi, rows, [&](int32_t x) { return make_int2(L.in_off[x], L.in_off[x + 1]); },
                [&](int32_t x, int32_t j) {
                    const int4 ie = L.in_rec[j];  // {tail, slot, threshold, 0}
                    const int32_t u = ie.x;
                    const bool seed = bit_set(q.excl, u);
                    if (!seed && stamp[u] >= e1) return;  // in the cone already (or a self-loop)
                    if (!live_edge(q, w, ie.y, (uint32_t)ie.z)) return;
                    if (seed) {
                        atomicMax(&stamp[x], e2);
                    } else if (atomicMax(&stamp[u], e1) < e1) {
                        const int at = atomicAdd(&s_n, 1);
                        if (at < g.n) list[at] = u;
                        else bad = true;
                    }
                });
            lo = hi;
            hi = min(s_n, g.n);
            __syncthreads();
        }
        // the entry nodes to the front of the list, in order: the workgroup
        // is one wave, so a chunk is read before any lane writes, and every
        // write lands at or before its lane's read
        int ne = 0;
        for (int c0 = 0; c0 < hi; c0 += kLrrNT) {
            const int c = c0 + t;
            int32_t x = 0;
            bool entry = false;
            if (c < hi) {
                x = list[c];
                entry = stamp[x] == e2;
            }
            const unsigned long long b = __ballot(entry);
            if (entry) list[ne + __popcll(b & ((1ull << t) - 1ull))] = x;
            ne += __popcll(b);
        }
        if (t == 0) s_n = ne;
        __syncthreads();
        // forward closure inside the cone from the entry nodes, a level at a
        // time
        int flo = 0, fhi = ne;
        while (flo < fhi) {
            lrr_expand(
                list, flo, fhi, rows, [&](int32_t x) { return make_int2(g.off[x], g.off[x + 1]); },
                [&](int32_t, int32_t e) {
                    const int32_t y = g.col[e];
                    if (stamp[y] != e1) return;  // outside the cone, or in the set already
                    if (!live_edge(q, w, e, g.thr[e])) return;
                    if (atomicCAS(&stamp[y], e1, e2) == e1) {
                        const int at = atomicAdd(&s_n, 1);
                        if (at < g.n) list[at] = y;
                        else bad = true;
                    }
                });
            flo = fhi;
            fhi = min(s_n, g.n);
            __syncthreads();
        }
        const int nl = fhi;
        if (out.cover == kCoverCount) {
            // does the set meet the marked nodes?
            int hit = 0;
            for (int c = t; c < nl; c += kLrrNT) hit |= bit_set(out.mark, list[c]) ? 1 : 0;
            hit = __syncthreads_or(hit);
            if (t == 0) {
                out.world_size[i] = hit ? 1 : 0;
                out.wloc[i] = 0;
                out.wlen[i] = 0;
            }
        } else if (nl == 0) {
            // an empty set (the target not reached): no entries, no room taken
            if (t == 0) {
                out.wloc[i] = 0;
                out.wlen[i] = 0;
                out.world_size[i] = 0;
            }
        } else {
            if (t == 0) s_base = out.big_base + atomicAdd(&ctl->big_count, (unsigned long long)nl);
            __syncthreads();
            const unsigned long long base = s_base;
            if (base + (unsigned long long)nl <= out.scr_cap) {
                for (int c = t; c < nl; c += kLrrNT) {
                    out.scr_node[base + c] = list[c];
                    out.scr_cnt[base + c] = 1;
                }
                if (t == 0) {
                    out.wloc[i] = (int64_t)base;
                    out.wlen[i] = nl;
                }
            } else if (t == 0) {
                atomicOr(&ctl->flags, (uint32_t)kFlagPairOverflow);  // the tile is redone with more room
                out.wloc[i] = 0;
                out.wlen[i] = 0;
            }
            if (t == 0) out.world_size[i] = 1;
        }
        __syncthreads();
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    if (t == 0) L.epoch[slot] = ep;
}

}  // namespace

hipError_t launch_lrr(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin, uint32_t count,
                      const LrrDev& L, const TileOut& out, hipStream_t s) {
    if (L.n_slots < 1 || L.nvp < 1) return hipErrorInvalidValue;
    k_lrr<<<(unsigned)L.n_slots, kLrrNT, 0, s>>>(g, q, ctl, w_begin, count, L, out);
    return hipGetLastError();
}

}  // namespace imin
