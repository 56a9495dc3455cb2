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
// One wave per sample.  Each slot (workgroup) owns a stamp per node and
// two lists sized for the whole graph, so any cone fits; a stamp of 2t+1
// marks the cone of the slot's t-th sample and 2t+2 its LRR set, so stamps
// are never cleared between samples.
#include <hip/hip_runtime.h>

#include "imin_device.hpp"
#include "imin_internal.hpp"

namespace imin {
namespace {

constexpr int kLrrNT = 64;  // one wave per sample: most cones are small

__device__ __forceinline__ bool coin_live(const GraphDev& g, const QueryDev& q, uint32_t w, int32_t e) {
    const uint32_t t = g.thr[e];
    if (t == kAlwaysLive) return true;
    const uint4 c = philox_block((uint32_t)e >> 2, w, q.key0, q.key1);
    const uint32_t x = ((e & 3) == 0) ? c.x : ((e & 3) == 1) ? c.y : ((e & 3) == 2) ? c.z : c.w;
    return x < t;
}

__global__ __launch_bounds__(kLrrNT) void k_lrr(GraphDev g, QueryDev q, RoundCtl* ctl, uint32_t w_begin,
                                                uint32_t count, LrrDev L, TileOut out) {
    __shared__ int s_ncone, s_nlst;
    __shared__ unsigned long long s_base;
    if (ctl->stop) return;
    const int t = threadIdx.x;
    const size_t n = (size_t)g.n;
    const size_t slot = blockIdx.x;
    int32_t* stamp = L.stamp + slot * n;
    int32_t* cone = L.cone + slot * n;
    int32_t* lst = L.lst + slot * n;
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
            cone[0] = v;
            s_ncone = 1;
            s_nlst = 0;
        }
        __syncthreads();
        // reverse search: v's cone, and the cone nodes with a live edge from a seed
        // (the wave's lanes share each frontier node's edges: most cones are
        // a few nodes with a few dozen in-edges between them)
        int lo = 0, hi = 1;
        while (lo < hi) {
            for (int c = lo; c < hi; ++c) {
                const int32_t x = cone[c];
                for (int32_t j = L.in_off[x] + t; j < L.in_off[x + 1]; j += kLrrNT) {
                    const int32_t u = L.in_src[j];
                    const bool seed = bit_set(q.excl, u);
                    if (!seed && stamp[u] >= e1) continue;  // in the cone already (or a self-loop)
                    if (!coin_live(g, q, w, L.in_eid[j])) continue;
                    if (seed) {
                        if (atomicCAS(&stamp[x], e1, e2) == e1) {
                            const int at = atomicAdd(&s_nlst, 1);
                            if (at < g.n) lst[at] = x;
                            else bad = true;
                        }
                    } else if (atomicMax(&stamp[u], e1) < e1) {
                        const int at = atomicAdd(&s_ncone, 1);
                        if (at < g.n) cone[at] = u;
                        else bad = true;
                    }
                }
            }
            __syncthreads();
            lo = hi;
            hi = min(s_ncone, g.n);
            __syncthreads();
        }
        // forward closure inside the cone from the entry nodes
        int flo = 0, fhi = min(s_nlst, g.n);
        while (flo < fhi) {
            for (int c = flo; c < fhi; ++c) {
                const int32_t x = lst[c];
                for (int32_t e = g.off[x] + t; e < g.off[x + 1]; e += kLrrNT) {
                    const int32_t y = g.col[e];
                    if (stamp[y] != e1) continue;  // outside the cone, or in the set already
                    if (!coin_live(g, q, w, e)) continue;
                    if (atomicCAS(&stamp[y], e1, e2) == e1) {
                        const int at = atomicAdd(&s_nlst, 1);
                        if (at < g.n) lst[at] = y;
                        else bad = true;
                    }
                }
            }
            __syncthreads();
            flo = fhi;
            fhi = min(s_nlst, g.n);
            __syncthreads();
        }
        const int nl = fhi;
        if (out.cover == kCoverCount) {
            // does the set meet the marked nodes?
            int hit = 0;
            for (int c = t; c < nl; c += kLrrNT) hit |= bit_set(out.mark, lst[c]) ? 1 : 0;
            hit = __syncthreads_or(hit);
            if (t == 0) {
                out.world_size[i] = hit ? 1 : 0;
                out.wloc[i] = 0;
                out.wlen[i] = 0;
            }
        } else {
            if (t == 0) s_base = out.big_base + atomicAdd(&ctl->big_count, (unsigned long long)nl);
            __syncthreads();
            const unsigned long long base = s_base;
            if (base + (unsigned long long)nl <= out.scr_cap) {
                for (int c = t; c < nl; c += kLrrNT) {
                    out.scr_node[base + c] = lst[c];
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
            if (t == 0) out.world_size[i] = nl > 0 ? 1 : 0;
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
