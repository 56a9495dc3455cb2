// Greedy selection (§2.2, the greedy framework): argmax of the gains over the
// candidates V \ (S ∪ B), ties to the smaller node id, and the round's
// bookkeeping.  Shared by the selection kernels and by the search for the
// changed worlds, which finishes the selection of the round before it.
#pragma once

#include "imin_device.hpp"
#include "imin_internal.hpp"

namespace imin {

__device__ __forceinline__ bool better(int64_t g1, int32_t u1, int64_t g2, int32_t u2) {
    if (u2 < 0) return u1 >= 0;
    if (u1 < 0) return false;
    return g1 > g2 || (g1 == g2 && u1 < u2);
}

// Workgroup-wide best (gain, node) and sum of the lost-node counts (256
// threads; every thread gets the result): each wave reduces with lane
// exchanges, then the four waves' results meet in LDS (sg, su, sd: four
// entries each).
__device__ __forceinline__ void select_block_best(int64_t& bg, int32_t& bu, long long& dl, int64_t* sg,
                                                  int32_t* su, long long* sd) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int64_t og = __shfl_xor(bg, d, 64);
        const int32_t ou = __shfl_xor(bu, d, 64);
        dl += __shfl_xor(dl, d, 64);
        if (better(og, ou, bg, bu)) {
            bg = og;
            bu = ou;
        }
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sg[wid] = bg;
        su[wid] = bu;
        sd[wid] = dl;
    }
    __syncthreads();
    bg = sg[0];
    bu = su[0];
    dl = sd[0];
#pragma unroll
    for (int x = 1; x < 4; ++x) {
        if (better(sg[x], su[x], bg, bu)) {
            bg = sg[x];
            bu = su[x];
        }
        dl += sd[x];
    }
    __syncthreads();  // the arrays may be reused
}

// Where a selection's parts are and where its results go.
struct SelectOut {
    int32_t parts;
    int64_t* pg;           // per part: best gain
    int32_t* pu;           //           its node
    long long* pd;         //           nodes lost by the round's changed worlds
    uint32_t* excl;        // bitmap of seeds and blockers
    int32_t k;
    int32_t* blockers;
    int64_t* gains;
    int64_t* totals;
    int32_t* n_selected;
};

// Combine the parts in one workgroup (every workgroup gets the same result).
__device__ __forceinline__ void select_combine(const SelectOut& so, int64_t& bg, int32_t& bu, long long& dl,
                                               int64_t* sg, int32_t* su, long long* sd) {
    bg = 0;
    bu = -1;
    dl = 0;
    // two parts per thread loaded before either is compared (512 parts in
    // one pass)
    for (int i0 = threadIdx.x; i0 < so.parts; i0 += 512) {
        const int i1 = i0 + 256;
        const int64_t g0 = so.pg[i0];
        const int32_t u0 = so.pu[i0];
        const long long d0 = so.pd[i0];
        int64_t g1 = 0;
        int32_t u1 = -1;
        long long d1 = 0;
        if (i1 < so.parts) {
            g1 = so.pg[i1];
            u1 = so.pu[i1];
            d1 = so.pd[i1];
        }
        if (better(g0, u0, bg, bu)) {
            bg = g0;
            bu = u0;
        }
        if (better(g1, u1, bg, bu)) {
            bg = g1;
            bu = u1;
        }
        dl += d0 + d1;
    }
    select_block_best(bg, bu, dl, sg, su, sd);
}

// The selection stops at round r when the budget is spent or no candidate
// with a positive gain is left.
__device__ __forceinline__ bool select_stops(int r, int32_t k, int32_t bu, int64_t bg) {
    return r >= k || bu < 0 || bg <= 0;
}

// Round r's bookkeeping (one thread): T_r, the check T_r = T_{r-1} - gain,
// the blocker, and the stop rule.
__device__ __forceinline__ void select_commit(RoundCtl* ctl, const SelectOut& so, int r, int64_t bg, int32_t bu,
                                              long long dl) {
    if (dl) ctl->total -= dl;
    const long long T = ctl->total;
    if (ctl->expect_total >= 0 && ctl->expect_total != T) atomicOr(&ctl->flags, (uint32_t)kFlagSpreadMismatch);
    so.totals[r] = T;
    if (select_stops(r, so.k, bu, bg)) {
        ctl->stop = 1;
        *so.n_selected = r;
        return;
    }
    so.blockers[r] = bu;
    so.gains[r] = bg;
    so.excl[bu >> 5] |= 1u << (bu & 31);
    ctl->ustar = bu;
    ctl->best_gain = bg;
    ctl->round = r + 1;
    ctl->expect_total = T - bg;
    if (r + 1 == so.k) {
        // T_k follows exactly from T_{k-1} - gain_{k-1}
        so.totals[so.k] = T - bg;
        ctl->stop = 1;
        *so.n_selected = so.k;
    }
}

}  // namespace imin
