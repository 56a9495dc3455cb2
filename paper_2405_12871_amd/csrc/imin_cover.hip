// Max-Coverage over stored CP sequences (Section 5.1, the procedure of
// Algorithm 4; the coverage of Section 4.1).
//
// A world's CP sets are its dominator tree: the CP set of v is v's chain of
// non-seed dominators, so B covers v exactly when some node of B is v or a
// dominator of v.  The store keeps every world's non-seed entries in
// dominator-tree preorder, each with its current count, its parent's
// position and its subtree size, so a node's subtree is a run of entries.
// The count of an uncovered entry u is its marginal coverage in that world:
// the entries of u's subtree not yet covered (a covered entry counts 0).
// Blocking u covers its subtree (those entries drop to 0) and lowers every
// ancestor by u's count, which is exactly the new marginal of each ancestor;
// the dominator trees themselves never change.  gain[v], the sum over worlds
// of v's count, is the marginal coverage Cov(B + v) - Cov(B).
//
// A round r is four launches, all enqueued:
//   selection   the partial argmax (shared with the greedy solve), then a
//               one-workgroup commit: Cov(B_r), the stop rule, the pick;
//   top-k       the sum of the k largest marginals over the candidates by a
//               most-significant-digit radix search, kTopkBits per pass:
//               each pass histograms (count and sum per digit) the positive
//               candidates whose higher digits match the prefix chosen so
//               far, then one workgroup picks the digit holding the k-th
//               largest; after the last digit the k-th largest value is
//               known exactly, and the top-k sum is the sums of the bins
//               above it plus the rest at that value;
//   update      the pick's index entries, one wave per world.
//
// The same rounds run over LRR sets (Section 4.2; GSBM, Section 5.2): each
// stored item is one set with every member entry counting 1 while the set is
// uncovered, so gain[v] is the number of uncovered sets holding v, and a pick
// covers whole sets.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "imin_device.hpp"
#include "imin_internal.hpp"
#include "imin_select.hpp"

namespace imin {
namespace {

constexpr int kHistNT = 256;
constexpr int kPickNT = 1024;
constexpr int kUpdNT = 256;
static_assert(kTopkBins == kPickNT, "one bin per thread of the pick");

// state[]: 0 prefix, 1 k remaining, 2 sum of the bins above, 3 done flag

__global__ __launch_bounds__(256) void k_cover_commit(SelectOut so, CoverOut co, RoundCtl* ctl, int r) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    __shared__ long long sd[4];
    int64_t bg;
    int32_t bu;
    long long dl;
    select_combine(so, bg, bu, dl, sg, su, sd);
    if (threadIdx.x != 0 || ctl->stop) return;
    if (dl) ctl->total -= dl;
    const long long T = ctl->total;
    // the covered counts of the last update add up to the last pick's gain
    if (ctl->expect_total >= 0 && ctl->expect_total != T) atomicOr(&ctl->flags, (uint32_t)kFlagSpreadMismatch);
    co.cov[r] = co.t0 - T;
    co.state[0] = 0;
    co.state[1] = co.k;
    co.state[2] = 0;
    co.state[3] = co.k <= 0 ? 1 : 0;
    if (co.k <= 0) co.cov_upper[r] = co.cov[r];  // the top-0 sum is 0
    if (r >= so.k || bu < 0 || bg <= 0 || (ctl->flags & kFlagFatalMask)) {
        ctl->stop = 1;
        ctl->ustar = -1;
        *so.n_selected = r;
        return;
    }
    so.blockers[r] = bu;
    so.gains[r] = bg;
    // the pick joins the exclusions in the update, after the top-k search
    // of this round has counted it among the candidates of B_r
    ctl->ustar = bu;
    ctl->expect_total = T - bg;
    ctl->round = r + 1;
    *so.n_selected = r + 1;
}

__global__ __launch_bounds__(kHistNT) void k_topk_hist(const int64_t* __restrict__ gain, const uint32_t* __restrict__ excl,
                                                       int32_t n, CoverOut co, int r, int shift) {
    __shared__ uint32_t hc[kTopkBins];
    __shared__ long long hs[kTopkBins];
    if (co.cov[r] < 0 || co.state[3]) return;  // round not reached, or nothing left to find
    const unsigned long long prefix = (unsigned long long)co.state[0];
    for (int b = threadIdx.x; b < kTopkBins; b += kHistNT) {
        hc[b] = 0u;
        hs[b] = 0;
    }
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kHistNT;
    for (int64_t v0 = (int64_t)blockIdx.x * kHistNT + threadIdx.x; v0 < n; v0 += 4 * stride) {
        int64_t gv[4];
        uint32_t ex[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = v0 + j * stride;
            gv[j] = v < n ? gain[v] : 0;
            ex[j] = v < n ? excl[(uint32_t)v >> 5] : ~0u;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t v = (uint32_t)(v0 + j * stride);
            if (gv[j] <= 0 || ((ex[j] >> (v & 31u)) & 1u)) continue;
            const unsigned long long key = (unsigned long long)gv[j];
            const unsigned long long hi = (shift + kTopkBits >= 64) ? 0ull : (key >> (shift + kTopkBits));
            if (hi != prefix) continue;
            const int b = (int)((key >> shift) & (unsigned long long)(kTopkBins - 1));
            atomicAdd(&hc[b], 1u);
            atomicAdd((unsigned long long*)&hs[b], key);
        }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kTopkBins; b += kHistNT) {
        if (hc[b]) {
            atomicAdd(&co.hist_cnt[b], hc[b]);
            atomicAdd((unsigned long long*)&co.hist_sum[b], (unsigned long long)hs[b]);
        }
    }
}

// one workgroup, one bin per thread: bins are read from the top, so thread t
// holds bin kTopkBins-1-t and an inclusive scan gives the count of its bin
// and every bin above it
__global__ __launch_bounds__(kPickNT) void k_topk_pick(CoverOut co, int r, int shift) {
    __shared__ long long sc[kPickNT];
    __shared__ int found;
    if (co.cov[r] < 0 || co.state[3]) return;
    const int t = threadIdx.x;
    const int b = kTopkBins - 1 - t;
    const long long c = (long long)co.hist_cnt[b];
    const long long sm = co.hist_sum[b];
    co.hist_cnt[b] = 0u;  // cleared for the next pass
    co.hist_sum[b] = 0;
    sc[t] = c;
    if (t == 0) found = -1;
    __syncthreads();
    for (int d = 1; d < kPickNT; d <<= 1) {
        const long long x = t >= d ? sc[t - d] : 0;
        __syncthreads();
        sc[t] += x;
        __syncthreads();
    }
    const long long krem = co.state[1];
    const long long above = sc[t] - c;  // candidates in the bins above this one
    if (c > 0 && above < krem && krem <= sc[t]) found = t;
    __syncthreads();
    const int f = found;
    // sums of the bins above the chosen one (all bins when fewer than krem
    // candidates matched)
    __shared__ long long ss[kPickNT];
    ss[t] = (f < 0 || t < f) ? sm : 0;
    __syncthreads();
    for (int d = kPickNT / 2; d >= 1; d >>= 1) {
        if (t < d) ss[t] += ss[t + d];
        __syncthreads();
    }
    if (t != 0) return;
    long long acc = co.state[2] + ss[0];
    if (f < 0) {
        // fewer positive candidates than krem: all of them are in the top k
        co.state[2] = acc;
        co.state[3] = 1;
        co.cov_upper[r] = co.cov[r] + acc;
        return;
    }
    // the candidates in bins above f are taken whole
    const long long taken = (f > 0) ? sc[f - 1] : 0;
    const long long k2 = krem - taken;
    const unsigned long long prefix = ((unsigned long long)co.state[0] << kTopkBits) | (unsigned long long)(kTopkBins - 1 - f);
    if (shift == 0) {
        // the k-th largest value is prefix itself: k2 more of it complete the sum
        acc += k2 * (long long)prefix;
        co.state[2] = acc;
        co.state[3] = 1;
        co.cov_upper[r] = co.cov[r] + acc;
        return;
    }
    co.state[0] = (long long)prefix;
    co.state[1] = k2;
    co.state[2] = acc;
}

// The pick's worlds: idx_ent[idx_off[u] .. idx_off[u+1]) are (position,
// world) of u's entries; one wave per entry.
template <bool SETS>
__global__ __launch_bounds__(kUpdNT) void k_cover_update(RoundCtl* ctl, TileOut out, const uint32_t* __restrict__ idx_off,
                                                         const int2* __restrict__ idx_ent, int64_t* gain, long long* dsz,
                                                         uint32_t* excl) {
    __shared__ long long part[kUpdNT / 64];
    if (ctl->stop) return;
    const int32_t u = ctl->ustar;
    if (blockIdx.x == 0 && threadIdx.x == 0) excl[u >> 5] |= 1u << (u & 31);
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    const int gw = blockIdx.x * (kUpdNT / 64) + wid;
    const int nwaves = gridDim.x * (kUpdNT / 64);
    long long acc = 0;
    bool bad = false;
    const uint32_t a = idx_off[u], b = idx_off[u + 1];
    for (uint32_t i = a + (uint32_t)gw; i < b; i += (uint32_t)nwaves) {
        const int2 e = idx_ent[i];
        const long long pos = index_pos(e);
        const int w = e.y;
        const int c = out.store_cnt[pos];
        if (c <= 0) continue;  // u is covered in this world already (uniform per wave)
        const long long base = out.store_off[w];
        const int len = out.store_len[w];
        if (pos < base || pos >= base + len || (unsigned long long)(base + len) > out.store_cap) {
            bad = true;
            continue;
        }
        if constexpr (SETS) {
            // an LRR set: every member entry is covered, and the set counts once
            for (int j = lane; j < len; j += 64) {
                const long long q = base + j;
                const int cj = out.store_cnt[q];
                if (cj > 0) {
                    out.store_cnt[q] = 0;
                    if (q != pos) atomicAdd((unsigned long long*)&gain[out.store_node[q]], (unsigned long long)(long long)-cj);
                }
            }
            if (lane == 0) acc += 1;
            continue;
        }
        const int size = (int)out.store_lab[pos];
        if (pos + size > base + len) {
            bad = true;
            continue;
        }
        // u's subtree: the run of entries after u's own
        for (int j = lane; j < size; j += 64) {
            const long long q = pos + j;
            const int cj = out.store_cnt[q];
            if (cj > 0) {
                out.store_cnt[q] = 0;
                if (j != 0) atomicAdd((unsigned long long*)&gain[out.store_node[q]], (unsigned long long)(long long)-cj);
            }
        }
        // u's ancestors lose u's count
        if (lane == 0) {
            int at = out.store_par[pos];
            int steps = 0;
            while (at >= 0) {
                if (at >= len || ++steps > len) {
                    bad = true;
                    break;
                }
                const long long q = base + at;
                out.store_cnt[q] -= c;
                atomicAdd((unsigned long long*)&gain[out.store_node[q]], (unsigned long long)(long long)-c);
                at = out.store_par[q];
            }
            acc += c;
        }
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if (lane == 0) part[wid] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long s = 0;
        for (int x = 0; x < kUpdNT / 64; ++x) s += part[x];
        dsz[blockIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_cover_round(const GraphDev& g, int64_t* gain, RoundCtl* ctl, const SelectOut& so,
                              const CoverOut& co, int r, int key_bits, const TileOut& out, const uint32_t* idx_off,
                              const int2* idx_ent, long long* dsz, int32_t dsz_n, int grid, bool sets,
                              hipStream_t s) {
    if (grid < 1 || grid > dsz_n || key_bits < 1 || key_bits > 62) return hipErrorInvalidValue;
    hipError_t e = launch_select(g, gain, ctl, so, dsz, dsz_n, false, s);
    if (e != hipSuccess) return e;
    k_cover_commit<<<1, 256, 0, s>>>(so, co, ctl, r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int passes = (key_bits + kTopkBits - 1) / kTopkBits;
    const unsigned hist_grid = (unsigned)std::max<long long>(1, std::min<long long>(1024, ((long long)g.n + 4 * kHistNT - 1) / (4 * kHistNT)));
    for (int p = 0; p < passes; ++p) {
        const int shift = (passes - 1 - p) * kTopkBits;
        k_topk_hist<<<hist_grid, kHistNT, 0, s>>>(gain, so.excl, g.n, co, r, shift);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_topk_pick<<<1, kPickNT, 0, s>>>(co, r, shift);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (r < so.k) {
        if (sets)
            k_cover_update<true><<<(unsigned)grid, kUpdNT, 0, s>>>(ctl, out, idx_off, idx_ent, gain, dsz, so.excl);
        else
            k_cover_update<false><<<(unsigned)grid, kUpdNT, 0, s>>>(ctl, out, idx_off, idx_ent, gain, dsz, so.excl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace imin
