// World evaluation on gfx950: one workgroup evaluates one live-edge world
// (a realization, Section 2.1, Eq. 1) end to end.
//
//   1. Level-synchronous BFS from the seeds over live edges, never entering a
//      seed again or a blocked node.  Coins are Philox4x32-10 blocks drawn
//      lazily, one block per 4-aligned group of CSR slots of a reached row
//      (unscanned edges cannot change the reached set).  Level 0 walks a
//      per-query table of the seeds' slot groups; deeper levels lay their
//      rows out with a block-wide scan.  A claimed node gets a local id in
//      BFS order and its BFS parent; every other live edge into a reached
//      non-seed is kept ("extra" edge).  Edges into seeds never matter: a
//      seed's only dominator is the virtual source (Section 3.1).
//   2. Immediate dominators under the virtual source: every dominator of v
//      lies on a shortest path, so a strict dominator has a smaller BFS level
//      and a smaller local id.  Starting from the BFS tree, levels are swept
//      in order and each v with extra edges gets
//        idom(v) = lowest common ancestor of {parent(v)} and its extra
//                  predecessors in the current tree,
//      computed as the smallest id among LCA(parent(v), u) (all lie on
//      parent(v)'s chain).  Sweeps repeat until nothing changes; one sweep
//      suffices when every extra edge goes exactly one level down.
//   3. Subtree sizes c(v) = 1 + sum over children, deepest level first
//      (Section 2.2: c(v) is the number of nodes v protects in this world).
//   4. (node, c) pairs of the reached non-seeds go to the tile's pair buffer.
//
// Three tiers share this code: a one-wave workgroup with everything in LDS
// (worlds of up to 256 non-seed nodes), a four-wave workgroup with a larger
// LDS store (up to 2048), and a four-wave workgroup whose per-world arrays
// live in HBM (any size).  A world that outgrows a tier is redone by the next
// one; every tier gives the same integers.
#include "imin_device.hpp"
#include "imin_internal.hpp"

#include <algorithm>

namespace imin {

constexpr int kMaxDomPasses = 4096;

template <int NT>
struct WorldShared {
    int count;    // local ids handed out (= nodes reached so far)
    int n_extra;  // extra edges recorded
    int overflow; // store out of room: hand the world to the next tier
    int changed;
    int nonfwd;   // some extra edge does not go exactly one level down
    unsigned long long pair_base;
    unsigned long long x_base;
    long long edges;  // CSR slots of reached rows
    int ndelta;       // count changes reported (incremental rounds)
    int nlevels;      // BFS levels holding nodes
    unsigned long long in_bytes;  // algorithmic bytes read by the BFS phase
    unsigned long long acc_worlds, acc_edges, acc_bytes;  // this workgroup's work so far
    long long acc_dsize;  // reached nodes lost by this workgroup's worlds (incremental rounds)
    int row_lid[NT];
    int row_node[NT];
    int row_e0[NT];
    int row_e1[NT];
    int row_start[NT];
    int scan_tmp[NT / 64];
    long long sum_tmp[NT / 64];
};

// ------------------------------------------------------------ LDS store
// Seeds are implicit (local ids 0..ns-1, nodes read from the seed array,
// parent and idom = virtual source); only non-seed nodes are stored, at
// index lid - ns.  Node -> local id is an open-addressing table.
template <int CAPNS, int HBITS, int XCAP, int LVCAP>
struct LdsStore {
    static constexpr int kHash = 1 << HBITS;
    static constexpr int kCapNonSeed = CAPNS;
    static constexpr int kCapX = XCAP;
    static constexpr int kMaxSeeds = 32767 - CAPNS;  // local ids fit int16
    int32_t keys[kHash];
    int16_t vals[kHash];
    int32_t nodes[CAPNS];
    int16_t parent[CAPNS];
    int16_t idom[CAPNS];
    int32_t aux[CAPNS];
    int32_t xv[XCAP];
    int16_t xu[XCAP];
    int32_t lvl[LVCAP + 2];
    int32_t ns;
    const int32_t* seeds;

    __device__ static constexpr int cap_lv() { return LVCAP; }
    __device__ static constexpr int cap_x() { return XCAP; }
    __device__ bool fits(int n_seeds) const { return n_seeds <= kMaxSeeds; }

    __device__ __forceinline__ static uint32_t hash(int32_t v) {
        return ((uint32_t)v * 0x9E3779B1u) >> (32 - HBITS);
    }
    template <int NT>
    __device__ void clear() {
        for (int i = threadIdx.x; i < kHash; i += NT) keys[i] = -1;
    }
    template <int NT>
    __device__ void init_seeds(const QueryDev& q) {
        if (threadIdx.x == 0) {
            ns = q.n_seeds;
            seeds = q.seeds;
        }
    }
    // New node: its local id.  Already present: -1.  Out of room: -2.
    __device__ int claim(int32_t v, int* counter) {
        uint32_t h = hash(v);
        for (int probe = 0; probe < kHash; ++probe) {
            const int32_t old = atomicCAS(&keys[h], -1, v);
            if (old == -1) {
                const int lid = atomicAdd(counter, 1);
                if (lid - ns >= CAPNS) return -2;
                vals[h] = (int16_t)(lid - ns);
                return lid;
            }
            if (old == v) return -1;
            h = (h + 1) & (kHash - 1);
        }
        return -2;
    }
    // Local id of v, or -1 when v was not reached (nothing is ever removed
    // from the table within a world, so an empty slot ends the probe).
    __device__ int lookup(int32_t v) const {
        uint32_t h = hash(v);
        for (int probe = 0; probe < kHash; ++probe) {
            const int32_t k = keys[h];
            if (k == v) return (int)vals[h] + ns;
            if (k == -1) return -1;
            h = (h + 1) & (kHash - 1);
        }
        return -1;
    }
    __device__ int32_t node(int lid) const { return lid < ns ? seeds[lid] : nodes[lid - ns]; }
    __device__ void set_node(int lid, int32_t v) { nodes[lid - ns] = v; }
    __device__ int get_parent(int lid) const { return lid < ns ? -1 : (int)parent[lid - ns]; }
    __device__ void set_parent(int lid, int p) { parent[lid - ns] = (int16_t)p; }
    __device__ int get_idom(int lid) const { return lid < ns ? -1 : (int)idom[lid - ns]; }
    __device__ void set_idom(int lid, int p) { idom[lid - ns] = (int16_t)p; }
    __device__ int32_t* aux_ptr(int lid) { return &aux[lid - ns]; }
    __device__ int get_xu(int64_t x) const { return xu[x]; }
    __device__ void set_xu(int64_t x, int u) { xu[x] = (int16_t)u; }
    __device__ int get_xv(int64_t x) const { return xv[x]; }
    __device__ void set_xv(int64_t x, int v) { xv[x] = v; }
    // the extra edges' heads are node ids until resolved to local ids
    __device__ void resolve_xv(int64_t x) { xv[x] = lookup(xv[x]); }
    // local id now of the node of stored entry i (incremental rounds)
    __device__ int delta_lid(int /*i*/, int32_t u) const { return lookup(u); }
    template <int NT>
    __device__ void reset(int /*count*/) { clear<NT>(); }
};

// ------------------------------------------------------------ HBM store
// Per-slot arrays sized for the whole graph, so a world never outgrows it.
struct HbmStore {
    int32_t* lid_of;  // node -> local id, -1 = absent
    int32_t* nodes;
    int32_t* parent_;
    int32_t* idom_;
    int32_t* aux;
    int32_t* lvl;
    int32_t* xv;
    int32_t* xu_;
    int32_t cap_lv_;
    int64_t cap_x_;

    __device__ int cap_lv() const { return cap_lv_; }
    __device__ int64_t cap_x() const { return cap_x_; }
    __device__ bool fits(int) const { return true; }
    template <int NT>
    __device__ void init_seeds(const QueryDev& q) {
        for (int i = threadIdx.x; i < q.n_seeds; i += NT) {
            const int32_t v = q.seeds[i];
            lid_of[v] = i;
            nodes[i] = v;
            parent_[i] = -1;
            idom_[i] = -1;
        }
    }
    __device__ int claim(int32_t v, int* counter) {
        if (atomicCAS(&lid_of[v], -1, -2) != -1) return -1;
        const int lid = atomicAdd(counter, 1);
        lid_of[v] = lid;
        return lid;
    }
    __device__ int lookup(int32_t v) const { return lid_of[v]; }
    __device__ int32_t node(int lid) const { return nodes[lid]; }
    __device__ void set_node(int lid, int32_t v) { nodes[lid] = v; }
    __device__ int get_parent(int lid) const { return parent_[lid]; }
    __device__ void set_parent(int lid, int p) { parent_[lid] = p; }
    __device__ int get_idom(int lid) const { return idom_[lid]; }
    __device__ void set_idom(int lid, int p) { idom_[lid] = p; }
    __device__ int32_t* aux_ptr(int lid) { return &aux[lid]; }
    __device__ int get_xu(int64_t x) const { return xu_[x]; }
    __device__ void set_xu(int64_t x, int u) { xu_[x] = u; }
    __device__ int get_xv(int64_t x) const { return xv[x]; }
    __device__ void set_xv(int64_t x, int v) { xv[x] = v; }
    __device__ void resolve_xv(int64_t x) { xv[x] = lookup(xv[x]); }
    __device__ int delta_lid(int /*i*/, int32_t u) const { return lookup(u); }
    template <int NT>
    __device__ void reset(int count) {
        for (int i = threadIdx.x; i < count; i += NT) lid_of[nodes[i]] = -1;
    }
};

// A 4-aligned group of CSR slots [4*blk, 4*blk+4) of row ulid (node unode),
// restricted to the row's slots [e0, e1).
struct SlotGroup {
    uint32_t blk;
    int ulid;
    int32_t unode;
    int e0, e1;
    bool valid;
};

// Draw the coins of U slot groups and claim or record every live edge.  The
// work is split in phases so that the U groups' loads are in flight
// together: columns and thresholds, then the Philox blocks, then the
// exclusion bits of the live heads, then the claims.
template <int NT, int U, class Store>
__device__ __forceinline__ void scan_slot_groups(const GraphDev& g, const QueryDev& q, uint32_t w,
                                                 const SlotGroup (&gr)[U], Store& st, WorldShared<NT>& sh) {
    int4 cv[U];
    uint4 tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t b = gr[u].valid ? (size_t)gr[u].blk : 0;
        cv[u] = *reinterpret_cast<const int4*>(g.col + 4 * b);
        tv[u] = *reinterpret_cast<const uint4*>(g.thr + 4 * b);
    }
    uint4 cn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cn[u] = philox_block(gr[u].blk, w, q.key0, q.key1);
    int32_t vv[U][4];
    uint32_t ex[U][4];
    bool lv[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t vs[4] = {cv[u].x, cv[u].y, cv[u].z, cv[u].w};
        const uint32_t ts[4] = {tv[u].x, tv[u].y, tv[u].z, tv[u].w};
        const uint32_t cs[4] = {cn[u].x, cn[u].y, cn[u].z, cn[u].w};
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            const int e = (int)(4 * gr[u].blk) + qd;
            const bool in = gr[u].valid && e >= gr[u].e0 && e < gr[u].e1;
            const bool live = in && (ts[qd] == kAlwaysLive || cs[qd] < ts[qd]) && vs[qd] != gr[u].unode;
            vv[u][qd] = vs[qd];
            lv[u][qd] = live;
            ex[u][qd] = live ? q.excl[(uint32_t)vs[qd] >> 5] : 0u;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            if (!lv[u][qd]) continue;
            const int32_t v = vv[u][qd];
            if ((ex[u][qd] >> ((uint32_t)v & 31u)) & 1u) continue;  // seed or blocker
            const int lid = st.claim(v, &sh.count);
            if (lid >= 0) {
                st.set_node(lid, v);
                st.set_parent(lid, gr[u].ulid);
            } else if (lid == -1) {
                const int x = atomicAdd(&sh.n_extra, 1);
                if (x < st.cap_x()) {
                    st.xv[x] = v;
                    st.set_xu(x, gr[u].ulid);
                } else {
                    sh.overflow = 1;
                }
            } else {
                sh.overflow = 1;
            }
        }
    }
}

constexpr int kGroupsPerLane = 2;

// Phase 1 of a world evaluation by sampling: the BFS with coins.  Returns
// false when the store ran out of room (uniform over the workgroup).
template <int NT, class Store>
__device__ bool bfs_sample(const GraphDev& g, const QueryDev& q, uint32_t w, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    if (!st.fits(ns)) return false;  // uniform

    st.template init_seeds<NT>(q);
    if (t == 0) {
        sh.count = ns;
        sh.edges = q.seed_edges;
        sh.ndelta = 0;
        sh.n_extra = 0;
        sh.overflow = 0;
        st.lvl[0] = 0;
        st.lvl[1] = ns;
    }
    __syncthreads();

    // ---- level 0: the seeds' slot groups from the per-query table
    for (int j0 = t; j0 < q.n_seed_chunks; j0 += NT * kGroupsPerLane) {
        SlotGroup gr[kGroupsPerLane];
#pragma unroll
        for (int u = 0; u < kGroupsPerLane; ++u) {
            const int j = j0 + u * NT;
            if (j < q.n_seed_chunks) {
                const int4 d = q.seed_chunk[j];  // {blk, seed lid, e0, e1}
                gr[u] = SlotGroup{(uint32_t)d.x, d.y, -1, d.z, d.w, true};
            } else {
                gr[u] = SlotGroup{0u, 0, -1, 0, 0, false};
            }
        }
        scan_slot_groups<NT, kGroupsPerLane>(g, q, w, gr, st, sh);
    }
    __syncthreads();
    if (sh.overflow) return false;
    if (t == 0) st.lvl[2] = sh.count;
    __syncthreads();

    // ---- deeper levels
    int nlev = 2;  // closed levels: lvl[0..nlev]
    for (;;) {
        const int f0 = st.lvl[nlev - 1];
        const int f1 = st.lvl[nlev];
        if (f0 == f1) break;
        for (int base = f0; base < f1; base += NT) {
            const int i = base + t;
            int nb = 0, u = 0, e0 = 0, e1 = 0;
            if (i < f1) {
                u = st.node(i);
                e0 = g.off[u];
                e1 = g.off[u + 1];
                nb = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
            }
            int total;
            const int start = block_excl_scan<NT>(nb, sh.scan_tmp, total);
            if (e1 > e0) atomicAdd((unsigned long long*)&sh.edges, (unsigned long long)(e1 - e0));
            sh.row_lid[t] = i;
            sh.row_node[t] = u;
            sh.row_e0[t] = e0;
            sh.row_e1[t] = e1;
            sh.row_start[t] = start;
            __syncthreads();
            const int nrows = (f1 - base < NT) ? (f1 - base) : NT;
            for (int j0 = t; j0 < total; j0 += NT * kGroupsPerLane) {
                SlotGroup gr[kGroupsPerLane];
#pragma unroll
                for (int u = 0; u < kGroupsPerLane; ++u) {
                    const int j = j0 + u * NT;
                    if (j < total) {
                        int lo = 0, hi = nrows - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (sh.row_start[mid] <= j) lo = mid; else hi = mid - 1;
                        }
                        gr[u] = SlotGroup{(uint32_t)(sh.row_e0[lo] >> 2) + (uint32_t)(j - sh.row_start[lo]),
                                          sh.row_lid[lo], sh.row_node[lo], sh.row_e0[lo], sh.row_e1[lo], true};
                    } else {
                        gr[u] = SlotGroup{0u, 0, -1, 0, 0, false};
                    }
                }
                scan_slot_groups<NT, kGroupsPerLane>(g, q, w, gr, st, sh);
            }
            __syncthreads();
            if (sh.overflow) break;
        }
        if (sh.overflow) break;
        if (nlev + 1 > st.cap_lv()) {
            sh.overflow = 1;  // same nlev in every thread: uniform
            break;
        }
        if (t == 0) st.lvl[nlev + 1] = sh.count;
        __syncthreads();
        ++nlev;
    }
    __syncthreads();
    if (sh.overflow) return false;
    if (t == 0) {
        sh.nlevels = nlev - 1;  // levels 0..nlevels-1 hold nodes
        sh.in_bytes = 8ull * (unsigned long long)sh.edges + 8ull * (unsigned long long)(sh.count - ns) +
                      16ull * (unsigned long long)q.n_seed_chunks;
    }
    __syncthreads();
    return true;
}

// Phase 2, shared by sampling and replay: immediate dominators, subtree
// sizes and the outputs of the mode.
template <int NT, int TIER, class Store>
__device__ void finish_world(const QueryDev& q, RoundCtl* ctl, uint32_t w, uint32_t wi, const TileOut& out,
                             Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const int nlevels = sh.nlevels;
    const int R = sh.count;
    const int nx = sh.n_extra;

    // ---- dominators
    for (int x = t; x < nx; x += NT) st.resolve_xv(x);
    for (int i = ns + t; i < R; i += NT) {
        const int p = st.get_parent(i);
        st.set_idom(i, p);
        *st.aux_ptr(i) = p;
    }
    if (t == 0) sh.nonfwd = 0;
    __syncthreads();
    for (int x = t; x < nx; x += NT) {
        const int v = st.get_xv(x);
        const int u = st.get_xu(x);
        int lo = 0, hi = nlevels - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (st.lvl[mid] <= v) lo = mid; else hi = mid - 1;
        }
        const bool fwd = (lo >= 1) && (u >= st.lvl[lo - 1]) && (u < st.lvl[lo]);
        if (!fwd) sh.nonfwd = 1;
    }
    __syncthreads();
    if (nx > 0) {
        // Every sweep that changes something lowers some idom id, so the
        // sweeps end; the cap only guards a broken invariant.
        for (int pass = 0;; ++pass) {
            if (pass >= kMaxDomPasses) {
                if (t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagDomPasses);
                break;
            }
            if (t == 0) sh.changed = 0;
            __syncthreads();
            for (int L = 1; L < nlevels; ++L) {
                const int v0 = st.lvl[L], v1 = st.lvl[L + 1];
                for (int x = t; x < nx; x += NT) {
                    const int v = st.get_xv(x);
                    if (v < v0 || v >= v1) continue;
                    int a = st.get_parent(v);
                    int b = st.get_xu(x);
                    while (a != b) {
                        if (a > b) a = st.get_idom(a); else b = st.get_idom(b);
                    }
                    atomicMin(st.aux_ptr(v), a);
                }
                __syncthreads();
                for (int x = t; x < nx; x += NT) {
                    const int v = st.get_xv(x);
                    if (v < v0 || v >= v1) continue;
                    const int nv = *st.aux_ptr(v);
                    if (nv != st.get_idom(v)) {
                        st.set_idom(v, nv);
                        sh.changed = 1;
                    }
                }
                __syncthreads();
            }
            const bool again = sh.nonfwd && sh.changed;
            __syncthreads();
            if (!again) break;
        }
    }

    // ---- subtree sizes of non-seeds, deepest level first
    for (int i = ns + t; i < R; i += NT) *st.aux_ptr(i) = 1;
    __syncthreads();
    for (int L = nlevels - 1; L >= 1; --L) {
        for (int i = st.lvl[L] + t; i < st.lvl[L + 1]; i += NT) {
            const int p = st.get_idom(i);
            if (p >= ns) atomicAdd(st.aux_ptr(p), *st.aux_ptr(i));
        }
        __syncthreads();
    }

    // ---- outputs
    const int len = R - ns;
    int read_len = 0;  // stored entries read back (incremental rounds)
    if (out.mode == kModeDelta) {
        // The stored list keeps the round-0 order; an entry whose count is 0
        // is a node no longer reached.  Blocking only removes nodes, so every
        // node reached now has a live entry: walking the live entries finds
        // every count that changed; each is updated in place and the change
        // written at the front of the world's own range of dl_*.
        const size_t so = (size_t)out.store_off[w];
        int list_len = out.store_len[w];
        if (so + (size_t)list_len > out.store_cap || so + (size_t)list_len > out.dl_cap) {
            if (t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            list_len = 0;  // uniform: every thread read the same values
        }
        read_len = list_len;
        const int lane = t & 63;
        for (int base = 0; base < list_len; base += NT) {
            const int i = base + t;
            int32_t u = 0;
            int d = 0;
            if (i < list_len) {
                const int c_old = out.store_cnt[so + i];
                if (c_old > 0) {
                    u = out.store_node[so + i];
                    const int lid = st.delta_lid(i, u);
                    const int c_new = (lid >= ns) ? *st.aux_ptr(lid) : 0;
                    d = c_new - c_old;
                    if (d != 0) out.store_cnt[so + i] = c_new;
                }
            }
            const unsigned long long mask = __ballot(d != 0);
            const int cnt = __popcll(mask);
            int wbase = 0;
            if (lane == 0 && cnt) wbase = atomicAdd(&sh.ndelta, cnt);
            wbase = __shfl(wbase, 0, 64);
            if (d != 0) {
                const size_t pos = so + (size_t)(wbase + __popcll(mask & ((1ull << lane) - 1ull)));
                out.dl_node[pos] = u;
                out.dl_cnt[pos] = d;
            }
        }
        __syncthreads();
        if (t == 0) out.wlen[w] = sh.ndelta;
    } else {
        if (t == 0) {
            sh.pair_base = (TIER == 0) ? (unsigned long long)wi * out.slot_cap0
                                       : out.big_base + atomicAdd(&ctl->big_count, (unsigned long long)len);
        }
        __syncthreads();
        const unsigned long long off = sh.pair_base;
        if (off + (unsigned long long)len <= out.scr_cap) {
            for (int i = t; i < len; i += NT) {
                out.scr_node[off + i] = st.node(ns + i);
                out.scr_cnt[off + i] = *st.aux_ptr(ns + i);
                if (out.keep_edges) out.scr_par[off + i] = st.get_parent(ns + i);
            }
            if (t == 0) {
                out.wloc[wi] = (int64_t)off;
                out.wlen[wi] = len;
            }
        } else if (t == 0) {
            atomicOr(&ctl->flags, (uint32_t)kFlagPairOverflow);  // bump region full: the tile is redone
        }
        if (out.keep_edges) {
            // the extra live edges, as local ids, for later replays
            if (t == 0) {
                sh.x_base = (TIER == 0) ? (unsigned long long)wi * out.xslot_cap0
                                        : out.xbig_base + atomicAdd(&ctl->xbig_count, (unsigned long long)nx);
            }
            __syncthreads();
            const unsigned long long xo = sh.x_base;
            if (xo + (unsigned long long)nx <= out.xscr_cap) {
                for (int x = t; x < nx; x += NT) {
                    out.xscr_v[xo + x] = st.get_xv(x);
                    out.xscr_u[xo + x] = st.get_xu(x);
                }
                if (t == 0) {
                    out.xloc[wi] = (int64_t)xo;
                    out.xlen[wi] = nx;
                }
            } else if (t == 0) {
                atomicOr(&ctl->flags, (uint32_t)kFlagPairOverflow);
            }
        }
    }
    long long s = 0;
    if (out.world_sum) {  // uniform
        for (int i = ns + t; i < R; i += NT) s += st.node(i);
        s = block_sum_ll<NT>(s, sh.sum_tmp);
    }
    if (t == 0) {
        if (out.mode == kModeDelta) sh.acc_dsize += (long long)out.world_size[wi] - (long long)R;
        if (out.world_size) out.world_size[wi] = R;
        if (out.world_sum) out.world_sum[wi] = s + q.seed_sum;
        if (out.world_edges) out.world_edges[wi] = sh.edges;
        unsigned long long bytes = sh.in_bytes;
        if (out.mode == kModeDelta)
            bytes += 8ull * (unsigned long long)read_len + 12ull * (unsigned long long)sh.ndelta;
        else
            bytes += (out.keep_edges ? 12ull : 8ull) * (unsigned long long)len + 12ull +
                     (out.keep_edges ? 8ull * (unsigned long long)nx + 12ull : 0ull);
        // per-workgroup tallies, added to the device counters once at exit
        sh.acc_worlds += 1;
        sh.acc_edges += (unsigned long long)sh.edges;
        sh.acc_bytes += bytes;
    }
}

// A world evaluated by sampling: false when the store ran out of room.
template <int NT, int TIER, class Store>
__device__ bool evaluate_world(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w, uint32_t wi,
                               const TileOut& out, Store& st, WorldShared<NT>& sh) {
    if (!bfs_sample<NT>(g, q, w, st, sh)) return false;
    finish_world<NT, TIER>(q, ctl, w, wi, out, st, sh);
    return true;
}

// ------------------------------------------------------------- kernels
// Tier 0 (one wave, small LDS store) and tier 1 (four waves, larger LDS
// store).  With range_count > 0 the kernel takes worlds 0..range_count-1 of
// the tile; otherwise it takes the list handed down by the previous tier.
using Tier0Store = LdsStore<256, 9, 128, 30>;
using Tier1Store = LdsStore<2048, 12, 1024, 254>;
constexpr int kTier0NT = 64;
constexpr int kTier1NT = 256;
constexpr int kTier2NT = 256;

// Per-workgroup work tallies, one slot per (tier, field, workgroup): no
// shared counter is touched.
__device__ __forceinline__ void add_work(const TileOut& out, int tier, unsigned long long worlds,
                                         unsigned long long edges, unsigned long long bytes) {
    if (!out.work || !worlds) return;
    const size_t st = (size_t)out.work_stride;
    unsigned long long* wk = out.work + (size_t)tier * 3 * st + blockIdx.x;
    wk[0] += worlds;
    wk[st] += edges;
    wk[2 * st] += bytes;
}

// Worlds are dealt to workgroups by a fixed stride (no shared work counter).
template <int NT, class Store, int TIER>
__global__ __launch_bounds__(NT) void k_world_lds(GraphDev g, QueryDev q, RoundCtl* ctl, uint32_t w_begin,
                                                  uint32_t range_count, const int32_t* in_list, int count_idx,
                                                  int32_t* next_list, TileOut out) {
    __shared__ Store st;
    __shared__ WorldShared<NT> sh;
    const int t = threadIdx.x;
    if (ctl->stop) return;
    const uint32_t n_items = in_list ? min(ctl->list_n[count_idx], count_idx ? out.next_cap : out.list_cap)
                                     : range_count;
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    st.template clear<NT>();
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    for (uint32_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const uint32_t wi = in_list ? (uint32_t)in_list[k] : k;
        const bool ok = evaluate_world<NT, TIER>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) {
            const uint32_t pos = atomicAdd(&ctl->list_n[TIER + 1], 1u);
            if (pos < out.next_cap) next_list[pos] = (int32_t)wi;
            else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        }
        st.template reset<NT>(0);
        __syncthreads();
    }
    if (t == 0) {
        add_work(out, TIER, sh.acc_worlds, sh.acc_edges, sh.acc_bytes);
        // incremental rounds keep T up to date: subtract the nodes lost
        if (sh.acc_dsize) atomicAdd((unsigned long long*)&ctl->total, (unsigned long long)(-sh.acc_dsize));
    }
}

// Tier 2: per-world arrays in HBM, one slot per resident workgroup.
__global__ __launch_bounds__(kTier2NT) void k_world_hbm(GraphDev g, QueryDev q, RoundCtl* ctl, uint32_t w_begin,
                                                        uint32_t range_count, const int32_t* in_list,
                                                        int count_idx, TileOut out, BigSlots bs) {
    __shared__ WorldShared<kTier2NT> sh;
    const int t = threadIdx.x;
    const size_t slot = blockIdx.x;
    const size_t n = (size_t)g.n;
    HbmStore st;
    st.lid_of = bs.lid_of + slot * n;
    st.nodes = bs.nodes + slot * n;
    st.parent_ = bs.parent + slot * n;
    st.idom_ = bs.idom + slot * n;
    st.aux = bs.aux + slot * n;
    st.lvl = bs.lvl + slot * (n + 3);
    st.xv = bs.xv + slot * (size_t)bs.xcap;
    st.xu_ = bs.xu + slot * (size_t)bs.xcap;
    st.cap_lv_ = g.n + 1;
    st.cap_x_ = bs.xcap;
    if (ctl->stop) return;
    const uint32_t n_items = in_list ? min(ctl->list_n[count_idx], count_idx ? out.next_cap : out.list_cap)
                                     : range_count;
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_dsize = 0;
    }
    for (uint32_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const uint32_t wi = in_list ? (uint32_t)in_list[k] : k;
        const bool ok = evaluate_world<kTier2NT, 2>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBigCapacity);
        __syncthreads();
        st.reset<kTier2NT>(sh.count < g.n ? sh.count : g.n);
        __syncthreads();
    }
    if (t == 0) {
        add_work(out, 2, sh.acc_worlds, sh.acc_edges, sh.acc_bytes);
        if (sh.acc_dsize) atomicAdd((unsigned long long*)&ctl->total, (unsigned long long)(-sh.acc_dsize));
    }
}

// ------------------------------------------------------------ compaction
// Items are the tile's worlds [0, count) (entries at wloc/wlen in scratch) or,
// in incremental rounds, the changed worlds of list[0 .. list_n[0]) (changes
// at store_off[w] in dl_*, wlen[w] of them).  Each workgroup scans its
// items' lengths, takes one range of the destination with one counter
// update, and copies with one wave per item.
constexpr int kCompactNT = 256;

__global__ __launch_bounds__(kCompactNT) void k_sum_lengths(const int32_t* len, uint32_t count,
                                                            unsigned long long* total, RoundCtl* ctl) {
    __shared__ long long tmp[kCompactNT / 64];
    if (ctl->stop) return;
    long long s = 0;
    for (uint32_t i = blockIdx.x * kCompactNT + threadIdx.x; i < count; i += gridDim.x * kCompactNT) s += len[i];
    s = block_sum_ll<kCompactNT>(s, tmp);
    if (threadIdx.x == 0 && s) atomicAdd(total, (unsigned long long)s);
}

__global__ __launch_bounds__(kCompactNT) void k_compact(CompactSpec sp, RoundCtl* ctl) {
    __shared__ int tmp[kCompactNT / 64];
    __shared__ unsigned long long base_sh;
    __shared__ long long src_sh[kCompactNT];
    __shared__ unsigned long long dst_sh[kCompactNT];
    __shared__ int len_sh[kCompactNT];
    if (ctl->stop) return;
    const uint32_t n_items = sp.list ? min(ctl->list_n[0], sp.count) : sp.count;
    unsigned long long* counter =
        sp.counter_id == 0 ? &ctl->pair_count : (sp.counter_id == 1 ? &ctl->store_count : &ctl->xstore_count);
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    for (uint32_t b0 = blockIdx.x * kCompactNT; b0 < n_items; b0 += gridDim.x * kCompactNT) {
        const uint32_t i = b0 + threadIdx.x;
        int len = 0;
        long long src = 0;
        uint32_t w = 0;
        if (i < n_items) {
            w = sp.list ? (uint32_t)sp.list[i] : sp.w_begin + i;
            const uint32_t key = sp.by_world ? w : i;
            src = sp.loc[key];
            len = sp.len[key];
            if (len < 0 || src < 0 || (unsigned long long)src + (unsigned long long)len > sp.src_cap) {
                atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
                len = 0;
            }
        }
        int tot;
        const int ex = block_excl_scan<kCompactNT>(len, tmp, tot);
        if (threadIdx.x == 0) {
            base_sh = atomicAdd(counter, (unsigned long long)tot);
            if (sp.counter_id == 1) atomicAdd(&ctl->pair_count, (unsigned long long)tot);
        }
        __syncthreads();
        const unsigned long long dst = base_sh + (unsigned long long)ex;
        const bool fits = base_sh + (unsigned long long)tot <= sp.dst_cap;
        if (i < n_items && sp.out_off && fits) {
            sp.out_off[w] = (int64_t)dst;
            sp.out_len[w] = len;
        }
        src_sh[threadIdx.x] = src;
        dst_sh[threadIdx.x] = dst;
        len_sh[threadIdx.x] = (i < n_items) ? len : 0;
        __syncthreads();
        if (fits) {
            for (int it = wid; it < kCompactNT; it += kCompactNT / 64) {
                const int L = len_sh[it];
                const long long sp0 = src_sh[it];
                const unsigned long long dp = dst_sh[it];
                for (int f = 0; f < sp.nf; ++f)
                    for (int e = lane; e < L; e += 64) sp.dst[f][dp + e] = sp.src[f][sp0 + e];
            }
        } else if (threadIdx.x == 0) {
            atomicOr(&ctl->flags, sp.overflow_flag);
        }
        __syncthreads();
    }
}

hipError_t launch_sum_lengths(const int32_t* len, uint32_t count, unsigned long long* total, RoundCtl* ctl,
                              hipStream_t s) {
    k_sum_lengths<<<128, kCompactNT, 0, s>>>(len, count, total, ctl);
    return hipGetLastError();
}

hipError_t launch_compact(const CompactSpec& spec, RoundCtl* ctl, hipStream_t s) {
    k_compact<<<256, kCompactNT, 0, s>>>(spec, ctl);
    return hipGetLastError();
}

int world_tier0_capacity() { return Tier0Store::kCapNonSeed; }
int world_tier0_xcapacity() { return Tier0Store::kCapX; }

int world_tier_blocks_per_cu(int tier) {
    size_t lds = 0;
    if (tier == 0) lds = sizeof(Tier0Store) + sizeof(WorldShared<kTier0NT>);
    else if (tier == 1) lds = sizeof(Tier1Store) + sizeof(WorldShared<kTier1NT>);
    else return 2;
    int b = (int)((160 * 1024) / lds);
    return b < 1 ? 1 : b;
}

hipError_t launch_world_tier(int tier, const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin,
                             uint32_t range_count, const int32_t* in_list, int count_idx, int32_t* next_list,
                             const TileOut& out, const BigSlots& bs, int grid, hipStream_t s) {
    if (tier == 0) {
        k_world_lds<kTier0NT, Tier0Store, 0><<<grid, kTier0NT, 0, s>>>(g, q, ctl, w_begin, range_count, in_list,
                                                                       count_idx, next_list, out);
    } else if (tier == 1) {
        k_world_lds<kTier1NT, Tier1Store, 1><<<grid, kTier1NT, 0, s>>>(g, q, ctl, w_begin, range_count, in_list,
                                                                       count_idx, next_list, out);
    } else {
        k_world_hbm<<<bs.n_slots, kTier2NT, 0, s>>>(g, q, ctl, w_begin, range_count, in_list, count_idx, out, bs);
    }
    return hipGetLastError();
}

// ----------------------------------------------- incremental-round index
// After round 0 every stored entry (world w, position p, node u) is indexed
// by u.  The worlds a new blocker u changes are those whose entry for u is
// still live (count > 0): every other world keeps its reached set and its
// dominator tree.

// count entries per node
__global__ void k_index_count(const int32_t* store_node, unsigned long long n_entries, int32_t* cnt) {
    for (size_t p = blockIdx.x * (size_t)blockDim.x + threadIdx.x; p < n_entries; p += (size_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[store_node[p]], 1);
}

// one wave per world: place (position, world) of each entry at its node's cursor
__global__ void k_index_fill(TileOut out, uint32_t theta, int32_t* cursor, int32_t* idx_pos, int32_t* idx_world) {
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * (uint32_t)blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * (uint32_t)blockDim.x) >> 6;
    for (uint32_t w = wave; w < theta; w += nwaves) {
        const size_t so = (size_t)out.store_off[w];
        const int len = out.store_len[w];
        for (int i = lane; i < len; i += 64) {
            const int pos = atomicAdd(&cursor[out.store_node[so + i]], 1);
            idx_pos[pos] = (int32_t)(so + i);
            idx_world[pos] = (int32_t)w;
        }
    }
}

// worlds whose entry for the last selected blocker is live -> list_n[0]
__global__ __launch_bounds__(256) void k_affected(TileOut out, RoundCtl* ctl, const int32_t* idx_off,
                                                  const int32_t* idx_pos, const int32_t* idx_world,
                                                  int32_t* list) {
    if (ctl->stop) return;
    const int32_t u = ctl->ustar;
    const int32_t a = idx_off[u], b = idx_off[u + 1];
    const int lane = threadIdx.x & 63;
    for (int i = a + blockIdx.x * 256 + threadIdx.x - lane; i < b; i += gridDim.x * 256) {
        const int k = i + lane;
        const bool live = (k < b) && out.store_cnt[idx_pos[k]] > 0;
        const unsigned long long mask = __ballot(live);
        const int cnt = __popcll(mask);
        uint32_t base = 0;
        if (lane == 0 && cnt) base = atomicAdd(&ctl->list_n[0], (uint32_t)cnt);
        base = __shfl(base, 0, 64);
        if (live) {
            const uint32_t pos = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
            if (pos < out.list_cap) list[pos] = idx_world[k];
            else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        }
    }
}

hipError_t launch_index_count(const TileOut& out, unsigned long long n_entries, int32_t* cnt, hipStream_t s) {
    unsigned blocks = (unsigned)std::min<unsigned long long>((n_entries + 255) / 256, 8192ull);
    if (blocks == 0) return hipSuccess;
    k_index_count<<<blocks, 256, 0, s>>>(out.store_node, n_entries, cnt);
    return hipGetLastError();
}

hipError_t launch_index_fill(const TileOut& out, uint32_t theta, int32_t* cursor, int32_t* idx_pos,
                             int32_t* idx_world, hipStream_t s) {
    unsigned blocks = (theta + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    k_index_fill<<<blocks, 256, 0, s>>>(out, theta, cursor, idx_pos, idx_world);
    return hipGetLastError();
}

hipError_t launch_affected(const TileOut& out, RoundCtl* ctl, const int32_t* idx_off, const int32_t* idx_pos,
                           const int32_t* idx_world, int32_t* list, hipStream_t s) {
    k_affected<<<256, 256, 0, s>>>(out, ctl, idx_off, idx_pos, idx_world, list);
    return hipGetLastError();
}

// --------------------------------------------------------------- replay
// A world re-evaluated without coins.  Reached sets only shrink as blockers
// are added, so every live edge that can matter in a later round joins two
// nodes reached in round 0, and round 0 kept all of them: the BFS tree edges
// (each entry's parent) and the extra edges, as round-0 local ids.  The BFS
// is redone over those edges with the blocked nodes (and the nodes already
// lost, count 0) removed; dominators, counts and changes then follow exactly
// as for a sampled world.  Old non-seed j = ns + i is stored entry i.
template <int CAP, int XCAP, int ECAP, int LVCAP>
struct ReplayStore {
    int32_t nl[CAP];     // old entry -> new local id; -1 not reached yet, -2 removed, -3 being claimed
    int16_t eu[ECAP];    // edge sources, round-0 local ids (seeds are 0..ns-1)
    int16_t ev[ECAP];    // edge heads, old entry index
    int16_t parent[CAP]; // by new local id - ns
    int16_t idom[CAP];
    int32_t aux[CAP];
    int32_t xv[XCAP];    // extra edges of the new BFS: head (old entry until resolved), source new id
    int16_t xu[XCAP];
    int32_t lvl[LVCAP + 2];
    int32_t ns;

    __device__ static constexpr int cap_lv() { return LVCAP; }
    __device__ static constexpr int cap_x() { return XCAP; }
    __device__ int get_parent(int lid) const { return lid < ns ? -1 : (int)parent[lid - ns]; }
    __device__ void set_parent(int lid, int p) { parent[lid - ns] = (int16_t)p; }
    __device__ int get_idom(int lid) const { return lid < ns ? -1 : (int)idom[lid - ns]; }
    __device__ void set_idom(int lid, int p) { idom[lid - ns] = (int16_t)p; }
    __device__ int32_t* aux_ptr(int lid) { return &aux[lid - ns]; }
    __device__ int get_xu(int64_t x) const { return xu[x]; }
    __device__ void set_xu(int64_t x, int u) { xu[x] = (int16_t)u; }
    __device__ int get_xv(int64_t x) const { return xv[x]; }
    __device__ void set_xv(int64_t x, int v) { xv[x] = v; }
    __device__ void resolve_xv(int64_t x) { xv[x] = nl[xv[x]]; }
    __device__ int delta_lid(int i, int32_t /*u*/) const { return nl[i]; }
    __device__ int32_t node(int) const { return 0; }  // node ids are not needed in incremental rounds
};

using ReplayStoreT = ReplayStore<512, 128, 768, 62>;
constexpr int kReplayNT = 64;

template <int NT, class RS>
__device__ bool bfs_replay(const QueryDev& q, uint32_t w, const TileOut& out, RS& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const size_t so = (size_t)out.store_off[w];
    const int L0 = out.store_len[w];
    const size_t xo = (size_t)out.xstore_off[w];
    const int X0 = out.xstore_len[w];
    const int E = L0 + X0;
    // room, and local ids that fit the 16-bit arrays (uniform checks)
    if (L0 > 512 || E > 768 || ns + L0 > 32767) return false;
    if (so + (size_t)L0 > out.store_cap || xo + (size_t)X0 > out.xstore_cap) return false;
    if (t == 0) {
        st.ns = ns;
        sh.count = ns;
        sh.edges = E;
        sh.ndelta = 0;
        sh.n_extra = 0;
        sh.overflow = 0;
        st.lvl[0] = 0;
        st.lvl[1] = ns;
    }
    for (int i = t; i < L0; i += NT) {
        const bool gone = out.store_cnt[so + i] == 0 || bit_set(q.excl, out.store_node[so + i]);
        st.nl[i] = gone ? -2 : -1;
        st.eu[i] = (int16_t)out.store_par[so + i];
        st.ev[i] = (int16_t)i;
    }
    for (int x = t; x < X0; x += NT) {
        st.eu[L0 + x] = (int16_t)out.xstore_u[xo + x];
        st.ev[L0 + x] = (int16_t)(out.xstore_v[xo + x] - ns);
    }
    __syncthreads();
    int nlev = 1;
    for (;;) {
        const int f0 = st.lvl[nlev - 1];
        const int f1 = st.lvl[nlev];
        if (f0 == f1) break;
        for (int e = t; e < E; e += NT) {
            const int u = st.eu[e];
            const int vi = st.ev[e];
            if (u < 0 || u >= ns + L0 || vi < 0 || vi >= L0) continue;  // not a stored local id
            const int nu = (u < ns) ? u : st.nl[u - ns];
            if (nu < f0 || nu >= f1) continue;  // the source is not in this level
            const int old = atomicCAS(&st.nl[vi], -1, -3);
            if (old == -1) {
                const int lid = atomicAdd(&sh.count, 1);
                st.nl[vi] = lid;
                st.set_parent(lid, nu);
            } else if (old != -2) {
                const int x = atomicAdd(&sh.n_extra, 1);
                if (x < st.cap_x()) {
                    st.xv[x] = vi;  // resolved to its new id in the dominator phase
                    st.xu[x] = (int16_t)nu;
                } else {
                    sh.overflow = 1;
                }
            }
        }
        __syncthreads();
        if (sh.overflow) return false;
        if (nlev + 1 > st.cap_lv()) return false;  // same nlev in every thread: uniform
        if (t == 0) st.lvl[nlev + 1] = sh.count;
        __syncthreads();
        ++nlev;
    }
    if (t == 0) {
        sh.nlevels = nlev - 1;
        sh.in_bytes = 12ull * (unsigned long long)L0 + 8ull * (unsigned long long)X0;
    }
    __syncthreads();
    return true;
}

// Incremental rounds: every changed world is first replayed; a world that
// does not fit the replay store goes on to the sampling tiers (list 1).
__global__ __launch_bounds__(kReplayNT) void k_world_replay(QueryDev q, RoundCtl* ctl, const int32_t* in_list,
                                                             int32_t* next_list, TileOut out) {
    __shared__ ReplayStoreT st;
    __shared__ WorldShared<kReplayNT> sh;
    const int t = threadIdx.x;
    if (ctl->stop) return;
    const uint32_t n_items = min(ctl->list_n[0], out.list_cap);
    if (blockIdx.x >= n_items) return;
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    for (uint32_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const uint32_t w = (uint32_t)in_list[k];
        if (bfs_replay<kReplayNT>(q, w, out, st, sh)) {
            finish_world<kReplayNT, 0>(q, ctl, w, w, out, st, sh);
        } else if (t == 0) {
            const uint32_t pos = atomicAdd(&ctl->list_n[1], 1u);
            if (pos < out.next_cap) next_list[pos] = (int32_t)w;
            else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        }
        __syncthreads();
    }
    if (t == 0) {
        add_work(out, 3, sh.acc_worlds, sh.acc_edges, sh.acc_bytes);
        if (sh.acc_dsize) atomicAdd((unsigned long long*)&ctl->total, (unsigned long long)(-sh.acc_dsize));
    }
}

int world_replay_blocks_per_cu() {
    const size_t lds = sizeof(ReplayStoreT) + sizeof(WorldShared<kReplayNT>);
    int b = (int)((160 * 1024) / lds);
    return b < 1 ? 1 : b;
}

hipError_t launch_world_replay(const QueryDev& q, RoundCtl* ctl, const int32_t* in_list, int32_t* next_list,
                               const TileOut& out, int grid, hipStream_t s) {
    k_world_replay<<<grid, kReplayNT, 0, s>>>(q, ctl, in_list, next_list, out);
    return hipGetLastError();
}

// ------------------------------------------------- level-0 slot table
// For seed i with row [e0, e1): nb_i = number of 4-aligned slot groups.
__global__ void k_seed_count(GraphDev g, const int32_t* seeds, int32_t ns, int32_t* cnt, RoundCtl* ctl) {
    long long sum = 0, edges = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        const int32_t v = seeds[i];
        int nb = 0;
        if (v >= 0 && v < g.n) {
            const int e0 = g.off[v], e1 = g.off[v + 1];
            nb = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
            sum += v;
            edges += e1 - e0;
        }
        cnt[i] = nb;
    }
    if (sum) atomicAdd((unsigned long long*)&ctl->seed_sum, (unsigned long long)sum);
    if (edges) atomicAdd((unsigned long long*)&ctl->seed_edges, (unsigned long long)edges);
}

// Single workgroup: exclusive scan of cnt[0..ns) in place, total to ctl.
__global__ __launch_bounds__(1024) void k_seed_scan(int32_t* cnt, int32_t ns, RoundCtl* ctl) {
    __shared__ int tmp[16];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < ns; base += 1024) {
        const int i = base + threadIdx.x;
        const int v = (i < ns) ? cnt[i] : 0;
        int tot;
        const int ex = block_excl_scan<1024>(v, tmp, tot);
        if (i < ns) cnt[i] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->seed_chunks = carry;
}

__global__ void k_seed_fill(GraphDev g, const int32_t* seeds, int32_t ns, const int32_t* start, int4* table) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ns; i += gridDim.x * blockDim.x) {
        const int32_t v = seeds[i];
        const int e0 = g.off[v], e1 = g.off[v + 1];
        if (e1 <= e0) continue;
        const int b0 = e0 >> 2, b1 = (e1 - 1) >> 2;
        for (int b = b0; b <= b1; ++b) table[start[i] + (b - b0)] = make_int4(b, i, e0, e1);
    }
}

hipError_t launch_seed_count(const GraphDev& g, const int32_t* seeds, int32_t ns, int32_t* cnt, RoundCtl* ctl,
                             hipStream_t s) {
    k_seed_count<<<(ns + 255) / 256, 256, 0, s>>>(g, seeds, ns, cnt, ctl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_seed_scan<<<1, 1024, 0, s>>>(cnt, ns, ctl);
    return hipGetLastError();
}

hipError_t launch_seed_fill(const GraphDev& g, const int32_t* seeds, int32_t ns, const int32_t* start,
                            int4* table, hipStream_t s) {
    k_seed_fill<<<(ns + 255) / 256, 256, 0, s>>>(g, seeds, ns, start, table);
    return hipGetLastError();
}

}  // namespace imin
