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
#include <hip/hip_ext.h>

#include "imin_device.hpp"
#include "imin_internal.hpp"
#include "imin_select.hpp"

#include <algorithm>
#include <cstdlib>

namespace imin {

constexpr int kMaxDomPasses = 4096;

// Limits of the replay of a changed world (entries, stored extra edges, all
// stored edges).  A world within them never fails its replay: the extra
// edges of a replay never outnumber the stored ones, and the level array
// has a slot per entry.
constexpr int kReplayCap = 512;
constexpr int kReplayXCap = 256;
constexpr int kReplayEdgeCap = 768;

// The rows of one BFS step: frontier nodes, their CSR ranges and the first
// slot group of each.
template <int NT>
struct BfsRows {
    int lid[NT];
    int node[NT];
    int e0[NT];
    int e1[NT];
    int start[NT];
};
// The stores lend the rows LDS that the BFS leaves unused: the LDS stores
// their dominator arrays, the HBM store its extra-edge staging.  (Tier 0
// gains a resident wave per SIMD from it, tier 2 a workgroup per CU.)

template <int NT>
struct WorldShared {
    int count;    // local ids handed out (= nodes reached so far)
    int n_extra;  // extra edges recorded
    int overflow; // store out of room: hand the world to the next tier
    int changed;
    int nonfwd;   // some extra edge does not go exactly one level down
    unsigned long long xlevels;  // bit L: some extra edge ends in level L (bit 63: level 63 or deeper)
    int root_cur;  // label placement of the dominator tree's roots
    unsigned long long pair_base;
    unsigned long long x_base;
    long long edges;  // CSR slots of reached rows
    int ndelta;       // count changes reported (incremental rounds)
    int nlevels;      // BFS levels holding nodes
    int covered;      // non-seeds whose CP set meets the marked set (coverage count)
    unsigned long long in_bytes;  // algorithmic bytes read by the BFS phase
    unsigned long long acc_worlds, acc_edges, acc_bytes;  // this workgroup's work so far
    unsigned long long acc_reached, acc_live;  // reached nodes (seeds included) and recorded live edges
    long long acc_dsize;  // reached nodes lost by this workgroup's worlds (incremental rounds)
    uint32_t sched;       // first world of the chunk just taken
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
    int16_t idom[CAPNS];  // idom and aux hold a one-wave BFS's rows until the dominator phase
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
    template <int NT>
    __device__ BfsRows<NT>& bfs_rows() {
        static_assert(sizeof(idom) % 4 == 0 && sizeof(BfsRows<NT>) <= sizeof(idom) + sizeof(aux),
                      "the rows fit idom and aux, which follow each other");
        return *reinterpret_cast<BfsRows<NT>*>(idom);
    }
    __device__ int get_xu(int64_t x) const { return xu[x]; }
    __device__ void set_xu(int64_t x, int u) { xu[x] = (int16_t)u; }
    __device__ int get_xv(int64_t x) const { return xv[x]; }
    __device__ void set_xv(int64_t x, int v) { xv[x] = v; }
    // the extra edges' heads are node ids until resolved to local ids
    __device__ void resolve_xv(int64_t x) { xv[x] = lookup(xv[x]); }
    // local id now of the node of stored entry i (incremental rounds)
    __device__ int delta_lid(int /*i*/, int32_t u) const { return lookup(u); }
    // dominator-tree labels, once the counts are known: the node table is
    // no longer needed and holds the placement cursors and preorder indexes
    static constexpr bool kLabels = true;
    __device__ int32_t* cur_ptr(int lid) { return &keys[lid - ns]; }
    __device__ void set_tin(int lid, int v) { vals[lid - ns] = (int16_t)v; }
    __device__ int get_tin(int lid) const { return (int)(uint16_t)vals[lid - ns]; }
    // once the labels are placed the cursors are free: the exit ranges of
    // the labels live there and in the rest of the table
    static_assert(kHash >= 2 * CAPNS, "room for the exit ranges");
    static constexpr bool kSortExtras = false;  // the extra edges are in LDS already
    __device__ int32_t* lo_ptr(int lid) { return &keys[lid - ns]; }
    __device__ int32_t* hi_ptr(int lid) { return &keys[CAPNS + lid - ns]; }
    template <int NT>
    __device__ void reset(int /*count*/) { clear<NT>(); }
    template <int NT>
    __device__ void stage(int) {}  // everything is in LDS already
};

// ------------------------------------------------------------ HBM store
// Per-slot arrays sized for the whole graph, so a world never outgrows it.
// A node is claimed in a visited bitset (in LDS when the graph's bitset
// fits, else the slot's own words in HBM); its claimer writes lid_of[v],
// which is read only while v's bit is set and so is never reset.  For the
// dominator phase the extra edges are staged in LDS when they fit.
struct HbmStore {
    uint32_t* vis;     // visited bitset, (n + 31) / 32 words
    int32_t vis_words;
    bool vis_lds;      // vis is in LDS (cleared whole after a world)
    int32_t* lid_of;   // node -> local id, valid while the node's bit is set
    int32_t* nodes;
    int32_t* parent_;
    int32_t* idom_;
    int32_t* aux;
    int32_t* lvl;
    int32_t* xv;
    int32_t* xu_;
    int32_t* xv_s;     // LDS copies of the extra edges (xs_cap of them)
    int32_t* xu_s;
    int32_t xs_cap;
    bool staged;       // the extra edges are read from and written to the LDS copies
    int32_t lid_cap;   // nodes a world may reach in this slot
    int32_t cap_lv_;
    int64_t cap_x_;

    __device__ int cap_lv() const { return cap_lv_; }
    __device__ int64_t cap_x() const { return cap_x_; }
    __device__ bool fits(int) const { return true; }
    template <int NT>
    __device__ void init_seeds(const QueryDev& q) {
        for (int i = threadIdx.x; i < q.n_seeds; i += NT) {
            const int32_t v = q.seeds[i];
            atomicOr(&vis[(uint32_t)v >> 5], 1u << ((uint32_t)v & 31u));
            lid_of[v] = i;
            nodes[i] = v;
            parent_[i] = -1;
            idom_[i] = -1;
        }
    }
    __device__ int claim(int32_t v, int* counter) {
        const uint32_t bit = 1u << ((uint32_t)v & 31u);
        if (atomicOr(&vis[(uint32_t)v >> 5], bit) & bit) return -1;
        const int lid = atomicAdd(counter, 1);
        if (lid >= lid_cap) return -2;  // out of room: the world goes to the next tier
        lid_of[v] = lid;
        return lid;
    }
    __device__ int lookup(int32_t v) const {
        return ((vis[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u) ? lid_of[v] : -1;
    }
    __device__ int32_t node(int lid) const { return nodes[lid]; }
    __device__ void set_node(int lid, int32_t v) { nodes[lid] = v; }
    __device__ int get_parent(int lid) const { return parent_[lid]; }
    __device__ void set_parent(int lid, int p) { parent_[lid] = p; }
    __device__ int get_idom(int lid) const { return idom_[lid]; }
    __device__ void set_idom(int lid, int p) { idom_[lid] = p; }
    __device__ int32_t* aux_ptr(int lid) { return &aux[lid]; }
    __device__ int get_xu(int64_t x) const { return staged ? xu_s[x] : xu_[x]; }
    __device__ void set_xu(int64_t x, int u) { xu_[x] = u; }  // written while sampling (not staged)
    __device__ int get_xv(int64_t x) const { return staged ? xv_s[x] : xv[x]; }
    __device__ void set_xv(int64_t x, int v) {
        if (staged) xv_s[x] = v;
        else xv[x] = v;
    }
    __device__ void resolve_xv(int64_t x) { set_xv(x, lookup(get_xv(x))); }
    __device__ int delta_lid(int /*i*/, int32_t u) const { return lookup(u); }
    // Extra edges that are not staged in LDS are sorted by their head's BFS
    // level (a counting sort into the slot's second pair of arrays, the level
    // cursors in the unused staging area), so that a dominator sweep over a
    // level reads only that level's extra edges instead of all of them.  The
    // pairs then trade places: the sorted one is read from here on, and the
    // other takes the next world's extra edges.
    static constexpr bool kSortExtras = true;
    int32_t* xv2;
    int32_t* xu2;
    bool sorted;
    __device__ int32_t* level_cursors() { return xv_s; }  // 2 * xs_cap ints while not staged
    // the BFS rows, in the staging words (2 * xs_cap ints, not yet staged)
    template <int NT>
    __device__ BfsRows<NT>& bfs_rows() { return *reinterpret_cast<BfsRows<NT>*>(xv_s); }
    __device__ int sort_cap() const { return 2 * xs_cap; }
    // after every head's level was counted into level_cursors(): the cursors
    // become level starts, every edge goes to its level's range, and the
    // cursors end as level ends
    template <int NT>
    __device__ __forceinline__ void sort_by_level(int nx, int nlevels) {
        int32_t* cur = level_cursors();
        if (threadIdx.x == 0) {
            int run = 0;
            for (int L = 0; L <= nlevels; ++L) {
                const int c = cur[L];
                cur[L] = run;
                run += c;
            }
        }
        __syncthreads();
        for (int x = threadIdx.x; x < nx; x += NT) {
            const int v = xv[x];
            int lo = 0, hi = nlevels - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (lvl[mid] <= v) lo = mid; else hi = mid - 1;
            }
            const int at = atomicAdd(&cur[lo], 1);
            xv2[at] = v;
            xu2[at] = xu_[x];
        }
        __syncthreads();
        int32_t* const v2 = xv2;
        int32_t* const u2 = xu2;
        xv2 = xv;
        xu2 = xu_;
        xv = v2;
        xu_ = u2;
        sorted = true;
    }
    // the extra edges a sweep over level L reads
    __device__ __forceinline__ void level_range(int L, int nx, int& xa, int& xb) {
        if (sorted) {
            xa = L == 0 ? 0 : level_cursors()[L - 1];
            xb = level_cursors()[L];
        } else {
            xa = 0;
            xb = nx;
        }
    }
    // the extra edges into LDS when they fit (every thread takes the same
    // decision); the caller synchronises before they are read
    template <int NT>
    __device__ void stage(int nx) {
        staged = nx <= xs_cap;
        if (!staged) return;
        for (int x = threadIdx.x; x < nx; x += NT) {
            xv_s[x] = xv[x];
            xu_s[x] = xu_[x];
        }
    }
    // Worlds of this tier carry no labels for the incremental rounds.  The
    // coverage store still places them in dominator-tree preorder: the
    // preorder index in tin_, the placement cursors in parent_ (the BFS
    // parents are not needed once the dominators are known).
    static constexpr bool kLabels = false;
    int32_t* tin_;
    __device__ int32_t* cur_ptr(int lid) { return &parent_[lid]; }
    __device__ void set_tin(int lid, int v) { tin_[lid] = v; }
    __device__ int get_tin(int lid) const { return tin_[lid]; }
    // clear the bitset for the next world: whole when it is in LDS or the
    // world ran out of room (claimed nodes past lid_cap are not listed),
    // else the words of the world's reached nodes
    template <int NT>
    __device__ void reset(int count, bool whole) {
        if (vis_lds || whole) {
            for (int i = threadIdx.x; i < vis_words; i += NT) vis[i] = 0u;
        } else {
            for (int i = threadIdx.x; i < count; i += NT) vis[(uint32_t)nodes[i] >> 5] = 0u;
        }
        staged = false;
        sorted = false;
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

// A live edge from local id ulid to node v: v is claimed (a new node of the
// next level, with ulid as its BFS parent) or, when it is reached already,
// the edge is kept as an extra edge; out of room, the world overflows.
template <int NT, class Store>
__device__ __forceinline__ void claim_live(Store& st, WorldShared<NT>& sh, int32_t v, int ulid) {
    const int lid = st.claim(v, &sh.count);
    if (lid >= 0) {
        st.set_node(lid, v);
        st.set_parent(lid, ulid);
    } else if (lid == -1) {
        const int x = atomicAdd(&sh.n_extra, 1);
        if (x < st.cap_x()) {
            st.xv[x] = v;
            st.set_xu(x, ulid);
        } else {
            sh.overflow = 1;
        }
    } else {
        sh.overflow = 1;
    }
}

// Draw the coins of U slot groups whose columns (cv) and thresholds (tv) are
// loaded, and claim or record every live edge.  Exclusions (seeds, blocked
// nodes) are already in the per-query thresholds when q.excl_in_thr is set
// (an excluded head's slots have threshold 0, never live); otherwise the
// exclusion bits of the live heads are loaded and tested.  Phases keep the U
// groups' work side by side: the Philox blocks, then the exclusion bits,
// then the claims.
template <int NT, int U, class Store>
__device__ __forceinline__ void claim_slot_groups(const QueryDev& q, uint32_t w, const SlotGroup (&gr)[U],
                                                  const int4 (&cv)[U], const uint4 (&tv)[U], Store& st,
                                                  WorldShared<NT>& sh) {
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
            ex[u][qd] = (live && !q.excl_in_thr) ? q.excl[(uint32_t)vs[qd] >> 5] : 0u;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            if (!lv[u][qd]) continue;
            const int32_t v = vv[u][qd];
            if ((ex[u][qd] >> ((uint32_t)v & 31u)) & 1u) continue;  // seed or blocker
            claim_live<NT>(st, sh, v, gr[u].ulid);
        }
    }
}


// Slot groups of reached rows: columns from the graph, thresholds from the
// query's own copy.
template <int NT, int U, class Store>
__device__ __forceinline__ void scan_slot_groups(const GraphDev& g, const QueryDev& q, uint32_t w,
                                                 const SlotGroup (&gr)[U], Store& st, WorldShared<NT>& sh) {
    int4 cv[U];
    uint4 tv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const size_t b = gr[u].valid ? (size_t)gr[u].blk : 0;
        cv[u] = *reinterpret_cast<const int4*>(g.col + 4 * b);
        tv[u] = *reinterpret_cast<const uint4*>(q.thr + 4 * b);
    }
    claim_slot_groups<NT, U>(q, w, gr, cv, tv, st, sh);
}

constexpr int kGroupsPerLane = 2;

// Phase 1 of a world evaluation by sampling: the BFS with coins.  Returns
// false when the store ran out of room (uniform over the workgroup).
template <int NT, class Store>
__device__ bool bfs_sample(const GraphDev& g, const QueryDev& q, uint32_t w, const uint32_t* l0, Store& st,
                           WorldShared<NT>& sh) {
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

    // ---- level 0: the seeds' slot groups from the per-query table, which
    // carries each group's columns and thresholds (one round trip); when the
    // live slots were drawn ahead (l0), only those are read and claimed
    if (l0) {
        const int nwords = (q.n_seed_chunks + 7) >> 3;
        for (int wd = t; wd < nwords; wd += NT) {
            uint32_t m = l0[wd];
            while (m) {
                const int b = __ffs((int)m) - 1;
                m &= m - 1u;
                const int j = wd * 8 + (b >> 2);
                const int qd = b & 3;
                const int seed_lid = q.seed_chunk[j].y;
                const int4 cv = q.seed_col[j];
                const int32_t v = qd == 0 ? cv.x : qd == 1 ? cv.y : qd == 2 ? cv.z : cv.w;
                claim_live<NT>(st, sh, v, seed_lid);
            }
        }
    }
    for (int j0 = l0 ? q.n_seed_chunks : t; j0 < q.n_seed_chunks; j0 += NT * kGroupsPerLane) {
        SlotGroup gr[kGroupsPerLane];
        int4 cv[kGroupsPerLane];
        uint4 tv[kGroupsPerLane];
#pragma unroll
        for (int u = 0; u < kGroupsPerLane; ++u) {
            const int j = j0 + u * NT;
            if (j < q.n_seed_chunks) {
                const int4 d = q.seed_chunk[j];  // {blk, seed lid, e0, e1}
                cv[u] = q.seed_col[j];
                tv[u] = q.seed_thr[j];
                gr[u] = SlotGroup{(uint32_t)d.x, d.y, -1, d.z, d.w, true};
            } else {
                cv[u] = make_int4(0, 0, 0, 0);
                tv[u] = make_uint4(0u, 0u, 0u, 0u);
                gr[u] = SlotGroup{0u, 0, -1, 0, 0, false};
            }
        }
        claim_slot_groups<NT, kGroupsPerLane>(q, w, gr, cv, tv, st, sh);
    }
    __syncthreads();
    if (sh.overflow) return false;
    if (t == 0) st.lvl[2] = sh.count;
    __syncthreads();

    // ---- deeper levels
    BfsRows<NT>& rows = st.template bfs_rows<NT>();
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
            rows.lid[t] = i;
            rows.node[t] = u;
            rows.e0[t] = e0;
            rows.e1[t] = e1;
            rows.start[t] = start;
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
                            if (rows.start[mid] <= j) lo = mid; else hi = mid - 1;
                        }
                        gr[u] = SlotGroup{(uint32_t)(rows.e0[lo] >> 2) + (uint32_t)(j - rows.start[lo]),
                                          rows.lid[lo], rows.node[lo], rows.e0[lo], rows.e1[lo], true};
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

// Phase 2, shared by sampling and replay: immediate dominators under the
// super-source and the dominator-subtree size (the count) of every reached
// non-seed, left in aux.
template <int NT, class Store>
__device__ void world_counts(const QueryDev& q, RoundCtl* ctl, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const int nlevels = sh.nlevels;
    const int R = sh.count;
    const int nx = sh.n_extra;

    // ---- dominators
    st.template stage<NT>(nx);
    __syncthreads();
    for (int x = t; x < nx; x += NT) st.resolve_xv(x);
    for (int i = ns + t; i < R; i += NT) {
        const int p = st.get_parent(i);
        st.set_idom(i, p);
        *st.aux_ptr(i) = p;
    }
    // extra edges that stay in HBM are sorted by head level (uniform)
    bool sort = false;
    if constexpr (Store::kSortExtras) {
        sort = !st.staged && nx > 0 && nlevels + 1 <= st.sort_cap();
        if (sort)
            for (int i = t; i <= nlevels; i += NT) st.level_cursors()[i] = 0;
    }
    if (t == 0) {
        sh.nonfwd = 0;
        sh.xlevels = 0;
    }
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
        atomicOr(&sh.xlevels, lo < 63 ? (1ull << lo) : (1ull << 63));  // levels holding an extra edge's head
        if constexpr (Store::kSortExtras)
            if (sort) atomicAdd(&st.level_cursors()[lo], 1);
    }
    __syncthreads();
    if constexpr (Store::kSortExtras)
        if (sort) st.template sort_by_level<NT>(nx, nlevels);
    if (nx > 0 && !sh.nonfwd) {
        // Every extra edge goes exactly one level down: the idom of a level-L
        // node depends only on final idoms of shallower levels, so one sweep
        // over the levels holding extra heads suffices, kept in aux.
        const unsigned long long xl = sh.xlevels;
        for (int L = 1; L < nlevels; ++L) {
            if (L < 63 && !((xl >> L) & 1ull)) continue;  // uniform
            const int v0 = st.lvl[L], v1 = st.lvl[L + 1];
            int xa = 0, xb = nx;
            if constexpr (Store::kSortExtras) st.level_range(L, nx, xa, xb);
            for (int x = xa + t; x < xb; x += NT) {
                const int v = st.get_xv(x);
                if (v < v0 || v >= v1) continue;
                int a = st.get_parent(v);
                int b = st.get_xu(x);
                while (a != b) {
                    if (a > b) a = (a < ns) ? -1 : *st.aux_ptr(a);
                    else b = (b < ns) ? -1 : *st.aux_ptr(b);
                }
                atomicMin(st.aux_ptr(v), a);
            }
            __syncthreads();
        }
        for (int i = ns + t; i < R; i += NT) st.set_idom(i, *st.aux_ptr(i));
        __syncthreads();
    } else if (nx > 0) {
        // Every sweep that changes something lowers some idom id, so the
        // sweeps end; the cap only guards a broken invariant.
        for (int pass = 0;; ++pass) {
            if (pass >= kMaxDomPasses) {
                if (t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagDomPasses);
                break;
            }
            if (t == 0) sh.changed = 0;
            __syncthreads();
            const unsigned long long xl = sh.xlevels;
            for (int L = 1; L < nlevels; ++L) {
                // a level without extra heads keeps idom = BFS parent
                if (L < 63 && !((xl >> L) & 1ull)) continue;  // uniform
                const int v0 = st.lvl[L], v1 = st.lvl[L + 1];
                int xa = 0, xb = nx;
                if constexpr (Store::kSortExtras) st.level_range(L, nx, xa, xb);
                for (int x = xa + t; x < xb; x += NT) {
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
                for (int x = xa + t; x < xb; x += NT) {
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
            const bool again = sh.changed;
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
}

// Dominator-tree labels: each non-seed gets a preorder index such that its
// subtree is the index range [index, index + count).  Nodes are placed level
// by level (an idom lies on every path, so on a shallower level): a node
// takes the next range of its idom's cursor (or of the roots' cursor when
// its idom is a seed or the super-source).  Sibling order is arbitrary.
template <int NT, class Store>
__device__ void world_labels(const QueryDev& q, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const int nlevels = sh.nlevels;
    if (t == 0) sh.root_cur = 0;
    __syncthreads();
    for (int L = 1; L < nlevels; ++L) {
        for (int v = st.lvl[L] + t; v < st.lvl[L + 1]; v += NT) {
            const int p = st.get_idom(v);
            const int size = *st.aux_ptr(v);
            const int at = (p < ns) ? atomicAdd(&sh.root_cur, size) : atomicAdd(st.cur_ptr(p), size);
            st.set_tin(v, at);
            *st.cur_ptr(v) = at + 1;
        }
        __syncthreads();
    }
}

// Exit bits of the labels.  For each non-seed v, [lo(v), hi(v)] spans the
// preorder indexes of the heads of the live edges that leave v's subtree's
// nodes; some edge leads out of the subtree when that span is not inside
// [tin(v), tin(v) + count(v)).  An edge whose head dominates its source is
// left out: a simple path reaches its source through its head already, so
// it never carries a path out of any subtree it leaves.  Each edge widens
// its source's span; spans are then merged into each idom, deepest level
// first (an idom lies on a shallower level).
template <int NT, class Store>
__device__ void exits_init(int ns, int R, Store& st) {
    for (int i = ns + (int)threadIdx.x; i < R; i += NT) {
        *st.lo_ptr(i) = 0x7FFFFFFF;
        *st.hi_ptr(i) = -1;
    }
}

// live edge a -> b between reached nodes (local ids)
template <class Store>
__device__ __forceinline__ void exits_edge(int ns, Store& st, int a, int b) {
    if (a < ns || b < ns) return;  // seeds lie in no non-seed's subtree
    const int ta = st.get_tin(a), tb = st.get_tin(b);
    if (tb <= ta && ta < tb + *st.aux_ptr(b)) return;  // b dominates a
    atomicMin(st.lo_ptr(a), tb);
    atomicMax(st.hi_ptr(a), tb);
}

template <int NT, class Store>
__device__ void exits_merge(int ns, Store& st, WorldShared<NT>& sh) {
    for (int L = sh.nlevels - 1; L >= 1; --L) {
        for (int i = st.lvl[L] + (int)threadIdx.x; i < st.lvl[L + 1]; i += NT) {
            const int p = st.get_idom(i);
            if (p >= ns) {
                atomicMin(st.lo_ptr(p), *st.lo_ptr(i));
                atomicMax(st.hi_ptr(p), *st.hi_ptr(i));
            }
        }
        __syncthreads();
    }
}

// whether some live edge leads out of lid's subtree (after exits_merge)
template <class Store>
__device__ __forceinline__ bool exits_of(Store& st, int lid, int count) {
    const int tv = st.get_tin(lid);
    return *st.lo_ptr(lid) < tv || *st.hi_ptr(lid) >= tv + count;
}

// The exits of a sampled world: its edges are the BFS tree edges and the
// extra edges.  A world without extra edges is a forest and has none (the
// caller skips it).
template <int NT, class Store>
__device__ void world_exits(const QueryDev& q, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const int R = sh.count;
    const int nx = sh.n_extra;
    exits_init<NT>(ns, R, st);
    __syncthreads();
    for (int i = ns + t; i < R; i += NT) exits_edge(ns, st, st.get_parent(i), i);
    for (int x = t; x < nx; x += NT) exits_edge(ns, st, st.get_xu(x), st.get_xv(x));
    __syncthreads();
    exits_merge<NT>(ns, st, sh);
}

// Coverage of a marked set in one world (Section 4.1): a non-seed's CP set
// is its chain of non-seed dominators up to and including itself, so it
// meets the marked set when the node is marked or its immediate dominator's
// set does.  Levels are walked shallowest first (a dominator lies on a
// shallower level); the flags replace the subtree sizes in aux, and their
// sum goes to sh.covered.
template <int NT, class Store>
__device__ void world_cover_marks(const QueryDev& q, const TileOut& out, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    for (int L = 1; L < sh.nlevels; ++L) {
        for (int v = st.lvl[L] + t; v < st.lvl[L + 1]; v += NT) {
            const uint32_t u = (uint32_t)st.node(v);
            const int p = st.get_idom(v);
            const bool m = ((out.mark[u >> 5] >> (u & 31u)) & 1u) != 0u;
            *st.aux_ptr(v) = (m || (p >= ns && *st.aux_ptr(p) != 0)) ? 1 : 0;
        }
        __syncthreads();
    }
    long long c = 0;
    for (int i = ns + t; i < sh.count; i += NT) c += *st.aux_ptr(i);
    c = block_sum_ll<NT>(c, sh.sum_tmp);
    if (t == 0) sh.covered = (int)c;
}

// Phase 3 of a sampled world: the outputs of the mode.
template <int NT, int TIER, class Store>
__device__ void world_outputs(const QueryDev& q, RoundCtl* ctl, uint32_t w, uint32_t wi, const TileOut& out,
                              Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const int R = sh.count;
    const int nx = sh.n_extra;
    const int len = (out.cover == kCoverCount || out.sizes_only) ? 0 : R - ns;  // entries written
    int read_len = 0;  // stored entries read back (incremental rounds)
    if (out.mode == kModeDelta) {
        // The stored list keeps the round-0 order; an entry whose count is 0
        // is a node no longer reached.  Blocking only removes nodes, so every
        // node reached now has a live entry: walking the live entries finds
        // every count that changed; each is updated in place and its change
        // added to gain.
        const size_t so = (size_t)out.store_off[w];
        int list_len = out.store_len[w];
        if (so + (size_t)list_len > out.store_cap) {
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
            if (lane == 0 && mask) atomicAdd(&sh.ndelta, __popcll(mask));
            if (d != 0 && u != ctl->ustar) atomicAdd((unsigned long long*)&out.gain[u], (unsigned long long)(long long)d);
        }
        __syncthreads();
        if (t == 0 && out.world_flags) out.world_flags[w] = 0;  // no labels from this evaluation
    } else {
        if (t == 0) {
            sh.pair_base = (TIER == 0) ? (unsigned long long)wi * out.slot_cap0
                                       : out.big_base + atomicAdd(&ctl->big_count, (unsigned long long)len);
        }
        __syncthreads();
        const unsigned long long off = sh.pair_base;
        if (off + (unsigned long long)len <= out.scr_cap && out.cover == kCoverStore) {
            // dominator-tree preorder: a subtree is a run of entries
            for (int i = t; i < len; i += NT) {
                const int lid = ns + i;
                const int at = st.get_tin(lid);
                const int p = st.get_idom(lid);
                const int c = *st.aux_ptr(lid);
                out.scr_node[off + at] = st.node(lid);
                out.scr_cnt[off + at] = c;
                out.scr_par[off + at] = (p >= ns) ? st.get_tin(p) : -1;
                out.scr_lab[off + at] = (uint32_t)c;
            }
            if (t == 0) {
                out.wloc[wi] = (int64_t)off;
                out.wlen[wi] = len;
            }
        } else if (off + (unsigned long long)len <= out.scr_cap) {
            for (int i = t; i < len; i += NT) {
                out.scr_node[off + i] = st.node(ns + i);
                out.scr_cnt[off + i] = out.unit_counts ? 1 : *st.aux_ptr(ns + i);
                if (out.keep_edges) {
                    out.scr_par[off + i] = st.get_parent(ns + i);
                    // A world without labels stores every entry with its exit
                    // bit set, so the label rule never takes one of its
                    // entries: the round-update launch's replay may label the
                    // world while a rule workgroup still reads the entry of
                    // the same blocker, whose label the replay leaves as it
                    // was (the blocker is no longer reached); with the exit
                    // bit set both roles agree that the rule does not hold.
                    uint32_t lab = kLabelExit;
                    if constexpr (Store::kLabels) {
                        const int c = *st.aux_ptr(ns + i);
                        lab = pack_label(st.get_tin(ns + i), c, nx > 0 && exits_of(st, ns + i, c));
                    }
                    out.scr_lab[off + i] = lab;
                }
            }
            if (t == 0) {
                out.wloc[wi] = (int64_t)off;
                out.wlen[wi] = len;
            }
        } else if (t == 0) {
            atomicOr(&ctl->flags, (uint32_t)kFlagPairOverflow);  // bump region full: the tile is redone
        }
        if (out.keep_edges) {
            // the labels serve the incremental rounds directly
            if (t == 0 && out.world_flags) out.world_flags[w] = Store::kLabels ? (uint8_t)kWorldLabelled : 0;
            // worlds beyond the replay's limits need the sampling tiers later
            if (t == 0 && (len > kReplayCap || nx > kReplayXCap || len + nx > kReplayEdgeCap || ns + len > 32767))
                atomicOr(&ctl->replay_big, 1u);
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
        if (out.world_size) out.world_size[wi] = (out.cover == kCoverCount) ? sh.covered : R;
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
        // live edges between non-excluded nodes: one BFS-tree edge per
        // reached non-seed plus the extra edges
        sh.acc_reached += (unsigned long long)R;
        sh.acc_live += (unsigned long long)(R - ns + nx);
    }
}

// A world evaluated by sampling: false when the store ran out of room.
template <int NT, int TIER, class Store>
__device__ bool evaluate_world(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w, uint32_t wi,
                               const TileOut& out, Store& st, WorldShared<NT>& sh) {
    const uint32_t* l0 = out.l0_bits ? out.l0_bits + (size_t)wi * (size_t)out.l0_words : nullptr;
    if (!bfs_sample<NT>(g, q, w, l0, st, sh)) return false;
    // reach counts and world sizes need no dominators (uniform)
    if (!out.sizes_only && !out.unit_counts) world_counts<NT>(q, ctl, st, sh);
    if (out.cover == kCoverStore) {  // uniform
        world_labels<NT>(q, st, sh);
    } else if (out.cover == kCoverCount) {
        world_cover_marks<NT>(q, out, st, sh);
    } else {
        if constexpr (Store::kLabels) {
            if (out.keep_edges && out.mode != kModeDelta) {  // uniform
                world_labels<NT>(q, st, sh);
                if (sh.n_extra > 0) world_exits<NT>(q, st, sh);
            }
        }
    }
    world_outputs<NT, TIER>(q, ctl, w, wi, out, st, sh);
    return true;
}

// The query as a world kernel runs it: the level-0 table's length and the
// seeds' id and edge sums come from the device counters that the set-up
// kernels wrote (a caller that enqueues a whole solve never reads them).
__device__ __forceinline__ QueryDev query_at_run(QueryDev q, const RoundCtl* ctl) {
    q.n_seed_chunks = min(ctl->seed_chunks, q.seed_cap);
    q.seed_sum = ctl->seed_sum;
    q.seed_edges = ctl->seed_edges;
    return q;
}

// ------------------------------------------------------------- kernels
// Tier 0 (one wave, small LDS store) and tier 1 (four waves, larger LDS
// store).  With range_count > 0 the kernel takes worlds 0..range_count-1 of
// the tile; otherwise it takes the list handed down by the previous tier.
// (32 extra live edges: the large trivalency workload's worlds keep 0.2 on
// average, and a world with more goes to tier 1)
using Tier0Store = LdsStore<256, 9, 32, 30>;
// tier 1 keeps a level slot for every node it can hold: a world that fitted it
// in a from-scratch pass fits it again after any blockers are added
using Tier1Store = LdsStore<2048, 12, 1024, 2050>;
constexpr int kTier0NT = 64;
// Tier 0 waits on dependent global loads level after level, so resident
// waves matter most: 6 per SIMD needs at most 80 VGPRs (the compiler keeps
// a few values in scratch) and at most 1/24 of the LDS per wave.
constexpr int kTier0WavesPerSimd = 6;
constexpr uint32_t kSchedChunk = 4;  // worlds per update of a tier's work counter
constexpr int kTier1NT = 256;
constexpr int kTier2NT = 256;

// Per-workgroup work tallies, one slot per (tier, field, workgroup): no
// shared counter is touched.  Fields: worlds, edges, bytes, reached nodes,
// live edges (the last two only for sampled worlds).
__device__ __forceinline__ void add_work_at(const TileOut& out, int tier, uint32_t slot, unsigned long long worlds,
                                            unsigned long long edges, unsigned long long bytes,
                                            unsigned long long reached = 0, unsigned long long live = 0) {
    if (!out.work || !worlds) return;
    const size_t st = (size_t)out.work_stride;
    unsigned long long* wk = out.work + (size_t)tier * kWorkFields * st + slot;
    wk[0] += worlds;
    wk[st] += edges;
    wk[2 * st] += bytes;
    wk[3 * st] += reached;
    wk[4 * st] += live;
}
__device__ __forceinline__ void add_work(const TileOut& out, int tier, unsigned long long worlds,
                                         unsigned long long edges, unsigned long long bytes,
                                         unsigned long long reached, unsigned long long live) {
    add_work_at(out, tier, blockIdx.x, worlds, edges, bytes, reached, live);
}

// Worlds are dealt to workgroups by a fixed stride (no shared work counter).
template <int NT, class Store, int TIER>
__global__ __launch_bounds__(NT, (NT == kTier0NT ? kTier0WavesPerSimd : 1))
void k_world_lds(GraphDev g, QueryDev q_in, RoundCtl* ctl, uint32_t w_begin, uint32_t range_count,
                 const int32_t* in_list, int count_idx, int32_t* next_list, TileOut out) {
    __shared__ Store st;
    __shared__ WorldShared<NT> sh;
    const int t = threadIdx.x;
    if (ctl->stop) return;
    const QueryDev q = query_at_run(q_in, ctl);
    const uint32_t n_items = in_list ? min(ctl->list_n[count_idx], count_idx ? out.next_cap : out.list_cap)
                                     : range_count;
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    st.template clear<NT>();
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_reached = sh.acc_live = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    // World costs vary widely, so after its first world (its block id) a
    // workgroup takes chunks of worlds from a counter: the workgroups finish
    // together, and the counter sees one update per chunk.  Chunks hold up to
    // kSchedChunk worlds, fewer when the worlds left after the first ones
    // would not give every workgroup several chunks.
    const uint32_t rest = n_items > gridDim.x ? n_items - gridDim.x : 0u;
    const uint32_t chunk = max(1u, min(kSchedChunk, rest / (gridDim.x * 4u)));
    uint32_t k = blockIdx.x, kend = blockIdx.x + 1;
    while (k < n_items) {
        const uint32_t wi = in_list ? (uint32_t)in_list[k] : k;
        const bool ok = evaluate_world<NT, TIER>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) {
            const uint32_t pos = atomicAdd(&ctl->list_n[TIER + 1], 1u);
            if (pos < out.next_cap) next_list[pos] = (int32_t)wi;
            else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        }
        st.template reset<NT>(0);
        if (++k == kend) {
            if (t == 0) sh.sched = gridDim.x + atomicAdd(&ctl->next[TIER], chunk);
            __syncthreads();
            k = sh.sched;
            kend = k + chunk;
        }
        __syncthreads();
    }
    if (t == 0) {
        add_work(out, TIER, sh.acc_worlds, sh.acc_edges, sh.acc_bytes, sh.acc_reached, sh.acc_live);
        // incremental rounds keep T up to date: the nodes lost, per workgroup
        if (sh.acc_dsize) out.dsz[out.dsz_off[TIER] + blockIdx.x] = sh.acc_dsize;
    }
}

// Tier 0 over the worlds of several queries (a batch of from-scratch
// passes).  A workgroup finds the query of its packed world by a binary
// search over the queries' first worlds, once per change of query (chunks
// are dealt in ascending order, so consecutive worlds mostly share one), and
// then evaluates the world exactly as that query's own tier-0 launch would;
// a world the tier cannot hold goes to that query's tier-1 list.  The
// workgroup is one wave, so the world index is made uniform and the query's
// fields are read with scalar loads.
template <int NT, class Store>
__global__ __launch_bounds__(NT, kTier0WavesPerSimd)
void k_world_lds_packed(GraphDev g, const PackedQuery* __restrict__ pq, int nq, uint32_t n_items,
                        uint32_t* counter) {
    static_assert(NT == 64, "the packed tier is one wave per workgroup");
    __shared__ Store st;
    __shared__ WorldShared<NT> sh;
    const int t = threadIdx.x;
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    st.template clear<NT>();
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_reached = sh.acc_live = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    const uint32_t rest = n_items > gridDim.x ? n_items - gridDim.x : 0u;
    const uint32_t chunk = max(1u, min(kSchedChunk, rest / (gridDim.x * 4u)));
    uint32_t k = blockIdx.x, kend = blockIdx.x + 1;
    uint32_t lo = 1, hi = 0;  // the current query's packed range (none yet)
    const PackedQuery* cur = pq;
    QueryDev q{};
    bool stopped = false;
    while (k < n_items) {
        if (k < lo || k >= hi) {
            int a = 0, b = nq - 1;
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (pq[mid].first <= k) a = mid;
                else b = mid - 1;
            }
            cur = pq + __builtin_amdgcn_readfirstlane(a);
            lo = cur->first;
            hi = cur->first + cur->count;
            q = query_at_run(cur->q, cur->ctl);
            stopped = cur->ctl->stop != 0;
        }
        const uint32_t wi = k - lo;
        if (!stopped) {
            RoundCtl* ctl = cur->ctl;
            const bool ok = evaluate_world<NT, 0>(g, q, ctl, cur->w_begin + wi, wi, cur->out, st, sh);
            if (!ok && t == 0) {
                const uint32_t pos = atomicAdd(&ctl->list_n[1], 1u);
                if (pos < cur->out.next_cap) cur->list1[pos] = (int32_t)wi;
                else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            }
            st.template reset<NT>(0);
        }
        if (++k == kend) {
            if (t == 0) sh.sched = gridDim.x + atomicAdd(counter, chunk);
            __syncthreads();
            k = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh.sched);
            kend = k + chunk;
        }
        __syncthreads();
    }
}

// Tier 1 over the tier-1 lists of several queries (those of a packed tier-0
// launch).  The lists' lengths are read on the device; the items of the
// lists in query order are dealt round-robin to the workgroups (item x to
// workgroup x mod grid), so no counter is shared.  Each world is evaluated
// as its query's own tier-1 launch would evaluate it, and one the tier
// cannot hold goes to that query's tier-2 list.
template <int NT, class Store>
__global__ __launch_bounds__(NT) void k_world_lds_packed_list(GraphDev g, const PackedQuery* __restrict__ pq,
                                                              int nq) {
    __shared__ Store st;
    __shared__ WorldShared<NT> sh;
    const int t = threadIdx.x;
    st.template clear<NT>();
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_reached = sh.acc_live = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    const uint32_t grid = gridDim.x;
    uint64_t base = 0;  // items of the queries before this one
    for (int j = 0; j < nq; ++j) {
        const PackedQuery* cur = pq + j;
        RoundCtl* ctl = cur->ctl;
        const uint32_t n_items = min(ctl->list_n[1], cur->out.next_cap);
        if (n_items == 0 || ctl->stop) continue;  // uniform
        const QueryDev q = query_at_run(cur->q, ctl);
        // this workgroup's first item of the query: the first i with
        // (base + i) mod grid == blockIdx.x
        const uint32_t first = (uint32_t)((blockIdx.x + grid - (uint32_t)(base % grid)) % grid);
        for (uint32_t k = first; k < n_items; k += grid) {
            const uint32_t wi = (uint32_t)cur->list1[k];
            const bool ok = evaluate_world<NT, 1>(g, q, ctl, cur->w_begin + wi, wi, cur->out, st, sh);
            if (!ok && t == 0) {
                const uint32_t pos = atomicAdd(&ctl->list_n[2], 1u);
                if (pos < cur->out.next_cap) cur->list2[pos] = (int32_t)wi;
                else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            }
            st.template reset<NT>(0);
            __syncthreads();
        }
        base += n_items;
    }
}

// Level 0 of a tile's worlds, drawn ahead of the world kernels.  A lane
// holds one level-0 slot group (its table entry read once) and draws its
// coins for kL0Worlds consecutive worlds, so the draws wait on no load; the
// nibbles of eight neighbouring lanes make one word of a world's bits.  The
// world kernels then read and claim only the live slots.
constexpr int kL0NT = 256;
constexpr int kL0Worlds = 32;
__global__ __launch_bounds__(kL0NT) void k_level0_bits(QueryDev q_in, const RoundCtl* ctl, uint32_t w_begin,
                                                       uint32_t count, uint32_t* bits, int words) {
    if (ctl->stop) return;
    const QueryDev q = query_at_run(q_in, ctl);
    const int j = (int)(blockIdx.y * kL0NT + threadIdx.x);  // slot group
    const int wd = j >> 3;                                   // its word
    const uint32_t wi0 = blockIdx.x * (uint32_t)kL0Worlds;
    uint32_t valid = 0u;  // slots of the group inside its seed's row
    int4 d = make_int4(0, 0, 0, 0);
    uint4 th = make_uint4(0u, 0u, 0u, 0u);
    if (j < q.n_seed_chunks) {
        d = q.seed_chunk[j];  // {blk, seed lid, e0, e1}
        th = q.seed_thr[j];
#pragma unroll
        for (int qd = 0; qd < 4; ++qd) {
            const int e = 4 * d.x + qd;
            if (e >= d.z && e < d.w) valid |= 1u << qd;
        }
    }
    const uint32_t ts[4] = {th.x, th.y, th.z, th.w};
    for (int r = 0; r < kL0Worlds; ++r) {
        const uint32_t wi = wi0 + (uint32_t)r;
        if (wi >= count) break;  // uniform over the workgroup
        uint32_t nib = 0u;
        if (valid) {
            const uint4 c = philox_block((uint32_t)d.x, w_begin + wi, q.key0, q.key1);
            const uint32_t cs[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
            for (int qd = 0; qd < 4; ++qd)
                if (((valid >> qd) & 1u) && (ts[qd] == kAlwaysLive || cs[qd] < ts[qd])) nib |= 1u << qd;
        }
        uint32_t word = nib << (4 * (threadIdx.x & 7));
        word |= __shfl_xor(word, 1);
        word |= __shfl_xor(word, 2);
        word |= __shfl_xor(word, 4);
        if ((threadIdx.x & 7) == 0 && wd < words) bits[(size_t)wi * (size_t)words + (size_t)wd] = word;
    }
}

hipError_t launch_level0_bits(const QueryDev& q, const RoundCtl* ctl, uint32_t w_begin, uint32_t count,
                              uint32_t* bits, int words, int32_t chunk_cap, hipStream_t s, const LaunchEvents& ev) {
    const int gy = (chunk_cap + kL0NT - 1) / kL0NT;
    if (count == 0 || chunk_cap < 1 || words < (chunk_cap + 7) / 8 || gy > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((count + kL0Worlds - 1) / kL0Worlds), (unsigned)gy);
    if (ev.start)
        hipExtLaunchKernelGGL(k_level0_bits, grid, dim3(kL0NT), 0, s, ev.start, ev.stop, 0, q, ctl, w_begin, count,
                              bits, words);
    else
        k_level0_bits<<<grid, kL0NT, 0, s>>>(q, ctl, w_begin, count, bits, words);
    return hipGetLastError();
}

// The packed kernel's store: tier 0's, as a type of its own, so that the
// packed kernel gets its own instances of the world functions and the
// single-query tier-0 kernel is compiled as if it were their only caller
// (sharing them changes the inliner's choices and costs that kernel two
// registers, one occupancy step).
struct PackedTier0Store : Tier0Store {};
struct PackedTier1Store : Tier1Store {};

hipError_t launch_world_tier0_packed(const GraphDev& g, const PackedQuery* pq, int nq, uint32_t n_items,
                                     uint32_t* counter, int grid, hipStream_t s) {
    if (nq < 1 || grid < 1) return hipErrorInvalidValue;
    k_world_lds_packed<kTier0NT, PackedTier0Store><<<(unsigned)grid, kTier0NT, 0, s>>>(g, pq, nq, n_items, counter);
    return hipGetLastError();
}

hipError_t launch_world_tier1_packed(const GraphDev& g, const PackedQuery* pq, int nq, int grid, hipStream_t s) {
    if (nq < 1 || grid < 1) return hipErrorInvalidValue;
    k_world_lds_packed_list<kTier1NT, PackedTier1Store><<<(unsigned)grid, kTier1NT, 0, s>>>(g, pq, nq);
    return hipGetLastError();
}

// Tiers 2 and 3: per-world arrays in HBM, one slot per resident workgroup;
// the visited bitset in LDS (VIS_LDS) or in the slot, and up to kStageX
// extra edges staged in LDS, both in dynamic LDS.  Tier 2's slots hold
// worlds of up to lid_cap nodes and xcap extra edges and hand larger ones
// on to tier 3, whose few slots are sized for any world of the graph.
constexpr int kStageX = 2048;
static_assert(2 * kStageX * sizeof(int32_t) >= sizeof(BfsRows<kTier2NT>), "the BFS rows fit the staging words");
constexpr int kVisLdsMaxWords = 4096;  // graphs of up to 2^17 nodes keep their bitset in LDS

template <bool VIS_LDS, int TIER>
__global__ __launch_bounds__(kTier2NT) void k_world_hbm(GraphDev g, QueryDev q_in, RoundCtl* ctl, uint32_t w_begin,
                                                        uint32_t range_count, const int32_t* in_list,
                                                        int count_idx, int32_t* next_list, TileOut out,
                                                        BigSlots bs) {
    __shared__ WorldShared<kTier2NT> sh;
    extern __shared__ int32_t t2_lds[];  // [2 * kStageX] staged edges, then the bitset (VIS_LDS)
    const int t = threadIdx.x;
    const size_t slot = blockIdx.x;
    const size_t n = (size_t)g.n;
    const size_t lc = (size_t)bs.lid_cap;
    HbmStore st;
    st.vis_words = bs.vis_words;
    st.vis_lds = VIS_LDS;
    st.vis = VIS_LDS ? reinterpret_cast<uint32_t*>(t2_lds + 2 * kStageX) : bs.vis + slot * (size_t)bs.vis_words;
    st.lid_of = bs.lid_of + slot * n;
    st.nodes = bs.nodes + slot * lc;
    st.parent_ = bs.parent + slot * lc;
    st.idom_ = bs.idom + slot * lc;
    st.aux = bs.aux + slot * lc;
    st.tin_ = bs.tin ? bs.tin + slot * lc : nullptr;  // only the coverage store uses it
    st.lvl = bs.lvl + slot * (lc + 3);
    st.xv = bs.xv + slot * (size_t)bs.xcap;
    st.xu_ = bs.xu + slot * (size_t)bs.xcap;
    st.xv2 = bs.xv2 + slot * (size_t)bs.xcap;
    st.xu2 = bs.xu2 + slot * (size_t)bs.xcap;
    st.sorted = false;
    st.xv_s = t2_lds;
    st.xu_s = t2_lds + kStageX;
    st.xs_cap = kStageX;
    st.staged = false;
    st.lid_cap = bs.lid_cap;
    st.cap_lv_ = bs.lid_cap + 1;
    st.cap_x_ = bs.xcap;
    if (ctl->stop) return;
    const QueryDev q = query_at_run(q_in, ctl);
    const uint32_t n_items = in_list ? min(ctl->list_n[count_idx], count_idx ? out.next_cap : out.list_cap)
                                     : range_count;
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    if (VIS_LDS)
        for (int i = t; i < bs.vis_words; i += kTier2NT) st.vis[i] = 0u;
    if (t == 0) {
        sh.acc_worlds = sh.acc_edges = sh.acc_bytes = 0;
        sh.acc_reached = sh.acc_live = 0;
        sh.acc_dsize = 0;
    }
    __syncthreads();
    for (uint32_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        const uint32_t wi = in_list ? (uint32_t)in_list[k] : k;
        const bool ok = evaluate_world<kTier2NT, 2>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) {
            if (TIER == 2) {
                const uint32_t pos = atomicAdd(&ctl->list_n[4], 1u);
                if (pos < out.next_cap) next_list[pos] = (int32_t)wi;
                else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            } else {
                atomicOr(&ctl->flags, (uint32_t)kFlagBigCapacity);
            }
        }
        __syncthreads();
        st.reset<kTier2NT>(min(sh.count, bs.lid_cap), !ok);
        __syncthreads();
    }
    if (t == 0) {
        add_work(out, 2, sh.acc_worlds, sh.acc_edges, sh.acc_bytes, sh.acc_reached, sh.acc_live);
        if (sh.acc_dsize) out.dsz[out.dsz_off[TIER == 2 ? 2 : 6] + blockIdx.x] = sh.acc_dsize;
    }
}

// ------------------------------------------------------------ compaction
// Items are the tile's worlds [0, count) (entries at wloc/wlen in scratch).
// Each workgroup scans its items' lengths, takes one range of the
// destination with one counter update, and copies with one wave per item.
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
    const uint32_t n_items = sp.count;
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
            w = sp.w_begin + i;
            src = sp.loc[i];
            len = sp.len[i];
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

// Launch kernel k on grid x block threads with `lds` bytes of dynamic LDS,
// with the kernel's own start and stop timestamps in ev when given.
template <class... P, class... A>
hipError_t launch_k_lds(void (*k)(P...), unsigned grid, unsigned block, size_t lds, hipStream_t s,
                        const LaunchEvents& ev, A... a) {
    if (ev.start)
        hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), lds, s, ev.start, ev.stop, 0, a...);
    else
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, s, a...);
    return hipGetLastError();
}

// Launch kernel k on grid x block threads, with the kernel's own start and
// stop timestamps in ev when given.
template <class... P, class... A>
hipError_t launch_k(void (*k)(P...), unsigned grid, unsigned block, hipStream_t s, const LaunchEvents& ev, A... a) {
    if (ev.start)
        hipExtLaunchKernelGGL(k, dim3(grid), dim3(block), 0, s, ev.start, ev.stop, 0, a...);
    else
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), 0, s, a...);
    return hipGetLastError();
}

hipError_t launch_world_tier(int tier, const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin,
                             uint32_t range_count, const int32_t* in_list, int count_idx, int32_t* next_list,
                             const TileOut& out, const BigSlots& bs, int grid, hipStream_t s,
                             const LaunchEvents& ev) {
    if (tier == 0)
        return launch_k(k_world_lds<kTier0NT, Tier0Store, 0>, (unsigned)grid, kTier0NT, s, ev, g, q, ctl, w_begin,
                        range_count, in_list, count_idx, next_list, out);
    if (tier == 1)
        return launch_k(k_world_lds<kTier1NT, Tier1Store, 1>, (unsigned)grid, kTier1NT, s, ev, g, q, ctl, w_begin,
                        range_count, in_list, count_idx, next_list, out);
    const bool vis_lds = bs.vis_words <= kVisLdsMaxWords;
    const size_t lds = (size_t)2 * kStageX * sizeof(int32_t) + (vis_lds ? (size_t)bs.vis_words * sizeof(uint32_t) : 0);
    if (tier == 2) {
        if (vis_lds)
            return launch_k_lds(k_world_hbm<true, 2>, (unsigned)bs.n_slots, kTier2NT, lds, s, ev, g, q, ctl, w_begin,
                                range_count, in_list, count_idx, next_list, out, bs);
        return launch_k_lds(k_world_hbm<false, 2>, (unsigned)bs.n_slots, kTier2NT, lds, s, ev, g, q, ctl, w_begin,
                            range_count, in_list, count_idx, next_list, out, bs);
    }
    if (vis_lds)
        return launch_k_lds(k_world_hbm<true, 3>, (unsigned)bs.n_slots, kTier2NT, lds, s, ev, g, q, ctl, w_begin,
                            range_count, in_list, count_idx, next_list, out, bs);
    return launch_k_lds(k_world_hbm<false, 3>, (unsigned)bs.n_slots, kTier2NT, lds, s, ev, g, q, ctl, w_begin,
                        range_count, in_list, count_idx, next_list, out, bs);
}

// ----------------------------------------------- incremental-round index
// After round 0 every stored entry (world w, position p, node u) is indexed
// by u.  The worlds a new blocker u changes are those whose entry for u is
// still live (count > 0): every other world keeps its reached set and its
// dominator tree.

// Building the index regroups world-major entries by node.  Nodes are cut
// into buckets of 2^shift consecutive ids.  A histogram pass counts the
// entries of each bucket, one workgroup turns the counts into bucket bases,
// and a partition pass copies every entry, as a record (position, world,
// node, count), into its bucket's range of a record array: each workgroup
// reserves its share of a bucket with one counter update.  Then one
// workgroup owns each bucket: it counts its nodes' entries (and sums their
// counts into the gains) in LDS, scans the counts into the nodes' offsets,
// and places the entries inside the bucket's range of the index, which is
// the same range as in the record array.  A node's counters live in the
// LDS of the one workgroup that owns it, so no per-node global counter is
// ever updated and every index write lands in that workgroup's own range.
constexpr int kIdxNT = 512;
constexpr int kIdxMaxBuckets = 8192;
constexpr uint32_t kIdxWorldsPerWG = 256;
constexpr int kOwnNT = 1024;
constexpr int kOwnSlots = 2048;  // nodes counted per pass over a bucket

// The first 256 entries of a world (four per lane) from position so.
template <bool CNT>
__device__ __forceinline__ void load_world_head(const TileOut& out, long long so, int len, int lane, int32_t (&u)[4],
                                                int32_t (&c)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int i = lane + 64 * j;
        u[j] = i < len ? out.store_node[so + i] : 0;
        c[j] = (CNT && i < len) ? out.store_cnt[so + i] : 0;
    }
}

// Calls f(node, count, position, world) for every stored entry of the
// worlds w0 + wave, w0 + wave + waves, ... below w1 taken by this wave.
// The next world's first 256 entries, and the range of the world after
// that, are loaded before f runs on the current world: a wave then waits
// for memory about once per world, and stores made by f (which the same
// in-order counter tracks) are not waited for by the next world's loads.
template <int NT, bool CNT, typename F>
__device__ __forceinline__ void for_stored_entries(const TileOut& out, uint32_t w0, uint32_t w1, F&& f) {
    constexpr uint32_t kStep = NT / 64;
    const int lane = threadIdx.x & 63;
    uint32_t w = w0 + (threadIdx.x >> 6);
    if (w >= w1) return;
    long long so = out.store_off[w];
    int len = out.store_len[w];
    int32_t u[4], c[4];
    load_world_head<CNT>(out, so, len, lane, u, c);
    long long so_n = 0;
    int len_n = 0;
    if (w + kStep < w1) {
        so_n = out.store_off[w + kStep];
        len_n = out.store_len[w + kStep];
    }
    while (true) {
        const uint32_t wn = w + kStep;
        int32_t un[4], cn[4];
        load_world_head<CNT>(out, so_n, len_n, lane, un, cn);
        long long so_nn = 0;
        int len_nn = 0;
        if (wn + kStep < w1) {
            so_nn = out.store_off[wn + kStep];
            len_nn = out.store_len[wn + kStep];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = lane + 64 * j;
            if (i < len) f(u[j], c[j], so + i, w);
        }
        for (int i0 = 256; i0 < len; i0 += 256) {  // worlds of more than 256 entries
            int32_t ut[4], ct[4];
            load_world_head<CNT>(out, so + i0, len - i0, lane, ut, ct);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int i = i0 + lane + 64 * j;
                if (i < len) f(ut[j], ct[j], so + i, w);
            }
        }
        if (wn >= w1) break;
        w = wn;
        so = so_n;
        len = len_n;
        so_n = so_nn;
        len_n = len_nn;
        for (int j = 0; j < 4; ++j) {  // register moves (unrolled by the compiler)
            u[j] = un[j];
            c[j] = cn[j];
        }
    }
}

// entries per bucket
__global__ __launch_bounds__(kIdxNT) void k_index_bucket_count(TileOut out, uint32_t theta, int shift, int nb,
                                                              uint32_t* bcnt, RoundCtl* ctl) {
    __shared__ int32_t h[kIdxMaxBuckets];
    const uint32_t w0 = blockIdx.x * kIdxWorldsPerWG;
    const uint32_t w1 = min(theta, w0 + kIdxWorldsPerWG);
    for (int i = threadIdx.x; i < nb; i += kIdxNT) h[i] = 0;
    __syncthreads();
    bool bad = false;
    for_stored_entries<kIdxNT, false>(out, w0, w1, [&](int32_t u, int32_t, long long, uint32_t) {
        const uint32_t bk = (uint32_t)u >> shift;
        if (bk < (uint32_t)nb) atomicAdd(&h[bk], 1);
        else bad = true;
    });
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kIdxNT)
        if (h[i]) atomicAdd(&bcnt[i], (uint32_t)h[i]);
}

__device__ __forceinline__ int bucket_size_class(uint32_t v) { return v ? 32 - __clz((int)v) : 0; }

// bucket bases: bbase[b] = entries of the buckets before b, bbase[nb] = all;
// the partition's cursors start at the bases.  border lists the buckets by
// decreasing size class (floor(log2(entries)) + 1), the order in which the
// owning workgroups start.
__global__ __launch_bounds__(1024) void k_index_bucket_scan(const uint32_t* bcnt, int nb, uint32_t* bbase,
                                                           uint32_t* bcur, int32_t* border) {
    __shared__ long long tmp[16];
    __shared__ int cls[33];
    if (threadIdx.x < 33) cls[threadIdx.x] = 0;
    __syncthreads();
    long long run = 0;  // the host keeps the total below kIndexPosLimit
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        const int i = c0 + threadIdx.x;
        const uint32_t v = i < nb ? bcnt[i] : 0u;
        long long tot;
        const long long ex = block_excl_scan_ll<1024>((long long)v, tmp, tot);
        if (i < nb) {
            bbase[i] = (uint32_t)(run + ex);
            bcur[i] = (uint32_t)(run + ex);
            atomicAdd(&cls[bucket_size_class(v)], 1);
        }
        run += tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        bbase[nb] = (uint32_t)run;
        int start = 0;
        for (int k = 32; k >= 0; --k) {
            const int c = cls[k];
            cls[k] = start;
            start += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += 1024) border[atomicAdd(&cls[bucket_size_class(bcnt[i])], 1)] = i;
}

// records of the workgroup's worlds into their buckets' ranges.  The
// workgroup's entries, numbered flat over its worlds, go in batches of
// kPartStage: each batch is counted per bucket in LDS, its share of every
// bucket reserved with one counter update, the records staged in LDS
// bucket by bucket, and each bucket's run written out to consecutive
// addresses (scattered 16-byte stores would cost one transaction each).
constexpr int kPartStage = 4096;
static_assert(kIdxWorldsPerWG <= (uint32_t)kIdxNT, "one world range per thread");
static_assert(kPartStage % kIdxNT == 0, "whole records per thread");

size_t index_partition_lds(int nb) {
    return (size_t)kPartStage * sizeof(int4) + kIdxWorldsPerWG * sizeof(long long) +
           (kIdxWorldsPerWG + 1) * sizeof(int32_t) + 2 * (size_t)nb * sizeof(int32_t);
}

__global__ __launch_bounds__(kIdxNT) void k_index_partition(TileOut out, uint32_t theta, int shift, int nb,
                                                           uint32_t* bcur, int4* rec, uint32_t rec_cap,
                                                           RoundCtl* ctl) {
    extern __shared__ int4 part_lds[];
    int4* stage = part_lds;                                                      // [kPartStage]
    long long* woff = reinterpret_cast<long long*>(stage + kPartStage);          // [worlds]
    int32_t* wpre = reinterpret_cast<int32_t*>(woff + kIdxWorldsPerWG);         // [worlds + 1]
    int32_t* bnum = wpre + kIdxWorldsPerWG + 1;                                  // [nb] count, then base
    uint32_t* bdel = reinterpret_cast<uint32_t*>(bnum + nb);                     // [nb] global - local (mod 2^32)
    __shared__ int tmp[kIdxNT / 64];
    constexpr int kPer = kPartStage / kIdxNT;
    const int t = threadIdx.x;
    const uint32_t w0 = blockIdx.x * kIdxWorldsPerWG;
    const int nw = (int)(min(theta, w0 + kIdxWorldsPerWG) - w0);
    int len = 0;
    if (t < nw) {
        woff[t] = out.store_off[w0 + t];
        len = max(out.store_len[w0 + t], 0);
    }
    int total;
    const int ex = block_excl_scan<kIdxNT>(len, tmp, total);
    if (t <= nw) wpre[t] = ex;  // wpre[nw] = total
    __syncthreads();
    bool bad = false;
    for (int k0 = 0; k0 < total; k0 += kPartStage) {
        const int k1 = min(total, k0 + kPartStage);
        for (int i = t; i < nb; i += kIdxNT) bnum[i] = 0;
        __syncthreads();
        int32_t ru[kPer], rc[kPer], rp[kPer], rw[kPer], rr[kPer];
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const int k = k0 + t + j * kIdxNT;
            ru[j] = -1;
            rc[j] = rp[j] = rw[j] = rr[j] = 0;
            if (k < k1) {
                // the world holding flat entry k: wpre[lo] <= k < wpre[lo + 1]
                int lo = 0, hi = nw;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (wpre[mid] <= k) lo = mid;
                    else hi = mid;
                }
                const long long pos = woff[lo] + (k - wpre[lo]);
                rp[j] = (int32_t)(uint32_t)pos;
                rw[j] = (int32_t)(w0 + (uint32_t)lo);
                ru[j] = out.store_node[pos];
                rc[j] = out.store_cnt[pos];
            }
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            if (ru[j] < 0) continue;
            const uint32_t bk = (uint32_t)ru[j] >> shift;
            if (bk < (uint32_t)nb) rr[j] = atomicAdd(&bnum[bk], 1);
            else ru[j] = -1;
        }
        __syncthreads();
        // local bases, and the batch's share of each bucket
        const int per = (nb + kIdxNT - 1) / kIdxNT;
        const int b0 = min(nb, t * per), b1 = min(nb, b0 + per);
        int sum = 0;
        for (int bk = b0; bk < b1; ++bk) sum += bnum[bk];
        int staged;
        int base = block_excl_scan<kIdxNT>(sum, tmp, staged);
        for (int bk = b0; bk < b1; ++bk) {
            const int c = bnum[bk];
            bnum[bk] = base;
            if (c) bdel[bk] = atomicAdd(&bcur[bk], (uint32_t)c) - (uint32_t)base;
            base += c;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (ru[j] >= 0) stage[bnum[(uint32_t)ru[j] >> shift] + rr[j]] = make_int4(rp[j], rw[j], ru[j], rc[j]);
        __syncthreads();
        for (int i = t; i < staged; i += kIdxNT) {
            const int4 r = stage[i];
            const uint32_t g = bdel[(uint32_t)r.z >> shift] + (uint32_t)i;
            if (g < rec_cap) rec[g] = r;
            else bad = true;
        }
        __syncthreads();
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
}

// The slot most lanes of a wave hold among those of lanes 0, 8, ..., 56
// (held by at least two lanes), or -1; the same value on every lane.
__device__ __forceinline__ int own_hot_slot(uint32_t d, bool ok) {
    const int key = ok ? (int)d : -1;
    int best = -1, best_n = 1;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int cand = __shfl(key, s * 8, 64);
        const int m = __popcll(__ballot(cand >= 0 && key == cand));
        if (m > best_n) {
            best_n = m;
            best = cand;
        }
    }
    return best;
}

// One workgroup per bucket, largest buckets first: the nodes' entry counts
// (and with GAIN the sums of the entries' counts: the from-scratch gains of
// round 0, Section 2.2, added to gain[u]) in LDS, their offsets idx_off[u]
// by a scan from the bucket's base, and each entry (position, world) at its
// node's offset plus a rank handed out in LDS.  Buckets wider than the LDS
// table take several passes over their records, one per slice of kOwnSlots
// nodes.  A hub can hold a third of its bucket's entries, and lanes updating
// one LDS counter are served one after another: each wave picks its most
// common node (its hot slot) from its first records, keeps that node's
// count and sum in registers while counting, and takes that node's ranks
// with one counter update per instruction while placing.
template <bool GAIN>
__global__ __launch_bounds__(kOwnNT) void k_index_own(const int4* rec, uint32_t rec_cap, const uint32_t* bbase,
                                                     const int32_t* border, int nb, int shift, int32_t n,
                                                     uint32_t* idx_off, int2* idx_ent, uint32_t ent_cap,
                                                     int64_t* gain, RoundCtl* ctl) {
    __shared__ uint32_t cnt[kOwnSlots];
    __shared__ unsigned long long gs[GAIN ? kOwnSlots : 1];
    __shared__ uint32_t tmp[kOwnNT / 64];
    const int b = border[blockIdx.x];
    if (b < 0 || b >= nb) {  // the order is a permutation of the buckets
        if (threadIdx.x == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        return;
    }
    // records [r0, r1) (within rec_cap even if the partition overflowed)
    const uint32_t r0 = min(bbase[b], rec_cap), r1 = min(bbase[b + 1], rec_cap);
    const int32_t lo = (int32_t)((long long)b << shift);
    const int32_t hi = (int32_t)min((long long)n, (long long)lo + (1ll << shift));
    const int t = threadIdx.x;
    const int lane = t & 63;
    uint32_t run = r0;
    bool bad = false;
    for (int32_t sub = lo; sub < hi; sub += kOwnSlots) {
        const int ns = min(kOwnSlots, hi - sub);
        for (int i = t; i < kOwnSlots; i += kOwnNT) {
            cnt[i] = 0;
            if (GAIN) gs[i] = 0;
        }
        __syncthreads();
        int hot = -1;
        int hot_n = 0;
        unsigned long long hot_s = 0;
        for (uint32_t q = r0; q < r1; q += 4 * kOwnNT) {
            int4 e[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t r = q + t + j * kOwnNT;
                e[j] = r < r1 ? rec[r] : make_int4(0, 0, -1, 0);
            }
            if (q == r0) hot = own_hot_slot((uint32_t)(e[0].z - sub), r0 + t < r1 && (uint32_t)(e[0].z - sub) < (uint32_t)ns);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t d = (uint32_t)(e[j].z - sub);
                if (q + t + j * kOwnNT < r1 && d < (uint32_t)ns) {
                    if ((int)d == hot) {
                        ++hot_n;
                        if (GAIN) hot_s += (uint32_t)e[j].w;
                    } else {
                        atomicAdd(&cnt[d], 1u);
                        if (GAIN) atomicAdd(&gs[d], (unsigned long long)(uint32_t)e[j].w);
                    }
                }
            }
        }
        if (hot >= 0) {  // the same on every lane of the wave
#pragma unroll
            for (int k = 32; k >= 1; k >>= 1) {
                hot_n += __shfl_xor(hot_n, k, 64);
                if (GAIN) hot_s += __shfl_xor(hot_s, k, 64);
            }
            if (lane == 0 && hot_n) {
                atomicAdd(&cnt[hot], (uint32_t)hot_n);
                if (GAIN) atomicAdd(&gs[hot], hot_s);
            }
        }
        __syncthreads();
        // two consecutive slots per thread
        const uint32_t a0 = cnt[2 * t], a1 = cnt[2 * t + 1];
        uint32_t tot;
        const uint32_t o0 = run + block_excl_scan<kOwnNT, uint32_t>(a0 + a1, tmp, tot);
        const uint32_t o1 = o0 + a0;
        cnt[2 * t] = o0;
        cnt[2 * t + 1] = o1;
        if (2 * t < ns) {
            idx_off[sub + 2 * t] = o0;
            if (GAIN) gain[sub + 2 * t] += (int64_t)gs[2 * t];
        }
        if (2 * t + 1 < ns) {
            idx_off[sub + 2 * t + 1] = o1;
            if (GAIN) gain[sub + 2 * t + 1] += (int64_t)gs[2 * t + 1];
        }
        run += tot;
        __syncthreads();
        // the next records are loaded before this batch's stores, which
        // the loads would otherwise wait for (one in-order counter)
        int4 e[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t r = r0 + t + j * kOwnNT;
            e[j] = r < r1 ? rec[r] : make_int4(0, 0, -1, 0);
        }
        for (uint32_t q = r0; q < r1; q += 4 * kOwnNT) {
            int4 en[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t r = q + 4 * kOwnNT + t + j * kOwnNT;
                en[j] = r < r1 ? rec[r] : make_int4(0, 0, -1, 0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t d = (uint32_t)(e[j].z - sub);
                const bool ok = q + t + j * kOwnNT < r1 && d < (uint32_t)ns;
                const bool is_hot = ok && (int)d == hot;
                const unsigned long long m = __ballot(is_hot);
                uint32_t p = 0;
                if (m) {
                    const int leader = __ffsll((long long)m) - 1;
                    uint32_t base = 0;
                    if (lane == leader) base = atomicAdd(&cnt[hot], (uint32_t)__popcll(m));
                    base = __shfl(base, leader, 64);
                    p = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                }
                if (ok && !is_hot) p = atomicAdd(&cnt[d], 1u);
                if (ok) {
                    if (p < ent_cap) idx_ent[p] = make_int2(e[j].x, e[j].y);
                    else bad = true;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) e[j] = en[j];
        }
        __syncthreads();
    }
    if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    if (b == nb - 1 && t == 0) idx_off[n] = run;
}
static_assert(kOwnSlots == 2 * kOwnNT, "the offset scan takes two slots per thread");

// Whether the label rule updates a world for the new blocker: the world is
// labelled and the blocker's exit bit is clear.
__device__ __forceinline__ bool label_rule_holds(uint8_t wflags, uint32_t lab) {
    return (wflags & kWorldLabelled) != 0 && !label_exits(lab);
}

// An incremental round without replay starts here (with replay,
// k_round_update takes this role).  Every workgroup combines the parts of
// the last selection (the same result everywhere); workgroup 0 commits it.
// Then the worlds whose entry for the new blocker u is live are listed in
// list[0 .. list_n[0]) for the sampling tiers.
__global__ __launch_bounds__(256) void k_affected_select(TileOut out, RoundCtl* ctl, const uint32_t* idx_off,
                                                         const int2* idx_ent,
                                                         int32_t* list, SelectOut so) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    __shared__ long long sd[4];
    if (ctl->stop) return;
    int64_t bg;
    int32_t bu;
    long long dl;
    select_combine(so, bg, bu, dl, sg, su, sd);
    const int r = ctl->round_snap;  // written by the partial launch; workgroup 0 updates ctl->round
    if (blockIdx.x == 0 && threadIdx.x == 0) select_commit(ctl, so, r, bg, bu, dl);
    if (select_stops(r, so.k, bu, bg) || r + 1 == so.k) return;  // no further round
    const int32_t u = bu;
    const uint32_t a = idx_off[u], b = idx_off[u + 1];
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (uint32_t i = a + blockIdx.x * 256 + threadIdx.x - lane; i < b; i += gridDim.x * 256) {
        const uint32_t k = i + lane;
        int32_t w = 0, c = 0;
        if (k < b) {
            const int2 e = idx_ent[k];
            w = e.y;
            c = out.store_cnt[index_pos(e)];
        }
        const bool live = c > 0;
        const unsigned long long mr = __ballot(live);
        uint32_t br = 0;
        if (lane == 0 && mr) br = atomicAdd(&ctl->list_n[0], (uint32_t)__popcll(mr));
        br = __shfl(br, 0, 64);
        if (live) {
            const uint32_t at = br + (uint32_t)__popcll(mr & below);
            if (at < out.list_cap) list[at] = w;
            else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        }
    }
}

hipError_t launch_index_build(const TileOut& out, uint32_t theta, int32_t n, const IndexBufs& ib, int64_t* gain,
                              RoundCtl* ctl, hipStream_t s) {
    if (ib.nb < 1 || ib.nb > kIdxMaxBuckets || ((long long)ib.nb << ib.shift) < (long long)n) return hipErrorInvalidValue;
    const unsigned groups = (theta + kIdxWorldsPerWG - 1) / kIdxWorldsPerWG;
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t*>(ib.bcnt), 0, (size_t)ib.nb, s);
    if (e != hipSuccess) return e;
    if (groups > 0) {
        k_index_bucket_count<<<groups, kIdxNT, 0, s>>>(out, theta, ib.shift, ib.nb, ib.bcnt, ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    k_index_bucket_scan<<<1, 1024, 0, s>>>(ib.bcnt, ib.nb, ib.bbase, ib.bcur, ib.border);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (groups > 0) {
        const size_t lds = index_partition_lds(ib.nb);
        if ((e = hipFuncSetAttribute((const void*)k_index_partition, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds)) != hipSuccess)
            return e;
        k_index_partition<<<groups, kIdxNT, lds, s>>>(out, theta, ib.shift, ib.nb, ib.bcur, ib.rec, ib.rec_cap, ctl);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (gain)
        k_index_own<true><<<(unsigned)ib.nb, kOwnNT, 0, s>>>(ib.rec, ib.rec_cap, ib.bbase, ib.border, ib.nb, ib.shift, n, ib.idx_off,
                                                              ib.idx_ent, ib.ent_cap, gain, ctl);
    else
        k_index_own<false><<<(unsigned)ib.nb, kOwnNT, 0, s>>>(ib.rec, ib.rec_cap, ib.bbase, ib.border, ib.nb, ib.shift, n, ib.idx_off,
                                                               ib.idx_ent, ib.ent_cap, nullptr, ctl);
    return hipGetLastError();
}

hipError_t launch_affected_select(const TileOut& out, RoundCtl* ctl, const uint32_t* idx_off, const int2* idx_ent,
                                  int32_t* list, const SelectOut& so, hipStream_t s) {
    k_affected_select<<<256, 256, 0, s>>>(out, ctl, idx_off, idx_ent, list, so);
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
template <int CAP, int XCAP, int LVCAP>
struct ReplayStore {
    int32_t nl[CAP];      // old entry -> new local id; -1 not reached yet, -2 removed, -3 being claimed
    int32_t cur[CAP];     // BFS: owner slot of each head claimed in a level; then label placement cursors
    int16_t parent[CAP];  // by new local id - ns; preorder index once the counts are known
    int16_t idom[CAP];
    int32_t aux[CAP];
    int32_t hi[CAP];      // upper ends of the exit spans (lower ends: cur, after the labels)
    int32_t xv[XCAP];     // extra edges of the new BFS: head (old entry until resolved), source new id
    int16_t xu[XCAP];
    int32_t lvl[LVCAP + 2];
    int32_t ns;

    static constexpr int kCap = CAP;
    static constexpr bool kSortExtras = false;  // the extra edges are in LDS
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
    static constexpr bool kLabels = true;
    __device__ int32_t* cur_ptr(int lid) { return &cur[lid - ns]; }
    __device__ void set_tin(int lid, int v) { parent[lid - ns] = (int16_t)v; }
    __device__ int get_tin(int lid) const { return (int)(uint16_t)parent[lid - ns]; }
    __device__ int32_t* lo_ptr(int lid) { return &cur[lid - ns]; }
    __device__ int32_t* hi_ptr(int lid) { return &hi[lid - ns]; }
    template <int NT>
    __device__ void stage(int) {}  // everything is in LDS already
};

// levels: at most one per entry plus the seeds' and a closing empty one
using ReplayStoreT = ReplayStore<kReplayCap, kReplayXCap, kReplayCap + 2>;
constexpr int kReplayNT = 256;                          // four waves per replayed world

// A replay configuration: workgroup size and store, with the world's
// entries and stored edges held in registers (kEntrySlots and kSlots per
// thread).
template <int NT_, int CAP, int XCAP, int EDGECAP>
struct ReplayCfg {
    static constexpr int NT = NT_;
    using Store = ReplayStore<CAP, XCAP, CAP + 2>;
    static constexpr int kEntrySlots = CAP / NT_;
    static constexpr int kSlots = EDGECAP / NT_;
    static_assert(CAP % NT_ == 0 && EDGECAP % NT_ == 0, "whole slots per thread");
    static_assert(kSlots <= 32, "the valid edge slots fit one 32-bit mask");
};
// the replay workgroups of the round-update launch
using ReplaySmall = ReplayCfg<kReplayNT, kReplayCap, kReplayXCap, kReplayEdgeCap>;

// The label rule on a world's entries held in registers: entries in u's
// label range lose their whole count, u's ancestors lose count(u), and T
// loses count(u).
template <class C>
__device__ __forceinline__ void replay_local_update(const ReplayItem& it, int32_t ustar, const TileOut& out,
                                    const int32_t (&ec)[C::kEntrySlots], const int32_t (&en)[C::kEntrySlots],
                                    const uint32_t (&el)[C::kEntrySlots]) {
    constexpr int NT = C::NT;
    const int t = threadIdx.x;
    const size_t so = (size_t)it.store_off;
    const int L0 = it.store_len;
    const int tj = label_tin(it.labj);
    const int szj = label_size(it.labj);
    const int cj = it.cj;
#pragma unroll
    for (int r = 0; r < C::kEntrySlots; ++r) {
        const int i = t + r * NT;
        if (i >= L0 || ec[r] <= 0) continue;
        const int ti = label_tin(el[r]);
        const int si = label_size(el[r]);
        int d = 0, cn = 0;
        if (ti >= tj && ti < tj + szj) {
            d = -ec[r];
        } else if (tj >= ti && tj < ti + si) {
            d = -cj;
            cn = ec[r] - cj;
        }
        if (d != 0) {
            if (en[r] != ustar) atomicAdd((unsigned long long*)&out.gain[en[r]], (unsigned long long)(long long)d);
            out.store_cnt[so + i] = cn;
        }
    }
    if (t == 0) out.world_size[it.w] = it.world_size - cj;
}

// The stored edges stay in registers (C::kSlots per thread); each level
// looks up the new id of every pending edge's source and claims the heads
// of the edges leaving the frontier.  Every edge is used once, when its
// source's level is expanded.  The world's entries (count, node) stay in
// registers too (thread t holds entries t, t+NT, ...) for the outputs.  An
// entry is removed when its count is 0 (lost in an earlier round, which
// includes every earlier blocker) or it is this round's blocker.
//
// Within a level, the edges into a head not reached before each write
// their slot id into cur[head]; the edge whose id stays there claims it,
// the other edges into reached heads become extra edges, and one
// workgroup-wide scan hands out the new local ids and extra-edge slots.
//
// Before the BFS, a world with valid labels is checked for a shortcut: if no
// stored live edge leads from a reached node of u's dominator subtree to a
// reached node outside it (edges into a dominator of their source aside),
// no simple path to a node outside the subtree passes through the subtree,
// so blocking u removes exactly the subtree and leaves every other dominator
// (and label) as it was: the label rule applies.  (The exit bit of u's label
// answers the same question for the edges as they were when the labels were
// made; the test here also sees the edges lost since.)  The stored edges are
// left in ed (source << 16 | head entry, old ids), act marking the valid
// ones.  Returns 1 when the world was replayed, 2 when the shortcut
// applied, 0 when the world exceeds the replay's limits.
template <class C>
__device__ __forceinline__ int bfs_replay(const QueryDev& q, int32_t ustar, const ReplayItem& it, const TileOut& out,
                          typename C::Store& st, WorldShared<C::NT>& sh, int32_t (&ec)[C::kEntrySlots],
                          int32_t (&en)[C::kEntrySlots], uint32_t (&ed)[C::kSlots], uint32_t& act0) {
    constexpr int NT = C::NT;
    using RS = typename C::Store;
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    const size_t so = (size_t)it.store_off;
    const int L0 = it.store_len;
    const size_t xo = (size_t)it.xstore_off;
    const int X0 = it.xstore_len;
    const int E = L0 + X0;
    // room, local ids that fit the 16-bit arrays, ranges inside the stores
    // (uniform checks)
    if (L0 < 0 || X0 < 0 || L0 > RS::kCap || X0 > RS::cap_x() || E > NT * C::kSlots || ns + L0 > 32767)
        return 0;
    if (it.store_off < 0 || it.xstore_off < 0 || so + (size_t)L0 > out.store_cap || xo + (size_t)X0 > out.xstore_cap)
        return 0;
    const bool labelled = (it.flags & kWorldLabelled) != 0;
    // one batch of loads: entries, then edges (the tree edge of entry e is
    // its round-0 parent; then the extras)
    uint32_t el[C::kEntrySlots];
#pragma unroll
    for (int r = 0; r < C::kEntrySlots; ++r) {
        const int i = t + r * NT;
        ec[r] = 0;
        en[r] = -1;
        el[r] = 0;
        if (i < L0) {
            ec[r] = out.store_cnt[so + i];
            en[r] = out.store_node[so + i];
            if (labelled) el[r] = out.store_lab[so + i];
        }
    }
    uint32_t act = 0;
#pragma unroll
    for (int r = 0; r < C::kSlots; ++r) {
        const int e = t + r * NT;
        int u = -1, vi = -1;
        if (e < L0) {
            u = out.store_par[so + e];
            vi = e;
        } else if (e < E) {
            u = out.xstore_u[xo + (e - L0)];
            vi = out.xstore_v[xo + (e - L0)] - ns;
        }
        const bool ok = u >= 0 && u < ns + L0 && vi >= 0 && vi < L0;
        ed[r] = ok ? (((uint32_t)u << 16) | (uint32_t)vi) : 0u;  // inactive slots read entry 0, harmlessly
        act |= ok ? (1u << r) : 0u;
    }
    act0 = act;
    if (labelled) {
        // reached entries' labels (-1: not reached) for the edge test; a
        // label is below 2^27
        const int tj = label_tin(it.labj);
        const int szj = label_size(it.labj);
#pragma unroll
        for (int r = 0; r < C::kEntrySlots; ++r) {
            const int i = t + r * NT;
            if (i < L0) st.cur[i] = (ec[r] > 0) ? (int)el[r] : -1;
        }
        __syncthreads();
        bool escape = false;
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r) {
            const int u = (int)(ed[r] >> 16);
            if (((act >> r) & 1u) && u >= ns) {
                const int ls = st.cur[u - ns];
                const int lh = st.cur[ed[r] & 0xFFFFu];
                if (ls >= 0 && lh >= 0) {
                    const int ts = label_tin((uint32_t)ls);
                    const int th = label_tin((uint32_t)lh);
                    const bool src_in = ts >= tj && ts < tj + szj;
                    const bool head_out = th < tj || th >= tj + szj;
                    const bool head_dominates = th <= ts && ts < th + label_size((uint32_t)lh);
                    escape |= src_in && head_out && !head_dominates;
                }
            }
        }
        if (!__syncthreads_or(escape)) {
            replay_local_update<C>(it, ustar, out, ec, en, el);
            return 2;
        }
    }
#pragma unroll
    for (int r = 0; r < C::kEntrySlots; ++r) {
        const int i = t + r * NT;
        if (i < L0) st.nl[i] = (ec[r] <= 0 || en[r] == ustar) ? -2 : -1;
    }
    if (t == 0) {
        st.ns = ns;
        st.lvl[0] = 0;
        st.lvl[1] = ns;
    }
    __syncthreads();
    int count = ns, nx = 0;  // uniform
    int f0 = 0, f1 = ns;     // the frontier: level nlev - 1
    int nlev = 1;            // closed levels: lvl[0..nlev]
    while (f0 != f1) {
        int nu[C::kSlots], hv[C::kSlots], own[C::kSlots];
        uint32_t hit = 0;
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r) {
            const int u = (int)(ed[r] >> 16);
            const int x = st.nl[(u >= ns) ? u - ns : 0];
            nu[r] = (u < ns) ? u : x;
            hv[r] = st.nl[ed[r] & 0xFFFFu];
        }
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r)
            hit |= (((act >> r) & 1u) && nu[r] >= f0 && nu[r] < f1) ? (1u << r) : 0u;
        act &= ~hit;
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r)
            if (((hit >> r) & 1u) && hv[r] == -1) st.cur[ed[r] & 0xFFFFu] = t * C::kSlots + r;
        __syncthreads();
        uint32_t win = 0, ext = 0;
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r) {
            own[r] = st.cur[ed[r] & 0xFFFFu];
            const bool h = (hit >> r) & 1u;
            const bool w = h && hv[r] == -1 && own[r] == t * C::kSlots + r;
            win |= w ? (1u << r) : 0u;
            ext |= (h && hv[r] != -2 && !w) ? (1u << r) : 0u;
        }
        // local ids and extra-edge slots: one scan of (claims, extras)
        int tot;
        const int ex = block_excl_scan<NT, int>(__popc(win) | (__popc(ext) << 16), sh.scan_tmp, tot);
        int lid = count + (ex & 0xFFFF);
        int xs = nx + (ex >> 16);
#pragma unroll
        for (int r = 0; r < C::kSlots; ++r) {
            const int vi = (int)(ed[r] & 0xFFFFu);
            if ((win >> r) & 1u) {
                st.nl[vi] = lid;
                st.set_parent(lid, nu[r]);
                ++lid;
            }
            if ((ext >> r) & 1u) {
                if (xs < st.cap_x()) {
                    st.xv[xs] = vi;  // resolved to its new id in the dominator phase
                    st.xu[xs] = (int16_t)nu[r];
                }
                ++xs;
            }
        }
        count += tot & 0xFFFF;
        nx += tot >> 16;
        if (nx > st.cap_x()) return 0;         // uniform (cannot happen within the limits)
        if (nlev + 1 > st.cap_lv()) return 0;  // uniform (cannot happen within the limits)
        if (t == 0) st.lvl[nlev + 1] = count;
        ++nlev;
        f0 = f1;
        f1 = count;
        __syncthreads();
    }
    if (t == 0) {
        sh.count = count;
        sh.n_extra = nx;
        sh.edges = E;
        sh.nlevels = nlev - 1;
    }
    __syncthreads();
    return 1;
}

// The exits of a replayed world: its edges are the stored edges whose
// endpoints are both reached again.
template <class C>
__device__ __forceinline__ void replay_exits(typename C::Store& st, WorldShared<C::NT>& sh,
                                             const uint32_t (&ed)[C::kSlots], uint32_t act) {
    constexpr int NT = C::NT;
    const int ns = st.ns;
    exits_init<NT>(ns, sh.count, st);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < C::kSlots; ++r) {
        if (!((act >> r) & 1u)) continue;
        const int u = (int)(ed[r] >> 16);
        const int a = (u < ns) ? -1 : st.nl[u - ns];
        const int b = st.nl[ed[r] & 0xFFFFu];
        exits_edge(ns, st, a, b);  // skips unreached (negative) ends
    }
    __syncthreads();
    exits_merge<NT>(ns, st, sh);
}

// Count changes of a replayed world: each entry's new count against the one
// held in registers; changes are added to gain and the counts updated in
// place.
template <class C>
__device__ __forceinline__ int replay_outputs(const ReplayItem& it, int32_t ustar, const TileOut& out,
                              typename C::Store& st, WorldShared<C::NT>& sh,
                              const int32_t (&ec)[C::kEntrySlots], const int32_t (&en)[C::kEntrySlots]) {
    constexpr int NT = C::NT;
    const int t = threadIdx.x;
    const int ns = st.ns;
    const size_t so = (size_t)it.store_off;
    const int L0 = it.store_len;
    if (t == 0) sh.ndelta = 0;
    __syncthreads();
    int nd = 0;
#pragma unroll
    for (int r = 0; r < C::kEntrySlots; ++r) {
        const int i = t + r * NT;
        int cn = 0, d = 0;
        if (i < L0 && ec[r] > 0) {
            const int lid = st.nl[i];
            cn = (lid >= ns) ? st.aux[lid - ns] : 0;
            d = cn - ec[r];
            // the dominator tree may have changed shape: every reached
            // entry takes its new label
            if (cn > 0)
                out.store_lab[so + i] = pack_label(st.get_tin(lid), cn, sh.n_extra > 0 && exits_of(st, lid, cn));
        }
        const unsigned long long mask = __ballot(d != 0);
        if (d != 0) {
            if (en[r] != ustar) atomicAdd((unsigned long long*)&out.gain[en[r]], (unsigned long long)(long long)d);
            out.store_cnt[so + i] = cn;
        }
        nd += __popcll(mask);
    }
    if ((t & 63) == 0 && nd) atomicAdd(&sh.ndelta, nd);
    __syncthreads();
    if (t == 0) {
        out.world_size[it.w] = sh.count;
        if (out.world_flags) out.world_flags[it.w] = kWorldLabelled;
    }
    return sh.ndelta;
}

// Changed worlds the label rule cannot take are replayed; a world that does
// not fit the replay store goes on (list 1) to the wide replay, and from
// there to the sampling tiers.  The replay workgroups find those worlds in
// the index themselves: workgroup
// `part` of `parts` takes slices of kReplaySlice index entries of u (slice
// part, part + parts, ...), lists in LDS the live entries the rule cannot
// take and replays them one by one.
constexpr int kReplaySlice = 32;

template <class C>
struct ReplaySharedT {
    typename C::Store st;
    WorldShared<C::NT> sh;
    ReplayItem lst[kReplaySlice];  // the listed worlds
    uint32_t lst_n;
};
using ReplayShared = ReplaySharedT<ReplaySmall>;

struct ReplayAcc {
    unsigned long long w = 0, e = 0, b = 0, lw = 0, le = 0, lb = 0;
    long long d = 0;
};

// Replay one listed world (every thread of the workgroup, uniform); a world
// beyond the configuration's limits is appended to over_list (counter
// list_n[over_idx]).
template <class C>
__device__ __forceinline__ void replay_one(const QueryDev& q, RoundCtl* ctl, int over_idx, int32_t* over_list,
                                           const TileOut& out, int32_t ustar, const ReplayItem& cur,
                                           ReplaySharedT<C>& rs, ReplayAcc& acc) {
    typename C::Store& st = rs.st;
    WorldShared<C::NT>& sh = rs.sh;
    const int t = threadIdx.x;
    int32_t ec[C::kEntrySlots], en[C::kEntrySlots];
    uint32_t ed[C::kSlots], act;
    const int how = bfs_replay<C>(q, ustar, cur, out, st, sh, ec, en, ed, act);
    if (how == 2) {
        // the shortcut: reported with the label-based updates
        acc.lw += 1;
        acc.le += (unsigned long long)(cur.store_len + cur.xstore_len);
        acc.lb += 37ull + 16ull * (unsigned long long)cur.store_len + 8ull * (unsigned long long)cur.xstore_len + 8ull;
        acc.d += cur.cj;
    } else if (how == 1) {
        world_counts<C::NT>(q, ctl, st, sh);
        world_labels<C::NT>(q, st, sh);
        if (sh.n_extra > 0) replay_exits<C>(st, sh, ed, act);  // uniform
        const int nd = replay_outputs<C>(cur, ustar, out, st, sh, ec, en);
        acc.w += 1;
        acc.e += (unsigned long long)(cur.store_len + cur.xstore_len);
        // index entry, count, label, the world's ranges, size and flags;
        // entries and edges; the changes; the new size
        acc.b += 37ull + 12ull * (unsigned long long)cur.store_len + 8ull * (unsigned long long)cur.xstore_len +
                 12ull * (unsigned long long)nd + 8ull;
        acc.d += (long long)cur.world_size - (long long)sh.count;
    } else if (t == 0) {
        const uint32_t pos = atomicAdd(&ctl->list_n[over_idx], 1u);
        if (pos < out.next_cap) over_list[pos] = cur.w;
        else atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    }
    __syncthreads();
}

__device__ __forceinline__ void replay_worlds(const QueryDev& q, RoundCtl* ctl, int32_t* next_list, const TileOut& out,
                                              const uint32_t* idx_off, const int2* idx_ent, int32_t ustar,
                                              ReplayShared& rs, uint32_t part, uint32_t parts) {
    static_assert(kReplaySlice <= kReplayNT, "one thread per entry of a slice");
    const int t = threadIdx.x;
    const uint32_t a = idx_off[ustar], b = idx_off[ustar + 1];
    if ((long long)a + (long long)part * kReplaySlice >= (long long)b) return;  // no slice for this workgroup
    ReplayAcc acc;
    for (long long base = (long long)a + (long long)part * kReplaySlice; base < (long long)b;
         base += (long long)parts * kReplaySlice) {
        if (t == 0) rs.lst_n = 0;
        __syncthreads();
        if (t < kReplaySlice && base + t < (long long)b) {
            const int2 ie = idx_ent[base + t];
            const uint32_t pos = index_pos(ie);
            const int32_t w = ie.y;
            // the world's record is read with u's entry, whether or not it
            // is listed: one round trip
            ReplayItem it;
            it.w = w;
            it.cj = out.store_cnt[pos];
            it.labj = out.store_lab ? out.store_lab[pos] : 0u;
            it.flags = out.world_flags ? out.world_flags[w] : (uint8_t)0;
            it.store_off = out.store_off[w];
            it.store_len = out.store_len[w];
            it.xstore_off = out.xstore_off[w];
            it.xstore_len = out.xstore_len[w];
            it.world_size = out.world_size[w];
            it.j = (int32_t)((int64_t)pos - it.store_off);
            if (it.cj > 0 && !label_rule_holds((uint8_t)it.flags, it.labj)) {
                const uint32_t at = atomicAdd(&rs.lst_n, 1u);
                rs.lst[at] = it;
            }
        }
        __syncthreads();
        const uint32_t nl = rs.lst_n;
        for (uint32_t li = 0; li < nl; ++li) {
            const ReplayItem cur = rs.lst[li];
            replay_one<ReplaySmall>(q, ctl, 1, next_list, out, ustar, cur, rs, acc);
        }
    }
    if (t == 0) {
        add_work_at(out, 3, part, acc.w, acc.e, acc.b);
        add_work_at(out, 5, part, acc.lw, acc.le, acc.lb);
        // T is lowered by the nodes the replayed worlds lost
        if (acc.d) out.dsz[out.dsz_off[3] + part] = acc.d;
    }
}

// Changed worlds too large for the replay workgroups of the round-update
// launch (list 1, world ids) are replayed by one workgroup of 1024 threads
// each, with four times the capacities; a world beyond those goes on to
// the sampling tiers (list 3).  The new blocker's entry in each world is
// found by scanning the world's entries.
using ReplayWide = ReplayCfg<1024, 4 * kReplayCap, 4 * kReplayXCap, 4 * kReplayEdgeCap>;

__global__ __launch_bounds__(ReplayWide::NT) void k_replay_wide(QueryDev q, RoundCtl* ctl, TileOut out,
                                                             const int32_t* in_list, int32_t* over_list) {
    __shared__ ReplaySharedT<ReplayWide> rs;
    __shared__ int32_t jpos;
    const int t = threadIdx.x;
    if (ctl->stop) return;
    const uint32_t n_items = min(ctl->list_n[1], out.next_cap);
    if (blockIdx.x >= n_items) return;  // no world for this workgroup
    const int32_t ustar = ctl->ustar;   // committed by the round-update launch
    ReplayAcc acc;
    for (uint32_t k = blockIdx.x; k < n_items; k += gridDim.x) {
        ReplayItem it;
        it.w = in_list[k];
        it.store_off = out.store_off[it.w];
        it.store_len = out.store_len[it.w];
        it.xstore_off = out.xstore_off[it.w];
        it.xstore_len = out.xstore_len[it.w];
        it.world_size = out.world_size[it.w];
        it.flags = out.world_flags ? out.world_flags[it.w] : (uint8_t)0;
        if (it.store_off < 0 || it.store_len < 0 || (size_t)it.store_off + (size_t)it.store_len > out.store_cap) {
            if (t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
            continue;  // uniform
        }
        if (t == 0) jpos = -1;
        __syncthreads();
        for (int i = t; i < it.store_len; i += ReplayWide::NT)
            if (out.store_node[it.store_off + i] == ustar) jpos = i;  // a node has one entry per world
        __syncthreads();
        it.j = jpos;
        __syncthreads();  // jpos is written again for the next world
        if (it.j < 0) {
            if (t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);  // listed without an entry for u
            continue;  // uniform
        }
        it.cj = out.store_cnt[it.store_off + it.j];
        it.labj = out.store_lab ? out.store_lab[it.store_off + it.j] : 0u;
        if (it.cj <= 0) continue;  // uniform: listed only while u's entry is live
        replay_one<ReplayWide>(q, ctl, 3, over_list, out, ustar, it, rs, acc);
    }
    if (t == 0) {
        add_work_at(out, 3, blockIdx.x, acc.w, acc.e, acc.b);
        add_work_at(out, 5, blockIdx.x, acc.lw, acc.le, acc.lb);
        // T is lowered by the nodes the replayed worlds lost
        if (acc.d) out.dsz[out.dsz_off[5] + blockIdx.x] = acc.d;
    }
}

hipError_t launch_replay_wide(const QueryDev& q, RoundCtl* ctl, const TileOut& out, const int32_t* in_list,
                              int32_t* over_list, int grid, hipStream_t s, const LaunchEvents& ev) {
    if (grid < 1) return hipErrorInvalidValue;
    return launch_k(k_replay_wide, (unsigned)grid, (unsigned)ReplayWide::NT, s, ev, q, ctl, out, in_list, over_list);
}

// ------------------------------------------------------- label rule
// When no live edge leads out of u's dominator subtree (u's exit bit is
// clear; always so where the reached live edges form a forest), no simple
// path to a node outside the subtree passes through it: blocking u removes
// exactly u's subtree (its entries' counts become 0) and lowers the count
// of each of u's ancestors by count(u); no other count and no other
// dominator changes.  Subtree and ancestors are read off the labels: entry
// i lies in u's subtree when tin(u) <= tin(i) < tin(u) + size(u), and is an
// ancestor of u when tin(i) <= tin(u) < tin(i) + size(i).  The rest of the
// tree keeps valid labels; exit bits can only have become stale in the safe
// direction (an edge lost with the subtree may have been some ancestor's
// only exit).
//
// The label-rule workgroups of the changed-world launch walk the index
// entries of u themselves (the search listed only the other worlds): each
// group of LANES lanes takes entries a + group, a + group + groups, ...;
// a live entry of a labelled world with a clear exit bit is updated by the
// group in one pass over the world's entries.  The loads of the next entry
// (index, then its count, label and world) are issued before the current
// world's pass; smaller groups keep more worlds in flight per wave.  The
// count changes of a workgroup's worlds are summed in LDS and added to gain
// once per node per workgroup.
constexpr int kRuleUnroll = 8;
using RuleSums = LdsSums<11>;

struct RuleShared {
    RuleSums sums;
    unsigned long long red[4];
};

// What is read of one index entry before deciding.
struct RuleMeta {
    uint32_t pos;
    int32_t w, c;
    uint32_t lab;
    uint8_t flags;
    int64_t off;
    int32_t len, wsize;
};

__device__ __forceinline__ void rule_meta(const TileOut& out, RuleMeta& m) {
    m.c = out.store_cnt[m.pos];
    m.lab = out.store_lab[m.pos];
    m.flags = out.world_flags[m.w];
    m.off = out.store_off[m.w];
    m.len = out.store_len[m.w];
    m.wsize = out.world_size[m.w];
}

// The rule on entries [i0, i1) of a world (group of LANES lanes): returns
// the number of entries changed.
template <int LANES>
__device__ __forceinline__ int rule_span(const TileOut& out, RuleSums& sums, size_t so0, int i0, int i1, uint32_t labj,
                                         int cj, int gl, unsigned long long gmask) {
    const int tj = label_tin(labj);
    const int szj = label_size(labj);
    int nd = 0;
    for (int b0 = i0; b0 < i1; b0 += LANES * kRuleUnroll) {
        int c[kRuleUnroll], v[kRuleUnroll];
        uint32_t lab[kRuleUnroll];
#pragma unroll
        for (int q = 0; q < kRuleUnroll; ++q) {
            const int i = b0 + q * LANES + gl;
            c[q] = 0;
            v[q] = 0;
            lab[q] = 0;
            if (i < i1) {
                c[q] = out.store_cnt[so0 + i];
                v[q] = out.store_node[so0 + i];
                lab[q] = out.store_lab[so0 + i];
            }
        }
#pragma unroll
        for (int q = 0; q < kRuleUnroll; ++q) {
            const int i = b0 + q * LANES + gl;
            int d = 0, cn = 0;
            if (c[q] > 0) {
                const int ti = label_tin(lab[q]);
                const int si = label_size(lab[q]);
                if (ti >= tj && ti < tj + szj) {
                    d = -c[q];  // u's subtree, u included: no longer reached
                } else if (tj >= ti && tj < ti + si) {
                    d = -cj;  // an ancestor of u
                    cn = c[q] - cj;
                }
            }
            const unsigned long long mask = __ballot(d != 0) & gmask;
            if (d != 0) {
                // u itself is blocked from now on: its gain is never read again
                if (label_tin(lab[q]) != tj) sums.add(v[q], d, out.gain);
                out.store_cnt[so0 + i] = cn;
            }
            nd += __popcll(mask);
        }
    }
    return nd;
}

template <int LANES>
__device__ __forceinline__ void rule_worlds(RoundCtl* ctl, const TileOut& out, const uint32_t* idx_off,
                                            const int2* idx_ent, int32_t ustar,
                                            RuleShared& fs, uint32_t part, uint32_t parts) {
    static_assert(LANES == 16 || LANES == 32 || LANES == 64, "a world per 16, 32 or 64 lanes");
    constexpr int kGroups = kRuleNT / LANES;  // worlds of a workgroup at a time
    const uint32_t a = idx_off[ustar], b = idx_off[ustar + 1];
    RuleSums& sums = fs.sums;
    sums.clear<kRuleNT>();  // while u's index range is on its way
    if (threadIdx.x < 4) fs.red[threadIdx.x] = 0;
    __syncthreads();
    if ((long long)a + (long long)part * kGroups >= (long long)b) return;  // no entry for this workgroup (uniform)
    const int lane = threadIdx.x & 63;
    const int gl = lane % LANES;  // lane within the world's group
    const int group = (int)threadIdx.x / LANES;
    const unsigned long long gmask = (LANES == 64) ? ~0ull : (((1ull << LANES) - 1ull) << (lane - gl));
    const uint32_t stride = parts * kGroups;
    unsigned long long acc_w = 0, acc_e = 0, acc_b = 0;
    long long acc_d = 0;

    // uniform over the group: entry k0 now, k1 next, k2 after that
    uint32_t k0 = a + part * kGroups + (uint32_t)group;
    RuleMeta m0{};
    if (k0 < b) {
        const int2 e = idx_ent[k0];
        m0.pos = index_pos(e);
        m0.w = e.y;
        rule_meta(out, m0);
    }
    uint32_t k1 = k0 + stride;
    uint32_t p1 = 0;
    int32_t w1 = 0;
    if (k1 < b) {
        const int2 e = idx_ent[k1];
        p1 = index_pos(e);
        w1 = e.y;
    }
    while (k0 < b) {
        // next entry's decision data, and the index of the one after
        RuleMeta m1{};
        const uint32_t k2 = k1 + stride;
        uint32_t p2 = 0;
        int32_t w2 = 0;
        if (k1 < b) {
            m1.pos = p1;
            m1.w = w1;
            rule_meta(out, m1);
        }
        if (k2 < b) {
            const int2 e = idx_ent[k2];
            p2 = index_pos(e);
            w2 = e.y;
        }
        const size_t so0 = (size_t)m0.off;
        const int L0 = m0.len;
        if (m0.c <= 0 || !label_rule_holds(m0.flags, m0.lab)) {
            // lost already, or listed for the replay
        } else if (m0.off < 0 || L0 < 0 || so0 + (size_t)L0 > out.store_cap) {
            if (gl == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
        } else {
            const int nd = rule_span<LANES>(out, sums, so0, 0, L0, m0.lab, m0.c, gl, gmask);
            if (gl == 0) {
                out.world_size[m0.w] = m0.wsize - m0.c;
                acc_w += 1;
                acc_e += (unsigned long long)L0;
                // index entry, count and label of u, the world's range, size
                // and flags; the entries; the changes; the new size
                acc_b += 33ull + 12ull * (unsigned long long)L0 + 12ull * (unsigned long long)nd + 4ull;
                acc_d += m0.c;
            }
        }
        k0 = k1;
        m0 = m1;
        k1 = k2;
        p1 = p2;
        w1 = w2;
    }
    if (gl == 0 && acc_w) {
        atomicAdd(&fs.red[0], acc_w);
        atomicAdd(&fs.red[1], acc_e);
        atomicAdd(&fs.red[2], acc_b);
        atomicAdd(&fs.red[3], (unsigned long long)acc_d);
    }
    __syncthreads();
    sums.flush<kRuleNT>(out.gain);
    if (threadIdx.x == 0) {
        add_work_at(out, 4, part, fs.red[0], fs.red[1], fs.red[2]);
        if (fs.red[3]) out.dsz[out.dsz_off[4] + part] = (long long)fs.red[3];
    }
}

// ------------------------------------------------- changed-world update
// One launch per incremental round: every workgroup combines the parts of
// the last selection (the same result everywhere) and workgroup 0 commits
// it; then the first rule_parts workgroups apply the label rule while the
// rest replay the other changed worlds, side by side.  LDS is shared
// between the roles.
static_assert(kReplayNT == kRuleNT, "both roles use the same workgroup size");
union UpdateShared {
    struct {
        int64_t sg[kReplayNT];
        int32_t su[kReplayNT];
        long long sd[kReplayNT / 64];
    } sel;
    ReplayShared r;
    RuleShared f;
};

template <int LANES>
__global__ __launch_bounds__(kReplayNT, 5) void k_round_update(QueryDev q, RoundCtl* ctl, int32_t* next_list, TileOut out,
                                                             uint32_t rule_parts, const uint32_t* idx_off,
                                                             const int2* idx_ent,
                                                             SelectOut so) {
    __shared__ UpdateShared u;
    // the stop flag, the round and the selection's parts are read together
    // (the parts are always valid memory): one round trip, not three
    const int32_t stop = ctl->stop;
    const int r = ctl->round_snap;  // written by the partial launch; workgroup 0 updates ctl->round
    int64_t bg;
    int32_t bu;
    long long dl;
    select_combine(so, bg, bu, dl, u.sel.sg, u.sel.su, u.sel.sd);
    if (stop) return;  // uniform
    if (blockIdx.x == 0 && threadIdx.x == 0) select_commit(ctl, so, r, bg, bu, dl);
    if (select_stops(r, so.k, bu, bg) || r + 1 == so.k) return;  // no further round (uniform)
    __syncthreads();  // the selection's LDS is reused below
    if (blockIdx.x < rule_parts)
        rule_worlds<LANES>(ctl, out, idx_off, idx_ent, bu, u.f, blockIdx.x, rule_parts);
    else
        replay_worlds(q, ctl, next_list, out, idx_off, idx_ent, bu, u.r, blockIdx.x - rule_parts,
                      gridDim.x - rule_parts);
}

hipError_t launch_round_update(const QueryDev& q, RoundCtl* ctl, int32_t* next_list, const TileOut& out,
                               int rule_parts, int replay_parts, int lanes, const uint32_t* idx_off,
                               const int2* idx_ent, const SelectOut& so, hipStream_t s, const LaunchEvents& ev) {
    const unsigned grid = (unsigned)(replay_parts + rule_parts);
    if (grid == 0 || replay_parts < 1 || rule_parts < 0) return hipErrorInvalidValue;
    // index cursors advance by the parts' stride, which must stay below 2^24
    if ((long long)grid * kReplaySlice >= (1ll << 24) || (long long)rule_parts * kRuleNT >= (1ll << 24))
        return hipErrorInvalidValue;
    const uint32_t rp = (uint32_t)rule_parts;
    if (lanes == 16)
        return launch_k(k_round_update<16>, grid, kReplayNT, s, ev, q, ctl, next_list, out, rp, idx_off, idx_ent, so);
    if (lanes == 32)
        return launch_k(k_round_update<32>, grid, kReplayNT, s, ev, q, ctl, next_list, out, rp, idx_off, idx_ent, so);
    return launch_k(k_round_update<64>, grid, kReplayNT, s, ev, q, ctl, next_list, out, rp, idx_off, idx_ent, so);
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

// A workgroup per seed: a hub's row has thousands of slot groups, which its
// threads fill side by side.
__global__ void k_seed_fill(GraphDev g, const int32_t* seeds, int32_t ns, const int32_t* start, int4* table,
                            int32_t cap, RoundCtl* ctl) {
    if (ctl->stop) return;  // bad seeds: nothing to read
    for (int i = blockIdx.x; i < ns; i += gridDim.x) {
        const int32_t v = seeds[i];
        const int e0 = g.off[v], e1 = g.off[v + 1];
        if (e1 <= e0) continue;
        const int b0 = e0 >> 2, b1 = (e1 - 1) >> 2;
        const int j0 = start[i];
        bool bad = false;
        for (int b = b0 + (int)threadIdx.x; b <= b1; b += (int)blockDim.x) {
            const int j = j0 + (b - b0);
            if (j < cap) table[j] = make_int4(b, i, e0, e1);
            else bad = true;
        }
        if (bad) atomicOr(&ctl->flags, (uint32_t)kFlagBounds);
    }
}

// The per-query thresholds: the graph's, with every slot whose head is a
// seed or a blocked node set to 0 (never live), and the level-0 table's
// copies of its slot groups' columns and thresholds.
__global__ void k_query_thr(GraphDev g, const uint32_t* excl, uint32_t* thr_q, const RoundCtl* ctl) {
    if (ctl->stop) return;
    const size_t groups = (size_t)g.m_pad / 4;
    for (size_t b = blockIdx.x * (size_t)blockDim.x + threadIdx.x; b < groups; b += (size_t)gridDim.x * blockDim.x) {
        const int4 c = *reinterpret_cast<const int4*>(g.col + 4 * b);
        uint4 th = *reinterpret_cast<const uint4*>(g.thr + 4 * b);
        const size_t e = 4 * b;
        if (e + 0 < (size_t)g.m && bit_set(excl, c.x)) th.x = 0u;
        if (e + 1 < (size_t)g.m && bit_set(excl, c.y)) th.y = 0u;
        if (e + 2 < (size_t)g.m && bit_set(excl, c.z)) th.z = 0u;
        if (e + 3 < (size_t)g.m && bit_set(excl, c.w)) th.w = 0u;
        *reinterpret_cast<uint4*>(thr_q + 4 * b) = th;
    }
}

// The same with the exclusion bits staged in LDS, for graphs whose bitset
// fits (up to about 1.3M nodes): a test from global memory pulls a whole
// L2 line into the compute unit for 4 bytes, and on the 10^7-slot graph
// those lines outweigh the thresholds.  One workgroup per compute unit,
// four slot groups in flight per thread.
constexpr int kQueryThrNT = 1024;
__global__ __launch_bounds__(kQueryThrNT) void k_query_thr_lds(GraphDev g, const uint32_t* excl, uint32_t* thr_q,
                                                               const RoundCtl* ctl, int words) {
    extern __shared__ uint32_t excl_lds[];
    if (ctl->stop) return;
    for (int i = threadIdx.x; i < words; i += kQueryThrNT) excl_lds[i] = excl[i];
    __syncthreads();
    const size_t groups = (size_t)g.m_pad / 4;
    const size_t stride = (size_t)gridDim.x * kQueryThrNT;
    for (size_t b0 = blockIdx.x * (size_t)kQueryThrNT + threadIdx.x; b0 < groups; b0 += 4 * stride) {
        int4 c[4];
        uint4 th[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t b = b0 + j * stride;
            if (b < groups) {
                c[j] = *reinterpret_cast<const int4*>(g.col + 4 * b);
                th[j] = *reinterpret_cast<const uint4*>(g.thr + 4 * b);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t b = b0 + j * stride;
            if (b >= groups) continue;
            const size_t e = 4 * b;
            if (e + 0 < (size_t)g.m && bit_set(excl_lds, c[j].x)) th[j].x = 0u;
            if (e + 1 < (size_t)g.m && bit_set(excl_lds, c[j].y)) th[j].y = 0u;
            if (e + 2 < (size_t)g.m && bit_set(excl_lds, c[j].z)) th[j].z = 0u;
            if (e + 3 < (size_t)g.m && bit_set(excl_lds, c[j].w)) th[j].w = 0u;
            *reinterpret_cast<uint4*>(thr_q + 4 * b) = th[j];
        }
    }
}

__global__ void k_seed_slots(GraphDev g, const uint32_t* thr_q, const int4* table, const RoundCtl* ctl,
                             int32_t cap, int4* scol, uint4* sthr) {
    if (ctl->stop) return;  // bad seeds: the table is not filled
    const int32_t nc = min(ctl->seed_chunks, cap);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += gridDim.x * blockDim.x) {
        const size_t b = (size_t)table[j].x;
        scol[j] = *reinterpret_cast<const int4*>(g.col + 4 * b);
        sthr[j] = *reinterpret_cast<const uint4*>(thr_q + 4 * b);
    }
}

hipError_t launch_query_thresholds(const GraphDev& g, const uint32_t* excl, uint32_t* thr_q, const int4* table,
                                   const RoundCtl* ctl, int32_t chunk_cap, int4* seed_col, uint4* seed_thr,
                                   hipStream_t s) {
    const int words = (g.n + 31) / 32;
    const size_t lds = (size_t)words * sizeof(uint32_t);
    int dev = 0, cus = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    // IMIN_QUERY_THR_LDS=0 keeps the bits in global memory (tests compare both ways)
    const char* env = std::getenv("IMIN_QUERY_THR_LDS");
    const bool lds_ok = !(env && env[0] == '0');
    if (lds_ok && lds <= (size_t)lds_max && cus > 0) {
        e = hipFuncSetAttribute((const void*)k_query_thr_lds, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        k_query_thr_lds<<<(unsigned)cus, kQueryThrNT, lds, s>>>(g, excl, thr_q, ctl, words);
    } else {
        k_query_thr<<<2048, 256, 0, s>>>(g, excl, thr_q, ctl);
    }
    e = hipGetLastError();
    if (e != hipSuccess || chunk_cap < 1) return e;
    k_seed_slots<<<(chunk_cap + 255) / 256, 256, 0, s>>>(g, thr_q, table, ctl, chunk_cap, seed_col, seed_thr);
    return hipGetLastError();
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
                            int4* table, int32_t cap, RoundCtl* ctl, hipStream_t s) {
    k_seed_fill<<<(unsigned)std::max(1, std::min(ns, 65535)), 256, 0, s>>>(g, seeds, ns, start, table, cap, ctl);
    return hipGetLastError();
}

}  // namespace imin
