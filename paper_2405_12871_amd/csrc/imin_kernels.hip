// Device code for the IMIN sampling estimator on gfx950 (wave64).
//
// One world is one live-edge realization (Section 2.1, Eq. 1).  A workgroup
// evaluates a world end to end:
//   1. level-synchronous BFS from the seeds over live edges, never entering a
//      blocked node; edge coins are Philox4x32-10 blocks drawn lazily, only
//      for the out-edges of reached nodes (unscanned edges cannot change the
//      reached set); each claimed node gets a local id in BFS order and its
//      BFS parent, and every other live edge between reached nodes is kept;
//   2. immediate dominators under the virtual source (Section 3.1) by
//      level-ordered passes: idom(v) = lowest common ancestor of all of v's
//      live predecessors in the current tree (a node whose only predecessor
//      is its BFS parent keeps it);
//   3. subtree sizes c(v) = 1 + sum over children, deepest level first
//      (Section 2.2: the estimator measures every subtree);
//   4. (node, c) pairs for the reached non-seeds go to a pair buffer.
// The per-node sums over worlds are formed without global atomics: pairs are
// counting-sorted into node buckets, each bucket is accumulated in LDS, and
// per-slice partial vectors are added in a fixed order.
#include "imin_internal.hpp"

#include <hip/hip_runtime.h>

namespace imin {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with counter words 2 and
// 3 fixed at zero: counter (c0, c1, 0, 0), key (k0, k1).
__device__ __forceinline__ uint4 philox_block(uint32_t c0, uint32_t c1, uint32_t k0, uint32_t k1) {
    uint32_t x0 = c0, x1 = c1, x2 = 0u, x3 = 0u;
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

__device__ __forceinline__ bool bit_set(const uint32_t* bits, int32_t v) {
    return (bits[(uint32_t)v >> 5] >> ((uint32_t)v & 31u)) & 1u;
}

// --------------------------------------------------------- block helpers
template <int NT>
__device__ __forceinline__ int block_excl_scan(int x, int* tmp, int& total) {
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    int inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if constexpr (NT == 64) {
        total = __shfl(inc, 63, 64);
        return inc - x;
    } else {
        if (lane == 63) tmp[wid] = inc;
        __syncthreads();
        int pre = 0, tot = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            const int v = tmp[i];
            pre += (i < wid) ? v : 0;
            tot += v;
        }
        __syncthreads();
        total = tot;
        return pre + inc - x;
    }
}

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

// ------------------------------------------------------ per-world shared
template <int NT>
struct WorldShared {
    int count;    // local ids handed out (= nodes reached so far)
    int n_extra;  // non-tree live edges recorded
    int overflow; // capacity exceeded: abandon the world
    int changed;
    int nonfwd;   // some non-tree edge does not go one level down
    int widx;
    unsigned long long pair_base;
    int row_lid[NT];
    int row_node[NT];
    int row_e0[NT];
    int row_e1[NT];
    int row_start[NT];
    int scan_tmp[NT / 64 > 0 ? NT / 64 : 1];
    long long sum_tmp[NT / 64 > 0 ? NT / 64 : 1];
    long long edges;  // CSR slots of reached nodes (coins this world needs)
};

// ---------------------------------------------------- small-world store
// Everything in LDS: an open-addressing node -> local id table and the
// per-local-id arrays.  Capacities bound the world; a world that exceeds any
// of them is handed to the big-world path.
constexpr int kMaxDomPasses = 4096;
constexpr int kSmallCap = 1024;      // reached nodes
constexpr int kSmallHashBits = 11;   // 2048 slots, load <= 1/2
constexpr int kSmallXCap = 256;      // non-tree live edges
constexpr int kSmallLvCap = 62;      // BFS levels

struct SmallStore {
    static constexpr int kHash = 1 << kSmallHashBits;
    int32_t keys[kHash];
    int16_t vals[kHash];
    int32_t nodes[kSmallCap];
    int16_t parent[kSmallCap];
    int16_t idom[kSmallCap];
    int32_t aux[kSmallCap];
    int32_t xv[kSmallXCap];
    int16_t xu[kSmallXCap];
    int32_t lvl[kSmallLvCap + 2];

    __device__ static constexpr int cap_r() { return kSmallCap; }
    __device__ static constexpr int cap_x() { return kSmallXCap; }
    __device__ static constexpr int cap_lv() { return kSmallLvCap; }

    __device__ __forceinline__ static uint32_t hash(int32_t v) {
        return ((uint32_t)v * 0x9E3779B1u) >> (32 - kSmallHashBits);
    }
    __device__ void seed(int32_t v, int lid) {
        uint32_t h = hash(v);
        for (int probe = 0; probe < kHash; ++probe) {
            if (atomicCAS(&keys[h], -1, v) == -1) {
                vals[h] = (int16_t)lid;
                return;
            }
            h = (h + 1) & (kHash - 1);
        }
    }
    // New node: its local id.  Already present: -1.  Out of room: -2.
    __device__ int claim(int32_t v, int* counter) {
        uint32_t h = hash(v);
        for (int probe = 0; probe < kHash; ++probe) {
            const int32_t old = atomicCAS(&keys[h], -1, v);
            if (old == -1) {
                const int lid = atomicAdd(counter, 1);
                if (lid >= kSmallCap) return -2;
                vals[h] = (int16_t)lid;
                return lid;
            }
            if (old == v) return -1;
            h = (h + 1) & (kHash - 1);
        }
        return -2;
    }
    __device__ int lookup(int32_t v) const {
        uint32_t h = hash(v);
        for (int probe = 0; probe < kHash; ++probe) {
            if (keys[h] == v) return vals[h];
            h = (h + 1) & (kHash - 1);
        }
        return -1;
    }
    __device__ int get_parent(int i) const { return parent[i]; }
    __device__ void set_parent(int i, int v) { parent[i] = (int16_t)v; }
    __device__ int get_idom(int i) const { return idom[i]; }
    __device__ void set_idom(int i, int v) { idom[i] = (int16_t)v; }
    __device__ int get_xu(int x) const { return xu[x]; }
    __device__ void set_xu(int x, int v) { xu[x] = (int16_t)v; }
    template <int NT>
    __device__ void reset(int /*count*/) {
        for (int i = threadIdx.x; i < kHash; i += NT) keys[i] = -1;
    }
};

// ------------------------------------------------------ big-world store
// Per-slot arrays in HBM, sized for the whole graph (a world can reach every
// node and keep every edge), so this path never runs out of room.
struct BigStore {
    int32_t* lid_of;
    int32_t* nodes;
    int32_t* parent_;
    int32_t* idom_;
    int32_t* aux;
    int32_t* lvl;
    int32_t* xv;
    int32_t* xu_;
    int32_t cap_r_;
    int32_t cap_lv_;
    int64_t cap_x_;

    __device__ int cap_r() const { return cap_r_; }
    __device__ int64_t cap_x() const { return cap_x_; }
    __device__ int cap_lv() const { return cap_lv_; }
    __device__ void seed(int32_t v, int lid) { lid_of[v] = lid; }
    __device__ int claim(int32_t v, int* counter) {
        if (atomicCAS(&lid_of[v], -1, -2) != -1) return -1;
        const int lid = atomicAdd(counter, 1);
        lid_of[v] = lid;
        return lid;
    }
    __device__ int lookup(int32_t v) const { return lid_of[v]; }
    __device__ int get_parent(int i) const { return parent_[i]; }
    __device__ void set_parent(int i, int v) { parent_[i] = v; }
    __device__ int get_idom(int i) const { return idom_[i]; }
    __device__ void set_idom(int i, int v) { idom_[i] = v; }
    __device__ int get_xu(int64_t x) const { return xu_[x]; }
    __device__ void set_xu(int64_t x, int v) { xu_[x] = v; }
    template <int NT>
    __device__ void reset(int count) {
        for (int i = threadIdx.x; i < count; i += NT) lid_of[nodes[i]] = -1;
    }
};

// ------------------------------------------------------- one world
// Returns false when the store ran out of room (the world is then redone by
// the big-world path).  On success writes the world's pairs and size.
template <int NT, class Store>
__device__ bool evaluate_world(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w,
                               uint32_t wi, const TileOut& out, Store& st, WorldShared<NT>& sh) {
    const int t = threadIdx.x;
    const int ns = q.n_seeds;
    if (ns > st.cap_r()) return false;  // uniform

    // ---- seeds: level 0, parent = virtual source (-1)
    for (int i = t; i < ns; i += NT) {
        const int32_t v = q.seeds[i];
        st.seed(v, i);
        st.nodes[i] = v;
        st.set_parent(i, -1);
    }
    if (t == 0) {
        sh.count = ns;
        sh.edges = 0;
        sh.n_extra = 0;
        sh.overflow = 0;
        st.lvl[0] = 0;
        st.lvl[1] = ns;
    }
    __syncthreads();

    // ---- level-synchronous BFS with lazy coins
    int nlev = 1;  // closed levels: lvl[0..nlev]
    for (;;) {
        const int f0 = st.lvl[nlev - 1];
        const int f1 = st.lvl[nlev];
        if (f0 == f1) break;
        for (int base = f0; base < f1; base += NT) {
            const int i = base + t;
            int nb = 0, u = 0, e0 = 0, e1 = 0;
            if (i < f1) {
                u = st.nodes[i];
                e0 = g.off[u];
                e1 = g.off[u + 1];
                nb = (e1 > e0) ? (((e1 - 1) >> 2) - (e0 >> 2) + 1) : 0;
            }
            int total;
            const int start = block_excl_scan<NT>(nb, sh.scan_tmp, total);
            if (out.world_edges && e1 > e0) atomicAdd((unsigned long long*)&sh.edges, (unsigned long long)(e1 - e0));
            sh.row_lid[t] = i;
            sh.row_node[t] = u;
            sh.row_e0[t] = e0;
            sh.row_e1[t] = e1;
            sh.row_start[t] = start;
            __syncthreads();
            const int nrows = (f1 - base < NT) ? (f1 - base) : NT;
            for (int j = t; j < total; j += NT) {
                int lo = 0, hi = nrows - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (sh.row_start[mid] <= j) lo = mid; else hi = mid - 1;
                }
                const int re0 = sh.row_e0[lo];
                const int re1 = sh.row_e1[lo];
                const int ulid = sh.row_lid[lo];
                const int32_t unode = sh.row_node[lo];
                const uint32_t blk = (uint32_t)(re0 >> 2) + (uint32_t)(j - sh.row_start[lo]);
                const uint4 coin = philox_block(blk, w, q.key0, q.key1);
                const int4 cv = *reinterpret_cast<const int4*>(g.col + 4 * (size_t)blk);
                const uint4 tv = *reinterpret_cast<const uint4*>(g.thr + 4 * (size_t)blk);
                const int ebase = (int)(4 * blk);
                const int32_t vv[4] = {cv.x, cv.y, cv.z, cv.w};
                const uint32_t tt[4] = {tv.x, tv.y, tv.z, tv.w};
                const uint32_t cc[4] = {coin.x, coin.y, coin.z, coin.w};
#pragma unroll
                for (int qd = 0; qd < 4; ++qd) {
                    const int e = ebase + qd;
                    if (e < re0 || e >= re1) continue;
                    const uint32_t th = tt[qd];
                    if (!(th == kAlwaysLive || cc[qd] < th)) continue;
                    const int32_t v = vv[qd];
                    if (v == unode || bit_set(q.excl, v)) continue;
                    const int lid = st.claim(v, &sh.count);
                    if (lid >= 0) {
                        st.nodes[lid] = v;
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
            }
            __syncthreads();
            if (sh.overflow) break;
        }
        if (sh.overflow) break;
        if (nlev + 1 > st.cap_lv()) {
            sh.overflow = 1;  // every thread sees the same nlev: uniform
            break;
        }
        if (t == 0) st.lvl[nlev + 1] = sh.count;
        __syncthreads();
        ++nlev;
    }
    __syncthreads();
    if (sh.overflow) return false;
    // The last closed level is empty: levels 0..nlev-2 hold nodes.
    const int nlevels = nlev - 1;
    const int R = sh.count;
    const int nx = sh.n_extra;

    // ---- dominators
    for (int x = t; x < nx; x += NT) st.xv[x] = st.lookup(st.xv[x]);
    for (int i = t; i < R; i += NT) {
        const int p = st.get_parent(i);
        st.set_idom(i, p);
        st.aux[i] = p;
    }
    if (t == 0) sh.nonfwd = 0;
    __syncthreads();
    for (int x = t; x < nx; x += NT) {
        // forward edge: u sits exactly one level above v
        const int v = st.xv[x];
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
        // Each pass that changes anything lowers some idom index, so the loop
        // ends; the cap only guards against a broken invariant.
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
                    const int v = st.xv[x];
                    if (v < v0 || v >= v1) continue;
                    int a = st.get_parent(v);
                    int b = st.get_xu(x);
                    while (a != b) {
                        if (a > b) a = st.get_idom(a); else b = st.get_idom(b);
                    }
                    atomicMin(&st.aux[v], a);
                }
                __syncthreads();
                for (int x = t; x < nx; x += NT) {
                    const int v = st.xv[x];
                    if (v < v0 || v >= v1) continue;
                    const int nv = st.aux[v];
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

    // ---- subtree sizes, deepest level first
    for (int i = t; i < R; i += NT) st.aux[i] = 1;
    __syncthreads();
    for (int L = nlevels - 1; L >= 1; --L) {
        for (int i = st.lvl[L] + t; i < st.lvl[L + 1]; i += NT) {
            const int p = st.get_idom(i);
            if (p >= 0) atomicAdd(&st.aux[p], st.aux[i]);
        }
        __syncthreads();
    }

    // ---- outputs
    const int len = R - ns;
    if (t == 0) sh.pair_base = atomicAdd(&ctl->pair_count, (unsigned long long)len);
    __syncthreads();
    const unsigned long long pb = sh.pair_base;
    if (pb + (unsigned long long)len <= out.pair_cap) {
        for (int i = t; i < len; i += NT) {
            out.pair_node[pb + i] = st.nodes[ns + i];
            out.pair_cnt[pb + i] = st.aux[ns + i];
        }
    } else if (t == 0) {
        atomicOr(&ctl->flags, (uint32_t)kFlagPairOverflow);
    }
    long long s = 0;
    for (int i = t; i < R; i += NT) s += st.nodes[i];
    s = block_sum_ll<NT>(s, sh.sum_tmp);
    if (t == 0) {
        if (out.world_size) out.world_size[wi] = R;
        if (out.world_sum) out.world_sum[wi] = s;
        if (out.world_edges) out.world_edges[wi] = sh.edges;
    }
    return true;
}

// ------------------------------------------------------- world kernels
constexpr int kSmallNT = 64;
constexpr int kBigNT = 256;

__global__ __launch_bounds__(kSmallNT) void k_world_small(GraphDev g, QueryDev q, RoundCtl* ctl,
                                                          uint32_t w_begin, uint32_t w_count,
                                                          TileOut out) {
    __shared__ SmallStore st;
    __shared__ WorldShared<kSmallNT> sh;
    const int t = threadIdx.x;
    for (int i = t; i < SmallStore::kHash; i += kSmallNT) st.keys[i] = -1;
    __syncthreads();
    for (;;) {
        if (t == 0) sh.widx = (int)atomicAdd(&ctl->next_world, 1u);
        __syncthreads();
        const uint32_t wi = (uint32_t)sh.widx;
        if (wi >= w_count) break;
        const bool ok = evaluate_world<kSmallNT>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) {
            const uint32_t pos = atomicAdd(&ctl->n_big, 1u);
            out.big_list[pos] = (int32_t)wi;
        }
        st.reset<kSmallNT>(0);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBigNT) void k_world_big(GraphDev g, QueryDev q, RoundCtl* ctl,
                                                      uint32_t w_begin, TileOut out, BigSlots bs) {
    __shared__ WorldShared<kBigNT> sh;
    const int t = threadIdx.x;
    const size_t slot = blockIdx.x;
    const size_t n = (size_t)g.n;
    BigStore st;
    st.lid_of = bs.lid_of + slot * n;
    st.nodes = bs.nodes + slot * n;
    st.parent_ = bs.parent + slot * n;
    st.idom_ = bs.idom + slot * n;
    st.aux = bs.aux + slot * n;
    st.lvl = bs.lvl + slot * (n + 3);
    st.xv = bs.xv + slot * (size_t)bs.xcap;
    st.xu_ = bs.xu + slot * (size_t)bs.xcap;
    st.cap_r_ = g.n;
    st.cap_lv_ = g.n + 1;
    st.cap_x_ = bs.xcap;
    const uint32_t n_big = ctl->n_big;
    for (;;) {
        if (t == 0) sh.widx = (int)atomicAdd(&ctl->next_big, 1u);
        __syncthreads();
        const uint32_t k = (uint32_t)sh.widx;
        if (k >= n_big) break;
        const uint32_t wi = (uint32_t)out.big_list[k];
        const bool ok = evaluate_world<kBigNT>(g, q, ctl, w_begin + wi, wi, out, st, sh);
        if (!ok && t == 0) atomicOr(&ctl->flags, (uint32_t)kFlagBigCapacity);
        __syncthreads();
        st.reset<kBigNT>(sh.count < g.n ? sh.count : g.n);
        __syncthreads();
    }
}

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
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, size_t c, hipStream_t s) { return fill(p, v, c, s); }
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
    ctl->total = 0;
    ctl->best_gain = 0;
}
__global__ void k_ctl_reset_tile(RoundCtl* ctl) {
    ctl->next_world = 0;
    ctl->n_big = 0;
    ctl->next_big = 0;
    ctl->pair_count = 0;
}
hipError_t launch_ctl_reset_round(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_round<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}
hipError_t launch_ctl_reset_tile(RoundCtl* ctl, hipStream_t s) {
    k_ctl_reset_tile<<<1, 1, 0, s>>>(ctl);
    return hipGetLastError();
}

int small_world_cap() { return kSmallCap; }
int small_world_blocks_per_cu() {
    const size_t lds = sizeof(SmallStore) + sizeof(WorldShared<kSmallNT>);
    int b = (int)((160 * 1024) / lds);
    return b < 1 ? 1 : b;
}

hipError_t launch_world_small(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin,
                              uint32_t w_count, const TileOut& out, int grid, hipStream_t s) {
    k_world_small<<<grid, kSmallNT, 0, s>>>(g, q, ctl, w_begin, w_count, out);
    return hipGetLastError();
}

hipError_t launch_world_big(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin,
                            const TileOut& out, const BigSlots& bs, hipStream_t s) {
    k_world_big<<<bs.n_slots, kBigNT, 0, s>>>(g, q, ctl, w_begin, out, bs);
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

__global__ __launch_bounds__(kRedNT) void k_hist(const RoundCtl* ctl, const int32_t* pair_node,
                                                 unsigned long long cap, ReduceBufs rb) {
    __shared__ int h[kMaxBuckets];
    unsigned long long P = ctl->pair_count;
    if (P > cap || (ctl->flags & kFlagPairOverflow)) P = 0;
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT) h[i] = 0;
    __syncthreads();
    unsigned long long a, b;
    chunk_range(P, rb.g1, blockIdx.x, a, b);
    for (unsigned long long i = a + threadIdx.x; i < b; i += kRedNT)
        atomicAdd(&h[pair_node[i] >> kBucketShift], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT) rb.hist[(size_t)i * rb.g1 + blockIdx.x] = h[i];
}

// single-workgroup exclusive scan of hist[0 .. nb*g1) in place; hist[nb*g1] = total
__global__ __launch_bounds__(1024) void k_scan(ReduceBufs rb) {
    __shared__ int tmp[16];
    __shared__ int carry;
    const int total = rb.nb * rb.g1;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < total; base += 1024 * 4) {
        int v[4];
        int loc = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int i = base + threadIdx.x * 4 + k;
            v[k] = (i < total) ? rb.hist[i] : 0;
            loc += v[k];
        }
        int tot;
        const int ex = block_excl_scan<1024>(loc, tmp, tot);
        int run = carry + ex;
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
    __shared__ int cur[kMaxBuckets];
    unsigned long long P = ctl->pair_count;
    if (P > cap || (ctl->flags & kFlagPairOverflow)) P = 0;
    for (int i = threadIdx.x; i < rb.nb; i += kRedNT) cur[i] = rb.hist[(size_t)i * rb.g1 + blockIdx.x];
    __syncthreads();
    unsigned long long a, b;
    chunk_range(P, rb.g1, blockIdx.x, a, b);
    for (unsigned long long i = a + threadIdx.x; i < b; i += kRedNT) {
        const int32_t v = pair_node[i];
        const int pos = atomicAdd(&cur[v >> kBucketShift], 1);
        rb.sorted_node[pos] = v;
        rb.sorted_cnt[pos] = pair_cnt[i];
    }
}

__global__ __launch_bounds__(kRedNT) void k_accum(int32_t n, ReduceBufs rb) {
    __shared__ unsigned long long acc[1 << kBucketShift];
    const int bucket = blockIdx.x / rb.slices;
    const int slice = blockIdx.x % rb.slices;
    for (int i = threadIdx.x; i < (1 << kBucketShift); i += kRedNT) acc[i] = 0ull;
    __syncthreads();
    const long long bs = rb.hist[(size_t)bucket * rb.g1];
    const long long be = (bucket + 1 < rb.nb) ? rb.hist[(size_t)(bucket + 1) * rb.g1] : rb.hist[(size_t)rb.nb * rb.g1];
    const long long len = be - bs;
    const long long a = bs + len * slice / rb.slices;
    const long long b = bs + len * (slice + 1) / rb.slices;
    const int32_t node0 = bucket << kBucketShift;
    for (long long i = a + threadIdx.x; i < b; i += kRedNT)
        atomicAdd(&acc[rb.sorted_node[i] - node0], (unsigned long long)(long long)rb.sorted_cnt[i]);
    __syncthreads();
    int64_t* out = rb.part + (size_t)slice * ((size_t)rb.nb << kBucketShift) + ((size_t)bucket << kBucketShift);
    for (int i = threadIdx.x; i < (1 << kBucketShift); i += kRedNT) out[i] = (int64_t)acc[i];
    (void)n;
}

__global__ void k_sum_slices(int32_t n, ReduceBufs rb, int64_t* gain) {
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
    k_scan<<<1, 1024, 0, s>>>(rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_scatter<<<rb.g1, kRedNT, 0, s>>>(ctl, out.pair_node, out.pair_cnt, out.pair_cap, rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_accum<<<rb.nb * rb.slices, kRedNT, 0, s>>>(g.n, rb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_sum_slices<<<1024, 256, 0, s>>>(g.n, rb, gain);
    return hipGetLastError();
}

__global__ void k_sum_sizes(const int32_t* ws, uint32_t count, RoundCtl* ctl) {
    __shared__ long long tmp[4];
    long long s = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        s += ws[i];
    s = block_sum_ll<256>(s, tmp);
    if (threadIdx.x == 0 && s) atomicAdd((unsigned long long*)&ctl->total, (unsigned long long)s);
}

hipError_t launch_sum_sizes(const int32_t* ws, uint32_t count, RoundCtl* ctl, hipStream_t s) {
    unsigned blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (blocks == 0) return hipSuccess;
    k_sum_sizes<<<blocks, 256, 0, s>>>(ws, count, ctl);
    return hipGetLastError();
}

// ----------------------------------------------------------- selection
// argmax over candidates (not seeds, not blocked) of (gain desc, id asc).
__device__ __forceinline__ bool better(int64_t g1, int32_t u1, int64_t g2, int32_t u2) {
    if (u2 < 0) return u1 >= 0;
    if (u1 < 0) return false;
    return g1 > g2 || (g1 == g2 && u1 < u2);
}

__global__ __launch_bounds__(256) void k_select_partial(int32_t n, const int64_t* gain, const uint32_t* excl,
                                                        int64_t* pg, int32_t* pu) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    int64_t bg = 0;
    int32_t bu = -1;
    for (int32_t u = blockIdx.x * 256 + threadIdx.x; u < n; u += gridDim.x * 256) {
        if (bit_set(excl, u)) continue;
        const int64_t gv = gain[u];
        if (better(gv, u, bg, bu)) { bg = gv; bu = u; }
    }
    sg[threadIdx.x] = bg;
    su[threadIdx.x] = bu;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            const int o = threadIdx.x + d;
            if (better(sg[o], su[o], sg[threadIdx.x], su[threadIdx.x])) {
                sg[threadIdx.x] = sg[o];
                su[threadIdx.x] = su[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pg[blockIdx.x] = sg[0];
        pu[blockIdx.x] = su[0];
    }
}

__global__ __launch_bounds__(256) void k_select_final(int parts, const int64_t* pg, const int32_t* pu,
                                                      uint32_t* excl, RoundCtl* ctl, int32_t k,
                                                      int32_t* blockers, int64_t* gains,
                                                      int64_t* totals, int32_t* n_selected) {
    __shared__ int64_t sg[256];
    __shared__ int32_t su[256];
    int64_t bg = 0;
    int32_t bu = -1;
    for (int i = threadIdx.x; i < parts; i += 256)
        if (better(pg[i], pu[i], bg, bu)) { bg = pg[i]; bu = pu[i]; }
    sg[threadIdx.x] = bg;
    su[threadIdx.x] = bu;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) {
            const int o = threadIdx.x + d;
            if (better(sg[o], su[o], sg[threadIdx.x], su[threadIdx.x])) {
                sg[threadIdx.x] = sg[o];
                su[threadIdx.x] = su[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x != 0 || ctl->stop) return;
    const int r = ctl->round;
    const long long T = ctl->total;
    if (ctl->expect_total >= 0 && ctl->expect_total != T) atomicOr(&ctl->flags, (uint32_t)kFlagSpreadMismatch);
    totals[r] = T;
    const int32_t u = su[0];
    const int64_t gbest = sg[0];
    if (r >= k || u < 0 || gbest <= 0) {
        ctl->stop = 1;
        *n_selected = r;
        return;
    }
    blockers[r] = u;
    gains[r] = gbest;
    excl[u >> 5] |= 1u << (u & 31);
    ctl->ustar = u;
    ctl->best_gain = gbest;
    ctl->round = r + 1;
    ctl->expect_total = T - gbest;
    if (r + 1 == k) {
        // T_k follows exactly from T_{k-1} - gain_{k-1}
        totals[k] = T - gbest;
        ctl->stop = 1;
        *n_selected = k;
    }
}

hipError_t launch_select(const GraphDev& g, const int64_t* gain, uint32_t* excl, RoundCtl* ctl,
                         int64_t* part_gain, int32_t* part_node, int parts, int32_t k,
                         int32_t* blockers, int64_t* gains, int64_t* totals, int32_t* n_selected,
                         hipStream_t s) {
    k_select_partial<<<parts, 256, 0, s>>>(g.n, gain, excl, part_gain, part_node);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_select_final<<<1, 256, 0, s>>>(parts, part_gain, part_node, excl, ctl, k, blockers, gains, totals,
                                     n_selected);
    return hipGetLastError();
}

} // namespace imin
