// Host side of the C ABI declared in include/imin.h.
#include "imin.h"
#include "imin_internal.hpp"
#include "imin_select.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

struct imin_graph {
    imin::GraphDev g;
    int device;
    // bump-region entries per world (1/1024 units) that earlier calls on this
    // graph needed, for worlds beyond tier 0's slots and for their extra
    // edges: later calls size their scratch from them and need not redo a
    // tile whose worlds overflowed it
    std::atomic<uint64_t> big_per_world{0};
    std::atomic<uint64_t> xbig_per_world{0};
    // shares of a pass's worlds (1/1024 units) that earlier calls handed on
    // to tier 1 and to tier 2: a call starts its worlds at the tier most of
    // them end up in
    std::atomic<uint64_t> tier1_share{0};
    std::atomic<uint64_t> tier2_share{0};
    std::atomic<bool> tier2_seen{false};  // some world of an earlier call needed the HBM tier
    // the same four figures as raised on the device by enqueued solves
    // (bump entries and extra edges per world, tier-1 and tier-2 shares)
    unsigned long long* hints_dev = nullptr;
    // launch shape chosen by imin_autotune: the tier-0 world launch's
    // workgroups in percent of its LDS residency (0: the default, 100)
    std::atomic<int32_t> tuned_grid0_pct{0};
    // made on first use and kept until destroy: host copies of the graph and
    // the in-edges on the device (Global Sampling)
    std::mutex aux_mu;
    std::unique_ptr<imin::HostGraph> host;
    int32_t* in_off = nullptr;
    int4* in_rec = nullptr;
    // Global Sampling's slots (a stamp and a list entry per node, an epoch
    // per slot), kept from one call to the next under aux_mu and lent to one
    // call at a time: a slot's epoch only grows, so its stamps stay valid and
    // a later call starts without clearing them
    int32_t* lrr_stamp = nullptr;
    int32_t* lrr_list = nullptr;
    int32_t* lrr_epoch = nullptr;
    size_t lrr_slots = 0;
    uint64_t lrr_epoch_bound = 0;  // no slot's epoch is above it
    bool lrr_lent = false;
    // V'_s of the last seed set (sorted) Global Sampling was called with
    bool vp_valid = false;
    std::vector<int32_t> vp_seeds;
    std::vector<int32_t> vp_nodes;
};

namespace {
void raise_hint(std::atomic<uint64_t>& a, uint64_t v) {
    uint64_t cur = a.load(std::memory_order_relaxed);
    while (v > cur && !a.compare_exchange_weak(cur, v, std::memory_order_relaxed)) {
    }
}
}  // namespace

namespace {

thread_local uint32_t g_last_flags = 0;
// rounds of this thread's last blocking solve: 1 incremental, 0 plain, -1 none
thread_local int32_t g_last_mode = -1;

// ---- optional per-kernel timing with HIP events
constexpr int kTimedKernels = 9;
constexpr int kWorkTiers = 6;  // tiers 0-2, replay, label rule (rule workgroups), label rule (replay workgroups)
struct Timing {
    std::atomic<bool> on{false};
    std::atomic<uint32_t> mask{0xFFFFFFFFu};  // kernels bracketed with events
    std::atomic<int> every{1};                // one launch in `every` of each selected kernel is timed
    std::atomic<bool> tallies{true};          // per-workgroup work tallies, summed at each call's end
    std::atomic<int64_t> seen[kTimedKernels] = {};  // launches of selected kernels, timed or not
    std::mutex mu;
    int64_t launches[kTimedKernels] = {};
    double ms[kTimedKernels] = {};
    int64_t work[kWorkTiers][imin::kWorkFields] = {};
};
Timing g_timing;

// Events are created once and reused across calls.
std::mutex g_event_mu;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t event_acquire() {
    {
        std::lock_guard<std::mutex> lk(g_event_mu);
        if (!g_event_pool.empty()) {
            hipEvent_t e = g_event_pool.back();
            g_event_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void event_release(hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(g_event_mu);
    g_event_pool.push_back(e);
}

// Event pairs recorded by one call, resolved after its final synchronisation.
struct TimedLaunches {
    struct Rec {
        int id;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    bool on = g_timing.on.load();
    uint32_t mask = g_timing.mask.load();
    void record(hipEvent_t e, hipStream_t s) {
        if (hipEventRecord(e, s) != hipSuccess) (void)hipGetLastError();  // best effort: leave no error behind
    }
    int every = g_timing.every.load();
    hipEvent_t begin(int id, hipStream_t s) {
        if (!on || !((mask >> id) & 1u)) return nullptr;
        const int64_t nth = g_timing.seen[id].fetch_add(1);
        if (every > 1 && nth % every != 0) return nullptr;
        hipEvent_t e = event_acquire();
        if (e) record(e, s);
        return e;
    }
    // Events for a launch that records them itself, around exactly its
    // kernel (null when this launch is not timed); then taken() after it.
    imin::LaunchEvents take(int id) {
        imin::LaunchEvents ev;
        if (!on || !((mask >> id) & 1u)) return ev;
        const int64_t nth = g_timing.seen[id].fetch_add(1);
        if (every > 1 && nth % every != 0) return ev;
        ev.start = event_acquire();
        ev.stop = ev.start ? event_acquire() : nullptr;
        if (!ev.stop) {
            event_release(ev.start);
            ev.start = nullptr;
        }
        return ev;
    }
    void taken(int id, const imin::LaunchEvents& ev) {
        if (ev.start) recs.push_back({id, ev.start, ev.stop});
    }
    void end(int id, hipEvent_t a, hipStream_t s) {
        if (!on || !a) return;
        hipEvent_t e = event_acquire();
        if (!e) {
            event_release(a);
            return;
        }
        record(e, s);
        recs.push_back({id, a, e});
    }
    void flush() {
        if (recs.empty()) return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        for (auto& r : recs) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                g_timing.launches[r.id] += 1;
                g_timing.ms[r.id] += ms;
            }
            event_release(r.a);
            event_release(r.b);
        }
        recs.clear();
    }
    ~TimedLaunches() { flush(); }
};

imin_status_t from_hip(hipError_t e) {
    if (e == hipSuccess) return IMIN_OK;
    return e == hipErrorOutOfMemory ? IMIN_ERR_NOMEM : IMIN_ERR_DEVICE;
}

// With IMIN_DEBUG set in the environment, a failing runtime call is named
// on stderr.
void report_hip(const char* what, hipError_t e) {
    static const bool on = std::getenv("IMIN_DEBUG") != nullptr;
    if (on) std::fprintf(stderr, "imin: %s failed: %s\n", what, hipGetErrorString(e));
}

#define IMIN_TRY(expr)                                  \
    do {                                                \
        const hipError_t imin_e_ = (expr);              \
        if (imin_e_ != hipSuccess) {                    \
            report_hip(#expr, imin_e_);                 \
            return from_hip(imin_e_);                   \
        }                                               \
    } while (0)

size_t env_size(const char* name, size_t dflt) {
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    char* end = nullptr;
    const unsigned long long x = std::strtoull(v, &end, 10);
    return (end && *end == '\0' && x > 0) ? (size_t)x : dflt;
}

// Device blocks kept between calls, per device.  Freeing gigabytes costs
// milliseconds per call (and the next call of the same query allocates the
// same sizes again), so released blocks stay cached up to a limit
// (IMIN_CACHE_BYTES, default 64 GiB; imin_cache_release frees them).  A block
// is handed out again for a request of at least half its size.  Blocks that a
// call releases while its stream may still use them wait in the call's
// ReleaseScope until the stream has drained.
struct BlockCache {
    std::mutex mu;
    std::map<int, std::multimap<size_t, void*>> free_blocks;
    size_t cached = 0;
    size_t limit = env_size("IMIN_CACHE_BYTES", (size_t)64 << 30);

    void* get(int dev, size_t bytes, size_t& got) {
        {
            std::lock_guard<std::mutex> lk(mu);
            auto& m = free_blocks[dev];
            auto it = m.lower_bound(bytes);
            if (it != m.end() && it->first / 2 <= bytes) {
                got = it->first;
                void* p = it->second;
                m.erase(it);
                cached -= got;
                return p;
            }
        }
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            release_device(dev);  // cached blocks may be what is missing
            if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        }
        got = bytes;
        return p;
    }
    void put(int dev, void* p, size_t bytes) {
        std::lock_guard<std::mutex> lk(mu);
        auto& m = free_blocks[dev];
        m.emplace(bytes, p);
        cached += bytes;
        while (cached > limit && !m.empty()) {  // the largest blocks go first
            auto it = std::prev(m.end());
            (void)hipFree(it->second);
            cached -= it->first;
            m.erase(it);
        }
    }
    void release_device(int dev) {
        std::lock_guard<std::mutex> lk(mu);
        free_locked(dev);
    }
    void release_all() {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& dm : free_blocks) free_locked(dm.first);
    }
    // frees every cached block of one device with that device current
    void free_locked(int dev) {
        auto& m = free_blocks[dev];
        if (m.empty()) return;
        int cur = dev;
        (void)hipGetDevice(&cur);
        if (cur != dev) (void)hipSetDevice(dev);
        for (auto& kv : m) {
            (void)hipFree(kv.second);
            cached -= kv.first;
        }
        m.clear();
        if (cur != dev) (void)hipSetDevice(cur);
    }
};
BlockCache g_cache;

struct CachedBlock {
    int dev;
    void* p;
    size_t bytes;
};
thread_local std::vector<CachedBlock>* t_deferred = nullptr;

// Blocks released during one call on one stream; they enter the cache once
// the owner has synchronised that stream (the scope's end).
struct ReleaseScope {
    std::vector<CachedBlock> blocks;
    std::vector<CachedBlock>* prev;
    ReleaseScope() : prev(t_deferred) { t_deferred = &blocks; }
    ReleaseScope(const ReleaseScope&) = delete;
    ReleaseScope& operator=(const ReleaseScope&) = delete;
    ~ReleaseScope() {
        t_deferred = prev;
        for (auto& b : blocks) g_cache.put(b.dev, b.p, b.bytes);
    }
};

// A caller's workspace, handed out in 256-byte-aligned pieces in the order
// they are asked for; nothing is given back.  Without a base it only adds up
// the sizes (the workspace size of a plan).
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    bool failed = false;
    void* take(size_t bytes) {
        const size_t at = (used + 255) & ~(size_t)255;
        used = at + bytes;
        if (!base) return reinterpret_cast<void*>((uintptr_t)256);  // sizing only: never dereferenced
        if (used > size) {
            failed = true;
            return nullptr;
        }
        return base + at;
    }
};
thread_local Arena* t_arena = nullptr;

// While alive, DevArray allocations of this thread come from the arena.
struct ArenaScope {
    Arena* prev;
    explicit ArenaScope(Arena* a) : prev(t_arena) { t_arena = a; }
    ~ArenaScope() { t_arena = prev; }
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;
};

// Device allocation owned by a scope; its block returns to the cache (or,
// taken from a caller's workspace, is simply dropped).
template <class T>
struct DevArray {
    T* p = nullptr;
    size_t count = 0;
    size_t bytes = 0;  // the block's size
    int dev = 0;
    bool borrowed = false;  // a piece of a caller's workspace
    DevArray() = default;
    DevArray(const DevArray&) = delete;
    DevArray& operator=(const DevArray&) = delete;
    ~DevArray() { release(); }
    void release() {
        if (p && !borrowed) {
            if (t_deferred)
                t_deferred->push_back({dev, p, bytes});
            else
                g_cache.put(dev, p, bytes);
        }
        p = nullptr;
        count = 0;
        bytes = 0;
        borrowed = false;
    }
    hipError_t alloc(size_t c) {
        release();
        if (t_arena) {
            void* q = t_arena->take(std::max<size_t>(c, 1) * sizeof(T));
            if (!q) return hipErrorOutOfMemory;
            p = static_cast<T*>(q);
            count = c;
            bytes = std::max<size_t>(c, 1) * sizeof(T);
            borrowed = true;
            return hipSuccess;
        }
        if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
        void* q = g_cache.get(dev, std::max<size_t>(c, 1) * sizeof(T), bytes);
        if (!q) return hipErrorOutOfMemory;
        p = static_cast<T*>(q);
        count = c;
        return hipSuccess;
    }
    void swap(DevArray& o) {
        std::swap(p, o.p);
        std::swap(count, o.count);
        std::swap(bytes, o.bytes);
        std::swap(dev, o.dev);
        std::swap(borrowed, o.borrowed);
    }
};

// Pinned host copies of the round counters, reused across calls.
std::mutex g_pinned_mu;
std::vector<imin::RoundCtl*> g_pinned;

struct HostCtl {
    imin::RoundCtl* p = nullptr;
    hipError_t get() {
        {
            std::lock_guard<std::mutex> lk(g_pinned_mu);
            if (!g_pinned.empty()) {
                p = g_pinned.back();
                g_pinned.pop_back();
                return hipSuccess;
            }
        }
        return hipHostMalloc((void**)&p, sizeof(imin::RoundCtl), hipHostMallocDefault);
    }
    ~HostCtl() {
        if (!p) return;
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        g_pinned.push_back(p);
    }
};

int cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

// How an enqueued solve lays out its workspace.
// The tier-0 world launch's workgroups, in percent of its LDS residency,
// unless the graph's handle holds a tuned shape: twice the residency, whose
// workgroups take smaller chunks of worlds as a pass ends (about 10% less
// tier-0 time than once the residency on the 1M-node trivalency workload).
constexpr int32_t kDefaultGrid0Pct = 200;

struct WsPlan {
    bool incremental = true;  // resident store and node index (else every round evaluates all worlds)
    size_t big_cap = 0;       // bump-region entries for worlds beyond tier 0 (and as many extra edges)
    size_t slots = 1;         // tier-2 slots (bounded per-world arrays)
    size_t slots3 = 1;        // tier-3 slots (any world), when some world can outgrow tier 2
    int32_t chunk_cap = 1;    // level-0 table entries
    int start_tier = 0;
};

// Everything one query needs on the device besides the graph.
struct Session {
    const imin::GraphDev& g;
    hipStream_t s;
    ReleaseScope scope;  // destroyed after every array below, and after the destructor's synchronisation
    DevArray<uint32_t> excl;
    DevArray<int64_t> gain;
    DevArray<imin::RoundCtl> ctl;
    HostCtl hctl;
    // per-world outputs of a tile: sizes, scratch locations and lengths
    DevArray<int32_t> world_size;
    DevArray<int64_t> wloc;
    DevArray<int32_t> wlen;
    DevArray<int32_t> scr_node, scr_cnt;  // per-world scratch (fixed tier-0 slots + bump region)
    size_t slot_cap0 = 0, big_cap = 0;
    DevArray<int32_t> list0, list1, list2, list3, list4;  // changed worlds; worlds handed on (RoundCtl::list_n)
    // the gain reduction's buffers (bucket counts, bases, cursors, records)
    DevArray<long long> g_bcnt, g_bbase, g_bcur;
    DevArray<int2> g_rec;
    imin::GainBufs gb{};
    // resident per-world (node, count) lists for incremental rounds
    DevArray<int32_t> store_node, store_cnt, store_len;
    DevArray<int64_t> store_off;
    // replay of changed worlds from their stored live edges: BFS parents
    // beside the pairs, extra edges (local ids) in a store of their own
    bool replay = false;
    bool label_rule = true;  // changed worlds updated from their labels where the rule holds (with replay)
    DevArray<int32_t> scr_par, xscr_v, xscr_u, xlen;
    DevArray<int64_t> xloc;
    size_t xslot_cap0 = 0, xbig_cap = 0;
    DevArray<int32_t> store_par, xstore_v, xstore_u, xstore_len;
    DevArray<int64_t> xstore_off;
    // dominator-tree labels and the labelled flag per world (with replay)
    DevArray<int32_t> scr_lab, store_lab;
    DevArray<uint8_t> world_flags;
    // nodes lost per (kernel, workgroup) in incremental rounds
    DevArray<long long> dsz;
    int32_t dsz_n = 0;
    int32_t dsz_off[7] = {0, 0, 0, 0, 0, 0, 0};
    int grid_l = 0;
    bool adopted = false;                  // the round-0 scratch serves as the store
    unsigned long long adopted_entries = 0;
    bool indexed = false;                  // idx_off / idx_ent hold the index
    int rule_lanes = 16;  // lanes per world in the label rule
    int grid_r = 0;
    int grid_w = 0;  // wide-replay workgroups
    bool incremental = false;
    size_t store_budget = 0;
    // node -> stored entries (position, world), built after round 0
    DevArray<uint32_t> idx_off, idx_bcnt, idx_bbase, idx_bcur;  // positions and offsets: uint32
    DevArray<int32_t> idx_border;
    DevArray<int4> idx_rec;  // the index build's entries grouped by bucket
    DevArray<int2> idx_ent;  // (store position, world) of each entry, grouped by node
    // level-0 slot groups of the seeds, with their columns and thresholds;
    // the query's thresholds (0 where the head is excluded)
    DevArray<int32_t> seed_cnt;
    DevArray<int4> seed_table, seed_col;
    DevArray<uint4> seed_thr;
    DevArray<uint32_t> thr_q;
    // HBM world tier
    // HBM-tier slots: tier 2's hold worlds of up to 2^16 nodes and 2^16
    // extra edges (many slots), tier 3's any world of the graph (a few)
    struct Slots {
        DevArray<int32_t> lid, nodes, parent, idom, aux, tin, lvl, xv, xu, xv2, xu2;
        DevArray<uint32_t> vis;
        imin::BigSlots bs{};
        bool ready() const { return lid.p != nullptr; }
    };
    Slots t2, t3;
    imin::BigSlots bs{};
    // selection
    DevArray<int64_t> sel_g;
    DevArray<int32_t> sel_u;
    DevArray<long long> sel_d;
    int sel_parts = 0;
    // per-workgroup work tallies
    DevArray<unsigned long long> work;
    int work_stride = 0;
    size_t tile_cap = 0;   // worlds per tile (buffer size)
    size_t tile = 0;       // worlds per tile in use
    int grid0 = 0, grid1 = 0;
    int start_tier = 0;    // first tier tried for every world of a tile
    // Some world of the from-scratch pass needed the HBM tier.  Worlds only
    // shrink as blockers are added and the large LDS tier holds any world
    // that fitted it before, so without such a world incremental rounds
    // never reach the HBM tier and do not launch it.
    bool any_tier2 = false;
    bool any_tier3 = false;  // likewise for the worlds tier 2's slots cannot hold
    bool replay_complete = false;  // every stored world fits the replay
    int last_tier() const { return any_tier3 ? 3 : (any_tier2 ? 2 : 1); }
    // Enqueue-only: every array is a piece of the caller's workspace, and
    // nothing is read back or waited for on the host.
    bool ws = false;
    TimedLaunches timed;
    // lower-bound coverage: the worlds' dominator trees as the store
    // (kCoverStore), or the coverage of the marked set cover_mark counted
    // per world (kCoverCount); unit_counts: every entry counts 1 (reach counts)
    int cover = imin::kCoverNone;
    const uint32_t* cover_mark = nullptr;
    int unit_counts = 0;
    int sizes_only = 0;  // |R_w| per world only
    // Global Sampling: samples are LRR sets (Algorithm 3) instead of worlds
    bool lrr = false;
    imin::LrrDev lrr_dev{};
    DevArray<int32_t> lrr_stamp, lrr_list, lrr_epoch, lrr_vprime;
    imin_graph* lrr_from = nullptr;  // the graph whose kept slots this call borrowed
    uint64_t lrr_epoch_bound = 0;    // no slot's epoch is above it

    // Stamps are int32 (2 * epoch + 2), so the slots are cleared before an
    // epoch could pass this.
    static constexpr uint64_t kLrrEpochLimit = (uint64_t)1 << 29;

    // the sampling slots and V'_s of Global Sampling: as many slots as
    // IMIN_LRR_BUDGET (default the smaller of 16 GiB and a quarter of the
    // free device memory) allows at 8 bytes per node, at most 32 per compute
    // unit (a sample is one wave and mostly waits on dependent loads, so many
    // are kept in flight).  The graph keeps its slots for later calls; a call
    // that finds them lent to another takes its own.
    imin_status_t setup_lrr(imin_graph_t h, const std::vector<int32_t>& vprime) {
        const int32_t* in_off = nullptr;
        const int4* in_rec = nullptr;
        if (!imin::graph_in_edges(h, &in_off, &in_rec)) return IMIN_ERR_NOMEM;
        const size_t n = (size_t)g.n;
        int32_t *stamp = nullptr, *list = nullptr, *epoch = nullptr;
        size_t slots = 0;
        {
            std::lock_guard<std::mutex> lk(h->aux_mu);
            if (!h->lrr_lent) {
                if (h->lrr_slots == 0) {
                    size_t free_b = 0, total_b = 0;
                    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                        (void)hipGetLastError();
                        return IMIN_ERR_DEVICE;
                    }
                    const size_t budget = env_size("IMIN_LRR_BUDGET", std::min<size_t>((size_t)16 << 30, free_b / 4));
                    const size_t want =
                        std::max<size_t>(1, std::min<size_t>(budget / (8 * n), (size_t)cu_count() * 32));
                    if (hipMalloc((void**)&h->lrr_stamp, want * n * sizeof(int32_t)) != hipSuccess ||
                        hipMalloc((void**)&h->lrr_list, want * n * sizeof(int32_t)) != hipSuccess ||
                        hipMalloc((void**)&h->lrr_epoch, want * sizeof(int32_t)) != hipSuccess) {
                        (void)hipGetLastError();
                        if (h->lrr_stamp) (void)hipFree(h->lrr_stamp);
                        if (h->lrr_list) (void)hipFree(h->lrr_list);
                        if (h->lrr_epoch) (void)hipFree(h->lrr_epoch);
                        h->lrr_stamp = h->lrr_list = h->lrr_epoch = nullptr;
                        return IMIN_ERR_NOMEM;
                    }
                    h->lrr_slots = want;
                    h->lrr_epoch_bound = kLrrEpochLimit + 1;  // cleared before the first launch
                }
                h->lrr_lent = true;
                lrr_from = h;
                stamp = h->lrr_stamp;
                list = h->lrr_list;
                epoch = h->lrr_epoch;
                slots = h->lrr_slots;
                lrr_epoch_bound = h->lrr_epoch_bound;
            }
        }
        if (!lrr_from) {
            slots = std::max<size_t>(1, std::min<size_t>(env_size("IMIN_LRR_BUDGET", (size_t)8 << 30) / (8 * n),
                                                         (size_t)cu_count() * 32));
            IMIN_TRY(lrr_stamp.alloc(slots * n));
            IMIN_TRY(lrr_list.alloc(slots * n));
            IMIN_TRY(lrr_epoch.alloc(slots));
            stamp = lrr_stamp.p;
            list = lrr_list.p;
            epoch = lrr_epoch.p;
            lrr_epoch_bound = kLrrEpochLimit + 1;
        }
        IMIN_TRY(lrr_vprime.alloc(std::max<size_t>(vprime.size(), 1)));
        if (!vprime.empty())
            IMIN_TRY(hipMemcpyAsync(lrr_vprime.p, vprime.data(), vprime.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s));
        IMIN_TRY(hipStreamSynchronize(s));  // vprime is a host vector
        lrr_dev.in_off = in_off;
        lrr_dev.in_rec = in_rec;
        lrr_dev.vprime = lrr_vprime.p;
        lrr_dev.nvp = (uint32_t)vprime.size();
        lrr_dev.n_slots = (int32_t)slots;
        lrr_dev.stamp = stamp;
        lrr_dev.list = list;
        lrr_dev.epoch = epoch;
        return IMIN_OK;
    }

    // before a launch of `count` samples, each slot taking at most
    // ceil(count / slots) of them: clear the slots first when an epoch could
    // otherwise pass the limit
    imin_status_t lrr_reserve(uint64_t count) {
        const uint64_t slots = (uint64_t)lrr_dev.n_slots;
        const uint64_t per = (count + slots - 1) / slots;
        if (per > kLrrEpochLimit) return IMIN_ERR_INVALID;
        if (lrr_epoch_bound + per > kLrrEpochLimit) {
            IMIN_TRY(imin::launch_fill_i32(lrr_dev.stamp, 0, (size_t)slots * (size_t)g.n, s));
            IMIN_TRY(imin::launch_fill_i32(lrr_dev.epoch, 0, (size_t)slots, s));
            lrr_epoch_bound = 0;
        }
        lrr_epoch_bound += per;
        return IMIN_OK;
    }

    Session(const imin::GraphDev& gd, hipStream_t st, imin_graph* h = nullptr) : g(gd), s(st), gh(h) {}
    imin_graph* gh;  // per-graph scratch hints (may be null)

    // the scratch a tile of `worlds` worlds is expected to need, from the
    // graph's hint (entries per world in 1/1024 units), with an eighth more;
    // at most 2^28 entries (a tile needing more grows its scratch and is
    // redone, as without a hint)
    size_t hinted(const std::atomic<uint64_t>* hint, size_t worlds, size_t dflt) const {
        if (!hint) return dflt;
        const unsigned long long per = hint->load(std::memory_order_relaxed);
        const unsigned long long need = (per * (unsigned long long)worlds) >> 10;
        const unsigned long long want = std::min<unsigned long long>(need + need / 8 + 1024, 1ull << 34);
        return std::max<size_t>(dflt, (size_t)want);
    }

    // a tile of nw worlds that asked for bc bump-region and xc extra-edge
    // entries raises the graph's hints
    void record_scratch(unsigned long long bc, unsigned long long xc, uint64_t nw) {
        if (!gh || nw == 0) return;
        raise_hint(gh->big_per_world, (uint64_t)((bc << 10) / nw));
        raise_hint(gh->xbig_per_world, (uint64_t)((xc << 10) / nw));
    }
    // the tier a call's worlds start at: the one most worlds of earlier calls
    // on the graph ended up in (IMIN_START_TIER overrides)
    int hinted_start_tier() const {
        if (const char* t = std::getenv("IMIN_START_TIER")) return std::max(0, std::min(2, std::atoi(t)));
        if (!gh) return 0;
        if (gh->tier2_share.load(std::memory_order_relaxed) > 512) return 2;
        if (gh->tier1_share.load(std::memory_order_relaxed) > 512) return 1;
        return 0;
    }
    // an early return may leave work queued: drain it before any block can
    // be handed to another call
    ~Session() {
        bool drained = true;
        if (!ws && hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            drained = false;
        }
        if (lrr_from) {
            // slots whose epochs a failed launch may not have written are
            // cleared before their next use
            std::lock_guard<std::mutex> lk(lrr_from->aux_mu);
            lrr_from->lrr_epoch_bound = drained ? lrr_epoch_bound : kLrrEpochLimit + 1;
            lrr_from->lrr_lent = false;
        }
    }
    Session(const Session&) = delete;
    Session& operator=(const Session&) = delete;

    // Every array of an enqueued solve, taken in a fixed order (so that
    // carving from an arena without a base gives the bytes a plan needs).
    imin_status_t carve(const WsPlan& p, uint64_t theta, int32_t n_seeds) {
        ws = true;
        timed.on = false;
        const size_t n = (size_t)g.n;
        tile_cap = tile = (size_t)theta;
        IMIN_TRY(ctl.alloc(1));
        IMIN_TRY(excl.alloc((n + 31) / 32));
        IMIN_TRY(gain.alloc(n));
        IMIN_TRY(world_size.alloc(theta));
        IMIN_TRY(wloc.alloc(theta));
        IMIN_TRY(wlen.alloc(theta));
        IMIN_TRY(list0.alloc(theta));
        IMIN_TRY(list1.alloc(theta));
        IMIN_TRY(list2.alloc(theta));
        IMIN_TRY(list3.alloc(theta));
        IMIN_TRY(list4.alloc(theta));
        IMIN_TRY(seed_cnt.alloc((size_t)n_seeds));
        IMIN_TRY(seed_table.alloc((size_t)p.chunk_cap));
        IMIN_TRY(seed_col.alloc((size_t)p.chunk_cap));
        IMIN_TRY(seed_thr.alloc((size_t)p.chunk_cap));
        IMIN_TRY(thr_q.alloc((size_t)g.m_pad));
        slot_cap0 = (size_t)imin::world_tier0_capacity();
        big_cap = p.big_cap;
        const size_t scr = tile_cap * slot_cap0 + big_cap;
        IMIN_TRY(scr_node.alloc(scr));
        IMIN_TRY(scr_cnt.alloc(scr));
        gb = imin::gain_buckets(g.n);
        IMIN_TRY(g_bcnt.alloc((size_t)gb.nb));
        IMIN_TRY(g_bbase.alloc((size_t)gb.nb + 1));
        IMIN_TRY(g_bcur.alloc((size_t)gb.nb));
        gb.bcnt = g_bcnt.p;
        gb.bbase = g_bbase.p;
        gb.bcur = g_bcur.p;
        const int cus = cu_count();
        IMIN_TRY(alloc_slots(t2, p.slots, t2_lid_cap(), t2_xcap()));
        if (tier3_possible()) IMIN_TRY(alloc_slots(t3, p.slots3, g.n, std::max<int64_t>(g.m, 1)));
        IMIN_TRY(alloc_grids(cus));
        start_tier = p.start_tier;
        any_tier2 = true;         // whether a world needs the HBM tiers is not known on the host
        any_tier3 = tier3_possible();
        replay_complete = false;  // nor whether every stored world fits the replay
        if (p.incremental) {
            incremental = true;
            replay = true;
            const char* fp = std::getenv("IMIN_LABEL_RULE");
            label_rule = !(fp && fp[0] == '0');
            xslot_cap0 = (size_t)imin::world_tier0_xcapacity();
            xbig_cap = big_cap;
            IMIN_TRY(scr_par.alloc(scr));
            IMIN_TRY(scr_lab.alloc(scr));
            IMIN_TRY(xscr_v.alloc(tile_cap * xslot_cap0 + xbig_cap));
            IMIN_TRY(xscr_u.alloc(tile_cap * xslot_cap0 + xbig_cap));
            IMIN_TRY(xloc.alloc(theta));
            IMIN_TRY(xlen.alloc(theta));
            IMIN_TRY(world_flags.alloc((theta + 3) & ~(uint64_t)3));
            IMIN_TRY(alloc_index(scr));  // every scratch entry can be indexed
        } else {
            IMIN_TRY(g_rec.alloc(scr));
        }
        return IMIN_OK;
    }

    // One from-scratch pass of an enqueued solve over all theta worlds (one
    // tile) under the current exclusions; round 0 of an incremental solve
    // keeps its scratch as the resident store and builds the node index,
    // whose pass also yields the gains.
    imin_status_t pass_ws(const imin::QueryDev& q, uint64_t theta, bool round0, unsigned long long* hints) {
        const bool keep = round0 && incremental;
        IMIN_TRY(imin::launch_query_thresholds(g, excl.p, thr_q.p, seed_table.p, ctl.p, q.seed_cap, seed_col.p,
                                               seed_thr.p, s));
        IMIN_TRY(imin::launch_ctl_reset_tile(ctl.p, s));
        imin::TileOut out = tile_out();
        out.world_size = world_size.p;
        out.keep_edges = keep ? 1 : 0;
        imin_status_t st = launch_tiers(q, 0, (uint32_t)theta, nullptr, out, start_tier, 0, 3);
        if (st != IMIN_OK) return st;
        IMIN_TRY(imin::launch_sum_lengths(wlen.p, (uint32_t)theta, &ctl.p->tile_total, ctl.p, s));
        if (keep) IMIN_TRY(imin::launch_sum_lengths(xlen.p, (uint32_t)theta, &ctl.p->xtile_total, ctl.p, s));
        // a world that found no room (or bad data) stops the solve here
        IMIN_TRY(imin::launch_guard(ctl.p, imin::kFlagFatalMask, s, round0 ? theta : 0, round0 ? hints : nullptr));
        if (keep) {
            store_node.swap(scr_node);
            store_cnt.swap(scr_cnt);
            store_off.swap(wloc);
            store_len.swap(wlen);
            store_par.swap(scr_par);
            store_lab.swap(scr_lab);
            xstore_v.swap(xscr_v);
            xstore_u.swap(xscr_u);
            xstore_off.swap(xloc);
            xstore_len.swap(xlen);
            adopted = true;
            st = build_index(theta, gain.p);
            if (st != IMIN_OK) return st;
        } else {
            imin::GainSrc src{};
            src.count = (uint32_t)theta;
            src.node = scr_node.p;
            src.cnt = scr_cnt.p;
            src.off = wloc.p;
            src.len = wlen.p;
            src.cap = scr_node.count;
            st = reduce_gains(src, 0);
            if (st != IMIN_OK) return st;
        }
        IMIN_TRY(imin::launch_sum_sizes(world_size.p, (uint32_t)theta, ctl.p, s));
        return IMIN_OK;
    }

    // A whole solve, enqueued: set-up, round 0 and k rounds, then the status.
    // Every kernel returns at once after the selection stops or a fatal flag
    // is raised, so nothing is decided on the host.
    imin_status_t run_ws(const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed,
                         int32_t chunk_cap, const imin::SelectOut& so, int32_t* device_status,
                         unsigned long long* hints) {
        IMIN_TRY(imin::launch_ctl_init(ctl.p, s));
        IMIN_TRY(imin::launch_fill_i64((int64_t*)dsz.p, 0, (size_t)dsz_n, s));
        IMIN_TRY(imin::launch_fill_i32((int32_t*)t2.vis.p, 0, t2.vis.count, s));
        if (t3.ready()) IMIN_TRY(imin::launch_fill_i32((int32_t*)t3.vis.p, 0, t3.vis.count, s));
        if (world_flags.p) IMIN_TRY(imin::launch_fill_u8(world_flags.p, 0, world_flags.count, s));
        IMIN_TRY(imin::launch_query_setup(g, seeds, n_seeds, nullptr, 0, excl.p, ctl.p, s));
        IMIN_TRY(imin::launch_seed_count(g, seeds, n_seeds, seed_cnt.p, ctl.p, s));
        IMIN_TRY(imin::launch_guard(ctl.p, imin::kFlagDataMask, s));
        IMIN_TRY(imin::launch_seed_fill(g, seeds, n_seeds, seed_cnt.p, seed_table.p, chunk_cap, ctl.p, s));
        const imin::QueryDev q = make_query(seeds, n_seeds, rng_seed, chunk_cap);
        IMIN_TRY(imin::launch_ctl_reset_round(ctl.p, s));
        IMIN_TRY(imin::launch_fill_i64_live(gain.p, 0, (size_t)g.n, ctl.p, s));
        imin_status_t st = pass_ws(q, theta, true, hints);
        if (st != IMIN_OK) return st;
        IMIN_TRY(imin::launch_select(g, gain.p, ctl.p, so, dsz.p, dsz_n, !incremental || k == 0, s));
        for (int32_t r = 1; r <= k; ++r) {
            if (incremental) {
                st = delta_round(q, theta, so);
            } else {
                IMIN_TRY(imin::launch_ctl_reset_round(ctl.p, s));
                IMIN_TRY(imin::launch_fill_i64_live(gain.p, 0, (size_t)g.n, ctl.p, s));
                st = pass_ws(q, theta, false, nullptr);
                if (st == IMIN_OK) IMIN_TRY(imin::launch_select(g, gain.p, ctl.p, so, dsz.p, dsz_n, true, s));
            }
            if (st != IMIN_OK) return st;
        }
        IMIN_TRY(imin::launch_solve_status(ctl.p, device_status, so.n_selected, theta, hints, s));
        return IMIN_OK;
    }

    // The query as the kernels take it (the level-0 table's length and the
    // seeds' sums are read on the device).
    imin::QueryDev make_query(const int32_t* seeds, int32_t n_seeds, uint64_t rng_seed, int32_t chunk_cap) const {
        imin::QueryDev q{};
        q.excl = excl.p;
        q.thr = thr_q.p;
        q.excl_in_thr = 1;
        q.seeds = seeds;
        q.n_seeds = n_seeds;
        q.key0 = (uint32_t)rng_seed;
        q.key1 = (uint32_t)(rng_seed >> 32);
        q.seed_chunk = seed_table.p;
        q.seed_col = seed_col.p;
        q.seed_thr = seed_thr.p;
        q.seed_cap = chunk_cap;
        q.n_seed_chunks = chunk_cap;
        return q;
    }

    imin::SelectOut select_out(int32_t k, int32_t* blockers, int64_t* gains, int64_t* totals,
                               int32_t* n_selected) const {
        imin::SelectOut so{};
        so.parts = sel_parts;
        so.pg = sel_g.p;
        so.pu = sel_u.p;
        so.pd = sel_d.p;
        so.excl = excl.p;
        so.k = k;
        so.blockers = blockers;
        so.gains = gains;
        so.totals = totals;
        so.n_selected = n_selected;
        return so;
    }

    // one incremental round: the last selection committed and the changed
    // worlds found, the changed worlds updated, then this round's partial
    // selection (committed by the next round, or by a final combining launch)
    imin_status_t delta_round(const imin::QueryDev& q, uint64_t theta, const imin::SelectOut& so) {
        imin_status_t st = evaluate_delta(q, theta, so);
        if (st != IMIN_OK) return st;
        hipEvent_t ev = timed.begin(3, s);
        IMIN_TRY(imin::launch_select(g, gain.p, ctl.p, so, dsz.p, dsz_n, false, s));
        timed.end(3, ev, s);
        return IMIN_OK;
    }

    // most tier-2 slots a call uses (one per resident workgroup: five per
    // compute unit, the register limit, which the LDS allows too unless the
    // visited bitset it holds is near its 16 KB maximum)
    static int max_slots(int cus) { return cus * 5; }

    static constexpr int32_t kT2Nodes = 1 << 16;  // nodes a world may reach in a tier-2 slot
    static constexpr int64_t kT2Edges = 1 << 16;  // extra edges it may keep there
    int32_t t2_lid_cap() const { return std::min<int32_t>(g.n, kT2Nodes); }
    int64_t t2_xcap() const { return std::min<int64_t>(std::max<int64_t>(g.m, 1), kT2Edges); }
    // whether some world of the graph could outgrow a tier-2 slot
    bool tier3_possible() const { return g.n > t2_lid_cap() || std::max<int64_t>(g.m, 1) > t2_xcap(); }

    // bytes of one HBM-tier slot: node -> local id, the visited bitset, four
    // per-node arrays (five with the coverage store's preorder indexes) and
    // the level offsets, and four extra-edge arrays (as found, and sorted by
    // head level)
    size_t slot_bytes(int32_t lid_cap, int64_t xcap) const {
        const size_t n = (size_t)g.n;
        const size_t per_node = cover == imin::kCoverStore ? 5 : 4;
        return n * 4 + (n + 31) / 32 * 4 + per_node * (size_t)lid_cap * 4 + ((size_t)lid_cap + 3) * 4 +
               4 * (size_t)xcap * 4;
    }
    size_t t2_slot_bytes() const { return slot_bytes(t2_lid_cap(), t2_xcap()); }
    size_t t3_slot_bytes() const { return slot_bytes(g.n, std::max<int64_t>(g.m, 1)); }

    // the slots of a call that takes its scratch from the block cache,
    // allocated when a tile first hands a world to their tier (or starts
    // there), so that calls whose worlds all fit the LDS tiers hold none:
    // tier 2 as many as IMIN_BIG_BUDGET (default 8 GiB) allows, at most
    // max_slots; tier 3 as many as IMIN_HUGE_BUDGET (default 2 GiB) allows,
    // at most one per compute unit
    // the HBM tiers' budgets; a batch's sessions, alive together, share them
    int32_t budget_share = 1;
    imin_status_t ensure_t2() {
        if (t2.ready()) return IMIN_OK;
        const size_t budget = env_size("IMIN_BIG_BUDGET", (size_t)8 << 30) / (size_t)budget_share;
        IMIN_TRY(alloc_slots(t2, std::min<size_t>(std::max<size_t>(budget / t2_slot_bytes(), 1),
                                                  (size_t)max_slots(cu_count())),
                             t2_lid_cap(), t2_xcap()));
        IMIN_TRY(imin::launch_fill_i32((int32_t*)t2.vis.p, 0, t2.vis.count, s));
        return IMIN_OK;
    }
    imin_status_t ensure_t3() {
        if (t3.ready()) return IMIN_OK;
        const size_t budget = env_size("IMIN_HUGE_BUDGET", (size_t)2 << 30) / (size_t)budget_share;
        IMIN_TRY(alloc_slots(t3, std::min<size_t>(std::max<size_t>(budget / t3_slot_bytes(), 1), (size_t)cu_count()),
                             g.n, std::max<int64_t>(g.m, 1)));
        IMIN_TRY(imin::launch_fill_i32((int32_t*)t3.vis.p, 0, t3.vis.count, s));
        return IMIN_OK;
    }

    // slots of one HBM tier (at most one per world of a tile)
    hipError_t alloc_slots(Slots& S, size_t slots, int32_t lid_cap, int64_t xcap) {
        const size_t n = (size_t)g.n;
        const size_t lc = (size_t)lid_cap;
        slots = std::max<size_t>(std::min<size_t>(slots, tile_cap), 1);
        S.bs.n_slots = (int32_t)slots;
        S.bs.lid_cap = lid_cap;
        S.bs.xcap = xcap;
        S.bs.vis_words = (int32_t)((n + 31) / 32);
        hipError_t e;
        if ((e = S.lid.alloc(slots * n)) != hipSuccess) return e;
        if ((e = S.nodes.alloc(slots * lc)) != hipSuccess) return e;
        if ((e = S.parent.alloc(slots * lc)) != hipSuccess) return e;
        if ((e = S.idom.alloc(slots * lc)) != hipSuccess) return e;
        if ((e = S.aux.alloc(slots * lc)) != hipSuccess) return e;
        if (cover == imin::kCoverStore && (e = S.tin.alloc(slots * lc)) != hipSuccess) return e;
        if ((e = S.lvl.alloc(slots * (lc + 3))) != hipSuccess) return e;
        if ((e = S.xv.alloc(slots * (size_t)xcap)) != hipSuccess) return e;
        if ((e = S.xu.alloc(slots * (size_t)xcap)) != hipSuccess) return e;
        if ((e = S.xv2.alloc(slots * (size_t)xcap)) != hipSuccess) return e;
        if ((e = S.xu2.alloc(slots * (size_t)xcap)) != hipSuccess) return e;
        if ((e = S.vis.alloc(slots * (size_t)S.bs.vis_words)) != hipSuccess) return e;
        S.bs.vis = S.vis.p;
        S.bs.lid_of = S.lid.p;
        S.bs.nodes = S.nodes.p;
        S.bs.parent = S.parent.p;
        S.bs.idom = S.idom.p;
        S.bs.aux = S.aux.p;
        S.bs.tin = S.tin.p;
        S.bs.lvl = S.lvl.p;
        S.bs.xv = S.xv.p;
        S.bs.xu = S.xu.p;
        S.bs.xv2 = S.xv2.p;
        S.bs.xu2 = S.xu2.p;
        return hipSuccess;
    }

    // launch shapes of the world and round kernels, the selection's parts
    // and the per-workgroup lost-node slots (not cleared here)
    hipError_t alloc_grids(int cus) {
        const size_t n = (size_t)g.n;
        // parts of the selection: few enough that combining them is cheap
        // for every workgroup of the search that reads them
        sel_parts = (int)std::min<size_t>(env_size("IMIN_SELECT_PARTS", 512), (n + 255) / 256);
        hipError_t e;
        if ((e = sel_g.alloc(sel_parts)) != hipSuccess) return e;
        if ((e = sel_u.alloc(sel_parts)) != hipSuccess) return e;
        if ((e = sel_d.alloc(sel_parts)) != hipSuccess) return e;
        int32_t pct = kDefaultGrid0Pct;
        if (gh && !ws) {  // an enqueued solve's layout is fixed when its workspace is sized
            const int32_t tuned = gh->tuned_grid0_pct.load(std::memory_order_relaxed);
            if (tuned > 0) pct = tuned;
        }
        grid0 = std::max(cus, (int)((long long)cus * imin::world_tier_blocks_per_cu(0) * pct / 100));
        grid1 = cus * imin::world_tier_blocks_per_cu(1);
        // changed-world update: label-rule and replay workgroups of one launch
        grid_r = cus * (int)env_size("IMIN_REPLAY_WG_PER_CU", 3);
        grid_l = cus * (int)env_size("IMIN_RULE_WG_PER_CU", 2);
        rule_lanes = (int)env_size("IMIN_RULE_LANES", 16);
        grid_w = cus;  // wide replay: one 1024-thread workgroup per CU
        const int sizes[7] = {grid0, grid1, max_slots(cus), grid_r, grid_l, grid_w, cus};
        int32_t at = 0;
        for (int i = 0; i < 7; ++i) {
            dsz_off[i] = at;
            at += sizes[i];
        }
        dsz_n = at;
        return dsz.alloc((size_t)dsz_n);
    }

    imin_status_t init(uint64_t theta, bool solve) {
        const size_t n = (size_t)g.n;
        IMIN_TRY(excl.alloc((n + 31) / 32));
        IMIN_TRY(gain.alloc(n));
        IMIN_TRY(ctl.alloc(1));
        IMIN_TRY(hctl.get());
        imin::RoundCtl c0{};
        c0.expect_total = -1;
        IMIN_TRY(hipMemcpyAsync(ctl.p, &c0, sizeof(c0), hipMemcpyHostToDevice, s));

        tile_cap = std::min<size_t>(theta, env_size("IMIN_TILE_WORLDS", (size_t)1 << 18));
        tile = tile_cap;
        IMIN_TRY(world_size.alloc(tile_cap));
        IMIN_TRY(wloc.alloc(tile_cap));
        // incremental rounds index change counts by world id
        IMIN_TRY(wlen.alloc(solve ? std::max<size_t>(tile_cap, theta) : tile_cap));
        // incremental rounds hand down changed worlds of the whole theta
        const size_t next_n = solve ? std::max<size_t>(tile_cap, theta) : tile_cap;
        IMIN_TRY(list1.alloc(next_n));
        IMIN_TRY(list2.alloc(next_n));
        IMIN_TRY(list3.alloc(next_n));
        IMIN_TRY(list4.alloc(next_n));
        IMIN_TRY(list0.alloc(1));
        slot_cap0 = lrr ? 0 : (size_t)imin::world_tier0_capacity();  // LRR sets use the bump region only
        big_cap = hinted(gh ? &gh->big_per_world : nullptr, tile_cap, env_size("IMIN_BIG_SCRATCH", (size_t)1 << 20));
        IMIN_TRY(scr_node.alloc(tile_cap * slot_cap0 + big_cap));
        IMIN_TRY(scr_cnt.alloc(tile_cap * slot_cap0 + big_cap));

        const int cus = cu_count();
        gb = imin::gain_buckets(g.n);
        IMIN_TRY(g_bcnt.alloc((size_t)gb.nb));
        IMIN_TRY(g_bbase.alloc((size_t)gb.nb + 1));
        IMIN_TRY(g_bcur.alloc((size_t)gb.nb));
        gb.bcnt = g_bcnt.p;
        gb.bbase = g_bbase.p;
        gb.bcur = g_bcur.p;
        IMIN_TRY(alloc_grids(cus));
        IMIN_TRY(hipMemsetAsync(dsz.p, 0, (size_t)dsz_n * sizeof(long long), s));
        start_tier = hinted_start_tier();
        if (start_tier == 2 || (gh && gh->tier2_seen.load(std::memory_order_relaxed))) {
            const imin_status_t st = ensure_t2();
            if (st != IMIN_OK) return st;
        }
        if (timed.on && g_timing.tallies.load()) {
            work_stride = std::max(std::max(std::max(grid0, grid1), grid_r + grid_l), max_slots(cus));
            const size_t wn = (size_t)imin::kWorkFields * kWorkTiers * work_stride;
            IMIN_TRY(work.alloc(wn));
            IMIN_TRY(hipMemsetAsync(work.p, 0, wn * sizeof(unsigned long long), s));
        }
        return IMIN_OK;
    }

    // Resolve this call's kernel timings and add its work tallies (after the
    // call's final synchronisation).
    void finish() {
        if (!timed.on) return;
        timed.flush();
        if (!work.p) return;  // no tallies taken
        constexpr int F = imin::kWorkFields;
        std::vector<unsigned long long> h((size_t)F * kWorkTiers * work_stride);
        if (work.p && hipMemcpy(h.data(), work.p, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) !=
                          hipSuccess)
            return;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        for (int tier = 0; tier < kWorkTiers; ++tier)
            for (int field = 0; field < F; ++field) {
                int64_t f = 0;
                for (int b = 0; b < work_stride; ++b) f += (int64_t)h[((size_t)tier * F + field) * work_stride + b];
                g_timing.work[tier][field] += f;
            }
    }

    imin_status_t read_ctl() {
        IMIN_TRY(hipMemcpyAsync(hctl.p, ctl.p, sizeof(imin::RoundCtl), hipMemcpyDeviceToHost, s));
        IMIN_TRY(hipStreamSynchronize(s));
        return IMIN_OK;
    }

    imin_status_t clear_flag(uint32_t bit) {
        hctl.p->flags &= ~bit;
        IMIN_TRY(hipMemcpyAsync(&ctl.p->flags, &hctl.p->flags, sizeof(uint32_t), hipMemcpyHostToDevice, s));
        return IMIN_OK;
    }

    // gain[u] += every count of u among the tile entries of src (`entries`
    // in all)
    imin_status_t reduce_gains(const imin::GainSrc& src, unsigned long long entries) {
        if (ws) entries = g_rec.count;  // carved for the most a tile can write
        else if (!g_rec.p || g_rec.count < entries) IMIN_TRY(g_rec.alloc((size_t)(entries + entries / 8 + 1024)));
        gb.rec = g_rec.p;
        gb.rec_cap = g_rec.count;
        gb.slices = imin::gain_slices(gb, entries, cu_count());
        IMIN_TRY(imin::launch_gain_reduce(src, gb, g.n, gain.p, ctl.p, s));
        return IMIN_OK;
    }

    // Resident store for incremental rounds: per-world offsets and lengths;
    // entries are allocated as round 0 produces them.
    imin_status_t enable_store(uint64_t theta) {
        // the index keeps store positions as uint32
        store_budget = std::min<size_t>(env_size("IMIN_STORE_CAP", (size_t)imin::kIndexPosLimit - 1),
                                        (size_t)imin::kIndexPosLimit - 1);
        if (store_off.alloc(theta) != hipSuccess || store_len.alloc(theta) != hipSuccess ||
            list0.alloc(theta) != hipSuccess) {
            store_off.release();
            store_len.release();
            (void)hipGetLastError();
            return IMIN_OK;  // plain rounds give the same integers
        }
        incremental = true;
        const char* fp = std::getenv("IMIN_LABEL_RULE");
        label_rule = !(fp && fp[0] == '0');
        const char* rp = std::getenv("IMIN_REPLAY");
        if (!(rp && rp[0] == '0')) {
            xslot_cap0 = (size_t)imin::world_tier0_xcapacity();
            xbig_cap = hinted(gh ? &gh->xbig_per_world : nullptr, tile_cap,
                              env_size("IMIN_XBIG_SCRATCH", (size_t)1 << 20));
            const size_t xn = tile_cap * xslot_cap0 + xbig_cap;
            replay = scr_par.alloc(scr_node.count) == hipSuccess && scr_lab.alloc(scr_node.count) == hipSuccess &&
                     xscr_v.alloc(xn) == hipSuccess && xscr_u.alloc(xn) == hipSuccess &&
                     xloc.alloc(tile_cap) == hipSuccess && xlen.alloc(tile_cap) == hipSuccess &&
                     xstore_off.alloc(theta) == hipSuccess && xstore_len.alloc(theta) == hipSuccess &&
                     world_flags.alloc(theta) == hipSuccess &&
                     hipMemsetAsync(world_flags.p, 0, theta, s) == hipSuccess;
            if (!replay) drop_replay();
        }
        return IMIN_OK;
    }

    // replay off for the rest of the solve: its buffers are released
    void drop_replay() {
        replay = false;
        scr_par.release();
        scr_lab.release();
        store_lab.release();
        world_flags.release();
        xscr_v.release();
        xscr_u.release();
        xloc.release();
        xlen.release();
        store_par.release();
        xstore_v.release();
        xstore_u.release();
        xstore_off.release();
        xstore_len.release();
        (void)hipGetLastError();
    }

    // grow the arrays of a store to hold `need` entries, keeping the first
    // `used`; false when the budget or the device memory is exhausted
    template <size_t N>
    bool grow_store(DevArray<int32_t>* (&arrs)[N], unsigned long long used, unsigned long long need,
                    unsigned long long budget) {
        if (need > budget) return false;
        if (arrs[0]->p && arrs[0]->count >= need) return true;
        const size_t want = (size_t)std::min<unsigned long long>(budget, need + need / 4 + 1024);
        DevArray<int32_t> fresh[N];
        for (size_t i = 0; i < N; ++i) {
            if (fresh[i].alloc(want) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
            if (used && hipMemcpyAsync(fresh[i].p, arrs[i]->p, used * sizeof(int32_t), hipMemcpyDeviceToDevice,
                                       s) != hipSuccess)
                return false;
        }
        for (size_t i = 0; i < N; ++i) arrs[i]->swap(fresh[i]);
        return hipStreamSynchronize(s) == hipSuccess;  // old arrays are freed on return
    }

    // room for `more` entries after the store's `used` ones
    bool ensure_store(unsigned long long used, unsigned long long more) {
        if (replay || cover == imin::kCoverStore) {
            DevArray<int32_t>* arrs[4] = {&store_node, &store_cnt, &store_par, &store_lab};
            return grow_store(arrs, used, used + more, store_budget);
        }
        DevArray<int32_t>* arrs[2] = {&store_node, &store_cnt};
        return grow_store(arrs, used, used + more, store_budget);
    }

    bool ensure_xstore(unsigned long long used, unsigned long long more) {
        DevArray<int32_t>* arrs[2] = {&xstore_v, &xstore_u};
        return grow_store(arrs, used, used + more, store_budget);
    }

    // node -> (store position, world) of every entry written in round 0,
    // for the incremental rounds; with gain_out also the from-scratch gains
    // of round 0, from the same pass over the store.  Nodes are grouped in
    // buckets of 2^IMIN_INDEX_BUCKET_LOG ids (default 10), widened until
    // there are at most 8192 buckets.
    imin_status_t build_index(uint64_t theta, int64_t* gain_out) {
        if (indexed) return IMIN_OK;
        if (!ws) {
            const unsigned long long entries = adopted ? adopted_entries : hctl.p->store_count;
            if (entries >= imin::kIndexPosLimit) return IMIN_ERR_INTERNAL;  // positions are uint32
            IMIN_TRY(alloc_index((size_t)entries));
        }
        imin::IndexBufs ib{};
        ib.shift = idx_shift;
        ib.nb = (int)idx_bcnt.count;
        ib.bcnt = idx_bcnt.p;
        ib.bbase = idx_bbase.p;
        ib.bcur = idx_bcur.p;
        ib.border = idx_border.p;
        ib.rec = idx_rec.p;
        ib.rec_cap = (uint32_t)idx_rec.count;
        ib.idx_off = idx_off.p;
        ib.idx_ent = idx_ent.p;
        ib.ent_cap = (uint32_t)idx_ent.count;
        IMIN_TRY(imin::launch_index_build(tile_out(), (uint32_t)theta, g.n, ib, gain_out, ctl.p, s));
        indexed = true;
        return IMIN_OK;
    }

    // arrays of the node index for `entries` stored entries (< kIndexPosLimit).
    // Nodes are grouped in buckets of 2^IMIN_INDEX_BUCKET_LOG ids (default
    // 10), widened until there are at most 8192 buckets.
    int idx_shift = 10;
    hipError_t alloc_index(size_t entries) {
        const unsigned long long n = (unsigned long long)g.n;
        int shift = (int)std::min<size_t>(std::max<size_t>(env_size("IMIN_INDEX_BUCKET_LOG", 10), 1), 30);
        while (((n + (1ull << shift) - 1) >> shift) > 8192ull) ++shift;
        idx_shift = shift;
        const size_t nb = (size_t)((n + (1ull << shift) - 1) >> shift);
        hipError_t e;
        if ((e = idx_off.alloc(n + 1)) != hipSuccess) return e;
        if ((e = idx_ent.alloc(entries)) != hipSuccess) return e;
        if ((e = idx_bcnt.alloc(nb)) != hipSuccess) return e;
        if ((e = idx_bbase.alloc(nb + 1)) != hipSuccess) return e;
        if ((e = idx_bcur.alloc(nb)) != hipSuccess) return e;
        if ((e = idx_border.alloc(nb)) != hipSuccess) return e;
        return idx_rec.alloc(entries);
    }

    imin::TileOut tile_out() const {
        imin::TileOut out{};
        out.mode = imin::kModePlain;
        out.scr_node = scr_node.p;
        out.scr_cnt = scr_cnt.p;
        out.slot_cap0 = slot_cap0;
        out.big_base = tile_cap * slot_cap0;
        out.scr_cap = scr_node.count;
        out.wloc = wloc.p;
        out.wlen = wlen.p;
        out.store_node = store_node.p;
        out.store_cnt = store_cnt.p;
        out.store_cap = store_node.count;
        out.store_off = store_off.p;
        out.store_len = store_len.p;
        out.gain = gain.p;
        out.list_cap = (uint32_t)std::min<size_t>(list0.count, 0xFFFFFFFFu);
        out.scr_lab = (uint32_t*)scr_lab.p;
        out.store_lab = (uint32_t*)store_lab.p;
        out.world_flags = label_rule ? world_flags.p : nullptr;
        out.dsz = dsz.p;
        for (int i = 0; i < 7; ++i) out.dsz_off[i] = dsz_off[i];
        out.next_cap =
            (uint32_t)std::min<size_t>(std::min(std::min(std::min(list1.count, list2.count), list3.count), list4.count),
                                       0xFFFFFFFFu);
        out.scr_par = scr_par.p;
        out.store_par = store_par.p;
        out.xscr_v = xscr_v.p;
        out.xscr_u = xscr_u.p;
        out.xslot_cap0 = xslot_cap0;
        out.xbig_base = tile_cap * xslot_cap0;
        out.xscr_cap = xscr_v.count;
        out.xloc = xloc.p;
        out.xlen = xlen.p;
        out.xstore_v = xstore_v.p;
        out.xstore_u = xstore_u.p;
        out.xstore_cap = xstore_v.count;
        out.xstore_off = xstore_off.p;
        out.xstore_len = xstore_len.p;
        out.work = work.p;
        out.work_stride = work_stride;
        out.cover = cover;
        out.mark = cover_mark;
        out.unit_counts = unit_counts;
        out.sizes_only = sizes_only;
        return out;
    }

    // Tiers first_tier..last_tier; the first reads first_list (count
    // list_n[first_idx]) or, without a list, worlds [wb, wb+range).  Tier t
    // hands the worlds it cannot hold to tier t+1's list (list1, list2,
    // list4); tiers 2 and 3 run only with their slots allocated.
    imin_status_t launch_tiers(const imin::QueryDev& q, uint32_t wb, uint32_t range, const int32_t* first_list,
                               const imin::TileOut& out, int first_tier, int first_idx = 0, int last_tier = 2) {
        if (last_tier > 2 && !tier3_possible()) last_tier = 2;
        for (int tier = first_tier; tier <= last_tier; ++tier) {
            if ((tier == 2 && !t2.ready()) || (tier == 3 && !t3.ready())) return IMIN_ERR_INTERNAL;
            const bool first = (tier == first_tier);
            const int32_t* in_list = first ? first_list : (tier == 1 ? list1.p : (tier == 2 ? list2.p : list4.p));
            const int count_idx = first ? first_idx : (tier == 3 ? 4 : tier);
            int32_t* next_list = tier == 0 ? list1.p : (tier == 1 ? list2.p : list4.p);
            const int timer_id = tier == 0 ? 0 : (tier == 1 ? 4 : 1);
            const imin::LaunchEvents ev = timed.take(timer_id);
            const hipError_t e = imin::launch_world_tier(tier, g, q, ctl.p, wb, first_list ? 0u : range, in_list,
                                                         count_idx, next_list, out, tier == 3 ? t3.bs : t2.bs,
                                                         tier == 0 ? grid0 : grid1, s, ev);
            timed.taken(timer_id, ev);
            IMIN_TRY(e);
        }
        return IMIN_OK;
    }

    // All tiers of a tile in a call with the block cache: the HBM tiers'
    // slots are allocated (and their launches made) only once some world of
    // the tile has been handed to them.
    // With packed, packed launches have already run tiers 0 and 1 over the
    // tile (its worlds too large for them are in list2).
    imin_status_t launch_tiers_checked(const imin::QueryDev& q, uint32_t wb, uint32_t nw, const imin::TileOut& out,
                                       bool packed = false) {
        imin_status_t st = IMIN_OK;
        if (start_tier >= 2 && (st = ensure_t2()) != IMIN_OK) return st;
        const bool three = tier3_possible();
        const int ready_last = !t2.ready() ? 1 : ((!three || t3.ready()) ? 3 : 2);
        if (!packed) st = launch_tiers(q, wb, nw, nullptr, out, start_tier, 0, ready_last);
        else if (ready_last >= 2) st = launch_tiers(q, wb, 0, list2.p, out, 2, 2, ready_last);
        if (st != IMIN_OK) return st;
        bool ran2 = ready_last >= 2;
        if (!t2.ready()) {
            if ((st = read_ctl()) != IMIN_OK) return st;
            if (hctl.p->list_n[2] > 0) {
                if ((st = ensure_t2()) != IMIN_OK) return st;
                if ((st = launch_tiers(q, wb, 0, list2.p, out, 2, 2, 2)) != IMIN_OK) return st;
                ran2 = true;
            }
        }
        if (three && ran2 && !t3.ready()) {
            if ((st = read_ctl()) != IMIN_OK) return st;
            if (hctl.p->list_n[4] > 0) {
                if ((st = ensure_t3()) != IMIN_OK) return st;
                if ((st = launch_tiers(q, wb, 0, list4.p, out, 3, 4, 3)) != IMIN_OK) return st;
            }
        }
        return IMIN_OK;
    }

    // One incremental round: worlds holding the last blocker are re-evaluated
    // and report their count changes; gain is updated in place.
    imin_status_t evaluate_delta(const imin::QueryDev& q0, uint64_t theta, const imin::SelectOut& so) {
        // blockers added since the thresholds were made are tested against
        // the exclusion bitmap
        imin::QueryDev q = q0;
        q.excl_in_thr = 0;
        imin::TileOut out = tile_out();
        out.mode = imin::kModeDelta;
        out.world_size = world_size.p;
        // the per-round counters were cleared by the last selection
        imin_status_t st;
        if (replay) {
            // one launch: the last selection is committed; worlds where no
            // live edge leaves the blocker's subtree lose it from their
            // labels; every other changed world is replayed, those too
            // large go on to sampling
            const imin::LaunchEvents ev = timed.take(6);
            const hipError_t e = imin::launch_round_update(q, ctl.p, list1.p, out, out.world_flags ? grid_l : 0,
                                                           grid_r, rule_lanes, idx_off.p, idx_ent.p, so, s, ev);
            timed.taken(6, ev);
            IMIN_TRY(e);
            // worlds the replay workgroups cannot hold are replayed by the
            // wide replay, and those too large for it sampled again; when
            // round 0 stored no such world, neither is launched
            if (!replay_complete) {
                const imin::LaunchEvents evw = timed.take(7);
                const hipError_t ew = imin::launch_replay_wide(q, ctl.p, out, list1.p, list3.p, grid_w, s, evw);
                timed.taken(7, evw);
                IMIN_TRY(ew);
                st = launch_tiers(q, 0, 0, list3.p, out, std::max(start_tier, 1), 3, last_tier());
            } else {
                st = IMIN_OK;
            }
        } else {
            // the search for the changed worlds, then their sampling
            hipEvent_t ev = timed.begin(5, s);
            IMIN_TRY(imin::launch_affected_select(out, ctl.p, idx_off.p, idx_ent.p, list0.p, so, s));
            timed.end(5, ev, s);
            st = launch_tiers(q, 0, 0, list0.p, out, start_tier, 0, last_tier());
        }
        if (st != IMIN_OK) return st;
        // T is carried over from the last round and lowered by the changed
        // worlds themselves: no pass over all theta sizes
        (void)theta;
        return IMIN_OK;
    }

    // Evaluate worlds [w_begin, w_begin+count) under the current excl bitmap;
    // gain += per-node sums, ctl.total += sum of sizes.  Optional per-world
    // outputs are written at [0, count).  With store_mode (round 0 of a
    // solve) the per-world lists also become the resident store.
    // Level 0 of a tile's worlds drawn ahead (launch_level0_bits), when the
    // tile gives every tier-0 workgroup four worlds or more (a smaller tile's
    // tier-0 launch is bound by one world's latency, and the extra launch
    // costs more than it saves), the bits fit IMIN_L0_BITS_BUDGET (default
    // 1 GiB), and IMIN_LEVEL0_BITS is not 0 (1 draws every tile ahead); out
    // then points the world kernels at them.
    DevArray<uint32_t> l0_bits;
    imin_status_t draw_level0(const imin::QueryDev& q, uint32_t wb, uint32_t nw, imin::TileOut& out) {
        const char* e = std::getenv("IMIN_LEVEL0_BITS");
        if ((e && e[0] == '0') || q.seed_cap < 1 || nw == 0) return IMIN_OK;
        if (!(e && e[0] == '1') && (uint64_t)nw < 4ull * (uint64_t)std::max(grid0, 1)) return IMIN_OK;
        const size_t words = ((size_t)q.seed_cap + 7) / 8;
        if ((size_t)(q.seed_cap + 255) / 256 > 65535) return IMIN_OK;
        const size_t need = (size_t)tile_cap * words;
        if (need * sizeof(uint32_t) > env_size("IMIN_L0_BITS_BUDGET", (size_t)1 << 30)) return IMIN_OK;
        if (l0_bits.count < need) IMIN_TRY(l0_bits.alloc(need));
        const imin::LaunchEvents ev = timed.take(8);
        const hipError_t le = imin::launch_level0_bits(q, ctl.p, wb, nw, l0_bits.p, (int)words, q.seed_cap, s, ev);
        timed.taken(8, ev);
        IMIN_TRY(le);
        out.l0_bits = l0_bits.p;
        out.l0_words = (int)words;
        return IMIN_OK;
    }

    // The outputs of the tile whose first world is `done`.
    imin::TileOut tile_out_at(uint64_t done, int32_t* ws_out, int64_t* wsum_out, int64_t* wedges_out, bool keep) {
        imin::TileOut out = tile_out();
        out.world_size = ws_out ? ws_out + done : world_size.p;
        out.world_sum = wsum_out ? wsum_out + done : nullptr;
        out.world_edges = wedges_out ? wedges_out + done : nullptr;
        out.keep_edges = keep ? 1 : 0;
        return out;
    }

    // Whether a from-scratch pass of `count` worlds can have its tier-0 and
    // tier-1 launches packed with other queries': one tile whose worlds do
    // not start at the HBM tier.  (A query the graph's hints would start at
    // tier 1 is packed from tier 0: its worlds that overflow go on to the
    // packed tier-1 launch, and the hints, the largest share any earlier
    // call handed to tier 1, may come from another seed set.)
    bool packable(uint64_t count) const {
        return !lrr && cover == imin::kCoverNone && !unit_counts && !sizes_only && start_tier <= 1 &&
               count <= (uint64_t)tile && count > 0;
    }

    // The set-up of such a pass (what evaluate does before its first tier-0
    // launch) and its entry in the packed launch.
    imin_status_t packed_prepare(const imin::QueryDev& q, uint64_t w_begin, uint64_t count, int32_t* ws_out,
                                 imin::PackedQuery& pq) {
        IMIN_TRY(imin::launch_query_thresholds(g, excl.p, thr_q.p, seed_table.p, ctl.p, q.seed_cap, seed_col.p,
                                               seed_thr.p, s));
        IMIN_TRY(imin::launch_ctl_reset_tile(ctl.p, s));
        start_tier = 0;  // the packed launches start at tier 0
        pq = imin::PackedQuery{};
        pq.q = q;
        pq.out = tile_out_at(0, ws_out, nullptr, nullptr, false);
        pq.out.work = nullptr;  // no per-workgroup tallies for packed launches

        pq.ctl = ctl.p;
        pq.list1 = list1.p;
        pq.list2 = list2.p;
        pq.w_begin = (uint32_t)w_begin;
        pq.count = (uint32_t)count;
        return IMIN_OK;
    }

    // With after_packed, packed_prepare and the packed tier-0 and tier-1
    // launches have already done the first tile's set-up and those tiers.
    imin_status_t evaluate(const imin::QueryDev& q, uint64_t w_begin, uint64_t count, int32_t* ws_out,
                           int64_t* wsum_out, int64_t* wedges_out, bool store_mode = false,
                           bool after_packed = false) {
        // the exclusions as they stand (blockers may have been added since
        // the last pass) go into the query's thresholds
        if (!after_packed)
            IMIN_TRY(imin::launch_query_thresholds(g, excl.p, thr_q.p, seed_table.p, ctl.p, q.seed_cap, seed_col.p,
                                                   seed_thr.p, s));
        uint64_t done = 0;
        bool packed_tile = after_packed;
        while (done < count) {
            const uint64_t nw = std::min<uint64_t>(tile, count - done);
            const bool keep = store_mode && incremental && replay;
            // entries carry parents and labels (replay) or parent positions
            // and subtree sizes (coverage store)
            const bool four = keep || cover == imin::kCoverStore;
            imin::TileOut out = tile_out_at(done, ws_out, wsum_out, wedges_out, keep);
            if (!packed_tile) IMIN_TRY(imin::launch_ctl_reset_tile(ctl.p, s));
            imin_status_t st = IMIN_OK;
            if (!lrr && !packed_tile && q.excl_in_thr) {
                st = draw_level0(q, (uint32_t)(w_begin + done), (uint32_t)nw, out);
                if (st != IMIN_OK) return st;
            }
            if (lrr) {
                st = lrr_reserve(nw);
                if (st == IMIN_OK && imin::launch_lrr(g, q, ctl.p, (uint32_t)(w_begin + done), (uint32_t)nw, lrr_dev,
                                                      out, s) != hipSuccess)
                    st = IMIN_ERR_DEVICE;
            } else {
                st = launch_tiers_checked(q, (uint32_t)(w_begin + done), (uint32_t)nw, out, packed_tile);
            }
            packed_tile = false;  // a redone tile runs every tier itself
            if (st != IMIN_OK) return st;
            IMIN_TRY(imin::launch_sum_lengths(wlen.p, (uint32_t)nw, &ctl.p->tile_total, ctl.p, s));
            if (keep) IMIN_TRY(imin::launch_sum_lengths(xlen.p, (uint32_t)nw, &ctl.p->xtile_total, ctl.p, s));
            st = read_ctl();
            if (st != IMIN_OK) return st;
            const uint32_t f = hctl.p->flags;
            if (hctl.p->list_n[2] > 0 || start_tier == 2) any_tier2 = true;
            if (hctl.p->list_n[4] > 0) any_tier3 = true;
            if (hctl.p->list_n[2] > 0 && gh) gh->tier2_seen.store(true, std::memory_order_relaxed);
            if (gh && nw > 0) {
                raise_hint(gh->tier1_share, ((uint64_t)hctl.p->list_n[1] << 10) / nw);
                raise_hint(gh->tier2_share, ((uint64_t)hctl.p->list_n[2] << 10) / nw);
            }
            replay_complete = (hctl.p->replay_big == 0);
            // route later tiles straight to the tier most worlds end up in
            if (start_tier < 2 && hctl.p->list_n[2] * 2 > nw) start_tier = 2;
            else if (start_tier < 1 && hctl.p->list_n[1] * 2 > nw) start_tier = 1;
            if (f & (imin::kFlagBigCapacity | imin::kFlagDomPasses | imin::kFlagBounds | imin::kFlagReduceCapacity)) {
                g_last_flags = f;
                return IMIN_ERR_INTERNAL;
            }
            if (!lrr) record_scratch(hctl.p->big_count, hctl.p->xbig_count, nw);
            if (f & imin::kFlagPairOverflow) {
                // a scratch bump region was too small: grow it, redo the tile
                st = clear_flag(imin::kFlagPairOverflow);
                if (st != IMIN_OK) return st;
                const unsigned long long bc = hctl.p->big_count, xc = hctl.p->xbig_count;
                big_cap = std::max<size_t>(big_cap, (size_t)(bc + bc / 8 + 1024));
                IMIN_TRY(scr_node.alloc(tile_cap * slot_cap0 + big_cap));
                IMIN_TRY(scr_cnt.alloc(tile_cap * slot_cap0 + big_cap));
                if (four) {
                    IMIN_TRY(scr_par.alloc(scr_node.count));
                    IMIN_TRY(scr_lab.alloc(scr_node.count));
                }
                if (keep) {
                    xbig_cap = std::max<size_t>(xbig_cap, (size_t)(xc + xc / 8 + 1024));
                    IMIN_TRY(xscr_v.alloc(tile_cap * xslot_cap0 + xbig_cap));
                    IMIN_TRY(xscr_u.alloc(tile_cap * xslot_cap0 + xbig_cap));
                }
                continue;
            }
            const unsigned long long total = hctl.p->tile_total;
            if (store_mode && incremental && done == 0 && nw == count && total < imin::kIndexPosLimit &&
                scr_node.count < imin::kIndexPosLimit) {
                // One tile holds every world: its scratch becomes the store
                // where it lies (fixed tier-0 slots and the bump region,
                // located by wloc / wlen), with no copy.  The gains follow
                // from the store in the pass that counts the index.
                store_node.swap(scr_node);
                store_cnt.swap(scr_cnt);
                store_off.swap(wloc);
                store_len.swap(wlen);
                if (four) {
                    store_par.swap(scr_par);
                    store_lab.swap(scr_lab);
                }
                if (keep) {
                    xstore_v.swap(xscr_v);
                    xstore_u.swap(xscr_u);
                    xstore_off.swap(xloc);
                    xstore_len.swap(xlen);
                }
                adopted = true;
                adopted_entries = total;
                hipEvent_t ev = timed.begin(2, s);
                const imin_status_t st2 = build_index((uint64_t)count, gain.p);
                if (st2 != IMIN_OK) return st2;
                timed.end(2, ev, s);
                IMIN_TRY(imin::launch_sum_sizes(out.world_size, (uint32_t)nw, ctl.p, s));
                done += nw;
                continue;
            }
            // dense destination for the tile's entries
            const unsigned long long store_base = hctl.p->store_count;
            bool use_store = store_mode && incremental;
            if (use_store && !ensure_store(store_base, total)) {
                incremental = false;  // the store does not fit: plain rounds from here on
                use_store = false;
                drop_replay();
            }
            bool use_x = keep && use_store;
            if (use_x && !ensure_xstore(hctl.p->xstore_count, hctl.p->xtile_total)) {
                drop_replay();  // incremental rounds go on by sampling
                use_x = false;
            }
            hipEvent_t ev = timed.begin(2, s);
            imin::GainSrc src{};
            src.count = (uint32_t)nw;
            if (use_store) {
                // pack the tile's entries densely into the store
                imin::CompactSpec cs{};
                cs.src[0] = scr_node.p;
                cs.src[1] = scr_cnt.p;
                cs.src[2] = scr_par.p;
                cs.src[3] = scr_lab.p;
                cs.nf = (use_x || cover == imin::kCoverStore) ? 4 : 2;
                cs.src_cap = scr_node.count;
                cs.loc = wloc.p;
                cs.len = wlen.p;
                cs.count = (uint32_t)nw;
                cs.w_begin = (uint32_t)(w_begin + done);
                cs.dst[0] = store_node.p;
                cs.dst[1] = store_cnt.p;
                cs.dst[2] = store_par.p;
                cs.dst[3] = store_lab.p;
                cs.dst_cap = store_node.count;
                cs.counter_id = 1;
                cs.out_off = store_off.p;
                cs.out_len = store_len.p;
                cs.overflow_flag = imin::kFlagStoreOverflow;
                IMIN_TRY(imin::launch_compact(cs, ctl.p, s));
                if (use_x) {
                    imin::CompactSpec xs{};
                    xs.src[0] = xscr_v.p;
                    xs.src[1] = xscr_u.p;
                    xs.dst[0] = xstore_v.p;
                    xs.dst[1] = xstore_u.p;
                    xs.nf = 2;
                    xs.src_cap = xscr_v.count;
                    xs.dst_cap = xstore_v.count;
                    xs.loc = xloc.p;
                    xs.len = xlen.p;
                    xs.count = (uint32_t)nw;
                    xs.w_begin = (uint32_t)(w_begin + done);
                    xs.counter_id = 2;
                    xs.out_off = xstore_off.p;
                    xs.out_len = xstore_len.p;
                    xs.overflow_flag = imin::kFlagStoreOverflow;
                    IMIN_TRY(imin::launch_compact(xs, ctl.p, s));
                }
                // the tile's worlds, by world id, where the compaction put them
                src.node = store_node.p;
                src.cnt = store_cnt.p;
                src.off = store_off.p + (w_begin + done);
                src.len = store_len.p + (w_begin + done);
                src.cap = store_node.count;
            } else {
                // the entries where the world kernels wrote them
                src.node = scr_node.p;
                src.cnt = scr_cnt.p;
                src.off = wloc.p;
                src.len = wlen.p;
                src.cap = scr_node.count;
            }
            st = reduce_gains(src, total);
            if (st != IMIN_OK) return st;
            timed.end(2, ev, s);
            IMIN_TRY(imin::launch_sum_sizes(out.world_size, (uint32_t)nw, ctl.p, s));
            done += nw;
        }
        return IMIN_OK;
    }
};

imin_status_t check_data_flags(uint32_t f) {
    if (f & imin::kFlagDataMask) {
        g_last_flags = f;
        return IMIN_ERR_DATA;
    }
    return IMIN_OK;
}

}  // namespace

extern "C" {

const char* imin_status_string(imin_status_t s) {
    switch (s) {
        case IMIN_OK: return "ok";
        case IMIN_ERR_INVALID: return "invalid argument";
        case IMIN_ERR_DATA: return "invalid input data (offsets, columns, probabilities, seeds or blockers)";
        case IMIN_ERR_DEVICE: return "HIP runtime error";
        case IMIN_ERR_NOMEM: return "out of device memory";
        case IMIN_ERR_INTERNAL: return "internal consistency check failed";
        case IMIN_ERR_WORKSPACE: return "workspace too small";
    }
    return "unknown status";
}

uint32_t imin_last_device_flags(void) { return g_last_flags; }

int32_t imin_last_solve_incremental(void) { return g_last_mode; }

imin_status_t imin_graph_create(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                const float* p, void* stream, imin_graph_t* out) {
    g_last_flags = 0;
    if (!out || !row_ptr) return IMIN_ERR_INVALID;
    *out = nullptr;
    if (n < 1 || n >= (1 << 24) || m < 0 || m > (int64_t)0x7FFFFFF0) return IMIN_ERR_INVALID;
    if (m > 0 && (!col || !p)) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    imin_graph* h = new (std::nothrow) imin_graph();
    if (!h) return IMIN_ERR_NOMEM;
    h->g.n = n;
    h->g.m = m;
    h->g.m_pad = ((m + 3) / 4) * 4 + 4;
    (void)hipGetDevice(&h->device);
    hipError_t e = hipMalloc((void**)&h->g.off, ((size_t)n + 1) * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&h->g.col, (size_t)h->g.m_pad * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&h->g.thr, (size_t)h->g.m_pad * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&h->hints_dev, 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemsetAsync(h->hints_dev, 0, 4 * sizeof(unsigned long long), s);
    imin::RoundCtl* ctl = nullptr;
    imin::RoundCtl* hc = nullptr;
    if (e == hipSuccess) e = hipMalloc((void**)&ctl, sizeof(imin::RoundCtl));
    if (e == hipSuccess) e = hipHostMalloc((void**)&hc, sizeof(imin::RoundCtl), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(ctl, 0, sizeof(imin::RoundCtl), s);
    if (e == hipSuccess) e = imin::launch_graph_ingest(h->g, row_ptr, col, p, ctl, s);
    // the largest out-degree bounds the level-0 table of any seed set
    if (e == hipSuccess) e = imin::launch_max_degree(h->g, &ctl->seed_chunks, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hc, ctl, sizeof(imin::RoundCtl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    imin_status_t st = from_hip(e);
    if (st == IMIN_OK) st = check_data_flags(hc->flags);
    if (st == IMIN_OK) h->g.max_deg = hc->seed_chunks;
    if (ctl) (void)hipFree(ctl);
    if (hc) (void)hipHostFree(hc);
    if (st != IMIN_OK) {
        imin_graph_destroy(h);
        return st;
    }
    *out = h;
    return IMIN_OK;
}

imin_status_t imin_graph_destroy(imin_graph_t g) {
    if (!g) return IMIN_OK;
    if (g->in_off) (void)hipFree(g->in_off);
    if (g->in_rec) (void)hipFree(g->in_rec);
    if (g->lrr_stamp) (void)hipFree(g->lrr_stamp);
    if (g->lrr_list) (void)hipFree(g->lrr_list);
    if (g->lrr_epoch) (void)hipFree(g->lrr_epoch);
    if (g->g.off) (void)hipFree(g->g.off);
    if (g->g.col) (void)hipFree(g->g.col);
    if (g->g.thr) (void)hipFree(g->g.thr);
    if (g->hints_dev) (void)hipFree(g->hints_dev);
    delete g;
    return IMIN_OK;
}

imin_status_t imin_graph_info(imin_graph_t g, int32_t* n, int64_t* m) {
    if (!g) return IMIN_ERR_INVALID;
    if (n) *n = g->g.n;
    if (m) *m = g->g.m;
    return IMIN_OK;
}

imin_status_t imin_graph_export(imin_graph_t g, int64_t* row_ptr, int32_t* col, uint32_t* thr) {
    if (!g || !row_ptr || !col || !thr) return IMIN_ERR_INVALID;
    const size_t n = (size_t)g->g.n, m = (size_t)g->g.m;
    std::vector<int32_t> off(n + 1);
    if (hipMemcpy(off.data(), g->g.off, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess ||
        (m > 0 && hipMemcpy(col, g->g.col, m * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) ||
        (m > 0 && hipMemcpy(thr, g->g.thr, m * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)) {
        (void)hipGetLastError();
        return IMIN_ERR_DEVICE;
    }
    for (size_t i = 0; i <= n; ++i) row_ptr[i] = off[i];
    return IMIN_OK;
}

static imin_status_t setup_query(Session& ss, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                                 int32_t n_blocked, uint64_t rng_seed, imin::QueryDev& q) {
    IMIN_TRY(imin::launch_query_setup(ss.g, seeds, n_seeds, blocked, n_blocked, ss.excl.p, ss.ctl.p, ss.s));
    imin_status_t st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    st = check_data_flags(ss.hctl.p->flags);
    if (st != IMIN_OK) return st;
    // level-0 table: slot groups of every seed's row
    IMIN_TRY(ss.seed_cnt.alloc((size_t)n_seeds));
    IMIN_TRY(imin::launch_seed_count(ss.g, seeds, n_seeds, ss.seed_cnt.p, ss.ctl.p, ss.s));
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    const int32_t chunks = std::max(ss.hctl.p->seed_chunks, 1);
    IMIN_TRY(ss.seed_table.alloc((size_t)chunks));
    IMIN_TRY(ss.seed_col.alloc((size_t)chunks));
    IMIN_TRY(ss.seed_thr.alloc((size_t)chunks));
    IMIN_TRY(ss.thr_q.alloc((size_t)ss.g.m_pad));
    IMIN_TRY(imin::launch_seed_fill(ss.g, seeds, n_seeds, ss.seed_cnt.p, ss.seed_table.p, chunks, ss.ctl.p, ss.s));
    q = ss.make_query(seeds, n_seeds, rng_seed, chunks);
    return IMIN_OK;
}

// a solve's status, also written to its device_status word when given
static imin_status_t with_device_status(imin_status_t st, int32_t* device_status, void* stream) {
    if (device_status) {
        const hipStream_t s = (hipStream_t)stream;
        if (imin::launch_fill_i32(device_status, (int32_t)st, 1, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            if (st == IMIN_OK) st = IMIN_ERR_DEVICE;
        }
    }
    return st;
}

static imin_status_t solve_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                                uint64_t rng_seed, void* stream, int32_t* blockers, int64_t* gains,
                                int64_t* spread_totals, int32_t* n_selected) {
    g_last_flags = 0;
    if (!g || !seeds || !blockers || !gains || !spread_totals || !n_selected) return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n || k < 0 || k > g->g.n) return IMIN_ERR_INVALID;
    if (theta < 1 || theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    Session ss(g->g, s, g);
    imin_status_t st = ss.init((uint64_t)theta, true);
    if (st != IMIN_OK) return st;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, nullptr, 0, rng_seed, q);
    if (st != IMIN_OK) return st;
    // worlds are resident: per-world sizes for all theta, and the per-world
    // count lists when they fit (incremental rounds)
    IMIN_TRY(ss.world_size.alloc((size_t)theta));
    // the resident store when earlier calls on the graph suggest its entries
    // can be indexed with 32-bit unsigned positions (else plain rounds from
    // the start)
    const char* inc_env = std::getenv("IMIN_INCREMENTAL");
    const unsigned long long est =
        ((g->big_per_world.load() * (unsigned long long)theta) >> 10) +
        (unsigned long long)theta * (unsigned long long)imin::world_tier0_capacity();
    if (!(inc_env && inc_env[0] == '0') && est < imin::kIndexPosLimit) {
        st = ss.enable_store((uint64_t)theta);
        if (st != IMIN_OK) return st;
    }
    // rounds enqueued between two reads of the round counters: doubling from
    // IMIN_ROUND_BATCH up to 4x that, so that a long solve waits on the host
    // a few times only and one that stops early wastes few empty launches
    const size_t batch0 = env_size("IMIN_ROUND_BATCH", 32);
    size_t batch = batch0;
    const imin::SelectOut so = ss.select_out(k, blockers, gains, spread_totals, n_selected);
    g_last_mode = -1;
    for (int32_t r = 0; r <= k;) {
        if (r > 0 && ss.incremental) {
            st = ss.build_index((uint64_t)theta, nullptr);  // built once
            if (st != IMIN_OK) return st;
            // incremental rounds need no host decision: enqueue a batch; once
            // the selection stops, every later kernel returns at once
            const int32_t nb = (int32_t)std::min<size_t>(batch, (size_t)(k + 1 - r));
            for (int32_t i = 0; i < nb; ++i) {
                st = ss.delta_round(q, (uint64_t)theta, so);
                if (st != IMIN_OK) return st;
            }
            r += nb;
            batch = std::min(batch * 2, batch0 * 4);
        } else {
            IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
            IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
            st = ss.evaluate(q, 0, (uint64_t)theta, ss.world_size.p, nullptr, nullptr, r == 0);
            if (st != IMIN_OK) return st;
            // when incremental rounds follow, the first of them commits this
            // selection; otherwise a combining launch does
            const bool combine = !ss.incremental || k == 0;
            hipEvent_t ev = ss.timed.begin(3, s);
            IMIN_TRY(imin::launch_select(g->g, ss.gain.p, ss.ctl.p, so, ss.dsz.p, ss.dsz_n, combine, s));
            ss.timed.end(3, ev, s);
            ++r;
        }
        st = ss.read_ctl();
        if (st != IMIN_OK) return st;
        if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
            g_last_flags = ss.hctl.p->flags;
            return IMIN_ERR_INTERNAL;
        }
        if (ss.hctl.p->stop) break;
    }
    g_last_mode = ss.incremental ? 1 : 0;
    ss.finish();
    return IMIN_OK;
}

// ---- enqueued solves: a caller's workspace, nothing read back

// the largest level-0 table a seed set of n_seeds seeds can need
static int32_t chunk_bound(const imin::GraphDev& g, int32_t n_seeds) {
    const long long per = (long long)g.max_deg / 4 + 2;
    const long long all = g.m_pad / 4 + n_seeds;
    return (int32_t)std::max(1ll, std::min((long long)n_seeds * per, all));
}

// bytes a plan takes from a workspace
static size_t plan_bytes(imin_graph_t g, const WsPlan& p, uint64_t theta, int32_t n_seeds) {
    Arena sizing;
    ArenaScope as(&sizing);
    Session ss(g->g, nullptr, g);
    (void)ss.carve(p, theta, n_seeds);
    return sizing.used;
}

static void fixed_plan(imin_graph_t g, WsPlan& p, int32_t n_seeds, uint64_t theta) {
    const size_t n = (size_t)g->g.n;
    const size_t m1 = (size_t)std::max<int64_t>(g->g.m, 1);
    const size_t lc2 = std::min<size_t>(n, (size_t)1 << 16), xc2 = std::min<size_t>(m1, (size_t)1 << 16);
    const size_t base = n * 4 + (n + 31) / 32 * 4;
    const size_t bytes2 = base + 5 * lc2 * 4 + 12 + 2 * xc2 * 4;
    const size_t bytes3 = base + 5 * n * 4 + 12 + 2 * m1 * 4;
    const int cus = cu_count();
    // tier-2 slots: up to 4 GiB once some world of the graph has needed that
    // tier, else up to 256 MiB; one per resident workgroup at most
    const bool big = g->tier2_seen.load(std::memory_order_relaxed) || g->tier2_share.load() > 0;
    const size_t budget = big ? ((size_t)4 << 30) : ((size_t)256 << 20);
    p.slots = std::max<size_t>(1, std::min<size_t>(std::min<size_t>(budget / bytes2, (size_t)cus * 4), (size_t)theta));
    p.slots3 = std::max<size_t>(1, std::min<size_t>(((size_t)1 << 30) / bytes3, 8));
    p.chunk_cap = chunk_bound(g->g, n_seeds);
    // worlds start in tier 0 (whose fixed slots the layout has anyway), or
    // in tier 2 when most worlds of earlier calls ended up there: both
    // routes put the same worlds in the bump region, so the record of bump
    // entries per world sizes it either way
    p.start_tier = 0;
    if (const char* t = std::getenv("IMIN_START_TIER")) p.start_tier = std::max(0, std::min(2, std::atoi(t)));
    else if (g->tier2_share.load(std::memory_order_relaxed) > 512) p.start_tier = 2;
}

// incremental rounds index every scratch entry with a uint32 position
static bool incremental_fits(uint64_t theta, size_t big_cap) {
    const char* inc_env = std::getenv("IMIN_INCREMENTAL");
    if (inc_env && inc_env[0] == '0') return false;
    return theta * (uint64_t)imin::world_tier0_capacity() + big_cap < imin::kIndexPosLimit;
}

// bump-region entries (and as many extra edges) that earlier calls on the
// graph needed for theta worlds beyond tier 0 (0 before any record)
static unsigned long long hinted_bump(imin_graph_t g, uint64_t theta) {
    const uint64_t per = std::max(g->big_per_world.load(), g->xbig_per_world.load());
    return (per * (unsigned long long)theta) >> 10;
}

// The layout for a workspace of `bytes`: incremental rounds when they fit
// with a bump region that holds what the graph's record asks for, else
// plain rounds; the bump region takes what the fixed arrays leave.
static imin_status_t plan_for(imin_graph_t g, int32_t n_seeds, uint64_t theta, size_t bytes, WsPlan& out) {
    WsPlan p;
    fixed_plan(g, p, n_seeds, theta);
    const unsigned long long need = hinted_bump(g, theta);
    for (int inc = 1; inc >= 0; --inc) {
        p.incremental = inc == 1;
        if (p.incremental && !incremental_fits(theta, 0)) continue;
        p.big_cap = 0;
        const size_t base = plan_bytes(g, p, theta, n_seeds);
        if (base > bytes) continue;
        p.big_cap = (size_t)1 << 20;
        const size_t per = (plan_bytes(g, p, theta, n_seeds) - base + ((size_t)1 << 20) - 1) >> 20;
        size_t big = (bytes - base) / std::max<size_t>(per, 1);
        if (p.incremental)
            big = std::min<size_t>(big, (size_t)imin::kIndexPosLimit - 1 - theta * (size_t)imin::world_tier0_capacity());
        p.big_cap = big;
        while (p.big_cap > 0 && plan_bytes(g, p, theta, n_seeds) > bytes) p.big_cap -= std::min<size_t>(p.big_cap, 4096);
        // the larger incremental layout only when its bump region is not the
        // one to run out
        if (p.incremental && p.big_cap < need) continue;
        out = p;
        return IMIN_OK;
    }
    return IMIN_ERR_WORKSPACE;
}

// the graph's device-side hints folded into its host-side ones
static void fold_device_hints(imin_graph_t g) {
    // a stream of this thread's own, so that the read waits for nothing else
    thread_local hipStream_t hs = nullptr;
    thread_local int hs_dev = -1;
    if (!hs || hs_dev != g->device) {
        if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            hs = nullptr;
            return;
        }
        hs_dev = g->device;
    }
    unsigned long long h[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(h, g->hints_dev, sizeof(h), hipMemcpyDeviceToHost, hs) != hipSuccess ||
        hipStreamSynchronize(hs) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    raise_hint(g->big_per_world, h[0]);
    raise_hint(g->xbig_per_world, h[1]);
    raise_hint(g->tier1_share, h[2]);
    raise_hint(g->tier2_share, h[3]);
    if (h[3] > 0) g->tier2_seen.store(true, std::memory_order_relaxed);
}

// The workspace of an enqueued solve: the incremental layout when its
// entries can be indexed and it takes at most `limit` bytes, else the plain
// one.
static imin_status_t workspace_size_impl(imin_graph_t g, int32_t n_seeds, int32_t k, int64_t theta, size_t limit,
                                         size_t* bytes) {
    if (!g || !bytes || n_seeds < 1 || n_seeds > g->g.n || k < 0 || k > g->g.n || theta < 1 ||
        theta > (int64_t)0xFFFFFFFFll)
        return IMIN_ERR_INVALID;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != g->device) (void)hipSetDevice(g->device);
    fold_device_hints(g);
    WsPlan p;
    fixed_plan(g, p, n_seeds, (uint64_t)theta);
    // bump entries (and as many extra edges) for the worlds beyond tier 0, from
    // what earlier calls on the graph needed, with an eighth more
    const unsigned long long need = hinted_bump(g, (uint64_t)theta);
    p.big_cap = std::max<size_t>((size_t)1 << 20, (size_t)(need + need / 8 + 1024));
    p.incremental = incremental_fits((uint64_t)theta, p.big_cap);
    size_t b = plan_bytes(g, p, (uint64_t)theta, n_seeds);
    if (p.incremental && b > limit) {
        p.incremental = false;
        b = plan_bytes(g, p, (uint64_t)theta, n_seeds);
    }
    *bytes = b;
    if (prev >= 0 && prev != g->device) (void)hipSetDevice(prev);
    return IMIN_OK;
}

static imin_status_t solve_ws_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                                   uint64_t rng_seed, void* workspace, size_t workspace_bytes, void* stream,
                                   int32_t* blockers, int64_t* gains, int64_t* spread_totals, int32_t* n_selected,
                                   int32_t* device_status) {
    g_last_flags = 0;
    if (!g || !seeds || !blockers || !gains || !spread_totals || !n_selected || !device_status || !workspace)
        return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n || k < 0 || k > g->g.n) return IMIN_ERR_INVALID;
    if (theta < 1 || theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
    if ((uintptr_t)workspace % 256 != 0) return IMIN_ERR_INVALID;
    WsPlan plan;
    imin_status_t st = plan_for(g, n_seeds, (uint64_t)theta, workspace_bytes, plan);
    if (st != IMIN_OK) return st;
    Arena arena;
    arena.base = static_cast<char*>(workspace);
    arena.size = workspace_bytes;
    ArenaScope as(&arena);
    hipStream_t s = (hipStream_t)stream;
    Session ss(g->g, s, g);
    st = ss.carve(plan, (uint64_t)theta, n_seeds);
    if (arena.failed) return IMIN_ERR_WORKSPACE;
    if (st != IMIN_OK) return st;
    const imin::SelectOut so = ss.select_out(k, blockers, gains, spread_totals, n_selected);
    return ss.run_ws(seeds, n_seeds, k, (uint64_t)theta, rng_seed, plan.chunk_cap, so, device_status, g->hints_dev);
}

static imin_status_t evaluate_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                                   int32_t n_blocked, int64_t w_begin, int64_t w_count, uint64_t rng_seed,
                                   void* stream, int64_t* gain, int64_t* total, int32_t* world_size,
                                   int64_t* world_sum, int64_t* world_edges) {
    g_last_flags = 0;
    if (!g || !seeds || !gain || !total) return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n || n_blocked < 0 || (n_blocked > 0 && !blocked)) return IMIN_ERR_INVALID;
    if (w_begin < 0 || w_count < 1 || w_begin + w_count > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    Session ss(g->g, s, g);
    imin_status_t st = ss.init((uint64_t)w_count, false);
    if (st != IMIN_OK) return st;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, blocked, n_blocked, rng_seed, q);
    if (st != IMIN_OK) return st;
    IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
    IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
    st = ss.evaluate(q, (uint64_t)w_begin, (uint64_t)w_count, world_size, world_sum, world_edges);
    if (st != IMIN_OK) return st;
    IMIN_TRY(hipMemcpyAsync(gain, ss.gain.p, (size_t)g->g.n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    IMIN_TRY(hipMemcpyAsync(total, &ss.ctl.p->total, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
        g_last_flags = ss.hctl.p->flags;
        return IMIN_ERR_INTERNAL;
    }
    ss.finish();
    return IMIN_OK;
}

// Several from-scratch passes on one graph: every query is set up as
// imin_evaluate would set it up; the tier-0 and tier-1 launches of those that
// fit one tile starting at tier 0 become one packed launch each, after which
// each query finishes its pass (HBM tiers, reduction) as usual.
static imin_status_t evaluate_batch_impl(imin_graph_t g, const imin_eval_query_t* qs, int32_t nq, void* stream) {
    g_last_flags = 0;
    if (!g || nq < 0 || (nq > 0 && !qs)) return IMIN_ERR_INVALID;
    for (int32_t j = 0; j < nq; ++j) {
        const imin_eval_query_t& a = qs[j];
        if (!a.seeds || !a.gain || !a.total) return IMIN_ERR_INVALID;
        if (a.n_seeds < 1 || a.n_seeds > g->g.n || a.n_blocked < 0 || (a.n_blocked > 0 && !a.blocked))
            return IMIN_ERR_INVALID;
        if (a.w_begin < 0 || a.w_count < 1 || a.w_begin + a.w_count > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;
    }
    hipStream_t s = (hipStream_t)stream;
    const int32_t group = (int32_t)std::max<size_t>(1, std::min<size_t>(env_size("IMIN_PACK_QUERIES", 64), 4096));
    // Sessions nest their release scopes (each defers the blocks released
    // while it is the newest), so they end newest first, on every path.
    struct SessionStack {
        std::vector<std::unique_ptr<Session>> v;
        ~SessionStack() {
            while (!v.empty()) v.pop_back();
        }
        Session& back() { return *v.back(); }
        Session& operator[](size_t i) { return *v[i]; }
    };
    for (int32_t j0 = 0; j0 < nq; j0 += group) {
        const int32_t nb = std::min(group, nq - j0);
        SessionStack ss;
        std::vector<imin::QueryDev> qd((size_t)nb);
        std::vector<imin::PackedQuery> pk;
        std::vector<uint8_t> packed((size_t)nb, 0);
        uint64_t first = 0;
        int grid = 0, grid1 = 0;
        for (int32_t j = 0; j < nb; ++j) {
            const imin_eval_query_t& a = qs[j0 + j];
            ss.v.push_back(std::make_unique<Session>(g->g, s, g));
            Session& x = ss.back();
            x.budget_share = nb;  // the group's sessions hold their HBM-tier slots together
            imin_status_t st = x.init((uint64_t)a.w_count, false);
            if (st != IMIN_OK) return st;
            st = setup_query(x, a.seeds, a.n_seeds, a.blocked, a.n_blocked, a.rng_seed, qd[(size_t)j]);
            if (st != IMIN_OK) return st;
            IMIN_TRY(imin::launch_fill_i64(x.gain.p, 0, (size_t)g->g.n, s));
            IMIN_TRY(imin::launch_ctl_reset_round(x.ctl.p, s));
            if (x.packable((uint64_t)a.w_count) && first + (uint64_t)a.w_count <= 0xFFFFFFFFull) {
                imin::PackedQuery pq;
                st = x.packed_prepare(qd[(size_t)j], (uint64_t)a.w_begin, (uint64_t)a.w_count, a.world_size, pq);
                if (st != IMIN_OK) return st;
                pq.first = (uint32_t)first;
                first += (uint64_t)a.w_count;
                pk.push_back(pq);
                packed[(size_t)j] = 1;
                grid = std::max(grid, x.grid0);
                grid1 = std::max(grid1, x.grid1);
            }
        }
        DevArray<imin::PackedQuery> pk_dev;
        DevArray<uint32_t> counter;
        if (!pk.empty()) {
            IMIN_TRY(pk_dev.alloc(pk.size()));
            IMIN_TRY(counter.alloc(1));
            IMIN_TRY(hipMemcpyAsync(pk_dev.p, pk.data(), pk.size() * sizeof(imin::PackedQuery),
                                    hipMemcpyHostToDevice, s));
            IMIN_TRY(imin::launch_fill_i32((int32_t*)counter.p, 0, 1, s));
            IMIN_TRY(imin::launch_world_tier0_packed(g->g, pk_dev.p, (int)pk.size(), (uint32_t)first, counter.p, grid,
                                                     s));
            IMIN_TRY(imin::launch_world_tier1_packed(g->g, pk_dev.p, (int)pk.size(), grid1, s));
        }
        for (int32_t j = 0; j < nb; ++j) {
            const imin_eval_query_t& a = qs[j0 + j];
            Session& x = ss[(size_t)j];
            imin_status_t st = x.evaluate(qd[(size_t)j], (uint64_t)a.w_begin, (uint64_t)a.w_count, a.world_size,
                                          nullptr, nullptr, false, packed[(size_t)j] != 0);
            if (st != IMIN_OK) return st;
            IMIN_TRY(hipMemcpyAsync(a.gain, x.gain.p, (size_t)g->g.n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
            IMIN_TRY(hipMemcpyAsync(a.total, &x.ctl.p->total, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
            st = x.read_ctl();
            if (st != IMIN_OK) return st;
            if (x.hctl.p->flags & ~imin::kFlagDataMask) {
                g_last_flags = x.hctl.p->flags;
                return IMIN_ERR_INTERNAL;
            }
            x.finish();
        }
    }
    return IMIN_OK;
}

// ---- lower-bound coverage (Sections 4.1 and 5.1)

static imin_status_t check_coverage_args(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t theta) {
    if (!g || !seeds) return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n) return IMIN_ERR_INVALID;
    if (theta < 1 || theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
    return IMIN_OK;
}

static int bit_length(unsigned long long v) {
    int b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

// V'_s of a seed set given in device memory (Global Sampling): seeds are
// checked on the host first (range), then the search runs on the handle's
// host copy of the graph.  The handle keeps the last seed set's V'_s, so the
// calls of one solver (every iteration samples for the same seeds) search
// once.
static imin_status_t lrr_vprime(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, hipStream_t s,
                                std::vector<int32_t>& vp) {
    std::vector<int32_t> hs((size_t)n_seeds);
    IMIN_TRY(hipMemcpyAsync(hs.data(), seeds, hs.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    IMIN_TRY(hipStreamSynchronize(s));
    for (int32_t v : hs)
        if (v < 0 || v >= g->g.n) return IMIN_ERR_DATA;
    std::vector<int32_t> key(hs);
    std::sort(key.begin(), key.end());
    {
        std::lock_guard<std::mutex> lk(g->aux_mu);
        if (g->vp_valid && g->vp_seeds == key) {
            vp = g->vp_nodes;
            return IMIN_OK;
        }
    }
    const imin::HostGraph* h = imin::graph_host(g);
    if (!h) return IMIN_ERR_DEVICE;
    vp = imin::reachable_nonseeds(*h, hs);
    std::lock_guard<std::mutex> lk(g->aux_mu);
    g->vp_seeds = std::move(key);
    g->vp_nodes = vp;
    g->vp_valid = true;
    return IMIN_OK;
}

// Max-Coverage over the CP sequences of worlds [0, theta) or, with lrr, over
// the LRR sets of samples [0, theta)
static imin_status_t max_coverage_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k,
                                       int64_t theta, uint64_t rng_seed, void* stream, int32_t* blockers,
                                       int64_t* gains, int64_t* cov, int64_t* cov_upper, int32_t* n_selected,
                                       bool lrr = false) {
    g_last_flags = 0;
    imin_status_t st = check_coverage_args(g, seeds, n_seeds, theta);
    if (st != IMIN_OK) return st;
    if (!blockers || !gains || !cov || !cov_upper || !n_selected || k < 0 || k > g->g.n) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> vp;
    if (lrr && (st = lrr_vprime(g, seeds, n_seeds, s, vp)) != IMIN_OK) return st;
    Session ss(g->g, s, g);
    ss.lrr = lrr;
    // before init: HBM-tier slots carry preorder indexes for the trees
    ss.cover = lrr ? imin::kCoverNone : imin::kCoverStore;
    st = ss.init((uint64_t)theta, true);
    if (st != IMIN_OK) return st;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, nullptr, 0, rng_seed, q);
    if (st != IMIN_OK) return st;
    if (lrr && vp.empty()) {
        // no node can be reached: every set is empty, nothing is selected
        IMIN_TRY(imin::launch_fill_i64(cov, -1, (size_t)k + 1, s));
        IMIN_TRY(imin::launch_fill_i64(cov_upper, -1, (size_t)k + 1, s));
        IMIN_TRY(imin::launch_fill_i64(cov, 0, 1, s));
        IMIN_TRY(imin::launch_fill_i64(cov_upper, 0, 1, s));
        IMIN_TRY(imin::launch_fill_i32(n_selected, 0, 1, s));
        IMIN_TRY(hipStreamSynchronize(s));
        return IMIN_OK;
    }
    if (lrr && (st = ss.setup_lrr(g, vp)) != IMIN_OK) return st;
    IMIN_TRY(ss.world_size.alloc((size_t)theta));
    // the store (dominator trees, or LRR sets): positions are uint32 in the index
    ss.store_budget = std::min<size_t>(env_size("IMIN_COVER_STORE_CAP", (size_t)imin::kIndexPosLimit - 1),
                                       (size_t)imin::kIndexPosLimit - 1);
    IMIN_TRY(ss.store_off.alloc((size_t)theta));
    IMIN_TRY(ss.store_len.alloc((size_t)theta));
    IMIN_TRY(ss.list0.alloc((size_t)theta));
    if (!lrr) {
        IMIN_TRY(ss.scr_par.alloc(ss.scr_node.count));
        IMIN_TRY(ss.scr_lab.alloc(ss.scr_node.count));
    }
    ss.incremental = true;
    ss.label_rule = false;
    IMIN_TRY(imin::launch_fill_i64(cov, -1, (size_t)k + 1, s));
    IMIN_TRY(imin::launch_fill_i64(cov_upper, -1, (size_t)k + 1, s));
    IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
    IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
    st = ss.evaluate(q, 0, (uint64_t)theta, ss.world_size.p, nullptr, nullptr, true);
    if (st != IMIN_OK) return st;
    if (!ss.incremental) return IMIN_ERR_NOMEM;  // the store did not fit
    // the index is sized from the store's entry count, which the last tile's
    // compaction raised after the pass last read the counters
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    st = ss.build_index((uint64_t)theta, nullptr);
    if (st != IMIN_OK) return st;
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
        g_last_flags = ss.hctl.p->flags;
        return IMIN_ERR_INTERNAL;
    }
    DevArray<uint32_t> hist_cnt;
    DevArray<long long> hist_sum, state;
    DevArray<int64_t> totals;
    IMIN_TRY(hist_cnt.alloc(imin::kTopkBins));
    IMIN_TRY(hist_sum.alloc(imin::kTopkBins));
    IMIN_TRY(state.alloc(4));
    IMIN_TRY(totals.alloc((size_t)k + 1));
    IMIN_TRY(imin::launch_fill_i32((int32_t*)hist_cnt.p, 0, imin::kTopkBins, s));
    IMIN_TRY(imin::launch_fill_i64((int64_t*)hist_sum.p, 0, imin::kTopkBins, s));
    imin::CoverOut co{};
    co.cov = cov;
    co.cov_upper = cov_upper;
    co.t0 = ss.hctl.p->total;
    co.k = k;
    co.hist_cnt = hist_cnt.p;
    co.hist_sum = hist_sum.p;
    co.state = state.p;
    const int key_bits = std::max(1, bit_length((unsigned long long)std::max<long long>(co.t0, 1)));
    const imin::SelectOut so = ss.select_out(k, blockers, gains, totals.p, n_selected);
    const imin::TileOut out = ss.tile_out();
    const int grid = std::min<int>(ss.dsz_n, cu_count() * 8);
    for (int32_t r = 0; r <= k; ++r) {
        IMIN_TRY(imin::launch_cover_round(g->g, ss.gain.p, ss.ctl.p, so, co, r, key_bits, out, ss.idx_off.p,
                                          ss.idx_ent.p, ss.dsz.p, ss.dsz_n, grid, lrr, s));
        if ((r & 31) == 31 || r == k) {
            st = ss.read_ctl();
            if (st != IMIN_OK) return st;
            if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
                g_last_flags = ss.hctl.p->flags;
                return IMIN_ERR_INTERNAL;
            }
            if (ss.hctl.p->stop) break;
        }
    }
    ss.finish();
    return IMIN_OK;
}

static imin_status_t coverage_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* set,
                                   int32_t n_set, int64_t theta, uint64_t rng_seed, void* stream, int64_t* covered,
                                   bool lrr = false) {
    g_last_flags = 0;
    imin_status_t st = check_coverage_args(g, seeds, n_seeds, theta);
    if (st != IMIN_OK) return st;
    if (!covered || n_set < 0 || (n_set > 0 && !set)) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> vp;
    if (lrr && (st = lrr_vprime(g, seeds, n_seeds, s, vp)) != IMIN_OK) return st;
    Session ss(g->g, s, g);
    ss.lrr = lrr;
    ss.cover = imin::kCoverCount;
    st = ss.init((uint64_t)theta, false);
    if (st != IMIN_OK) return st;
    if (lrr && vp.empty()) {
        IMIN_TRY(imin::launch_fill_i64(covered, 0, 1, s));
        IMIN_TRY(hipStreamSynchronize(s));
        return IMIN_OK;
    }
    if (lrr && (st = ss.setup_lrr(g, vp)) != IMIN_OK) return st;
    // the marked set, checked as a blocked set would be (in range, no seed)
    DevArray<uint32_t> mark;
    IMIN_TRY(mark.alloc(((size_t)g->g.n + 31) / 32));
    IMIN_TRY(imin::launch_query_setup(g->g, seeds, n_seeds, set, n_set, mark.p, ss.ctl.p, s));
    ss.cover_mark = mark.p;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, nullptr, 0, rng_seed, q);
    if (st != IMIN_OK) return st;
    IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
    IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
    st = ss.evaluate(q, 0, (uint64_t)theta, nullptr, nullptr, nullptr);
    if (st != IMIN_OK) return st;
    IMIN_TRY(hipMemcpyAsync(covered, &ss.ctl.p->total, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
        g_last_flags = ss.hctl.p->flags;
        return IMIN_ERR_INTERNAL;
    }
    ss.finish();
    return IMIN_OK;
}

static imin_status_t world_sizes_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                                      int32_t n_blocked, int64_t w_begin, int64_t w_count, uint64_t rng_seed,
                                      void* stream, int32_t* world_size) {
    g_last_flags = 0;
    if (!g || !seeds || !world_size) return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n || n_blocked < 0 || (n_blocked > 0 && !blocked)) return IMIN_ERR_INVALID;
    if (w_begin < 0 || w_count < 1 || w_begin + w_count > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    Session ss(g->g, s, g);
    ss.sizes_only = 1;
    imin_status_t st = ss.init((uint64_t)w_count, false);
    if (st != IMIN_OK) return st;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, blocked, n_blocked, rng_seed, q);
    if (st != IMIN_OK) return st;
    IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
    IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
    st = ss.evaluate(q, (uint64_t)w_begin, (uint64_t)w_count, world_size, nullptr, nullptr);
    if (st != IMIN_OK) return st;
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
        g_last_flags = ss.hctl.p->flags;
        return IMIN_ERR_INTERNAL;
    }
    ss.finish();
    return IMIN_OK;
}

static imin_status_t reach_counts_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t w_begin,
                                       int64_t w_count, uint64_t rng_seed, void* stream, int64_t* counts,
                                       int32_t* world_size) {
    g_last_flags = 0;
    if (!g || !seeds || !counts) return IMIN_ERR_INVALID;
    if (n_seeds < 1 || n_seeds > g->g.n) return IMIN_ERR_INVALID;
    if (w_begin < 0 || w_count < 1 || w_begin + w_count > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;
    hipStream_t s = (hipStream_t)stream;
    Session ss(g->g, s, g);
    ss.unit_counts = 1;
    imin_status_t st = ss.init((uint64_t)w_count, false);
    if (st != IMIN_OK) return st;
    imin::QueryDev q{};
    st = setup_query(ss, seeds, n_seeds, nullptr, 0, rng_seed, q);
    if (st != IMIN_OK) return st;
    IMIN_TRY(imin::launch_fill_i64(ss.gain.p, 0, (size_t)g->g.n, s));
    IMIN_TRY(imin::launch_ctl_reset_round(ss.ctl.p, s));
    st = ss.evaluate(q, (uint64_t)w_begin, (uint64_t)w_count, world_size, nullptr, nullptr);
    if (st != IMIN_OK) return st;
    IMIN_TRY(hipMemcpyAsync(counts, ss.gain.p, (size_t)g->g.n * sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    st = ss.read_ctl();
    if (st != IMIN_OK) return st;
    if (ss.hctl.p->flags & ~imin::kFlagDataMask) {
        g_last_flags = ss.hctl.p->flags;
        return IMIN_ERR_INTERNAL;
    }
    ss.finish();
    return IMIN_OK;
}

// Launch-shape tuning: from-scratch passes of the caller's query at several
// tier-0 grid sizes, the fastest kept on the handle.  Every candidate must
// give the same gains and total (the world-to-workgroup mapping never
// changes an integer); a difference is reported as IMIN_ERR_INTERNAL.
static imin_status_t autotune_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t theta,
                                   uint64_t rng_seed, void* stream, int32_t* best_pct, float* best_ms) {
    if (!g || !seeds || !best_pct || theta < 1 || theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
    static const int32_t kPct[] = {kDefaultGrid0Pct, 50, 75, 100, 150, 300};  // the default first
    constexpr int kCand = (int)(sizeof(kPct) / sizeof(kPct[0]));
    constexpr int kReps = 7;  // the first round warms the caches
    hipStream_t s = (hipStream_t)stream;
    const size_t n = (size_t)g->g.n;
    DevArray<int64_t> gain, total;
    IMIN_TRY(gain.alloc(n));
    IMIN_TRY(total.alloc(1));
    std::vector<int64_t> ref, cur;
    int64_t ref_total = -1;
    hipEvent_t e0 = event_acquire(), e1 = event_acquire();
    if (!e0 || !e1) {
        event_release(e0);
        event_release(e1);
        return IMIN_ERR_DEVICE;
    }
    const int32_t saved = g->tuned_grid0_pct.load();
    std::vector<std::vector<float>> times(kCand);
    imin_status_t st = IMIN_OK;
    // candidates interleaved, so that drift in the device's state spreads
    // over all of them
    for (int rep = 0; rep < kReps && st == IMIN_OK; ++rep) {
        for (int c = 0; c < kCand && st == IMIN_OK; ++c) {
            g->tuned_grid0_pct.store(kPct[c]);
            if (hipEventRecord(e0, s) != hipSuccess) st = IMIN_ERR_DEVICE;
            if (st == IMIN_OK)
                st = evaluate_impl(g, seeds, n_seeds, nullptr, 0, 0, theta, rng_seed, stream, gain.p, total.p,
                                   nullptr, nullptr, nullptr);
            float t = 0.f;
            if (st == IMIN_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                  hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                st = IMIN_ERR_DEVICE;
            if (st != IMIN_OK) break;
            if (rep > 0) times[(size_t)c].push_back(t);
            if (rep == 0) {
                // every shape gives the same integers
                cur.resize(n);
                int64_t tot = 0;
                if (hipMemcpy(cur.data(), gain.p, n * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
                    hipMemcpy(&tot, total.p, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess) {
                    st = IMIN_ERR_DEVICE;
                } else if (ref_total < 0) {
                    ref.swap(cur);
                    ref_total = tot;
                } else if (tot != ref_total || cur != ref) {
                    st = IMIN_ERR_INTERNAL;
                }
            }
        }
    }
    event_release(e0);
    event_release(e1);
    (void)hipGetLastError();
    if (st != IMIN_OK) {
        g->tuned_grid0_pct.store(saved);
        return st;
    }
    auto median = [](std::vector<float> v) {
        std::sort(v.begin(), v.end());
        return v[v.size() / 2];
    };
    // another shape replaces the default only when its median pass is at
    // least 3% faster
    int best = 0;
    float best_t = median(times[0]);
    for (int c = 1; c < kCand; ++c) {
        const float t = median(times[(size_t)c]);
        if (t < best_t * 0.97f && (best == 0 || t < best_t)) {
            best = c;
            best_t = t;
        }
    }
    g->tuned_grid0_pct.store(kPct[best]);
    *best_pct = kPct[best];
    if (best_ms) *best_ms = best_t;
    return IMIN_OK;
}

// No C++ exception crosses the boundary: host allocations that fail inside a
// call end it with IMIN_ERR_NOMEM (its session drains its stream while
// unwinding).
}  // extern "C"

namespace imin {
imin_status_t solve_workspace_size_within(imin_graph_t g, int32_t n_seeds, int32_t k, int64_t theta, size_t limit,
                                          size_t* bytes) {
    try {
        return workspace_size_impl(g, n_seeds, k, theta, limit, bytes);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t solve_enqueued(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                             uint64_t rng_seed, void* workspace, size_t workspace_bytes, void* stream,
                             int32_t* blockers, int64_t* gains, int64_t* spread_totals, int32_t* n_selected,
                             int32_t* device_status) {
    try {
        return solve_ws_impl(g, seeds, n_seeds, k, theta, rng_seed, workspace, workspace_bytes, stream, blockers,
                             gains, spread_totals, n_selected, device_status);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

int graph_device(imin_graph_t g) { return g ? g->device : -1; }

const HostGraph* graph_host(imin_graph_t g) {
    if (!g) return nullptr;
    std::lock_guard<std::mutex> lk(g->aux_mu);
    if (g->host) return g->host.get();
    auto h = std::make_unique<HostGraph>();
    h->n = g->g.n;
    h->m = g->g.m;
    h->row_ptr.resize((size_t)h->n + 1);
    h->col.resize((size_t)std::max<int64_t>(h->m, 1));
    h->thr.resize((size_t)std::max<int64_t>(h->m, 1));
    if (imin_graph_export(g, h->row_ptr.data(), h->col.data(), h->thr.data()) != IMIN_OK) return nullptr;
    g->host = std::move(h);
    return g->host.get();
}

bool graph_in_edges(imin_graph_t g, const int32_t** in_off, const int4** in_rec) {
    const HostGraph* h = graph_host(g);
    if (!h) return false;
    std::lock_guard<std::mutex> lk(g->aux_mu);
    if (!g->in_off) {
        // counting sort of the edges by head
        const size_t n = (size_t)h->n, m = (size_t)h->m;
        std::vector<int32_t> off(n + 1, 0);
        std::vector<int4> rec(std::max<size_t>(m, 1), int4{0, 0, 0, 0});
        for (size_t e = 0; e < m; ++e) off[(size_t)h->col[e] + 1] += 1;
        for (size_t v = 0; v < n; ++v) off[v + 1] += off[v];
        std::vector<int32_t> cur(off.begin(), off.end() - 1);
        for (size_t u = 0; u < n; ++u)
            for (int64_t e = h->row_ptr[u]; e < h->row_ptr[u + 1]; ++e) {
                const int32_t at = cur[(size_t)h->col[(size_t)e]]++;
                rec[(size_t)at] = int4{(int32_t)u, (int32_t)e, (int32_t)h->thr[(size_t)e], 0};
            }
        int32_t* a = nullptr;
        int4* b = nullptr;
        if (hipMalloc((void**)&a, off.size() * sizeof(int32_t)) != hipSuccess ||
            hipMalloc((void**)&b, rec.size() * sizeof(int4)) != hipSuccess ||
            hipMemcpy(a, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b, rec.data(), rec.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            if (a) (void)hipFree(a);
            if (b) (void)hipFree(b);
            return false;
        }
        g->in_off = a;
        g->in_rec = b;
    }
    *in_off = g->in_off;
    *in_rec = g->in_rec;
    return true;
}

std::vector<int32_t> reachable_nonseeds(const HostGraph& h, const std::vector<int32_t>& seeds) {
    std::vector<uint8_t> seen((size_t)h.n, 0), is_seed((size_t)h.n, 0);
    std::vector<int32_t> queue;
    for (int32_t v : seeds) {
        is_seed[(size_t)v] = 1;
        if (!seen[(size_t)v]) {
            seen[(size_t)v] = 1;
            queue.push_back(v);
        }
    }
    for (size_t head = 0; head < queue.size(); ++head) {
        const int32_t u = queue[head];
        for (int64_t e = h.row_ptr[(size_t)u]; e < h.row_ptr[(size_t)u + 1]; ++e) {
            const int32_t x = h.col[(size_t)e];
            if (h.thr[(size_t)e] == 0u || seen[(size_t)x]) continue;
            seen[(size_t)x] = 1;
            queue.push_back(x);
        }
    }
    std::vector<int32_t> out;
    for (int32_t v = 0; v < h.n; ++v)
        if (seen[(size_t)v] && !is_seed[(size_t)v]) out.push_back(v);
    return out;
}
}  // namespace imin

extern "C" {

imin_status_t imin_solve(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                         uint64_t rng_seed, void* workspace, size_t workspace_bytes, void* stream, int32_t* blockers,
                         int64_t* gains, int64_t* spread_totals, int32_t* n_selected, int32_t* device_status) {
    try {
        if (workspace)
            return solve_ws_impl(g, seeds, n_seeds, k, theta, rng_seed, workspace, workspace_bytes, stream, blockers,
                                 gains, spread_totals, n_selected, device_status);
        const imin_status_t st = solve_impl(g, seeds, n_seeds, k, theta, rng_seed, stream, blockers, gains,
                                            spread_totals, n_selected);
        return st == IMIN_ERR_INVALID ? st : with_device_status(st, device_status, stream);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_solve_workspace_size(imin_graph_t g, int32_t n_seeds, int32_t k, int64_t theta, size_t* bytes) {
    try {
        // the incremental layout while it fits the device's memory
        size_t limit = SIZE_MAX;
        if (g) {
            int prev = -1;
            (void)hipGetDevice(&prev);
            if (prev != g->device) (void)hipSetDevice(g->device);
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) limit = total_b;
            else (void)hipGetLastError();
            if (prev >= 0 && prev != g->device) (void)hipSetDevice(prev);
        }
        return workspace_size_impl(g, n_seeds, k, theta, limit, bytes);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_evaluate(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                            int32_t n_blocked, int64_t w_begin, int64_t w_count, uint64_t rng_seed, void* stream,
                            int64_t* gain, int64_t* total, int32_t* world_size, int64_t* world_sum,
                            int64_t* world_edges) {
    try {
        return evaluate_impl(g, seeds, n_seeds, blocked, n_blocked, w_begin, w_count, rng_seed, stream, gain, total,
                             world_size, world_sum, world_edges);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_evaluate_batch(imin_graph_t g, const imin_eval_query_t* queries, int32_t n_queries,
                                  void* stream) {
    try {
        return evaluate_batch_impl(g, queries, n_queries, stream);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_max_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                                uint64_t rng_seed, void* stream, int32_t* blockers, int64_t* gains, int64_t* cov,
                                int64_t* cov_upper, int32_t* n_selected) {
    try {
        return max_coverage_impl(g, seeds, n_seeds, k, theta, rng_seed, stream, blockers, gains, cov, cov_upper,
                                 n_selected);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* set, int32_t n_set,
                            int64_t theta, uint64_t rng_seed, void* stream, int64_t* covered) {
    try {
        return coverage_impl(g, seeds, n_seeds, set, n_set, theta, rng_seed, stream, covered);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_lrr_max_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                                    uint64_t key, void* stream, int32_t* blockers, int64_t* gains, int64_t* cov,
                                    int64_t* cov_upper, int32_t* n_selected) {
    try {
        return max_coverage_impl(g, seeds, n_seeds, k, theta, key, stream, blockers, gains, cov, cov_upper,
                                 n_selected, true);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_lrr_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* set,
                                int32_t n_set, int64_t theta, uint64_t key, void* stream, int64_t* covered) {
    try {
        return coverage_impl(g, seeds, n_seeds, set, n_set, theta, key, stream, covered, true);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_vprime(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, void* stream, int32_t* out,
                          int32_t* count) {
    if (!g || !seeds || !count || n_seeds < 1 || n_seeds > g->g.n) return IMIN_ERR_INVALID;
    try {
        std::vector<int32_t> vp;
        const imin_status_t st = lrr_vprime(g, seeds, n_seeds, (hipStream_t)stream, vp);
        if (st != IMIN_OK) return st;
        *count = (int32_t)vp.size();
        if (out && !vp.empty() &&
            hipMemcpy(out, vp.data(), vp.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            return IMIN_ERR_DEVICE;
        }
        return IMIN_OK;
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    }
}

imin_status_t imin_world_sizes(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                               int32_t n_blocked, int64_t w_begin, int64_t w_count, uint64_t rng_seed, void* stream,
                               int32_t* world_size) {
    try {
        return world_sizes_impl(g, seeds, n_seeds, blocked, n_blocked, w_begin, w_count, rng_seed, stream,
                                world_size);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_reach_counts(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t w_begin,
                                int64_t w_count, uint64_t rng_seed, void* stream, int64_t* counts,
                                int32_t* world_size) {
    try {
        return reach_counts_impl(g, seeds, n_seeds, w_begin, w_count, rng_seed, stream, counts, world_size);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_autotune(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t theta, uint64_t rng_seed,
                            void* stream, int32_t* grid0_pct, float* pass_ms) {
    try {
        return autotune_impl(g, seeds, n_seeds, theta, rng_seed, stream, grid0_pct, pass_ms);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

imin_status_t imin_set_launch_shape(imin_graph_t g, int32_t grid0_pct) {
    if (!g || grid0_pct < 0 || grid0_pct > 1000) return IMIN_ERR_INVALID;
    g->tuned_grid0_pct.store(grid0_pct);
    return IMIN_OK;
}

imin_status_t imin_cache_release(void) {
    g_cache.release_all();
    return IMIN_OK;
}

imin_status_t imin_timing_enable(int on) {
    g_timing.on.store(on != 0);
    return IMIN_OK;
}

imin_status_t imin_timing_mask(uint32_t kernel_mask) {
    g_timing.mask.store(kernel_mask);
    return IMIN_OK;
}

imin_status_t imin_timing_sample(int every) {
    if (every < 1) return IMIN_ERR_INVALID;
    g_timing.every.store(every);
    return IMIN_OK;
}

imin_status_t imin_timing_tallies(int on) {
    g_timing.tallies.store(on != 0);
    return IMIN_OK;
}

imin_status_t imin_timing_launches(int kernel_id, int64_t* all) {
    if (kernel_id < 0 || kernel_id >= kTimedKernels || !all) return IMIN_ERR_INVALID;
    *all = g_timing.seen[kernel_id].load();
    return IMIN_OK;
}

imin_status_t imin_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    for (int i = 0; i < kTimedKernels; ++i) {
        g_timing.launches[i] = 0;
        g_timing.ms[i] = 0.0;
        g_timing.seen[i].store(0);
    }
    for (int i = 0; i < kWorkTiers; ++i)
        for (int f = 0; f < imin::kWorkFields; ++f) g_timing.work[i][f] = 0;
    return IMIN_OK;
}

imin_status_t imin_timing_work(int tier, int64_t* worlds, int64_t* edges, int64_t* bytes, int64_t* reached,
                               int64_t* live) {
    if (tier < 0 || tier >= kWorkTiers) return IMIN_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    int64_t* const outs[imin::kWorkFields] = {worlds, edges, bytes, reached, live};
    for (int f = 0; f < imin::kWorkFields; ++f)
        if (outs[f]) *outs[f] = g_timing.work[tier][f];
    return IMIN_OK;
}

imin_status_t imin_timing_read(int kernel_id, int64_t* launches, double* total_ms) {
    if (kernel_id < 0 || kernel_id >= kTimedKernels) return IMIN_ERR_INVALID;
    std::lock_guard<std::mutex> lk(g_timing.mu);
    if (launches) *launches = g_timing.launches[kernel_id];
    if (total_ms) *total_ms = g_timing.ms[kernel_id];
    return IMIN_OK;
}

}  // extern "C"
