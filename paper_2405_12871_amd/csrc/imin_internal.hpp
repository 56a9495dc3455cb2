// Internal declarations shared by the device code and the host C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace imin {

constexpr uint32_t kAlwaysLive = 0xFFFFFFFFu;

// Device status bits (RoundCtl::flags).
enum : uint32_t {
    kFlagBadCol = 1u << 0,
    kFlagBadProb = 1u << 1,
    kFlagBadOffsets = 1u << 2,
    kFlagBadSeed = 1u << 3,
    kFlagDupSeed = 1u << 4,
    kFlagBlockedSeed = 1u << 5,
    kFlagBadBlocked = 1u << 6,
    kFlagDataMask = 0xFFu,
    kFlagPairOverflow = 1u << 8,   // pair buffer too small for the tile: redo
    kFlagBigCapacity = 1u << 9,    // big-world scratch too small
    kFlagSpreadMismatch = 1u << 10, // T_{r+1} != T_r - gain_r
    kFlagDomPasses = 1u << 11,      // dominator passes did not settle
    kFlagStoreOverflow = 1u << 12,  // resident per-world store too small
    kFlagReduceCapacity = 1u << 13, // more entries than the reduction's buffers hold
    kFlagBounds = 1u << 14,         // a per-world range fell outside its buffer
    // a solve cannot go on once any of these is set
    kFlagFatalMask = kFlagDataMask | kFlagPairOverflow | kFlagBigCapacity | kFlagSpreadMismatch | kFlagDomPasses |
                     kFlagStoreOverflow | kFlagReduceCapacity | kFlagBounds,
    // of those, the ones that mean a caller's workspace was too small
    kFlagCapacityMask = kFlagPairOverflow | kFlagStoreOverflow | kFlagReduceCapacity
};

// Graph as kept by a handle.  col/thr are padded with 4..7 trailing entries
// so that 16-byte loads of any 4-aligned group of slots stay in bounds.
struct GraphDev {
    int32_t n;
    int64_t m;
    int64_t m_pad;
    int32_t* off;  // [n+1]
    int32_t* col;  // [m_pad]
    uint32_t* thr; // [m_pad]
    int32_t max_deg;  // largest out-degree
};

// Round and tile counters, one instance in device memory per call.
struct RoundCtl {
    uint32_t flags;
    int32_t stop;
    int32_t round;
    int32_t round_snap;      // the round as the last partial selection saw it
    int32_t ustar;
    uint32_t next[3];        // work counters of the LDS world tiers (chunks handed out)
    // worlds listed for a later kernel: [0] changed worlds (rounds without
    // replay), [1] from tier 0 or the replay workgroups, [2] from tier 1,
    // [3] from the wide replay, [4] from tier 2 (for tier 3)
    uint32_t list_n[5];
    unsigned long long pair_count;
    long long total;         // sum of |R_w| over the worlds evaluated this round
    long long expect_total;  // T_r - gain_r from the previous selection (-1: none)
    long long best_gain;
    long long seed_sum;      // sum of the seed ids
    long long seed_edges;    // CSR slots leaving the seeds
    int32_t seed_chunks;     // entries of the level-0 slot-group table
    int32_t pad1;
    unsigned long long store_count;  // pairs held by the resident per-world store
    unsigned long long big_count;    // entries bump-allocated by tier-1/2 worlds this tile
    unsigned long long tile_total;   // entries the tile's worlds wrote (sum of lengths)
    unsigned long long xbig_count;   // extra edges bump-allocated this tile
    unsigned long long xtile_total;  // extra edges the tile's worlds wrote
    unsigned long long xstore_count; // extra edges held for replay
    uint32_t replay_big;             // some world stored in round 0 exceeds the replay's limits
};

// Fields of a per-workgroup work tally: worlds, edges, bytes, reached nodes,
// live edges.
constexpr int kWorkFields = 5;

// How a world evaluation reports its counts.
enum : int {
    kModePlain = 0,  // (node, c) pairs of the world into the tile pair buffer
    kModeStore = 1,  // pairs into the resident store, which the reduction reads
    kModeDelta = 2   // re-evaluation: (node, c_new - c_old) for every change
                     // against the stored list, then the list is replaced
};

// Scratch of the workgroup-per-world path, one slot per resident workgroup.
struct BigSlots {
    int32_t n_slots;
    int32_t lid_cap;   // nodes a world may reach (nodes/parent/idom/aux entries; lvl has lid_cap + 3)
    int64_t xcap;      // extra-edge capacity per slot
    int32_t vis_words; // (n + 31) / 32
    uint32_t* vis;     // [slots][vis_words] visited bitsets (zero between worlds; unused when they fit LDS)
    int32_t* lid_of;   // [slots][n]   node -> local id, valid while its visited bit is set
    int32_t* nodes;    // [slots][lid_cap]
    int32_t* parent;   // [slots][lid_cap]
    int32_t* idom;     // [slots][lid_cap]
    int32_t* aux;      // [slots][lid_cap]
    int32_t* tin;      // [slots][lid_cap] dominator-tree preorder indexes (coverage store)
    int32_t* lvl;      // [slots][lid_cap+3]
    int32_t* xv;       // [slots][xcap]
    int32_t* xu;       // [slots][xcap]
    int32_t* xv2;      // [slots][xcap] the extra edges sorted by their head's BFS level
    int32_t* xu2;      // [slots][xcap]
};

// Everything a tile of world evaluations writes.
//
// World evaluations first write their (node, count) entries to a scratch
// space with no shared counter: a tier-0 world at its own fixed slot
// (wi * slot_cap0), a larger world at a bump-allocated place after big_base
// (few and large, so the shared counter is cheap).  With one tile for all
// worlds that scratch is kept as the resident store; otherwise a compaction
// kernel packs the entries densely, with one counter update per workgroup.
// In incremental rounds a world's counts are updated in place, at its own
// stored-list positions, which it alone owns.
// A changed world of an incremental round with what its replay reads first
// (gathered by the replay workgroup that lists it).
struct ReplayItem {
    int64_t store_off;   // its (node, count, parent, label) entries
    int64_t xstore_off;  // its extra live edges (replay only)
    int32_t w;
    int32_t store_len;
    int32_t xstore_len;
    int32_t world_size;  // reached nodes before this round
    int32_t j;           // entry of the new blocker
    int32_t cj;          // its count
    uint32_t labj;       // its label
    int32_t flags;       // the world's kWorld* flags
};

// Per-world state of the resident store.
enum : uint8_t {
    kWorldLabelled = 2,  // the stored labels describe the world's dominator tree
};

// Dominator-tree label of a stored entry: preorder index (bits 16-31), the
// length of its subtree's index range (bits 0-14; the subtree of an entry is
// the entries whose preorder index lies in [index, index + length)), and an
// exit bit (15): set when some live edge between reached nodes leads from
// the subtree to a node outside it.  Labelled worlds hold at most 2048
// non-seeds, so both fields fit.
constexpr uint32_t kLabelExit = 0x8000u;
__host__ __device__ constexpr uint32_t pack_label(int tin, int size, bool exits) {
    return ((uint32_t)tin << 16) | (exits ? kLabelExit : 0u) | ((uint32_t)size & 0x7FFFu);
}
__host__ __device__ constexpr int label_tin(uint32_t lab) { return (int)(lab >> 16); }
__host__ __device__ constexpr int label_size(uint32_t lab) { return (int)(lab & 0x7FFFu); }
__host__ __device__ constexpr bool label_exits(uint32_t lab) { return (lab & kLabelExit) != 0; }

struct TileOut {
    int mode;
    int32_t* scr_node;
    int32_t* scr_cnt;
    unsigned long long slot_cap0;  // entries per tier-0 slot
    unsigned long long big_base;   // first entry of the bump region
    unsigned long long scr_cap;    // entries in the scratch space
    int64_t* wloc;                 // [tile] scratch start of each world's entries
    int32_t* wlen;                 // [tile] entries per world; [theta] changes per world (incremental)
    // resident per-world store (solve only), indexed by world id
    int32_t* store_node;
    int32_t* store_cnt;
    unsigned long long store_cap;
    int64_t* store_off;  // [theta]
    int32_t* store_len;  // [theta]
    int64_t* gain;       // incremental rounds: count changes are added here
    uint32_t list_cap;   // entries of the changed-world list
    uint32_t next_cap;   // entries of each list handed down to tier 1 / 2
    int32_t* world_size; // [tile] or nullptr
    int64_t* world_sum;  // [tile] or nullptr
    int64_t* world_edges;// [tile] or nullptr: CSR slots scanned (coins drawn)
    unsigned long long* work;  // [tiers][kWorkFields fields][work_stride] per-workgroup tallies
    int work_stride;
    // Live edges kept for replay (solve only).  In round 0 each world also
    // writes, aligned with its entries, the BFS parent of each node, and its
    // extra live edges (v, u); all as local ids of that round-0 evaluation.
    int keep_edges;
    int32_t* scr_par;     // aligned with scr_node
    int32_t* store_par;   // aligned with store_node
    int32_t* xscr_v;      // extra-edge scratch: fixed tier-0 slots, then a bump region
    int32_t* xscr_u;
    unsigned long long xslot_cap0;
    unsigned long long xbig_base;
    unsigned long long xscr_cap;
    int64_t* xloc;        // [tile]
    int32_t* xlen;        // [tile]
    int32_t* xstore_v;
    int32_t* xstore_u;
    unsigned long long xstore_cap;
    int64_t* xstore_off;  // [theta]
    int32_t* xstore_len;  // [theta]
    // Label rule: when no live edge leads out of the new blocker's dominator
    // subtree, blocking it removes exactly that subtree and leaves the rest
    // of the dominator tree as it was; the entries carry their labels.
    uint32_t* scr_lab;     // aligned with scr_node
    uint32_t* store_lab;   // aligned with store_node
    uint8_t* world_flags;  // [theta] kWorld* flags
    // Incremental rounds: nodes each workgroup's worlds lost, one slot per
    // (kernel, workgroup); summed and cleared by the selection.
    long long* dsz;
    int32_t dsz_off[7];   // slot ranges of tier 0, 1, 2, replay, label rule, wide replay, tier 3
    // Lower-bound coverage (kCover*): worlds are sampled without blockers and
    // their dominator trees kept (kCoverStore) or met against a set of
    // marked nodes (kCoverCount); unit_counts makes every entry count 1, so
    // that the reduced gains are per-node reach counts.
    int cover;
    const uint32_t* mark;  // [n bits] kCoverCount: the set whose coverage is counted
    int unit_counts;
    // only |R_w| per world: no dominators, no entries (stopping rules)
    int sizes_only;
    // Level 0 drawn ahead for the tile's worlds (or null): world i's live
    // seed slots as bits, words [i * l0_words, (i + 1) * l0_words), bit
    // 4j + q for slot q of level-0 slot group j.  Set only for tiles of
    // consecutive worlds whose thresholds carry every exclusion.
    const uint32_t* l0_bits;
    int l0_words;
};

// World outputs for lower-bound coverage.
enum : int {
    kCoverNone = 0,
    // entries in dominator-tree preorder: node, count (the subtree size, the
    // node's marginal coverage so far), the parent's position in the world
    // (-1 under a seed or the super-source) in scr_par and the subtree size
    // in scr_lab, so that a node's subtree is the run of entries
    // [position, position + size)
    kCoverStore = 1,
    // no entries: world_size gets the number of non-seeds whose CP set meets
    // the marked set
    kCoverCount = 2
};

// Global Sampling (Algorithm 3): the graph's in-edges, the pool's V'_s, and
// per-slot state (one slot per workgroup of the sampling launch).
struct LrrDev {
    const int32_t* in_off;  // [n+1] in-edges of each node
    const int4* in_rec;     // [m]   each in-edge as {tail, CSR slot (the coin's edge id), threshold, 0}
    const int32_t* vprime;  // [nvp] V'_s ascending
    uint32_t nvp;
    int32_t n_slots;
    int32_t* stamp;         // [slots][n] 2t+1: in the slot's t-th sample's cone, 2t+2: in its LRR set
    int32_t* list;          // [slots][n] the cone, then the LRR set over its front
    int32_t* epoch;         // [slots] samples the slot has taken; every stamp is at most 2 * epoch + 2
};

// Coverage greedy state per round (device): the top-k search over the gains
// and the coverage of each prefix of the selection.
struct CoverOut {
    int64_t* cov;        // [k+1] Cov(B_r), -1 where round r was never reached
    int64_t* cov_upper;  // [k+1] Cov(B_r) + sum of the k largest marginals given B_r
    long long t0;        // sum of |R_w| over the pool (Cov(B_r) = t0 - total)
    int32_t k;
    uint32_t* hist_cnt;  // [kTopkBins]
    long long* hist_sum; // [kTopkBins]
    long long* state;    // [4]: prefix, k remaining, sum of the bins above, matched total
};
constexpr int kTopkBits = 10;
constexpr int kTopkBins = 1 << kTopkBits;

// A compaction job: per-item ranges of up to four 32-bit fields are packed
// densely into the destination, one counter update per workgroup.
struct CompactSpec {
    const int32_t* src[4];
    int32_t* dst[4];
    int nf;
    unsigned long long src_cap;
    unsigned long long dst_cap;
    const int64_t* loc;       // source start per item
    const int32_t* len;       // entries per item
    uint32_t count;           // items: the tile's worlds 0 .. count-1
    uint32_t w_begin;         // world id of item 0
    int counter_id;           // 0: pair_count, 1: store_count (+ pair_count), 2: xstore_count
    int64_t* out_off;         // per world id: where its entries went (optional)
    int32_t* out_len;
    uint32_t overflow_flag;
};

struct QueryDev {
    const uint32_t* excl;    // bitmap: seeds and blocked nodes
    const uint32_t* thr;     // [m_pad] the query's coin thresholds: the graph's, 0 where the head is excluded
    int32_t excl_in_thr;     // thr reflects every bit of excl (else live heads are tested against excl)
    const int32_t* seeds;
    int32_t n_seeds;
    uint32_t key0, key1;
    const int4* seed_chunk;  // level-0 slot groups {blk, seed lid, e0, e1}
    const int4* seed_col;    // their columns
    const uint4* seed_thr;   // their thresholds (from thr)
    int32_t seed_cap;        // entries the table holds (kernels take the length from RoundCtl::seed_chunks)
    int32_t n_seed_chunks;
    long long seed_sum;
    long long seed_edges;
};

// Entries of a tile's worlds, world by world, for the gain reduction:
// world i's (node, count) entries are node/cnt[off[i] .. off[i] + len[i]).
struct GainSrc {
    const int32_t* node;
    const int32_t* cnt;
    const int64_t* off;       // [count]
    const int32_t* len;       // [count]
    uint32_t count;           // worlds
    unsigned long long cap;   // entries node / cnt hold
};

// Buffers of the gain reduction: nb buckets of 2^shift node ids, each summed
// by `slices` workgroups; rec holds every entry of the tile as (node, count).
constexpr int kGainMaxBuckets = 512;
struct GainBufs {
    int shift;
    int nb;
    int slices;
    long long* bcnt;   // [nb]
    long long* bbase;  // [nb + 1]
    long long* bcur;   // [nb]
    int2* rec;         // [rec_cap]
    unsigned long long rec_cap;
};

// ---- launchers (imin_kernels.hip) ----
hipError_t launch_graph_ingest(const GraphDev& g, const int64_t* row_ptr, const int32_t* col_in,
                               const float* p, RoundCtl* ctl, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int32_t v, size_t count, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t v, size_t count, hipStream_t s);
hipError_t launch_fill_i64_live(int64_t* p, int64_t v, size_t count, const RoundCtl* ctl, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, size_t count, hipStream_t s);
hipError_t launch_query_setup(const GraphDev& g, const int32_t* seeds, int32_t n_seeds,
                              const int32_t* blocked, int32_t n_blocked, uint32_t* excl,
                              RoundCtl* ctl, hipStream_t s);
hipError_t launch_ctl_reset_round(RoundCtl* ctl, hipStream_t s);
hipError_t launch_ctl_reset_tile(RoundCtl* ctl, hipStream_t s);
// Events a launch records itself, around exactly its kernel (both null: an
// ordinary launch).  Used to time a kernel without separate event packets
// on the stream, whose own dispatch would be counted too.
struct LaunchEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

// One query of a packed tier-0 launch (device memory): its worlds are
// packed worlds [first, first + count), world first + i being its world
// w_begin + i, evaluated as its own tier-0 launch would evaluate it.
struct PackedQuery {
    QueryDev q;
    TileOut out;
    RoundCtl* ctl;
    int32_t* list1;  // its tier-1 list (count ctl->list_n[1])
    int32_t* list2;  // its tier-2 list (count ctl->list_n[2])
    uint32_t w_begin;
    uint32_t first;
    uint32_t count;
    uint32_t pad;
};

// Tier 0 over the worlds of nq queries (ascending `first`, n_items packed
// worlds in all) in one launch; counter (zero at launch) deals out chunks.
hipError_t launch_world_tier0_packed(const GraphDev& g, const PackedQuery* pq, int nq, uint32_t n_items,
                                     uint32_t* counter, int grid, hipStream_t s);
// Tier 1 over the tier-1 lists of the same queries, after that launch.
hipError_t launch_world_tier1_packed(const GraphDev& g, const PackedQuery* pq, int nq, int grid, hipStream_t s);

// Level 0 of worlds [w_begin, w_begin + count) ahead of the world kernels:
// their live seed slots as bits (TileOut::l0_bits; words = ceil(chunk_cap /
// 8) per world).  q's thresholds must carry every exclusion.
struct LaunchEvents;
hipError_t launch_level0_bits(const QueryDev& q, const RoundCtl* ctl, uint32_t w_begin, uint32_t count,
                              uint32_t* bits, int words, int32_t chunk_cap, hipStream_t s, const LaunchEvents& ev);

// Tiers 0 and 1 (LDS), 2 (HBM slots with bounded per-world arrays) and 3
// (HBM slots with arrays for any world); bs gives the slots of tier 2 or 3.
hipError_t launch_world_tier(int tier, const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin,
                             uint32_t range_count, const int32_t* in_list, int count_idx, int32_t* next_list,
                             const TileOut& out, const BigSlots& bs, int grid, hipStream_t s,
                             const LaunchEvents& ev = LaunchEvents());
hipError_t launch_sum_lengths(const int32_t* len, uint32_t count, unsigned long long* total, RoundCtl* ctl,
                              hipStream_t s);
hipError_t launch_compact(const CompactSpec& spec, RoundCtl* ctl, hipStream_t s);
// An incremental round with replay, one launch: the last selection is
// combined and committed, then rule_parts workgroups apply the label rule to
// the worlds it holds for (a world per `lanes` lanes: 16, 32 or 64) and
// replay_parts (>= 1) workgroups replay the other changed worlds (those too
// large go to next_list); both find the worlds through the index.
struct SelectOut;
// The wide replay of an incremental round: worlds of in_list (count
// list_n[1]) too large for the round-update launch's replay; those beyond
// its limits are appended to over_list (count list_n[3]).  grid workgroups
// of 1024 threads.
hipError_t launch_replay_wide(const QueryDev& q, RoundCtl* ctl, const TileOut& out, const int32_t* in_list,
                              int32_t* over_list, int grid, hipStream_t s, const LaunchEvents& ev = LaunchEvents());
hipError_t launch_round_update(const QueryDev& q, RoundCtl* ctl, int32_t* next_list, const TileOut& out,
                               int rule_parts, int replay_parts, int lanes, const uint32_t* idx_off,
                               const int2* idx_ent, const SelectOut& so, hipStream_t s,
                               const LaunchEvents& ev = LaunchEvents());
constexpr int kRuleNT = 256;  // four worlds at a time per workgroup
// Store positions and index offsets are unsigned 32-bit: the first word of
// an index entry or partition record is a position read as uint32_t.  The
// store's capacity and the index's entries stay below kIndexPosLimit, which
// leaves every cursor plus any launch's stride (< 2^24) below 2^32.
constexpr unsigned long long kIndexPosLimit = 0xFF000000ull;
__host__ __device__ constexpr uint32_t index_pos(int2 e) { return (uint32_t)e.x; }

// Buffers of the index build: nodes fall in nb buckets of 2^shift ids
// (nb <= 8192, nb << shift >= n); rec and idx_ent hold every stored entry.
struct IndexBufs {
    int shift;
    int nb;
    uint32_t* bcnt;  // [nb] entries per bucket
    uint32_t* bbase; // [nb + 1] first entry of each bucket
    uint32_t* bcur;  // [nb] partition cursors
    int32_t* border; // [nb] buckets by decreasing size class
    int4* rec;       // [rec_cap] (position, world, node, count) grouped by bucket
    uint32_t rec_cap;
    uint32_t* idx_off;  // [n + 1] first index entry of each node
    int2* idx_ent;      // [ent_cap] (store position, world) grouped by node
    uint32_t ent_cap;
};
// node -> (store position, world) of every entry of the resident store;
// with gain non-null also the from-scratch gains (gain[u] += every count of u)
hipError_t launch_index_build(const TileOut& out, uint32_t theta, int32_t n, const IndexBufs& ib, int64_t* gain,
                              RoundCtl* ctl, hipStream_t s);
hipError_t launch_affected_select(const TileOut& out, RoundCtl* ctl, const uint32_t* idx_off, const int2* idx_ent,
                                  int32_t* list, const SelectOut& so, hipStream_t s);
hipError_t launch_seed_count(const GraphDev& g, const int32_t* seeds, int32_t ns, int32_t* cnt, RoundCtl* ctl,
                             hipStream_t s);
hipError_t launch_seed_fill(const GraphDev& g, const int32_t* seeds, int32_t ns, const int32_t* start,
                            int4* table, int32_t cap, RoundCtl* ctl, hipStream_t s);
// ctl = {0, expect_total = -1}, by a kernel (no host copy)
hipError_t launch_ctl_init(RoundCtl* ctl, hipStream_t s);
// stop every later kernel once a flag of `mask` is set; with hints, also
// raise hints[2] / hints[3] to the shares of the tile's theta worlds handed
// on to tier 1 / tier 2 (1/1024 units)
hipError_t launch_guard(RoundCtl* ctl, uint32_t mask, hipStream_t s, uint64_t theta = 0,
                        unsigned long long* hints = nullptr);
// the end of an enqueued solve: device_status from the flags (0, or an
// imin_status_t code), n_selected = 0 when the solve stopped on an error,
// and the graph's per-world scratch hints raised by what round 0 asked for
// (entries * 1024 / theta, for bump-region entries and extra edges)
hipError_t launch_solve_status(RoundCtl* ctl, int32_t* device_status, int32_t* n_selected, uint64_t theta,
                               unsigned long long* hints, hipStream_t s);
// largest out-degree of the graph into *out (device)
hipError_t launch_max_degree(const GraphDev& g, int32_t* out, hipStream_t s);
// thr_q[e] = 0 where col[e] is excluded, else the graph's threshold; then the
// level-0 table's columns and thresholds (ctl->seed_chunks entries, at most
// chunk_cap)
hipError_t launch_query_thresholds(const GraphDev& g, const uint32_t* excl, uint32_t* thr_q, const int4* table,
                                   const RoundCtl* ctl, int32_t chunk_cap, int4* seed_col, uint4* seed_thr,
                                   hipStream_t s);
int world_tier_blocks_per_cu(int tier);
int world_tier0_capacity();   // non-seed nodes a tier-0 world may reach
int world_tier0_xcapacity();  // extra live edges a tier-0 world may record
// gain[u] += every count of u among src's entries (bounds and capacity
// problems raise kFlagBounds / kFlagReduceCapacity).
hipError_t launch_gain_reduce(const GainSrc& src, const GainBufs& gb, int32_t n, int64_t* gain, RoundCtl* ctl,
                              hipStream_t s);
// bucket width for n nodes (one slice, the buffers left null), and the
// slices per bucket for a tile of `entries` entries on `cus` compute units
GainBufs gain_buckets(int32_t n);
int gain_slices(const GainBufs& gb, unsigned long long entries, int cus);
hipError_t launch_sum_sizes(const int32_t* world_size, uint32_t count, RoundCtl* ctl, hipStream_t s);
// Argmax of gain over the candidates (ties to the smaller id), the stop rule
// and the round's T; the partial launch also sums and clears the dsz slots
// (nodes lost by the round's changed worlds) and clears the next round's
// counters.  With `combine` a second launch commits the selection; else the
// next incremental round's search does.
hipError_t launch_select(const GraphDev& g, const int64_t* gain, RoundCtl* ctl, const SelectOut& so, long long* dsz,
                         int32_t dsz_n, bool combine, hipStream_t s);

// Coverage greedy, round r (all enqueued; every kernel returns at once after
// the selection stopped): the selection over the coverage marginals (ties to
// the smaller id; it stops when the best marginal is 0 or r == k), Cov(B_r)
// into co.cov[r], the sum of the k largest marginals into co.cov_upper[r],
// then the coverage update of the pick: in each world whose entry for it is
// still uncovered its subtree's entries are covered and its ancestors lose
// its count.  dsz (dsz_n slots, grid <= dsz_n) carries the newly covered
// counts to the next round's selection.  key_bits bounds every gain.
// With `sets` the stored items are LRR sets (Section 4.2) instead of
// dominator trees: covering a set zeroes every member entry, and the
// newly covered count is one per set.
hipError_t launch_cover_round(const GraphDev& g, int64_t* gain, RoundCtl* ctl, const SelectOut& so,
                              const CoverOut& co, int r, int key_bits, const TileOut& out, const uint32_t* idx_off,
                              const int2* idx_ent, long long* dsz, int32_t dsz_n, int grid, bool sets,
                              hipStream_t s);
// LRR sets of samples [w_begin, w_begin + count) of the pool keyed by q's
// key, as (node, 1) entries in the tile's bump region (wloc / wlen per
// sample; world_size 1 for a non-empty set), or with out.cover ==
// kCoverCount whether each set meets out.mark (world_size 0 or 1).
hipError_t launch_lrr(const GraphDev& g, const QueryDev& q, RoundCtl* ctl, uint32_t w_begin, uint32_t count,
                      const LrrDev& L, const TileOut& out, hipStream_t s);


// An enqueued solve in a given workspace (imin_solve with a workspace),
// and the device a graph handle lives on.
}  // namespace imin
#include "imin.h"
namespace imin {
imin_status_t solve_enqueued(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                             uint64_t rng_seed, void* workspace, size_t workspace_bytes, void* stream,
                             int32_t* blockers, int64_t* gains, int64_t* spread_totals, int32_t* n_selected,
                             int32_t* device_status);
int graph_device(imin_graph_t g);
// Host copies of a handle's graph (CSR offsets, heads, thresholds), made on
// first use and kept until the handle is destroyed; null on failure.
struct HostGraph {
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<uint32_t> thr;
};
const HostGraph* graph_host(imin_graph_t g);
// The handle's in-edges on the device (made on first use): in_off [n+1] and
// in_rec [m] = {tail, CSR slot, threshold, 0} grouped by head; false on
// failure.
bool graph_in_edges(imin_graph_t g, const int32_t** in_off, const int4** in_rec);
// V'_s: the non-seed nodes reachable from the seeds over edges that can be
// live (threshold > 0), ascending (host arrays; seeds validated by the caller).
std::vector<int32_t> reachable_nonseeds(const HostGraph& h, const std::vector<int32_t>& seeds);

} // namespace imin
