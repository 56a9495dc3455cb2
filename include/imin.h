/*
 * imin.h -- C ABI of the MI355X (gfx950) library for influence minimization
 * by node blocking: the sampling estimator of Wang et al., "Efficient
 * Influence Minimization via Node Blocking" (PVLDB), Section 2.2.
 *
 * The library picks up to k blockers for a seed set S on a directed graph
 * with edge probabilities.  For every candidate u it counts, over theta
 * sampled live-edge worlds (Section 2.1, Eq. 1), the nodes that lose every
 * path from S once u is blocked; these counts are dominator-subtree sizes
 * under a virtual source joined to every seed (Section 2.2, the estimator of
 * Xie et al.; Section 3.1, the unified seed).  Greedy selection adds the
 * candidate with the largest summed count, ties to the smaller node id, and
 * stops early when no candidate protects anything (problem statement: at
 * most k blockers).
 *
 * Worlds are drawn by counter-based coins: edge e (its CSR slot) is live in
 * world w iff its threshold is 0xFFFFFFFF (p == 1) or
 *   Philox4x32-10(counter = (e >> 2, w, 0, 0),
 *                 key = (lo32(rng_seed), hi32(rng_seed)))[e & 3] < thr[e],
 * with thr[e] = floor(p[e] * 2^32) for p[e] < 1.  A world is therefore a pure
 * function of (rng_seed, w), and every greedy round reuses the same theta
 * worlds.  All counts are exact integers; results do not depend on launch
 * shapes, tiling or thread timing.
 *
 * Conventions for every call:
 *   - array arguments are DEVICE pointers (HBM of the current HIP device)
 *     unless stated otherwise; scalars are passed by value;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - calls are synchronous with respect to the host (they return after the
 *     results are in place; work is ordered on `stream`), except imin_solve
 *     given a workspace, which only enqueues, and imin_server_submit;
 *   - no C++ exception crosses this boundary; every call returns a status.
 */
#ifndef IMIN_H
#define IMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IMIN_OK = 0,
    IMIN_ERR_INVALID = 1, /* bad argument, detected on the host               */
    IMIN_ERR_DATA = 2,    /* bad input data, detected on the device: a column
                             index out of range, a probability outside [0, 1]
                             or NaN, non-monotone row offsets, a seed out of
                             range or repeated, a blocker that is a seed      */
    IMIN_ERR_DEVICE = 3,  /* a HIP runtime call failed                        */
    IMIN_ERR_NOMEM = 4,   /* device memory could not be allocated             */
    IMIN_ERR_INTERNAL = 5,/* an internal consistency check failed             */
    IMIN_ERR_WORKSPACE = 6/* a caller's workspace is too small for the call   */
} imin_status_t;

typedef struct imin_graph* imin_graph_t;

/*
 * imin_graph_create -- ingest a graph (Section 2.1: G = (V, E) with
 * p(u, v) in [0, 1] on every edge).
 *
 *   n        number of nodes, 1 <= n < 2^24
 *   m        number of edges (CSR slots), 0 <= m < 2^31 - 8
 *   row_ptr  int64[n+1], device: out-edges of u are slots row_ptr[u] ..
 *            row_ptr[u+1]-1; row_ptr[0] == 0, row_ptr[n] == m, non-decreasing
 *   col      int32[m], device: head of each slot, in [0, n)
 *   p        float32[m], device: propagation probability of each slot
 *   stream   stream the ingest runs on
 *   out      host pointer receiving the handle
 *
 * The handle owns device copies of everything it needs (int32 offsets, a
 * padded column array and the coin thresholds), so the caller's arrays may
 * be freed once the call returns.  Parallel edges are allowed (each slot has
 * its own coin); self-loops are allowed and never matter.  Errors:
 * IMIN_ERR_INVALID (sizes, NULL pointers), IMIN_ERR_DATA (see above; no
 * handle is returned), IMIN_ERR_NOMEM, IMIN_ERR_DEVICE.
 */
imin_status_t imin_graph_create(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col,
                                const float* p, void* stream, imin_graph_t* out);

/* Release a handle and its device memory.  NULL is accepted. */
imin_status_t imin_graph_destroy(imin_graph_t g);

/* Node and edge counts of a handle (host pointers; either may be NULL). */
imin_status_t imin_graph_info(imin_graph_t g, int32_t* n, int64_t* m);

/*
 * Host copies of a handle's graph: row_ptr int64[n+1], col int32[m] and the
 * coin thresholds thr uint32[m] the handle derived from p (Section 2.1, the
 * live-edge process; 0xFFFFFFFF for p == 1, else floor(p * 2^32)).  All three
 * are HOST pointers.  Synchronous.
 */
imin_status_t imin_graph_export(imin_graph_t g, int64_t* row_ptr, int32_t* col, uint32_t* thr);

/*
 * imin_solve -- greedy blocker selection (Section 2.1, problem statement:
 * given G, p, the seed set S and a budget k, find at most k blockers
 * minimising the expected spread; Section 2.2: the greedy framework driven
 * by the dominator-tree estimator; Section 3.1, Algorithm 1: its inputs are
 * the graph, the seed set and the budget, its output the blocker set).
 *
 *   seeds          int32[n_seeds], device: the misinformation seed set S,
 *                  distinct ids in [0, n); 1 <= n_seeds <= n
 *   k              budget, 0 <= k <= n
 *   theta          worlds per round, 1 <= theta < 2^32 (the number of
 *                  realizations the greedy evaluates, Section 6)
 *   rng_seed       key of the coin generator
 *   workspace      device scratch owned by the caller, 256-byte aligned, of
 *                  workspace_bytes bytes (see imin_solve_workspace_size); or
 *                  NULL, see below
 *   stream         the stream every kernel of the call is enqueued on
 *   blockers       int32[max(k,1)], device, out: u*_0 .. u*_{n_selected-1}
 *   gains          int64[max(k,1)], device, out: gains[r] = sum over worlds
 *                  of nodes protected by u*_r given u*_0..u*_{r-1} blocked
 *   spread_totals  int64[k+1], device, out: T_r = sum over worlds of
 *                  |R_w(B_r)| for r = 0 .. n_selected (seeds included), so
 *                  T_{r+1} = T_r - gains[r] and the estimated spread after
 *                  blocking is T_{n_selected} / theta
 *   n_selected     int32[1], device, out: number of blockers chosen (<= k;
 *                  fewer when every remaining candidate protects nothing)
 *   device_status  int32[1], device, out: 0 when the solve succeeded, else
 *                  an imin_status_t code (may be NULL when workspace is NULL)
 *
 * With a workspace the call only enqueues: it allocates nothing, reads
 * nothing back and does not wait (so it can be captured into a HIP graph).
 * Every piece of scratch is carved from the workspace, which the call uses
 * until the stream reaches the end of its work; the caller keeps it, the
 * seeds and the outputs alive until then and must not share one workspace
 * between solves that overlap.  Problems found on the host (bad arguments,
 * a workspace smaller than the fixed part of the layout) return
 * IMIN_ERR_INVALID / IMIN_ERR_WORKSPACE at once and enqueue nothing.
 * Problems found on the device are written to device_status when the
 * stream gets there, and every later kernel of the solve then does nothing
 * (n_selected is set to 0): IMIN_ERR_DATA for bad seeds, IMIN_ERR_WORKSPACE
 * when the worlds beyond the smallest world tier need more bump-region
 * entries than the workspace holds (the graph then remembers how many were
 * needed, so imin_solve_workspace_size returns enough next time),
 * IMIN_ERR_INTERNAL when a consistency check fails.  The layout takes
 * incremental rounds (a resident per-world store and a node index) when the
 * stored entries can be indexed with unsigned 32-bit positions and the
 * workspace holds that layout with the bump region the graph's record asks
 * for, else every round evaluates all theta worlds again; both give the
 * same integers.
 *
 * With workspace == NULL the call takes its scratch from the library's
 * block cache (see imin_cache_release), waits for its work and returns the
 * solve's status (also written to device_status when that is not NULL).
 * Entries past n_selected are left untouched.  Errors: IMIN_ERR_INVALID,
 * IMIN_ERR_DATA (bad seeds), IMIN_ERR_NOMEM, IMIN_ERR_DEVICE,
 * IMIN_ERR_INTERNAL.
 */
imin_status_t imin_solve(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                         uint64_t rng_seed, void* workspace, size_t workspace_bytes, void* stream,
                         int32_t* blockers, int64_t* gains, int64_t* spread_totals, int32_t* n_selected,
                         int32_t* device_status);

/*
 * imin_solve_workspace_size -- bytes of workspace an enqueued imin_solve on
 * this graph with these sizes needs (host pointer `bytes`).  The fixed part
 * depends on n, m, n_seeds and theta; the bump region for worlds beyond the
 * smallest world tier is data-dependent and sized from what earlier calls on
 * the graph needed per world (at least 2^20 entries), with an eighth more.
 * A solve given more bytes uses them for that region.  The size is that of
 * the incremental-rounds layout while it fits the device's memory, else that
 * of the plain-rounds layout.  Waits for the device (it reads the graph's
 * device-side record of those needs).  IMIN_ERR_INVALID for bad arguments.
 */
imin_status_t imin_solve_workspace_size(imin_graph_t g, int32_t n_seeds, int32_t k, int64_t theta, size_t* bytes);

/*
 * imin_solve_static -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): imin_solve with its workspace taken from a fixed array of
 * 256 MiB that the library declares, one copy per device, held until the
 * process ends.  Arguments and outputs are those of imin_solve (device_status
 * required); the call only enqueues on `stream` and allocates nothing.  The
 * graph's device must be current.
 *
 * Limit: the solve's layout must fit the 256 MiB array; a larger one returns
 * IMIN_ERR_WORKSPACE at once, and worlds that need more bump-region entries
 * than the array leaves report IMIN_ERR_WORKSPACE in device_status.  Every
 * call on a device shares that device's array and leaves the last call's
 * contents in it: calls that overlap on one GPU (any streams) race, so the
 * caller must order them.  IMIN_ERR_INVALID for bad arguments or when the
 * graph's device is not current; IMIN_ERR_DEVICE if the array's address
 * cannot be looked up.
 */
imin_status_t imin_solve_static(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, int64_t theta,
                                uint64_t rng_seed, void* stream, int32_t* blockers, int64_t* gains,
                                int64_t* spread_totals, int32_t* n_selected, int32_t* device_status);

/*
 * One query of imin_solve_many and of the serving loop: its graph (NULL: the
 * batch's or server's own graph; any graph on the same device), the
 * arguments of imin_solve (device arrays, the same meaning and sizes) and,
 * written by the call, the query's status (an imin_status_t, from the
 * device_status of its solve) and device flags.
 */
typedef struct imin_query {
    imin_graph_t graph;
    const int32_t* seeds;
    int32_t n_seeds;
    int32_t k;
    int64_t theta;
    uint64_t rng_seed;
    int32_t* blockers;
    int64_t* gains;
    int64_t* spread_totals;
    int32_t* n_selected;
    int32_t status;         /* out: an imin_status_t */
    uint32_t device_flags;  /* out */
} imin_query_t;

/*
 * Batches and serving (many queries of Section 2.1's problem on resident
 * graphs).  Both run every query as an enqueued imin_solve whose workspace is
 * a range of one pool of device memory, allocated once when the batch or
 * server starts (hbm_budget bytes; 0 = half the device's free memory, at
 * most 96 GiB).  A query is admitted when the workspace its layout needs
 * (imin_solve_workspace_size) fits a free range of the pool: queries wait
 * in arrival order, and while the first waiting one does not fit a few
 * later ones that do may start.  Each admitted query goes to the stream
 * with the fewest queries in flight, so queries overlap on the device; its
 * workspace returns to the pool when its last kernel has run.  A query
 * whose worlds need more scratch than its workspace held
 * (IMIN_ERR_WORKSPACE found on the device) is admitted again with the size
 * its graph now records.  A query larger than the whole pool fails with
 * IMIN_ERR_WORKSPACE.  Every query's worlds are keyed by its own rng_seed,
 * so each result is identical to the query solved alone.
 *
 * The device arrays of a query must be ready on the host's side of every
 * stream (e.g. the device synchronised after they were written).  streams:
 * host array of n_streams distinct hipStream_t (as void*) on the graphs'
 * device, n_streams >= 1.
 *
 * imin_solve_many  solves queries[0 .. n_queries) (largest theta * (k + 1)
 *                  first) and returns when all have finished: IMIN_OK when
 *                  every query succeeded, else the status of the first
 *                  failing one (by index); IMIN_ERR_INVALID for bad
 *                  arguments (no query run), IMIN_ERR_NOMEM when the pool
 *                  cannot be allocated.
 */
imin_status_t imin_solve_many(imin_graph_t g, imin_query_t* queries, int32_t n_queries, void* const* streams,
                              int32_t n_streams, size_t hbm_budget);

/*
 * A serving loop: one dispatcher thread admits submitted queries as the
 * pool and the streams allow (see above) and hands back finished ones.
 *
 * imin_server_create   g is the default graph of queries with graph NULL;
 *                      the graphs must outlive the server.
 * imin_server_submit   queues one query and returns at once.  The query
 *                      entry and its device arrays must stay valid, and its
 *                      inputs ready on every stream, until imin_server_next
 *                      has returned it.  IMIN_ERR_INVALID after
 *                      imin_server_destroy has begun.
 * imin_server_next     blocks until a submitted query has finished and
 *                      returns it in *done (status and device_flags
 *                      written); every query is returned once, in the order
 *                      they finish.  IMIN_ERR_INVALID when no submitted
 *                      query is outstanding.
 * imin_server_destroy  lets every queued query finish, joins the dispatcher
 *                      and frees the server and its pool (queries not yet
 *                      returned by imin_server_next are finished but not
 *                      returned).
 *
 * One thread may submit while another waits in imin_server_next;
 * imin_server_destroy must not overlap any other call on the same server.
 */
typedef struct imin_server* imin_server_t;
imin_status_t imin_server_create(imin_graph_t g, void* const* streams, int32_t n_streams, size_t hbm_budget,
                                 imin_server_t* out);
imin_status_t imin_server_submit(imin_server_t s, imin_query_t* query);
imin_status_t imin_server_next(imin_server_t s, imin_query_t** done);
imin_status_t imin_server_destroy(imin_server_t s);

/*
 * imin_evaluate -- one pass of the estimator (Section 2.2: sample worlds,
 * build each world's dominator tree under the super-source, measure every
 * subtree) over the worlds [w_begin, w_begin + w_count) with a given blocked
 * set B.
 *
 *   seeds       int32[n_seeds], device, as for imin_solve
 *   blocked     int32[n_blocked], device (may be NULL when n_blocked == 0):
 *               nodes removed from the graph; never seeds; repeats allowed
 *   w_begin, w_count  world range, w_begin + w_count <= 2^32, w_count >= 1
 *   gain        int64[n], device, out: gain[u] = sum over the range of
 *               c_w(u|B) = |R_w(B)| - |R_w(B + u)|; 0 for seeds and for B
 *   total       int64[1], device, out: sum over the range of |R_w(B)|
 *   world_size  int32[w_count], device, out, optional (NULL): |R_w(B)|
 *   world_sum   int64[w_count], device, out, optional (NULL): sum of the
 *               node ids in R_w(B), an order-free fingerprint of the set
 *   world_edges int64[w_count], device, out, optional (NULL): number of CSR
 *               slots leaving the nodes of R_w(B), i.e. the edges whose coins
 *               the world needs (the unit of sampling work)
 *
 * Gains over disjoint world ranges add up to the gains over their union.
 * Errors as for imin_solve.
 */
imin_status_t imin_evaluate(imin_graph_t g, const int32_t* seeds, int32_t n_seeds,
                            const int32_t* blocked, int32_t n_blocked, int64_t w_begin,
                            int64_t w_count, uint64_t rng_seed, void* stream, int64_t* gain,
                            int64_t* total, int32_t* world_size, int64_t* world_sum,
                            int64_t* world_edges);

/*
 * imin_evaluate_batch -- imin_evaluate for several queries on one graph
 * (each its own seeds, blocked set, world range and rng_seed), whose passes
 * share their world launches: the worlds of every query that fits one tile
 * and whose worlds start at tier 0 are packed into a single tier-0 launch,
 * and the worlds those hand on into a single tier-1 launch; the HBM tiers,
 * the gain reductions and every other query run per query.  Each query's
 * outputs are those imin_evaluate gives it alone.
 *
 *   queries     imin_eval_query_t[n_queries], HOST; the pointers in each
 *               are device pointers, with the meanings of imin_evaluate's
 *               arguments of the same names (world_size may be NULL)
 *   n_queries   >= 0; at most IMIN_PACK_QUERIES (default 64) queries share
 *               a launch, and larger batches are taken in groups
 *
 * The queries of a group are set up together, each with its own arrays
 * (thresholds, gains, scratch: about 4m + 8n bytes plus 8 bytes per world
 * slot); they share the HBM tiers' slot budgets (IMIN_BIG_BUDGET,
 * IMIN_HUGE_BUDGET) instead of each taking them whole.
 *
 * Every query's pointers and sizes are checked before any work.  Errors
 * as for imin_evaluate: the first failing query's status is returned, and
 * the outputs of the other queries of its group are then not all written.
 */
typedef struct {
    const int32_t* seeds;
    int32_t n_seeds;
    const int32_t* blocked;
    int32_t n_blocked;
    int64_t w_begin;
    int64_t w_count;
    uint64_t rng_seed;
    int64_t* gain;
    int64_t* total;
    int32_t* world_size;
} imin_eval_query_t;
imin_status_t imin_evaluate_batch(imin_graph_t g, const imin_eval_query_t* queries, int32_t n_queries,
                                  void* stream);

/*
 * Lower-bound coverage (Section 3.2, the lower bounding function D^L;
 * Section 4.1, CP sequences and coverage; Section 5.1, Max-Coverage).
 *
 * In a world w (drawn as above, with no blockers) the CP set C_w(s, v) of a
 * reached non-seed v is the set of non-seed nodes on every path from the
 * seeds to v, v included (Definition 4.1): v's chain of non-seed dominators.
 * Cov(B) over worlds [0, theta) counts the pairs (w, v) whose CP set meets B;
 * Cov(B) / theta estimates D^L(B) without bias (Lemma 4.2).
 */

/*
 * imin_max_coverage -- the procedure Max-Coverage of Algorithm 4 on the CP
 * sequences of worlds [0, theta): k greedy steps, each adding the node of
 * V \ (S + B) with the largest marginal coverage Cov(B + v) - Cov(B), ties to
 * the smaller id; it stops early when the best marginal is 0.
 *
 *   blockers   int32[k], out: picks in order (n_selected of them)
 *   gains      int64[k], out: the marginal coverage of each pick
 *   cov        int64[k+1], out: cov[i] = Cov(B_i) for the prefixes
 *              B_0 .. B_{n_selected}; -1 beyond
 *   cov_upper  int64[k+1], out: cov[i] + the sum of the k largest marginal
 *              coverages given B_i (over V \ (S + B_i)); Algorithm 4 bounds
 *              the optimum's coverage by their minimum
 *   n_selected int32[1], out
 *
 * The worlds' dominator trees stay resident (16 bytes per reached non-seed
 * per world, plus 8 for the node index): IMIN_ERR_NOMEM when they exceed the
 * device or 0xFF000000 - 1 entries (store positions are unsigned 32-bit).
 * Errors otherwise as for imin_solve.
 */
imin_status_t imin_max_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k,
                                int64_t theta, uint64_t rng_seed, void* stream, int32_t* blockers,
                                int64_t* gains, int64_t* cov, int64_t* cov_upper, int32_t* n_selected);

/*
 * imin_coverage -- Cov(set) over the CP sequences of worlds [0, theta)
 * (Section 4.1).  set: int32[n_set], device, non-seeds (repeats allowed; a
 * seed or an id out of range is IMIN_ERR_DATA); covered: int64[1], out.
 */
imin_status_t imin_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* set,
                            int32_t n_set, int64_t theta, uint64_t rng_seed, void* stream,
                            int64_t* covered);

/*
 * imin_reach_counts -- in how many of the worlds [w_begin, w_begin + w_count)
 * each non-seed is reached from S (no blockers): counts[v] / w_count
 * estimates Pr[s -> v] (Section 5.1, OPT^L).  counts: int64[n], out (0 for
 * seeds); world_size: int32[w_count], out, optional: |R_w|.
 */
imin_status_t imin_reach_counts(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t w_begin,
                                int64_t w_count, uint64_t rng_seed, void* stream, int64_t* counts,
                                int32_t* world_size);

/*
 * imin_lsbm -- LSBM (Algorithm 4, Section 5.1): a blocker set B_L whose lower
 * bound D^L(B_L) is within 1 - 1/e - eps of the best size-k set's with
 * probability at least 1 - delta (Section 5.1, the theorem after Lemma 5.3).
 *
 *   1. ON = nodes a seed reaches by one edge that can be live (threshold > 0),
 *      seeds left out; when |ON| <= k the answer is ON (ascending).
 *   2. I_hat, E[I_G(s)] within relative error beta with probability
 *      1 - delta/6, by the Stopping Rule Algorithm of Dagum, Karp, Luby and
 *      Ross (SIAM J. Comput. 2000) on Z_w = |R_w| / b, b the nodes reachable
 *      from S over edges with threshold > 0: worlds 0, 1, ... are drawn until
 *      sum |R_w| >= b * Upsilon_1, with Upsilon = 4 (e - 2) ln(2 / (delta/6)) /
 *      beta^2 and Upsilon_1 = 1 + (1 + beta) Upsilon; then
 *      I_hat = b * Upsilon_1 / N for the N worlds drawn.
 *   3. OPT^L = sum over the k nodes of ON with the largest reach counts in
 *      those N worlds of count / N (1 / N when that sum is 0).
 *   4. theta_max = 2 I_hat ((1 - 1/e) sqrt(ln(12/delta)) +
 *      sqrt((1 - 1/e)(ln C(n - |S|, k) + ln(12/delta))))^2 /
 *      ((1 - beta) eps^2 OPT^L), with ln C(N, k) = sum over j = 1..k of
 *      ln((N - k + j) / j); theta_0 = theta_max (1 - beta) eps^2 OPT^L / I_hat;
 *      i_max = max(1, ceil(log2(theta_max / theta_0)));
 *      a_1 = a_2 = ln(3 i_max / delta).
 *   5. For i = 1 .. i_max, with both pools of theta_i = ceil(theta_0) 2^(i-1)
 *      worlds: B_L = Max-Coverage on pool 1; sigma^L from Cov(B_L) on pool 2
 *      and sigma^U from min_i cov_upper on pool 1 (Lemma 5.3, as Algorithm 4
 *      states them); return B_L when sigma^L / sigma^U >= 1 - 1/e - eps or
 *      i = i_max.
 *
 * Pool 1's worlds are those of key rng_seed (the worlds of imin_solve);
 * pool 2 uses key rng_seed ^ 0x9E3779B97F4A7C15 and the stopping rule
 * rng_seed ^ 0xC2B2AE3D27D4EB4F.  Floating-point steps are evaluated in
 * double, left to right as written above.
 *
 *   blockers    int32[k], device, out; n_selected int32[1], device, out
 *   info        host, out, optional: every intermediate quantity
 *   eps in (0, 1), beta in [0, 1), delta in (0, 1); k >= 1.
 */
typedef struct imin_lsbm_info {
    int32_t returned_on;  /* 1: |ON| <= k, the answer is ON */
    int32_t on_size;
    int64_t reach_bound;  /* b */
    int64_t sra_worlds;   /* N */
    double i_hat;
    double opt_l;
    double theta_max;
    double theta_0;
    int32_t i_max;
    int32_t iterations;   /* pool doublings + 1 */
    int64_t theta;        /* worlds per pool in the last iteration */
    int64_t cov1;         /* Cov(B_L) on pool 1 */
    int64_t cov2;         /* Cov(B_L) on pool 2 */
    int64_t cov_upper;    /* min_i cov_upper on pool 1 */
    double sigma_l;
    double sigma_u;
    double a1;
} imin_lsbm_info_t;

imin_status_t imin_lsbm(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps,
                        double beta, double delta, uint64_t rng_seed, void* stream, int32_t* blockers,
                        int32_t* n_selected, imin_lsbm_info_t* info);

/*
 * imin_world_sizes -- |R_w(B)| of every world in [w_begin, w_begin + w_count)
 * with the blocked set B (Section 2.1), without dominators: the samples of
 * the stopping rules of Algorithms 1 and 4.  blocked as for imin_evaluate;
 * world_size: int32[w_count], device, out.  Errors as for imin_evaluate.
 */
imin_status_t imin_world_sizes(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* blocked,
                               int32_t n_blocked, int64_t w_begin, int64_t w_count, uint64_t rng_seed,
                               void* stream, int32_t* world_size);

/*
 * Global Sampling (Section 4.2, Algorithm 3; Definition 4.3) and the upper
 * bound D^U (Section 3.3).
 *
 * V'_s is the set of non-seed nodes reachable from S over edges that can be
 * live (threshold > 0), ascending.  Sample i of key `key` is world i of that
 * key; its target is v = V'_s[(r * |V'_s|) >> 32], with r word 0 of
 * Philox4x32-10 at counter (0, i, 1, 0) and the same key (the coins use
 * counter word 2 = 0).  Its LRR set is empty when v is not reached from S in
 * the world, else the nodes that reach v in phi^s, the live subgraph
 * induced by the reached non-seeds (v included).  Cov(B) over samples
 * [0, theta) counts the sets that meet B, and |V'_s| Cov(B) / theta
 * estimates D^U(B) without bias (Lemma 4.4).
 *
 * imin_vprime: V'_s into out (int32[count], device; may be NULL to ask for
 * the count only); count: int32, HOST, out.
 * imin_lrr_max_coverage: the procedure Max-Coverage over the LRR sets of
 * samples [0, theta); outputs as imin_max_coverage.
 * imin_lrr_coverage: Cov(set) over the LRR sets of samples [0, theta).
 * The graph's in-edges and a host copy of the graph are made on a handle's
 * first use here and kept until imin_graph_destroy.  Sampling takes 8 bytes
 * per node per sampling slot: IMIN_LRR_BUDGET (default the smaller of 16 GiB
 * and a quarter of the device memory free at the first call) bounds the
 * slots.  The handle keeps them until imin_graph_destroy and lends them to
 * one call at a time; a call that finds them lent takes its own, within
 * IMIN_LRR_BUDGET (default 8 GiB), for its duration.
 */
imin_status_t imin_vprime(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, void* stream, int32_t* out,
                          int32_t* count);
imin_status_t imin_lrr_max_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k,
                                    int64_t theta, uint64_t key, void* stream, int32_t* blockers,
                                    int64_t* gains, int64_t* cov, int64_t* cov_upper, int32_t* n_selected);
imin_status_t imin_lrr_coverage(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, const int32_t* set,
                                int32_t n_set, int64_t theta, uint64_t key, void* stream, int64_t* covered);

/*
 * imin_gsbm -- GSBM (Section 5.2): Algorithm 4's loop over LRR sets, with
 *   theta_max = 2 |V'_s| ((1 - 1/e) sqrt(ln(6/delta)) +
 *     sqrt((1 - 1/e)(ln C(n - |S|, k) + ln(6/delta))))^2 / (eps^2 OPT^L),
 *   theta_0 = theta_max eps^2 OPT^L / |V'_s|, i_max and a_1 = a_2 as LSBM,
 *   sigma^L = ((sqrt(Cov_2(B_U) + 2 a_1/9) - sqrt(a_1/2))^2 - a_1/18) |V'_s| / theta,
 *   sigma^U = (sqrt(Cov^u_1 + a_2/2) + sqrt(a_2/2))^2 |V'_s| / theta,
 * where the binomial follows the section's proof (n - |S| candidates), and ON
 * and OPT^L are computed as for imin_lsbm (beta and delta set the stopping
 * rule behind OPT^L).  Pool 1 uses key rng_seed ^ 0x2545F4914F6CDD1D, pool
 * 2 rng_seed ^ 0x9FB21C651E98DF25.
 *
 * imin_lhga -- LHGA (Section 5.3): ON when |ON| <= k, else the k nodes of ON
 * with the largest Pr[s -> v] deg(v), ties to the smaller id, with Pr[s -> v]
 * the reach frequency over imin_lsbm's stopping-rule worlds (scores compare
 * as count(v) * out-degree(v), exact integers; the out-degree counts CSR
 * slots).  blockers in decreasing score order.
 *
 * imin_sandimin -- SandIMIN (Algorithm 1, Section 3.1): B_L = LSBM, B_U =
 * GSBM, B_R = LHGA on the same stopping-rule worlds; for each, the
 * (gamma, delta) estimate of E[I_{G[V \ B]}(s)] by the Stopping Rule
 * Algorithm on |R_w(B)| / b over the worlds of key rng_seed ^
 * 0xD6E8FEB86659FD93 (Upsilon from gamma and failure probability delta);
 * the answer is the set with the smallest estimate (ties: L, then U, then
 * R).  candidates: int32[3k], device, optional: B_L, B_U, B_R at offsets
 * 0, k, 2k (their sizes in info->n_blockers).
 */
typedef struct imin_gsbm_info {
    int32_t returned_on;
    int32_t on_size;
    int64_t nvp;          /* |V'_s| */
    int64_t sra_worlds;   /* N of the stopping rule behind OPT^L */
    double opt_l;
    double theta_max;
    double theta_0;
    int32_t i_max;
    int32_t iterations;
    int64_t theta;
    int64_t cov1;
    int64_t cov2;
    int64_t cov_upper;
    double sigma_l;
    double sigma_u;
    double a1;
} imin_gsbm_info_t;

imin_status_t imin_gsbm(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps,
                        double beta, double delta, uint64_t rng_seed, void* stream, int32_t* blockers,
                        int32_t* n_selected, imin_gsbm_info_t* info);
imin_status_t imin_lhga(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double beta,
                        double delta, uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected);

typedef struct imin_sandimin_info {
    int32_t choice;           /* 0: B_L, 1: B_U, 2: B_R */
    int32_t n_blockers[3];
    double estimate[3];       /* estimated E[I_{G[V \ B]}(s)] of B_L, B_U, B_R */
    int64_t eval_worlds[3];   /* worlds each estimate drew */
    imin_lsbm_info_t lsbm;
    imin_gsbm_info_t gsbm;
} imin_sandimin_info_t;

imin_status_t imin_sandimin(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps,
                            double beta, double gamma, double delta, uint64_t rng_seed, void* stream,
                            int32_t* blockers, int32_t* n_selected, int32_t* candidates,
                            imin_sandimin_info_t* info);

/*
 * imin_autotune -- choose the launch shape of the from-scratch world passes
 * for a graph: the tier-0 world launch's workgroup count, as a percentage
 * (50, 75, 100, 150, 200 or 300) of its LDS residency on the device.  Each
 * candidate runs seven from-scratch passes of the given query (worlds
 * [0, theta)), the candidates taking turns, the first round warming the
 * caches; every candidate must produce the same gains and total (a
 * difference is IMIN_ERR_INTERNAL).  A shape replaces the default (200) only
 * when its median pass is at least 3% faster, and the choice is kept on the
 * handle for every later call on it.  grid0_pct: HOST, out; pass_ms: HOST,
 * out, optional (the chosen shape's median pass time).
 * imin_set_launch_shape sets the percentage directly (0: the default).
 * Launch shapes never change any result; they only move time.  Calls given a
 * workspace keep the default shape (their layout is fixed when sized).
 */
imin_status_t imin_autotune(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int64_t theta,
                            uint64_t rng_seed, void* stream, int32_t* grid0_pct, float* pass_ms);
imin_status_t imin_set_launch_shape(imin_graph_t g, int32_t grid0_pct);

/*
 * Scratch device memory of imin_solve and imin_evaluate comes from a block
 * cache, per device: a block released at the end of a call stays allocated
 * for the next call (a request reuses a cached block of at most twice its
 * size), because freeing and allocating gigabytes costs milliseconds per
 * call.  The cache holds at most IMIN_CACHE_BYTES bytes (environment,
 * default 64 GiB; the largest blocks are freed first beyond it), and an
 * allocation that fails frees the device's cached blocks and tries again.
 * imin_cache_release frees every cached block on every device.  Blocks in
 * use by calls still running are not cached and are not touched.  Never
 * fails.
 */
imin_status_t imin_cache_release(void);

/*
 * Kernel timing, for measurement.  While enabled, the library brackets its
 * own kernel launches with HIP events on the stream they run on and adds
 * each launch's duration to a per-kernel tally (process-wide).  The world
 * kernels (ids 0, 1, 4, 6, 7, 8) take the events into their own launch
 * (hipExtLaunchKernel), so that the interval is the kernel's alone; the
 * others are bracketed by separate event records.  Kernel ids:
 *   0  world evaluation, small LDS tier (one wave per world)
 *   1  world evaluation, HBM tier (four waves per world, any size)
 *   2  gain reduction of a from-scratch pass (bucket histogram, scan,
 *      scatter, accumulate, sum), or in a solve whose round-0 worlds stay
 *      where they were written, the build of the node index that yields the
 *      gains; incremental rounds add their changes to the gains inside
 *      kernels 1, 4, 6 and 7
 *   3  greedy selection
 *   4  world evaluation, large LDS tier (four waves per world)
 *   5  search for the worlds a new blocker changes (incremental rounds
 *      without replay, whose changed worlds are sampled again)
 *   6  an incremental round with replay, one launch: the last selection is
 *      committed, the worlds where no live edge leaves the new blocker's
 *      dominator subtree are updated from their dominator-tree labels, and
 *      the other changed worlds are replayed from their stored live edges
 *      (worlds too large for the replay go on to kernel 7)
 *   7  the wide replay of an incremental round: worlds too large for kernel
 *      6's replay, one 1024-thread workgroup each, with four times its
 *      capacities (worlds too large for it go on to kernels 4 and 1)
 *   8  level 0 drawn ahead: the live seed slots of a tile's worlds as bits,
 *      read by the world kernels of that tile (from-scratch passes)
 * imin_timing_read returns the number of launches and their summed duration
 * in milliseconds (host pointers).  Enabling adds a small per-launch cost.
 */
imin_status_t imin_timing_enable(int on);
/* Bit i set: kernel id i is bracketed with events while timing is enabled
 * (default: all).  Work tallies are kept whatever the mask. */
imin_status_t imin_timing_mask(uint32_t kernel_mask);
/* Time one launch in `every` (>= 1, default 1) of each selected kernel: the
 * events themselves take time on the stream.  IMIN_ERR_INVALID if every < 1. */
imin_status_t imin_timing_sample(int every);
/* Whether calls made while timing is enabled keep the work tallies that
 * imin_timing_work reports (default 1).  Taking them costs each call a
 * clear, a copy to the host and a sum of per-workgroup slots, which grow with
 * the launch shapes; with 0 only the selected kernels' events are taken. */
imin_status_t imin_timing_tallies(int on);
/* Launches of a selected kernel while timing was enabled, timed or not, since
 * the last reset (host pointer). */
imin_status_t imin_timing_launches(int kernel_id, int64_t* all);
imin_status_t imin_timing_reset(void);
imin_status_t imin_timing_read(int kernel_id, int64_t* launches, double* total_ms);

/*
 * Work done while timing was enabled, per world tier (0 small LDS, 1 large
 * LDS, 2 HBM, 3 replay, 4 label-based update by the label-rule workgroups,
 * which take a world per 16, 32 or 64 lanes, 5 label-based update of worlds
 * handed to the replay that reduce to it): worlds finished, edges walked (for
 * tiers 4 and 5: stored entries scanned), algorithmic HBM bytes, reached
 * nodes and live edges.  For tiers 0-2 the edges are the CSR slots of the
 * reached rows (the edges whose coins were needed), the bytes are 8 per such
 * slot (column and threshold) + 8 per reached non-seed (row offsets) + 16 per
 * level-0 table entry + 8 per (node, count) entry written (12 with its BFS
 * parent kept for replay, + 8 per extra live edge kept), the reached nodes
 * count the seeds, and the live edges are the live edges between reached
 * nodes that are not seeds or blocked (one BFS-tree edge per reached
 * non-seed plus every other such edge).  For the replay tier the edges are
 * the stored live edges and the bytes are 12 per stored entry (node, count,
 * parent) + 8 per stored extra edge.  Incremental rounds add, for every tier,
 * 8 per stored entry read back and 12 per change reported (the change and
 * the count updated in place).  Reached nodes and live edges are tallied for
 * tiers 0-2 only.  Host pointers; any may be NULL.
 */
imin_status_t imin_timing_work(int tier, int64_t* worlds, int64_t* edges, int64_t* bytes, int64_t* reached,
                               int64_t* live);

/*
 * Measurement probes: the ceilings the sampling kernels are held against.
 * Each launches one kernel on `stream`, waits for it and writes its duration
 * in milliseconds (from events recorded by the launch) to *ms (host).
 *
 * imin_probe_philox  draws Philox4x32-10 blocks with the coin layout of the
 *                    world kernels (counter (group, world, 0, 0), key
 *                    (lo32(key), hi32(key))) for groups 0..groups_per_world-1
 *                    of worlds 0..worlds-1, touching no memory but one word
 *                    per thread of `out` (device, out_count >= grid * 256
 *                    entries, overwritten); 4 coins per block.
 * imin_probe_copy    copies `bytes` (a multiple of 16; both pointers 16-byte
 *                    aligned, device) from src to dst with 16-byte accesses;
 *                    2 * bytes cross HBM.
 * `grid` is the number of 256-thread workgroups.  IMIN_ERR_INVALID for bad
 * arguments, IMIN_ERR_DEVICE when a runtime call fails.
 */
imin_status_t imin_probe_philox(int64_t worlds, int32_t groups_per_world, uint64_t key, uint32_t* out,
                                int64_t out_count, int32_t grid, void* stream, float* ms);
imin_status_t imin_probe_copy(void* dst, const void* src, size_t bytes, int32_t grid, void* stream, float* ms);

/* Static description of a status code. */
const char* imin_status_string(imin_status_t s);

/*
 * Device status bits of the last failed call on this thread (0 if none):
 * a host-readable detail for IMIN_ERR_DATA / IMIN_ERR_INTERNAL.
 */
uint32_t imin_last_device_flags(void);

/*
 * Whether this thread's last blocking imin_solve ran incremental rounds (1)
 * or re-evaluated every world each round (0: its resident store would have
 * exceeded IMIN_STORE_CAP entries, at most 0xFF000000 - 1, or the device;
 * the results are the same integers, only slower); -1 before any completed
 * solve.
 */
int32_t imin_last_solve_incremental(void);

#ifdef __cplusplus
}
#endif

#endif /* IMIN_H */
