/*
 * CPU oracle for the sampling estimator of influence minimization by node
 * blocking (Wang et al., "Efficient Influence Minimization via Node
 * Blocking", PVLDB).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  It
 * is plain, slow and written for a reader holding the paper: every function
 * follows one passage and cites it.  It shares no code, header, table or
 * constant with the GPU path; only the tests, the smoke check and the CPU leg
 * of the benchmark load it.
 *
 * What it computes, per query (G, p, S, k, theta, rng_seed):
 *
 *   thr[e]     integer coin threshold of edge e from its float32 probability
 *              (the live-edge process of Section 2.1, Eq. 1: an edge is kept
 *              with probability p(u, v)); p == 1 is "always live", otherwise
 *              thr = floor(p * 2^32) computed exactly in double.
 *   coin(w,e)  word (e mod 4) of Philox4x32-10 (Salmon et al., SC'11) at
 *              counter (floor(e/4), w, 0, 0), key (lo32(seed), hi32(seed));
 *              edge e is live in world w iff thr[e] is "always live" or
 *              coin < thr[e].
 *   R_w(B)     nodes reachable from S in world w once the blockers B are
 *              removed (Section 2.1: a blocker's in-edges get probability 0;
 *              blockers are never seeds; the spread counts S itself).
 *   c_w(u|B)   |R_w(B)| - |R_w(B + u)|: the nodes that u protects.  By the
 *              dominator-tree lemma quoted in Section 2.2 this equals the size
 *              of u's subtree in the dominator tree of world w rooted at the
 *              virtual source s, whose edges to every seed have probability 1
 *              (Section 3.1).  It counts u itself (Example 1).
 *   gain_r[u]  sum over worlds w < theta of c_w(u|B_r)   (Section 2.2, the
 *              estimator of Xie et al.: D_s(u) is estimated by the average
 *              subtree size; the sum is that average times theta).
 *   T_r        sum over worlds of |R_w(B_r)|.
 *   greedy     the greedy framework of Section 2.2 (AdvancedGreedy): k
 *              iterations, each adding argmax_u gain_r[u] over V \ (S + B_r),
 *              ties to the smaller id; stop early when no candidate is left
 *              or the best gain is 0 ("at most k" blockers, problem
 *              statement).  Worlds are shared by every round.
 *
 * Two ways to get c_w are provided and must agree:
 *   mode 0 (dominator): breadth-first reachability, then the iterative
 *          dominator algorithm of Cooper, Harvey and Kennedy ("A Simple, Fast
 *          Dominance Algorithm", 2001) over the reached live subgraph plus
 *          the virtual source, then subtree sizes;
 *   mode 1 (definition): one extra reachability pass per reached candidate u.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from Salmon, Moraes, Dror and Shaw, "Parallel random        */
/* numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit key,  */
/* ten rounds of two 32x32->64 multiplies (multipliers 0xD2511F53 and         */
/* 0xCD9E8D57) with the key bumped by the Weyl increments 0x9E3779B9 and      */
/* 0xBB67AE85 between rounds.                                                 */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Edge thresholds.  Section 2.1 keeps each edge with probability p(u, v).    */
/* The coin is a uniform 32-bit word, so the edge is kept when the word is    */
/* below floor(p * 2^32); p == 1 must always keep the edge, which no 32-bit   */
/* word can express as a strict bound, so it gets the reserved value          */
/* 0xFFFFFFFF ("always live").  The largest float32 below 1 maps to           */
/* 0xFFFFFF00, so the reserved value is never produced by the floor.          */
/* Returns -1 when every p is in [0, 1], else the first offending index.      */
/* ------------------------------------------------------------------------ */
#define ORACLE_ALWAYS_LIVE 0xFFFFFFFFu

int64_t oracle_thresholds(int64_t m, const float* p, uint32_t* thr) {
    for (int64_t e = 0; e < m; ++e) {
        float pe = p[e];
        if (!(pe >= 0.0f && pe <= 1.0f)) return e; /* also catches NaN */
        if (pe == 1.0f) {
            thr[e] = ORACLE_ALWAYS_LIVE;
        } else {
            double scaled = (double)pe * 4294967296.0; /* exact: 24-bit mantissa times 2^32 */
            thr[e] = (uint32_t)scaled;                 /* truncation == floor for scaled >= 0 */
        }
    }
    return -1;
}

uint32_t oracle_coin(uint64_t seed, uint64_t w, int64_t e) {
    uint32_t ctr[4] = {(uint32_t)((uint64_t)e >> 2), (uint32_t)w, 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[(uint64_t)e & 3u];
}

static int edge_live(uint32_t thr, uint64_t seed, uint64_t w, int64_t e) {
    if (thr == ORACLE_ALWAYS_LIVE) return 1;
    return oracle_coin(seed, w, e) < thr;
}

/* ------------------------------------------------------------------------ */
/* Query and per-thread scratch                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;
    int64_t m;
    const int64_t* row_ptr;
    const int32_t* col;
    const uint32_t* thr;
    const int32_t* seeds;
    int32_t n_seeds;
    uint64_t rng_seed;
} query_t;

typedef struct {
    int32_t n;
    int32_t* stamp;     /* [n] world visit stamps                     */
    int32_t stamp_now;
    int32_t* local_of;  /* [n] node -> local id (1-based; 0 = root)  */
    int32_t* queue;     /* [n] BFS order of reached nodes             */
    uint8_t* blocked;   /* [n] private copy of the blocked set        */
    /* live subgraph over local ids 0..R (0 = virtual source s) */
    int64_t cap_e;
    int32_t* e_src;
    int32_t* e_dst;
    int32_t* pred_off; /* [n+2] */
    int32_t* pred;     /* [cap_e] */
    int32_t* succ_off; /* [n+2] */
    int32_t* succ;     /* [cap_e] */
    int32_t* fill;     /* [n+2] */
    int32_t* po;       /* [n+1] postorder number of each local id */
    int32_t* rpo;      /* [n+1] local ids in reverse postorder     */
    int32_t* idom;     /* [n+1] */
    int32_t* size;     /* [n+1] dominator subtree sizes */
    int32_t* stack;    /* [n+1] DFS stack: local ids */
    int32_t* it;       /* [n+1] DFS stack: next successor index */
    int32_t* c;        /* [n] per-node counts of the current world  */
    int oom;
} scratch_t;

static void scratch_free(scratch_t* s) {
    free(s->stamp); free(s->local_of); free(s->queue); free(s->blocked);
    free(s->e_src); free(s->e_dst); free(s->pred_off); free(s->pred);
    free(s->succ_off); free(s->succ); free(s->fill); free(s->po); free(s->rpo);
    free(s->idom); free(s->size); free(s->stack); free(s->it); free(s->c);
    memset(s, 0, sizeof(*s));
}

static int scratch_init(scratch_t* s, int32_t n, const uint8_t* blocked) {
    memset(s, 0, sizeof(*s));
    s->n = n;
    size_t nn = (size_t)n + 2;
    s->stamp = calloc(nn, sizeof(int32_t));
    s->local_of = calloc(nn, sizeof(int32_t));
    s->queue = calloc(nn, sizeof(int32_t));
    s->blocked = calloc(nn, 1);
    s->pred_off = calloc(nn + 1, sizeof(int32_t));
    s->succ_off = calloc(nn + 1, sizeof(int32_t));
    s->fill = calloc(nn + 1, sizeof(int32_t));
    s->po = calloc(nn, sizeof(int32_t));
    s->rpo = calloc(nn, sizeof(int32_t));
    s->idom = calloc(nn, sizeof(int32_t));
    s->size = calloc(nn, sizeof(int32_t));
    s->stack = calloc(nn, sizeof(int32_t));
    s->it = calloc(nn, sizeof(int32_t));
    s->c = calloc(nn, sizeof(int32_t));
    s->cap_e = 1024;
    s->e_src = malloc(s->cap_e * sizeof(int32_t));
    s->e_dst = malloc(s->cap_e * sizeof(int32_t));
    s->pred = malloc(s->cap_e * sizeof(int32_t));
    s->succ = malloc(s->cap_e * sizeof(int32_t));
    if (!s->stamp || !s->local_of || !s->queue || !s->blocked || !s->pred_off || !s->succ_off ||
        !s->fill || !s->po || !s->rpo || !s->idom || !s->size || !s->stack || !s->it || !s->c ||
        !s->e_src || !s->e_dst || !s->pred || !s->succ) {
        scratch_free(s);
        return -1;
    }
    if (blocked) memcpy(s->blocked, blocked, (size_t)n);
    return 0;
}

static int push_edge(scratch_t* s, int64_t* ne, int32_t a, int32_t b) {
    if (*ne == s->cap_e) {
        int64_t cap = s->cap_e * 2;
        int32_t* p1 = realloc(s->e_src, cap * sizeof(int32_t));
        if (p1) s->e_src = p1;
        int32_t* p2 = realloc(s->e_dst, cap * sizeof(int32_t));
        if (p2) s->e_dst = p2;
        int32_t* p3 = realloc(s->pred, cap * sizeof(int32_t));
        if (p3) s->pred = p3;
        int32_t* p4 = realloc(s->succ, cap * sizeof(int32_t));
        if (p4) s->succ = p4;
        if (!p1 || !p2 || !p3 || !p4) { s->oom = 1; return -1; }
        s->cap_e = cap;
    }
    s->e_src[*ne] = a;
    s->e_dst[*ne] = b;
    ++*ne;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* R_w(B): breadth-first search from S over live edges of world w, never     */
/* entering a blocked node (Section 2.1, live-edge process and blocking;     */
/* Section 3.1, the virtual source reaches every seed with probability 1).   */
/* Fills s->queue with the reached nodes in BFS order and returns |R_w(B)|.  */
/* ------------------------------------------------------------------------ */
static int32_t reach(const query_t* q, scratch_t* s, uint64_t w) {
    int32_t stamp = ++s->stamp_now;
    int32_t head = 0, tail = 0;
    for (int32_t i = 0; i < q->n_seeds; ++i) {
        int32_t v = q->seeds[i];
        if (s->stamp[v] != stamp) {
            s->stamp[v] = stamp;
            s->queue[tail++] = v;
        }
    }
    while (head < tail) {
        int32_t u = s->queue[head++];
        for (int64_t e = q->row_ptr[u]; e < q->row_ptr[u + 1]; ++e) {
            int32_t v = q->col[e];
            if (s->blocked[v]) continue;
            if (!edge_live(q->thr[e], q->rng_seed, w, e)) continue;
            if (s->stamp[v] == stamp) continue;
            s->stamp[v] = stamp;
            s->queue[tail++] = v;
        }
    }
    return tail;
}

/* Cooper-Harvey-Kennedy intersect: walk the two fingers up the current tree,  */
/* always moving the one with the smaller postorder number.                    */
static int32_t intersect(const int32_t* idom, const int32_t* po, int32_t a, int32_t b) {
    while (a != b) {
        while (po[a] < po[b]) a = idom[a];
        while (po[b] < po[a]) b = idom[b];
    }
    return a;
}

/* ------------------------------------------------------------------------ */
/* Mode 0: c_w(u|B) for every node as dominator-subtree sizes (Section 2.2,   */
/* the estimator of Xie et al.: sample a realization, build its dominator     */
/* tree rooted at s, measure every subtree).  Writes s->c[v] for all v in     */
/* R_w (seeds included; callers skip them) and returns |R_w(B)|.              */
/* ------------------------------------------------------------------------ */
static int32_t world_counts_dominator(const query_t* q, scratch_t* s, uint64_t w) {
    int32_t R = reach(q, s, w);
    int32_t N = R + 1; /* local ids: 0 = s, 1..R = reached nodes in BFS order */
    for (int32_t i = 0; i < R; ++i) s->local_of[s->queue[i]] = i + 1;

    /* live subgraph: s -> every seed, and every live edge u -> v with u      */
    /* reached and v not blocked (v is then reached too).  Self-loops never   */
    /* change reachability or dominance and are left out.                     */
    int64_t ne = 0;
    for (int32_t i = 0; i < q->n_seeds; ++i)
        if (push_edge(s, &ne, 0, s->local_of[q->seeds[i]])) return -1;
    for (int32_t i = 0; i < R; ++i) {
        int32_t u = s->queue[i];
        for (int64_t e = q->row_ptr[u]; e < q->row_ptr[u + 1]; ++e) {
            int32_t v = q->col[e];
            if (v == u || s->blocked[v]) continue;
            if (!edge_live(q->thr[e], q->rng_seed, w, e)) continue;
            if (push_edge(s, &ne, i + 1, s->local_of[v])) return -1;
        }
    }
    /* predecessor and successor lists (CSR over local ids) */
    for (int32_t v = 0; v <= N; ++v) { s->pred_off[v] = 0; s->succ_off[v] = 0; }
    for (int64_t i = 0; i < ne; ++i) { s->pred_off[s->e_dst[i] + 1]++; s->succ_off[s->e_src[i] + 1]++; }
    for (int32_t v = 0; v < N; ++v) { s->pred_off[v + 1] += s->pred_off[v]; s->succ_off[v + 1] += s->succ_off[v]; }
    for (int32_t v = 0; v < N; ++v) s->fill[v] = s->pred_off[v];
    for (int64_t i = 0; i < ne; ++i) s->pred[s->fill[s->e_dst[i]]++] = s->e_src[i];
    for (int32_t v = 0; v < N; ++v) s->fill[v] = s->succ_off[v];
    for (int64_t i = 0; i < ne; ++i) s->succ[s->fill[s->e_src[i]]++] = s->e_dst[i];

    /* depth-first postorder from s (iterative) */
    for (int32_t v = 0; v < N; ++v) s->po[v] = -1;
    int32_t top = 0, counter = 0;
    int32_t* onstack = s->idom; /* reuse as a visited flag before idom is computed */
    for (int32_t v = 0; v < N; ++v) onstack[v] = 0;
    s->stack[top] = 0; s->it[top] = s->succ_off[0]; top = 1; onstack[0] = 1;
    while (top > 0) {
        int32_t v = s->stack[top - 1];
        if (s->it[top - 1] < s->succ_off[v + 1]) {
            int32_t x = s->succ[s->it[top - 1]++];
            if (!onstack[x]) {
                onstack[x] = 1;
                s->stack[top] = x;
                s->it[top] = s->succ_off[x];
                ++top;
            }
        } else {
            s->po[v] = counter++;
            --top;
        }
    }
    /* every local id is reachable from s by construction */
    for (int32_t v = 0; v < N; ++v) s->rpo[N - 1 - s->po[v]] = v;

    /* Cooper-Harvey-Kennedy: iterate idom(v) = intersection over the        */
    /* processed predecessors until nothing changes.                          */
    for (int32_t v = 0; v < N; ++v) s->idom[v] = -1;
    s->idom[0] = 0;
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int32_t i = 1; i < N; ++i) {
            int32_t v = s->rpo[i];
            int32_t nd = -1;
            for (int32_t j = s->pred_off[v]; j < s->pred_off[v + 1]; ++j) {
                int32_t p = s->pred[j];
                if (s->idom[p] == -1) continue;
                nd = (nd == -1) ? p : intersect(s->idom, s->po, p, nd);
            }
            if (s->idom[v] != nd) { s->idom[v] = nd; changed = 1; }
        }
    }

    /* subtree sizes: children before parents = increasing postorder */
    for (int32_t v = 0; v < N; ++v) s->size[v] = 1;
    for (int32_t i = N - 1; i >= 1; --i) {
        int32_t v = s->rpo[i];
        s->size[s->idom[v]] += s->size[v];
    }
    for (int32_t i = 0; i < R; ++i) s->c[s->queue[i]] = s->size[i + 1];
    return R;
}

/* ------------------------------------------------------------------------ */
/* Mode 1: c_w(u|B) = |R_w(B)| - |R_w(B + u)| literally (Section 2.1, the     */
/* decreased spread D_S(B) = E[I_G(S)] - E[I_{G[V\B]}(S)] on one world).     */
/* ------------------------------------------------------------------------ */
static int32_t world_counts_definition(const query_t* q, scratch_t* s, uint64_t w, int32_t* reached_buf) {
    int32_t R = reach(q, s, w);
    memcpy(reached_buf, s->queue, (size_t)R * sizeof(int32_t));
    for (int32_t i = 0; i < R; ++i) {
        int32_t u = reached_buf[i];
        s->c[u] = 0;
        int is_seed = 0;
        for (int32_t j = 0; j < q->n_seeds; ++j) is_seed |= (q->seeds[j] == u);
        if (is_seed) continue;
        s->blocked[u] = 1;
        int32_t R2 = reach(q, s, w);
        s->blocked[u] = 0;
        s->c[u] = R - R2;
    }
    /* leave queue holding R_w(B) for the caller */
    memcpy(s->queue, reached_buf, (size_t)R * sizeof(int32_t));
    return R;
}

/* ------------------------------------------------------------------------ */
/* Evaluation over a world range, threaded over contiguous sub-ranges.       */
/* gain[u] += sum_w c_w(u|B) for u not in S; *total += sum_w |R_w(B)|.       */
/* Optional per-world outputs: rsize[w - w0] = |R_w(B)| and                  */
/* rsum[w - w0] = sum of the reached node ids (an order-free fingerprint).   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const query_t* q;
    const uint8_t* blocked;
    const uint8_t* is_seed;
    int mode;
    int count_gain; /* 0: reachability only */
    uint64_t w_begin, w_end, w0;
    int64_t* gain;  /* [n] private partial */
    int64_t total;
    int32_t* rsize;
    int64_t* rsum;
    int status;
} job_t;

static void* eval_job(void* arg) {
    job_t* j = (job_t*)arg;
    const query_t* q = j->q;
    scratch_t s;
    if (scratch_init(&s, q->n, j->blocked)) { j->status = -1; return NULL; }
    int32_t* buf = NULL;
    if (j->mode == 1) {
        buf = malloc(((size_t)q->n + 1) * sizeof(int32_t));
        if (!buf) { scratch_free(&s); j->status = -1; return NULL; }
    }
    for (uint64_t w = j->w_begin; w < j->w_end; ++w) {
        int32_t R;
        if (!j->count_gain) R = reach(q, &s, w);
        else if (j->mode == 1) R = world_counts_definition(q, &s, w, buf);
        else R = world_counts_dominator(q, &s, w);
        if (R < 0 || s.oom) { j->status = -1; break; }
        j->total += R;
        int64_t sum = 0;
        for (int32_t i = 0; i < R; ++i) {
            int32_t v = s.queue[i];
            sum += v;
            if (j->count_gain && !j->is_seed[v]) j->gain[v] += s.c[v];
        }
        if (j->rsize) j->rsize[w - j->w0] = R;
        if (j->rsum) j->rsum[w - j->w0] = sum;
    }
    free(buf);
    scratch_free(&s);
    return NULL;
}

static int run_eval(const query_t* q, const uint8_t* blocked, int mode, int count_gain,
                    uint64_t w0, uint64_t nw, int nthreads, int64_t* gain, int64_t* total,
                    int32_t* rsize, int64_t* rsum) {
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > nw && nw > 0) nthreads = (int)nw;
    uint8_t* is_seed = calloc((size_t)q->n + 1, 1);
    job_t* jobs = calloc((size_t)nthreads, sizeof(job_t));
    pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
    if (!is_seed || !jobs || !th) { free(is_seed); free(jobs); free(th); return -1; }
    for (int32_t i = 0; i < q->n_seeds; ++i) is_seed[q->seeds[i]] = 1;
    int status = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].q = q;
        jobs[t].blocked = blocked;
        jobs[t].is_seed = is_seed;
        jobs[t].mode = mode;
        jobs[t].count_gain = count_gain;
        jobs[t].w0 = w0;
        jobs[t].w_begin = w0 + nw * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].w_end = w0 + nw * (uint64_t)(t + 1) / (uint64_t)nthreads;
        jobs[t].rsize = rsize;
        jobs[t].rsum = rsum;
        jobs[t].gain = count_gain ? calloc((size_t)q->n, sizeof(int64_t)) : NULL;
        if (count_gain && !jobs[t].gain) status = -1;
    }
    if (status == 0) {
        for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, eval_job, &jobs[t]);
        eval_job(&jobs[0]);
        for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    /* merge in thread order; integer sums make the order immaterial */
    for (int t = 0; t < nthreads; ++t) {
        if (jobs[t].status) status = -1;
        *total += jobs[t].total;
        if (count_gain && jobs[t].gain) {
            for (int32_t v = 0; v < q->n; ++v) gain[v] += jobs[t].gain[v];
        }
        free(jobs[t].gain);
    }
    free(is_seed); free(jobs); free(th);
    return status;
}

static int check_query(int32_t n, const int32_t* seeds, int32_t n_seeds, const uint8_t* blocked) {
    if (n < 1 || n_seeds < 1 || n_seeds > n) return -1;
    uint8_t* seen = calloc((size_t)n, 1);
    if (!seen) return -1;
    int bad = 0;
    for (int32_t i = 0; i < n_seeds && !bad; ++i) {
        int32_t v = seeds[i];
        if (v < 0 || v >= n || seen[v]) bad = 1;
        else {
            seen[v] = 1;
            if (blocked && blocked[v]) bad = 1; /* blockers are never seeds */
        }
    }
    free(seen);
    return bad ? -1 : 0;
}

/* Public: evaluate gains under a given blocked set over worlds [w0, w0+nw).  */
/* gain[n] and *total are overwritten.  rsize/rsum may be NULL.               */
int oracle_eval(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                const int32_t* seeds, int32_t n_seeds, const uint8_t* blocked, uint64_t rng_seed,
                uint64_t w0, uint64_t nw, int mode, int nthreads,
                int64_t* gain, int64_t* total, int32_t* rsize, int64_t* rsum) {
    if (check_query(n, seeds, n_seeds, blocked)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* blk = calloc((size_t)n, 1);
    if (!blk) return -1;
    if (blocked) memcpy(blk, blocked, (size_t)n);
    memset(gain, 0, (size_t)n * sizeof(int64_t));
    *total = 0;
    int st = run_eval(&q, blk, mode, 1, w0, nw, nthreads, gain, total, rsize, rsum);
    free(blk);
    return st;
}

/* Public: per-node counts and reached list of one world (for fixtures).      */
/* c_out[n] gets c_w(v|B) for reached non-seeds and 0 elsewhere; reached_out  */
/* (capacity n) gets R_w(B) in BFS order.  Returns |R_w(B)| or -1.            */
int32_t oracle_world(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                     const int32_t* seeds, int32_t n_seeds, const uint8_t* blocked, uint64_t rng_seed,
                     uint64_t w, int mode, int32_t* c_out, int32_t* reached_out) {
    if (check_query(n, seeds, n_seeds, blocked)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    scratch_t s;
    if (scratch_init(&s, n, blocked)) return -1;
    int32_t* buf = malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!buf) { scratch_free(&s); return -1; }
    int32_t R = (mode == 1) ? world_counts_definition(&q, &s, w, buf) : world_counts_dominator(&q, &s, w);
    if (R >= 0) {
        memset(c_out, 0, (size_t)n * sizeof(int32_t));
        for (int32_t i = 0; i < R; ++i) {
            int32_t v = s.queue[i];
            reached_out[i] = v;
            c_out[v] = s.c[v];
        }
        for (int32_t i = 0; i < n_seeds; ++i) c_out[seeds[i]] = 0;
    }
    free(buf);
    scratch_free(&s);
    return R;
}

/* ------------------------------------------------------------------------ */
/* The greedy framework of Section 2.2 driven by the dominator-tree           */
/* estimator (AdvancedGreedy), on worlds shared by every round.               */
/* Outputs: blockers[k] in selection order, gains[k] = gain_r[u*_r],          */
/* totals[k+1] = T_0 .. T_{n_selected}, *n_selected <= k.                     */
/* ------------------------------------------------------------------------ */
int oracle_solve(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                 const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed,
                 int mode, int nthreads,
                 int32_t* blockers, int64_t* gains, int64_t* totals, int32_t* n_selected) {
    if (k < 0 || theta < 1) return -1;
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* blk = calloc((size_t)n, 1);
    uint8_t* is_seed = calloc((size_t)n, 1);
    int64_t* gain = calloc((size_t)n, sizeof(int64_t));
    if (!blk || !is_seed || !gain) { free(blk); free(is_seed); free(gain); return -1; }
    for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
    int status = 0;
    int32_t r = 0;
    int64_t T = 0;
    for (;;) {
        if (r == k) {
            /* T_k by definition: reachability under the final blocked set */
            T = 0;
            status = run_eval(&q, blk, mode, 0, 0, theta, nthreads, NULL, &T, NULL, NULL);
            totals[r] = T;
            break;
        }
        memset(gain, 0, (size_t)n * sizeof(int64_t));
        T = 0;
        status = run_eval(&q, blk, mode, 1, 0, theta, nthreads, gain, &T, NULL, NULL);
        if (status) break;
        totals[r] = T;
        int32_t best = -1;
        for (int32_t u = 0; u < n; ++u) {
            if (is_seed[u] || blk[u]) continue;
            if (best < 0 || gain[u] > gain[best]) best = u; /* strict: ties keep the smaller id */
        }
        if (best < 0 || gain[best] == 0) break;
        blockers[r] = best;
        gains[r] = gain[best];
        blk[best] = 1;
        ++r;
    }
    *n_selected = r;
    free(blk); free(is_seed); free(gain);
    return status;
}

/* ======================================================================== */
/* Lower-bound coverage (Section 4.1) and Max-Coverage (Section 5.1).        */
/*                                                                          */
/*   CP set     C_w(s,v): the non-seed nodes that lie on every path from s   */
/*              to v in world w (Definition 4.1).  Algorithm 2 builds them   */
/*              from the dominator tree: walking R_w in depth-first preorder */
/*              from s, a node whose immediate dominator is a seed (or s)   */
/*              gets {v}; any other node gets its immediate dominator's set  */
/*              plus itself.                                                */
/*   CP seq.    the CP sets of every v in R_w \ S.                           */
/*   Cov(B)     number of (world, v) pairs whose CP set meets B; Cov/theta  */
/*              is unbiased for the lower bound D^L(B) (Lemma 4.2).          */
/*   Max-Cov.   k greedy steps, each adding argmax over V \ S of the        */
/*              marginal coverage (ties to the smaller id); stops when the  */
/*              best marginal is 0.                                         */
/*   Cov^u      for every greedy prefix B_i (0 <= i <= n_selected):          */
/*              Cov(B_i) + the sum of the k largest marginal coverages given */
/*              B_i; Algorithm 4 takes their minimum as its upper bound.    */
/* Worlds are drawn exactly as for the greedy above, without blockers.      */
/* ======================================================================== */

/* CP sets of the current world once world_counts_dominator has run on it:  */
/* entries (non-seed reached nodes) in depth-first preorder from s, each    */
/* with its set.  node_out[i] is entry i's node, its set is                  */
/* cp[cp_off[i] .. cp_off[i+1]).  Returns the entry count, or -1 when the   */
/* set storage (cp_cap node slots) is too small.                             */
static int32_t world_cp_sets(scratch_t* s, int32_t R, const uint8_t* is_seed,
                             int32_t* node_out, int64_t* cp_off, int32_t* cp, int64_t cp_cap,
                             int32_t* set_of /* [R+1]: entry index of each local id, -1 none */) {
    int32_t N = R + 1;
    /* depth-first preorder of the live subgraph from s (local id 0) */
    int32_t* seen = s->po; /* postorder numbers are no longer needed */
    for (int32_t v = 0; v < N; ++v) { seen[v] = 0; set_of[v] = -1; }
    int32_t top = 0, ne = 0;
    int64_t used = 0;
    cp_off[0] = 0;
    s->stack[top] = 0; s->it[top] = s->succ_off[0]; top = 1; seen[0] = 1;
    for (;;) {
        if (top == 0) break;
        int32_t v = s->stack[top - 1];
        if (s->it[top - 1] < s->succ_off[v + 1]) {
            int32_t x = s->succ[s->it[top - 1]++];
            if (seen[x]) continue;
            seen[x] = 1;
            s->stack[top] = x;
            s->it[top] = s->succ_off[x];
            ++top;
            /* x is visited now (preorder): its immediate dominator was      */
            /* visited earlier, since every path from s to x passes it       */
            int32_t node = s->queue[x - 1];
            if (is_seed[node]) continue;
            int32_t d = s->idom[x];
            int32_t dn = (d == 0) ? -1 : s->queue[d - 1];
            if (d != 0 && !is_seed[dn]) {
                int32_t pe = set_of[d];
                if (pe < 0) return -1; /* cannot happen: d is a visited non-seed */
                int64_t len = cp_off[pe + 1] - cp_off[pe];
                if (used + len + 1 > cp_cap) return -1;
                memcpy(cp + used, cp + cp_off[pe], (size_t)len * sizeof(int32_t));
                used += len;
            }
            if (used + 1 > cp_cap) return -1;
            cp[used++] = node;
            set_of[x] = ne;
            node_out[ne] = node;
            cp_off[ne + 1] = used;
            ++ne;
        } else {
            --top;
        }
    }
    return ne;
}

/* Public: the CP sequence of world w (for fixtures and the tests).          */
/* Returns the entry count, -1 on a bad query, -2 when cp_cap is too small. */
int32_t oracle_cp_world(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, uint64_t rng_seed, uint64_t w,
                        int32_t* node_out, int64_t* cp_off, int32_t* cp, int64_t cp_cap) {
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    scratch_t s;
    if (scratch_init(&s, n, NULL)) return -1;
    uint8_t* is_seed = calloc((size_t)n, 1);
    int32_t* set_of = malloc(((size_t)n + 2) * sizeof(int32_t));
    int32_t ret = -1;
    if (is_seed && set_of) {
        for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
        int32_t R = world_counts_dominator(&q, &s, w);
        if (R >= 0 && !s.oom) {
            ret = world_cp_sets(&s, R, is_seed, node_out, cp_off, cp, cp_cap, set_of);
            if (ret < 0) ret = -2;
        }
    }
    free(is_seed); free(set_of);
    scratch_free(&s);
    return ret;
}

/* The CP sequences of a world range, kept for the greedy: one flat list of */
/* sets per thread, a covered flag per set.                                  */
typedef struct {
    const query_t* q;
    const uint8_t* is_seed;
    uint64_t w_begin, w_end;
    int64_t n_sets;
    int64_t* set_off;  /* [n_sets + 1] */
    int32_t* cp;       /* set members */
    uint8_t* covered;  /* [n_sets] */
    int64_t* marg;     /* [n] this thread's marginal coverages */
    const uint8_t* in_b; /* [n] blocker flags (coverage of a given set) */
    int64_t count;     /* coverage counted by this thread */
    int status;
    /* sets: 0 = the CP sets of every world (Section 4.1); 1 = one LRR set per */
    /* sample (Section 4.2), its target drawn from vprime[0 .. nvp)            */
    int kind;
    const int32_t* vprime;
    uint32_t nvp;
} cov_job_t;

static int grow(void** p, int64_t* cap, int64_t need, size_t elem) {
    if (need <= *cap) return 0;
    int64_t c = *cap ? *cap : 1024;
    while (c < need) c *= 2;
    void* np = realloc(*p, (size_t)c * elem);
    if (!np) return -1;
    *p = np;
    *cap = c;
    return 0;
}

static int32_t world_lrr_set(const query_t* q, scratch_t* s, uint64_t w, const uint8_t* is_seed,
                             const int32_t* vprime, uint32_t nvp, int32_t* out);

/* Build every CP set of the job's worlds (Algorithm 2 on each world), or   */
/* one LRR set per sample (Algorithm 3).                                    */
static void* cov_build_job(void* arg) {
    cov_job_t* j = (cov_job_t*)arg;
    const query_t* q = j->q;
    scratch_t s;
    if (scratch_init(&s, q->n, NULL)) { j->status = -1; return NULL; }
    int32_t* node_out = malloc(((size_t)q->n + 1) * sizeof(int32_t));
    int64_t* off = malloc(((size_t)q->n + 2) * sizeof(int64_t));
    int32_t* set_of = malloc(((size_t)q->n + 2) * sizeof(int32_t));
    int64_t tmp_cap = 1 << 16;
    int32_t* tmp = malloc((size_t)tmp_cap * sizeof(int32_t));
    int64_t off_cap = 0, cp_cap = 0, cov_cap = 0;
    j->n_sets = 0;
    j->set_off = NULL; j->cp = NULL; j->covered = NULL;
    if (!node_out || !off || !set_of || !tmp || grow((void**)&j->set_off, &off_cap, 1, sizeof(int64_t))) {
        j->status = -1;
        goto done;
    }
    j->set_off[0] = 0;
    for (uint64_t w = j->w_begin; w < j->w_end; ++w) {
        if (j->kind == 1) {
            /* one set: node_out holds its members */
            int32_t len = world_lrr_set(q, &s, w, j->is_seed, j->vprime, j->nvp, node_out);
            if (len < 0 || s.oom) { j->status = -1; break; }
            if (len == 0) continue; /* an empty set is never covered */
            int64_t base = j->set_off[j->n_sets];
            if (grow((void**)&j->set_off, &off_cap, j->n_sets + 2, sizeof(int64_t)) ||
                grow((void**)&j->cp, &cp_cap, base + len, sizeof(int32_t)) ||
                grow((void**)&j->covered, &cov_cap, j->n_sets + 1, 1)) {
                j->status = -1;
                break;
            }
            memcpy(j->cp + base, node_out, (size_t)len * sizeof(int32_t));
            j->set_off[j->n_sets + 1] = base + len;
            j->covered[j->n_sets] = 0;
            j->n_sets += 1;
            continue;
        }
        int32_t R = world_counts_dominator(q, &s, w);
        if (R < 0 || s.oom) { j->status = -1; break; }
        int32_t ne;
        while ((ne = world_cp_sets(&s, R, j->is_seed, node_out, off, tmp, tmp_cap, set_of)) < 0) {
            int32_t* nt = realloc(tmp, (size_t)tmp_cap * 2 * sizeof(int32_t));
            if (!nt) { j->status = -1; goto done; }
            tmp = nt;
            tmp_cap *= 2;
        }
        int64_t base = j->set_off[j->n_sets];
        if (grow((void**)&j->set_off, &off_cap, j->n_sets + ne + 1, sizeof(int64_t)) ||
            grow((void**)&j->cp, &cp_cap, base + off[ne], sizeof(int32_t)) ||
            grow((void**)&j->covered, &cov_cap, j->n_sets + ne, 1)) {
            j->status = -1;
            break;
        }
        memcpy(j->cp + base, tmp, (size_t)off[ne] * sizeof(int32_t));
        for (int32_t i = 0; i < ne; ++i) {
            j->set_off[j->n_sets + i + 1] = base + off[i + 1];
            j->covered[j->n_sets + i] = 0;
        }
        j->n_sets += ne;
    }
done:
    free(node_out); free(off); free(set_of); free(tmp);
    scratch_free(&s);
    return NULL;
}

/* Marginal coverage of every node given the covered flags: each uncovered  */
/* set adds one to each of its members.                                      */
static void* cov_marg_job(void* arg) {
    cov_job_t* j = (cov_job_t*)arg;
    memset(j->marg, 0, (size_t)j->q->n * sizeof(int64_t));
    for (int64_t i = 0; i < j->n_sets; ++i) {
        if (j->covered[i]) continue;
        for (int64_t x = j->set_off[i]; x < j->set_off[i + 1]; ++x) j->marg[j->cp[x]] += 1;
    }
    return NULL;
}

/* Mark the sets that contain the flagged nodes; count the newly covered.  */
static void* cov_mark_job(void* arg) {
    cov_job_t* j = (cov_job_t*)arg;
    j->count = 0;
    for (int64_t i = 0; i < j->n_sets; ++i) {
        if (j->covered[i]) continue;
        for (int64_t x = j->set_off[i]; x < j->set_off[i + 1]; ++x) {
            if (j->in_b[j->cp[x]]) {
                j->covered[i] = 1;
                j->count += 1;
                break;
            }
        }
    }
    return NULL;
}

static void run_jobs(cov_job_t* jobs, int nthreads, void* (*fn)(void*)) {
    pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
    int started = 0;
    if (th) {
        for (int t = 1; t < nthreads; ++t) {
            if (pthread_create(&th[t], NULL, fn, &jobs[t]) == 0) ++started;
            else break;
        }
    }
    fn(&jobs[0]);
    for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
    for (int t = started + 1; t < nthreads; ++t) fn(&jobs[t]); /* threads that could not start */
    free(th);
}

static int cmp_desc_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x < y) - (x > y);
}

static void cov_free_jobs(cov_job_t* jobs, int nthreads) {
    for (int t = 0; t < nthreads; ++t) {
        free(jobs[t].set_off); free(jobs[t].cp); free(jobs[t].covered); free(jobs[t].marg);
    }
    free(jobs);
}

static cov_job_t* cov_build_sets(const query_t* q, const uint8_t* is_seed, uint64_t theta, int nthreads,
                                 int with_marg, int kind, const int32_t* vprime, uint32_t nvp) {
    cov_job_t* jobs = calloc((size_t)nthreads, sizeof(cov_job_t));
    if (!jobs) return NULL;
    int bad = 0;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t].q = q;
        jobs[t].is_seed = is_seed;
        jobs[t].kind = kind;
        jobs[t].vprime = vprime;
        jobs[t].nvp = nvp;
        jobs[t].w_begin = theta * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].w_end = theta * (uint64_t)(t + 1) / (uint64_t)nthreads;
        if (with_marg && !(jobs[t].marg = malloc((size_t)q->n * sizeof(int64_t)))) bad = 1;
    }
    if (!bad) run_jobs(jobs, nthreads, cov_build_job);
    for (int t = 0; t < nthreads; ++t) bad |= jobs[t].status;
    if (bad) { cov_free_jobs(jobs, nthreads); return NULL; }
    return jobs;
}

static cov_job_t* cov_build(const query_t* q, const uint8_t* is_seed, uint64_t theta, int nthreads, int with_marg) {
    return cov_build_sets(q, is_seed, theta, nthreads, with_marg, 0, NULL, 0);
}

/* Public: Max-Coverage over the CP sequences of worlds [0, theta) (Section  */
/* 5.1, procedure Max-Coverage of Algorithm 4), with the coverage of every   */
/* prefix and its upper-bound term.  Outputs: blockers[k], gains[k] (the     */
/* marginal coverage of each pick), cov[k+1] = Cov(B_0..B_{n_selected}),     */
/* cov_upper[k+1] = Cov(B_i) + sum of the k largest marginals given B_i.     */
static int max_coverage_sets(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                             const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed,
                             int nthreads, int kind, const int32_t* vprime, uint32_t nvp, int32_t* blockers,
                             int64_t* gains, int64_t* cov, int64_t* cov_upper, int32_t* n_selected) {
    if (k < 0 || theta < 1) return -1;
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > theta) nthreads = (int)theta;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* is_seed = calloc((size_t)n, 1);
    uint8_t* in_b = calloc((size_t)n, 1);  /* the pick whose sets are being covered */
    uint8_t* chosen = calloc((size_t)n, 1); /* B_r */
    int64_t* marg = malloc((size_t)n * sizeof(int64_t));
    int64_t* sorted = malloc((size_t)n * sizeof(int64_t));
    if (!is_seed || !in_b || !chosen || !marg || !sorted) {
        free(is_seed); free(in_b); free(chosen); free(marg); free(sorted);
        return -1;
    }
    for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
    cov_job_t* jobs = cov_build_sets(&q, is_seed, theta, nthreads, 1, kind, vprime, nvp);
    if (!jobs) { free(is_seed); free(in_b); free(chosen); free(marg); free(sorted); return -1; }
    for (int t = 0; t < nthreads; ++t) jobs[t].in_b = in_b;
    int64_t covered = 0;
    int32_t r = 0;
    for (;;) {
        /* marginal coverage of every candidate given B_r */
        run_jobs(jobs, nthreads, cov_marg_job);
        memset(marg, 0, (size_t)n * sizeof(int64_t));
        for (int t = 0; t < nthreads; ++t)
            for (int32_t v = 0; v < n; ++v) marg[v] += jobs[t].marg[v];
        /* the k largest marginals over V \ S \ B_r (nodes with none add 0) */
        int64_t nz = 0;
        for (int32_t v = 0; v < n; ++v)
            if (!is_seed[v] && !chosen[v] && marg[v] > 0) sorted[nz++] = marg[v];
        qsort(sorted, (size_t)nz, sizeof(int64_t), cmp_desc_i64);
        int64_t top = 0;
        for (int64_t i = 0; i < nz && i < k; ++i) top += sorted[i];
        cov[r] = covered;
        cov_upper[r] = covered + top;
        if (r == k) break;
        int32_t best = -1;
        for (int32_t v = 0; v < n; ++v) {
            if (is_seed[v] || chosen[v]) continue;
            if (best < 0 || marg[v] > marg[best]) best = v; /* ties keep the smaller id */
        }
        if (best < 0 || marg[best] == 0) break;
        blockers[r] = best;
        gains[r] = marg[best];
        chosen[best] = 1;
        /* cover the sets that contain the pick (sets covered before are     */
        /* skipped, so only the new pick is flagged)                         */
        memset(in_b, 0, (size_t)n);
        in_b[best] = 1;
        run_jobs(jobs, nthreads, cov_mark_job);
        int64_t add = 0;
        for (int t = 0; t < nthreads; ++t) add += jobs[t].count;
        covered += add;
        ++r;
    }
    *n_selected = r;
    cov_free_jobs(jobs, nthreads);
    free(is_seed); free(in_b); free(chosen); free(marg); free(sorted);
    return 0;
}

int oracle_max_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed,
                        int nthreads, int32_t* blockers, int64_t* gains, int64_t* cov, int64_t* cov_upper,
                        int32_t* n_selected) {
    return max_coverage_sets(n, m, row_ptr, col, thr, seeds, n_seeds, k, theta, rng_seed, nthreads, 0, NULL, 0,
                             blockers, gains, cov, cov_upper, n_selected);
}

static int coverage_sets(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                         const int32_t* seeds, int32_t n_seeds, const int32_t* blockers, int32_t n_blockers,
                         uint64_t theta, uint64_t rng_seed, int nthreads, int kind, const int32_t* vprime,
                         uint32_t nvp, int64_t* cov);

/* Public: Cov(B) over the CP sequences of worlds [0, theta) (Section 4.1). */
int oracle_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                    const int32_t* seeds, int32_t n_seeds, const int32_t* blockers, int32_t n_blockers,
                    uint64_t theta, uint64_t rng_seed, int nthreads, int64_t* cov) {
    return coverage_sets(n, m, row_ptr, col, thr, seeds, n_seeds, blockers, n_blockers, theta, rng_seed, nthreads,
                         0, NULL, 0, cov);
}

static int coverage_sets(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                         const int32_t* seeds, int32_t n_seeds, const int32_t* blockers, int32_t n_blockers,
                         uint64_t theta, uint64_t rng_seed, int nthreads, int kind, const int32_t* vprime,
                         uint32_t nvp, int64_t* cov) {
    if (theta < 1 || n_blockers < 0) return -1;
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > theta) nthreads = (int)theta;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* is_seed = calloc((size_t)n, 1);
    uint8_t* in_b = calloc((size_t)n, 1);
    if (!is_seed || !in_b) { free(is_seed); free(in_b); return -1; }
    for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
    int bad = 0;
    for (int32_t i = 0; i < n_blockers; ++i) {
        if (blockers[i] < 0 || blockers[i] >= n) bad = 1;
        else in_b[blockers[i]] = 1;
    }
    cov_job_t* jobs = bad ? NULL : cov_build_sets(&q, is_seed, theta, nthreads, 0, kind, vprime, nvp);
    if (!jobs) { free(is_seed); free(in_b); return -1; }
    for (int t = 0; t < nthreads; ++t) jobs[t].in_b = in_b;
    run_jobs(jobs, nthreads, cov_mark_job);
    *cov = 0;
    for (int t = 0; t < nthreads; ++t) *cov += jobs[t].count;
    cov_free_jobs(jobs, nthreads);
    free(is_seed); free(in_b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-node reach counts over worlds [w0, w0+nw): counts[v] = number of      */
/* worlds in which v is reached from S (no blockers).  counts[v]/nw          */
/* estimates Pr[s -> v] (Section 5.1, the lower bound OPT^L).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    const query_t* q;
    uint64_t w_begin, w_end;
    int64_t* counts;
    int status;
} reach_job_t;

static void* reach_job(void* arg) {
    reach_job_t* j = (reach_job_t*)arg;
    scratch_t s;
    if (scratch_init(&s, j->q->n, NULL)) { j->status = -1; return NULL; }
    for (uint64_t w = j->w_begin; w < j->w_end; ++w) {
        int32_t R = reach(j->q, &s, w);
        for (int32_t i = 0; i < R; ++i) j->counts[s.queue[i]] += 1;
    }
    scratch_free(&s);
    return NULL;
}

int oracle_reach_counts(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, uint64_t rng_seed, uint64_t w0, uint64_t nw,
                        int nthreads, int64_t* counts) {
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nw > 0 && (uint64_t)nthreads > nw) nthreads = (int)nw;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    reach_job_t* jobs = calloc((size_t)nthreads, sizeof(reach_job_t));
    pthread_t* th = calloc((size_t)nthreads, sizeof(pthread_t));
    int status = (jobs && th) ? 0 : -1;
    for (int t = 0; t < nthreads && status == 0; ++t) {
        jobs[t].q = &q;
        jobs[t].w_begin = w0 + nw * (uint64_t)t / (uint64_t)nthreads;
        jobs[t].w_end = w0 + nw * (uint64_t)(t + 1) / (uint64_t)nthreads;
        if (!(jobs[t].counts = calloc((size_t)n, sizeof(int64_t)))) status = -1;
    }
    if (status == 0) {
        for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, reach_job, &jobs[t]);
        reach_job(&jobs[0]);
        for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
        memset(counts, 0, (size_t)n * sizeof(int64_t));
        for (int t = 0; t < nthreads; ++t) {
            if (jobs[t].status) status = -1;
            for (int32_t v = 0; v < n; ++v) counts[v] += jobs[t].counts[v];
        }
    }
    if (jobs)
        for (int t = 0; t < nthreads; ++t) free(jobs[t].counts);
    free(jobs); free(th);
    return status;
}

/* Public: |R_w(B)| of every world in [w0, w0+nw) (blocked may be NULL): the */
/* samples of the stopping-rule estimates of E[I_G(s)] in Algorithm 4 and of */
/* E[I_{G[V\B]}(s)] in Algorithm 1.                                          */
int oracle_world_sizes(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                       const int32_t* seeds, int32_t n_seeds, const uint8_t* blocked, uint64_t rng_seed,
                       uint64_t w0, uint64_t nw, int nthreads, int32_t* rsize) {
    if (check_query(n, seeds, n_seeds, blocked)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* blk = calloc((size_t)n, 1);
    if (!blk) return -1;
    if (blocked) memcpy(blk, blocked, (size_t)n);
    int64_t total = 0;
    int st = run_eval(&q, blk, 0, 0, w0, nw, nthreads, NULL, &total, rsize, NULL);
    free(blk);
    return st;
}

/* Public: the marginal coverage of every node given B over the CP sequences */
/* of worlds [0, theta): marg[v] = Cov(B + v) - Cov(B) for v not in B (0 for */
/* seeds and for B), and *cov = Cov(B) (Section 4.1).                         */
int oracle_cover_marginals(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                           const int32_t* seeds, int32_t n_seeds, const int32_t* blockers, int32_t n_blockers,
                           uint64_t theta, uint64_t rng_seed, int nthreads, int64_t* marg, int64_t* cov) {
    if (theta < 1 || n_blockers < 0) return -1;
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > theta) nthreads = (int)theta;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, rng_seed};
    uint8_t* is_seed = calloc((size_t)n, 1);
    uint8_t* in_b = calloc((size_t)n, 1);
    if (!is_seed || !in_b) { free(is_seed); free(in_b); return -1; }
    for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
    int bad = 0;
    for (int32_t i = 0; i < n_blockers; ++i) {
        if (blockers[i] < 0 || blockers[i] >= n) bad = 1;
        else in_b[blockers[i]] = 1;
    }
    cov_job_t* jobs = bad ? NULL : cov_build(&q, is_seed, theta, nthreads, 1);
    if (!jobs) { free(is_seed); free(in_b); return -1; }
    for (int t = 0; t < nthreads; ++t) jobs[t].in_b = in_b;
    run_jobs(jobs, nthreads, cov_mark_job);
    *cov = 0;
    for (int t = 0; t < nthreads; ++t) *cov += jobs[t].count;
    run_jobs(jobs, nthreads, cov_marg_job);
    memset(marg, 0, (size_t)n * sizeof(int64_t));
    for (int t = 0; t < nthreads; ++t)
        for (int32_t v = 0; v < n; ++v) marg[v] += jobs[t].marg[v];
    for (int32_t v = 0; v < n; ++v)
        if (in_b[v]) marg[v] = 0;
    cov_free_jobs(jobs, nthreads);
    free(is_seed); free(in_b);
    return 0;
}


/* ======================================================================== */
/* Global Sampling (Section 4.2, Algorithm 3; Definition 4.3).              */
/*                                                                          */
/*   V'_s     the non-seed nodes reachable from S in G over edges that can   */
/*            be live (threshold > 0), ascending (the caller's vprime).      */
/*   sample i world i of the key; its target v = vprime[(r * |V'_s|) >> 32]  */
/*            with r = word 0 of Philox4x32-10 at counter (0, i, 1, 0) (the  */
/*            edge coins use counter word 2 = 0, so the draws never meet).   */
/*   LRR set  empty when v is not reached from S in world i; otherwise the  */
/*            nodes that reach v in phi^s, the live subgraph induced by the  */
/*            reached non-seeds (v included).                                */
/*   Cov      sets that meet B; |V'_s| Cov(B) / theta is unbiased for the    */
/*            upper bound D^U(B) (Lemma 4.4).                                */
/* ======================================================================== */

uint32_t oracle_lrr_pick(uint64_t key, uint64_t i, uint32_t nvp) {
    uint32_t ctr[4] = {0u, (uint32_t)i, 1u, 0u};
    uint32_t k[2] = {(uint32_t)key, (uint32_t)(key >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, k, out);
    return (uint32_t)(((uint64_t)out[0] * (uint64_t)nvp) >> 32);
}

/* The LRR set of sample w into out (capacity n); returns its size, -1 on  */
/* failure.                                                                 */
static int32_t world_lrr_set(const query_t* q, scratch_t* s, uint64_t w, const uint8_t* is_seed,
                             const int32_t* vprime, uint32_t nvp, int32_t* out) {
    if (nvp == 0) return 0;
    const int32_t v = vprime[oracle_lrr_pick(q->rng_seed, w, nvp)];
    int32_t R = reach(q, s, w);
    int32_t now = s->stamp_now;
    if (s->stamp[v] != now) return 0; /* v is not reached: the empty set */
    /* local ids 1..R over the reached nodes; the live edges of phi^s,      */
    /* stored reversed (head -> tail) as a CSR over local ids               */
    for (int32_t i = 0; i < R; ++i) s->local_of[s->queue[i]] = i + 1;
    int64_t ne = 0;
    for (int32_t i = 0; i < R; ++i) {
        int32_t u = s->queue[i];
        if (is_seed[u]) continue;
        for (int64_t e = q->row_ptr[u]; e < q->row_ptr[u + 1]; ++e) {
            int32_t x = q->col[e];
            if (x == u || is_seed[x] || s->stamp[x] != now) continue;
            if (!edge_live(q->thr[e], q->rng_seed, w, e)) continue;
            if (push_edge(s, &ne, s->local_of[x], i + 1)) return -1;
        }
    }
    int32_t N = R + 1;
    for (int32_t x = 0; x <= N; ++x) s->pred_off[x] = 0;
    for (int64_t i = 0; i < ne; ++i) s->pred_off[s->e_src[i] + 1]++;
    for (int32_t x = 0; x < N; ++x) s->pred_off[x + 1] += s->pred_off[x];
    for (int32_t x = 0; x < N; ++x) s->fill[x] = s->pred_off[x];
    for (int64_t i = 0; i < ne; ++i) s->pred[s->fill[s->e_src[i]]++] = s->e_dst[i];
    /* breadth-first search from v along the reversed edges */
    int32_t* seen = s->idom;
    for (int32_t x = 0; x < N; ++x) seen[x] = 0;
    int32_t head = 0, tail = 0;
    int32_t lv = s->local_of[v];
    seen[lv] = 1;
    s->stack[tail++] = lv;
    while (head < tail) {
        int32_t x = s->stack[head++];
        for (int32_t j = s->pred_off[x]; j < s->pred_off[x + 1]; ++j) {
            int32_t u = s->pred[j];
            if (!seen[u]) {
                seen[u] = 1;
                s->stack[tail++] = u;
            }
        }
    }
    for (int32_t i = 0; i < tail; ++i) out[i] = s->queue[s->stack[i] - 1];
    return tail;
}

/* Public: the LRR set of sample w (members in out, capacity n). */
int32_t oracle_lrr_set(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                       const int32_t* seeds, int32_t n_seeds, uint64_t key, uint64_t w, const int32_t* vprime,
                       uint32_t nvp, int32_t* out) {
    if (check_query(n, seeds, n_seeds, NULL)) return -1;
    query_t q = {n, m, row_ptr, col, thr, seeds, n_seeds, key};
    scratch_t s;
    if (scratch_init(&s, n, NULL)) return -1;
    uint8_t* is_seed = calloc((size_t)n, 1);
    int32_t r = -1;
    if (is_seed) {
        for (int32_t i = 0; i < n_seeds; ++i) is_seed[seeds[i]] = 1;
        r = world_lrr_set(&q, &s, w, is_seed, vprime, nvp, out);
        if (s.oom) r = -1;
    }
    free(is_seed);
    scratch_free(&s);
    return r;
}

/* Public: Max-Coverage over the LRR sets of samples [0, theta) (Section    */
/* 5.2: GSBM runs the procedure of Algorithm 4 on LRR sets).  Outputs as   */
/* oracle_max_coverage.                                                     */
int oracle_lrr_max_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                            const int32_t* seeds, int32_t n_seeds, const int32_t* vprime, uint32_t nvp, int32_t k,
                            uint64_t theta, uint64_t key, int nthreads, int32_t* blockers, int64_t* gains,
                            int64_t* cov, int64_t* cov_upper, int32_t* n_selected) {
    return max_coverage_sets(n, m, row_ptr, col, thr, seeds, n_seeds, k, theta, key, nthreads, 1, vprime, nvp,
                             blockers, gains, cov, cov_upper, n_selected);
}

/* Public: Cov(B) over the LRR sets of samples [0, theta). */
int oracle_lrr_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, const int32_t* vprime, uint32_t nvp,
                        const int32_t* blockers, int32_t n_blockers, uint64_t theta, uint64_t key, int nthreads,
                        int64_t* cov) {
    return coverage_sets(n, m, row_ptr, col, thr, seeds, n_seeds, blockers, n_blockers, theta, key, nthreads, 1,
                         vprime, nvp, cov);
}
