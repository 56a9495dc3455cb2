// Batches and serving on top of the enqueued solve (imin_solve with a
// workspace): many queries, on one or several resident graphs of a device,
// share a pool of device memory and a set of streams.
//
// A dispatcher admits a query when the workspace its layout needs
// (imin_solve_workspace_size, with the plain-rounds layout when the
// incremental one exceeds the pool) fits a free range of the pool, enqueues its
// whole solve on the least loaded stream and records an event after it; the
// query's device_status word lives in pinned host memory, so once the event
// has completed the dispatcher reads the outcome without a copy.  A query
// whose worlds turn out to need more scratch than its workspace held
// (IMIN_ERR_WORKSPACE on the device) raised its graph's record and is
// admitted again with the larger size.  Queries wait in arrival order; when
// the first waiting query does not fit, a few later ones that do may start
// before it.  Worlds are keyed by each query's own rng_seed, so a query's
// result does not depend on what runs beside it.
#include "imin.h"
#include "imin_internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace imin {
// imin_solve_workspace_size for workspaces carved from a pool of `limit`
// bytes: the incremental layout only when it fits that limit (imin_api.cpp)
imin_status_t solve_workspace_size_within(imin_graph_t g, int32_t n_seeds, int32_t k, int64_t theta, size_t limit,
                                          size_t* bytes);
}  // namespace imin

namespace {

constexpr int kMaxInFlight = 4096;    // status words in pinned memory
constexpr int kBackfill = 16;         // waiting queries looked at beyond the first
constexpr int kWorkspaceRetries = 4;  // re-admissions after IMIN_ERR_WORKSPACE

// With IMIN_DEBUG set in the environment, admission decisions are written
// to stderr.
bool debug_on() {
    static const bool on = std::getenv("IMIN_DEBUG") != nullptr;
    return on;
}

struct Engine {
    int device = -1;
    imin_graph_t default_graph = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_load;  // queries in flight per stream
    char* pool = nullptr;
    size_t pool_bytes = 0;
    std::map<size_t, size_t> free_ranges;  // offset -> bytes, coalesced
    int32_t* status_host = nullptr;        // [kMaxInFlight], pinned
    std::vector<int> free_slots;
    std::vector<hipEvent_t> events;        // idle events for reuse

    struct Flight {
        imin_query_t* q;
        int stream;
        size_t off, bytes;
        int slot;
        hipEvent_t ev;
    };
    struct Waiting {
        imin_query_t* q;
        int retries;
    };
    std::vector<Flight> flights;
    std::deque<Waiting> waiting;

    imin_status_t init(imin_graph_t g, void* const* st, int32_t n_streams, size_t budget) {
        default_graph = g;
        device = imin::graph_device(g);
        streams.assign((hipStream_t*)st, (hipStream_t*)st + n_streams);
        stream_load.assign((size_t)n_streams, 0);
        if (budget == 0) {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
                (void)hipGetLastError();
                return IMIN_ERR_DEVICE;
            }
            budget = std::min<size_t>(free_b / 2, (size_t)96 << 30);
        }
        budget &= ~(size_t)255;
        if (budget == 0) return IMIN_ERR_INVALID;
        if (hipMalloc((void**)&pool, budget) != hipSuccess) {
            (void)hipGetLastError();
            pool = nullptr;
            return IMIN_ERR_NOMEM;
        }
        pool_bytes = budget;
        free_ranges[0] = budget;
        if (hipHostMalloc((void**)&status_host, kMaxInFlight * sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            status_host = nullptr;
            return IMIN_ERR_NOMEM;
        }
        free_slots.reserve(kMaxInFlight);
        for (int i = kMaxInFlight - 1; i >= 0; --i) free_slots.push_back(i);
        return IMIN_OK;
    }

    ~Engine() {
        for (Flight& f : flights) (void)hipEventSynchronize(f.ev);
        for (Flight& f : flights) (void)hipEventDestroy(f.ev);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (pool) (void)hipFree(pool);
        if (status_host) (void)hipHostFree(status_host);
    }

    // first range of the pool that holds `bytes` (256-aligned offsets)
    bool take(size_t bytes, size_t& off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const size_t left = it->second - bytes;
            free_ranges.erase(it);
            if (left) free_ranges[off + bytes] = left;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_ranges.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_ranges.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_ranges.erase(next);
        }
        if (it != free_ranges.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_ranges.erase(it);
            }
        }
    }

    hipEvent_t event() {
        if (!events.empty()) {
            hipEvent_t e = events.back();
            events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }

    imin_graph_t graph_of(const imin_query_t* q) const { return q->graph ? q->graph : default_graph; }

    // Admit w if its workspace fits now: true when it left the waiting list
    // (started, or finished with an error found on the host).
    bool try_start(const Waiting& w, std::vector<imin_query_t*>& finished) {
        imin_query_t* q = w.q;
        imin_graph_t g = graph_of(q);
        auto fail = [&](imin_status_t st) {
            if (debug_on()) std::fprintf(stderr, "imin: query %p failed on the host with status %d\n", (void*)q, (int)st);
            q->status = (int32_t)st;
            q->device_flags = 0;
            finished.push_back(q);
            return true;
        };
        if (!g || imin::graph_device(g) != device) return fail(IMIN_ERR_INVALID);
        size_t bytes = 0;
        imin_status_t st = imin::solve_workspace_size_within(g, q->n_seeds, q->k, q->theta, pool_bytes, &bytes);
        if (st != IMIN_OK) return fail(st);
        if (bytes > pool_bytes) {
            if (debug_on())
                std::fprintf(stderr, "imin: query %p needs %zu workspace bytes, more than the pool's %zu\n", (void*)q,
                             bytes, pool_bytes);
            return fail(IMIN_ERR_WORKSPACE);  // can never fit
        }
        if (free_slots.empty()) return false;
        size_t off = 0;
        if (!take(bytes, off)) return false;
        int s = 0;
        for (int i = 1; i < (int)streams.size(); ++i)
            if (stream_load[(size_t)i] < stream_load[(size_t)s]) s = i;
        const int slot = free_slots.back();
        status_host[slot] = -1;
        hipEvent_t ev = event();
        if (!ev) {
            give(off, bytes);
            return fail(IMIN_ERR_DEVICE);
        }
        st = imin_solve(g, q->seeds, q->n_seeds, q->k, q->theta, q->rng_seed, pool + off, bytes, streams[(size_t)s],
                        q->blockers, q->gains, q->spread_totals, q->n_selected, status_host + slot);
        if (st == IMIN_OK && hipEventRecord(ev, streams[(size_t)s]) != hipSuccess) st = IMIN_ERR_DEVICE;
        if (st != IMIN_OK) {
            (void)hipGetLastError();
            // whatever was enqueued must finish before its range is reused
            (void)hipStreamSynchronize(streams[(size_t)s]);
            give(off, bytes);
            events.push_back(ev);
            return fail(st);
        }
        free_slots.pop_back();
        ++stream_load[(size_t)s];
        flights.push_back(Flight{q, s, off, bytes, slot, ev});
        return true;
    }

    // start what fits: the first waiting query, else one of the next few
    void admit(std::vector<imin_query_t*>& finished) {
        for (;;) {
            bool started = false;
            const size_t look = std::min<size_t>(waiting.size(), kBackfill + 1);
            for (size_t i = 0; i < look; ++i) {
                if (try_start(waiting[i], finished)) {
                    waiting.erase(waiting.begin() + (long)i);
                    started = true;
                    break;
                }
            }
            if (!started) return;
        }
    }

    // collect the queries whose solves have completed; true if any did
    bool poll(std::vector<imin_query_t*>& finished) {
        bool any = false;
        for (size_t i = 0; i < flights.size();) {
            Flight& f = flights[i];
            const hipError_t e = hipEventQuery(f.ev);
            if (e == hipErrorNotReady) {
                ++i;
                continue;
            }
            any = true;
            const int32_t code = (e == hipSuccess) ? status_host[f.slot] : (int32_t)IMIN_ERR_DEVICE;
            if (e != hipSuccess) (void)hipGetLastError();
            give(f.off, f.bytes);
            free_slots.push_back(f.slot);
            --stream_load[(size_t)f.stream];
            events.push_back(f.ev);
            imin_query_t* q = f.q;
            flights[i] = flights.back();
            flights.pop_back();
            if (debug_on())
                std::fprintf(stderr, "imin: query %p finished with status %d in a workspace of %zu bytes\n", (void*)q,
                             (int)code, f.bytes);
            if (code == (int32_t)IMIN_ERR_WORKSPACE && retries_of(q) < kWorkspaceRetries) {
                // the graph now records what its worlds need: admit it again
                retry_count[q] = retries_of(q) + 1;
                waiting.push_front(Waiting{q, retry_count[q]});
                continue;
            }
            retry_count.erase(q);
            q->status = code;
            q->device_flags = 0;
            finished.push_back(q);
        }
        return any;
    }
    std::map<imin_query_t*, int> retry_count;
    int retries_of(imin_query_t* q) const {
        auto it = retry_count.find(q);
        return it == retry_count.end() ? 0 : it->second;
    }

    bool idle() const { return flights.empty() && waiting.empty(); }

    // Right after admit(): with nothing in flight the whole pool was free,
    // so a first waiting query that did not start never will.
    void drop_unstartable(std::vector<imin_query_t*>& finished) {
        if (!flights.empty() || waiting.empty()) return;
        imin_query_t* q = waiting.front().q;
        waiting.pop_front();
        retry_count.erase(q);
        if (debug_on()) std::fprintf(stderr, "imin: query %p cannot start on an empty pool\n", (void*)q);
        q->status = (int32_t)IMIN_ERR_WORKSPACE;
        q->device_flags = 0;
        finished.push_back(q);
    }
};

}  // namespace

extern "C" {

imin_status_t imin_solve_many(imin_graph_t g, imin_query_t* queries, int32_t n_queries, void* const* streams,
                              int32_t n_streams, size_t hbm_budget) {
    if (!g || n_queries < 0 || (n_queries > 0 && !queries) || n_streams < 1 || !streams) return IMIN_ERR_INVALID;
    for (int32_t i = 0; i < n_streams; ++i)
        for (int32_t j = 0; j < i; ++j)
            if (streams[i] == streams[j]) return IMIN_ERR_INVALID;
    for (int32_t q = 0; q < n_queries; ++q) {
        queries[q].status = (int32_t)IMIN_ERR_INTERNAL;  // until the query has run
        queries[q].device_flags = 0;
    }
    if (n_queries == 0) return IMIN_OK;
    try {
        int prev = -1;
        (void)hipGetDevice(&prev);
        const int dev = imin::graph_device(g);
        if (prev != dev) (void)hipSetDevice(dev);
        imin_status_t st;
        {
            Engine eng;
            st = eng.init(g, streams, n_streams, hbm_budget);
            if (st == IMIN_OK) {
                // largest first (theta * (k + 1) bounds a query's work), so
                // that a long query does not start last and stretch the batch
                std::vector<int32_t> order((size_t)n_queries);
                for (int32_t q = 0; q < n_queries; ++q) order[(size_t)q] = q;
                std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                    const double wa = (double)queries[a].theta * ((double)queries[a].k + 1.0);
                    const double wb = (double)queries[b].theta * ((double)queries[b].k + 1.0);
                    return wa > wb;
                });
                for (int32_t i : order) eng.waiting.push_back(Engine::Waiting{&queries[i], 0});
                std::vector<imin_query_t*> finished;
                while (!eng.idle()) {
                    eng.admit(finished);
                    eng.drop_unstartable(finished);
                    if (!eng.poll(finished) && !eng.flights.empty())
                        std::this_thread::sleep_for(std::chrono::microseconds(50));
                }
            }
        }
        if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
        if (st != IMIN_OK) return st;
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
    for (int32_t q = 0; q < n_queries; ++q)
        if (queries[q].status != (int32_t)IMIN_OK) return (imin_status_t)queries[q].status;
    return IMIN_OK;
}

struct imin_server {
    Engine eng;
    std::thread dispatcher;
    std::mutex mu;
    std::condition_variable submitted_cv;  // a query was submitted, or the server stops
    std::condition_variable done_cv;       // a query finished
    std::deque<imin_query_t*> inbox;       // submitted, not yet seen by the dispatcher
    std::deque<imin_query_t*> done;        // finished, not yet returned
    int64_t outstanding = 0;               // submitted, not yet returned
    bool stopping = false;

    void run() {
        (void)hipSetDevice(eng.device);
        std::vector<imin_query_t*> finished;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                if (eng.idle()) submitted_cv.wait(lk, [&] { return stopping || !inbox.empty(); });
                while (!inbox.empty()) {
                    eng.waiting.push_back(Engine::Waiting{inbox.front(), 0});
                    inbox.pop_front();
                }
                if (stopping && eng.idle()) return;
            }
            eng.admit(finished);
            eng.drop_unstartable(finished);
            const bool progressed = eng.poll(finished);
            if (!finished.empty()) {
                {
                    std::lock_guard<std::mutex> lk(mu);
                    for (imin_query_t* q : finished) done.push_back(q);
                }
                finished.clear();
                done_cv.notify_all();
            } else if (!progressed && !eng.flights.empty()) {
                std::unique_lock<std::mutex> lk(mu);
                submitted_cv.wait_for(lk, std::chrono::microseconds(50), [&] { return !inbox.empty(); });
            }
        }
    }
};

imin_status_t imin_server_create(imin_graph_t g, void* const* streams, int32_t n_streams, size_t hbm_budget,
                                 imin_server_t* out) {
    if (!g || !streams || n_streams < 1 || !out) return IMIN_ERR_INVALID;
    for (int32_t i = 0; i < n_streams; ++i)
        for (int32_t j = 0; j < i; ++j)
            if (streams[i] == streams[j]) return IMIN_ERR_INVALID;
    *out = nullptr;
    imin_server* sv = new (std::nothrow) imin_server();
    if (!sv) return IMIN_ERR_NOMEM;
    imin_status_t st;
    try {
        st = sv->eng.init(g, streams, n_streams, hbm_budget);
        if (st == IMIN_OK) sv->dispatcher = std::thread([sv] { sv->run(); });
    } catch (...) {
        st = IMIN_ERR_NOMEM;
    }
    if (st != IMIN_OK) {
        delete sv;
        return st;
    }
    *out = sv;
    return IMIN_OK;
}

imin_status_t imin_server_submit(imin_server_t s, imin_query_t* query) {
    if (!s || !query) return IMIN_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return IMIN_ERR_INVALID;
        query->status = (int32_t)IMIN_ERR_INTERNAL;  // until it has run
        query->device_flags = 0;
        try {
            s->inbox.push_back(query);
        } catch (...) {
            return IMIN_ERR_NOMEM;
        }
        ++s->outstanding;
    }
    s->submitted_cv.notify_one();
    return IMIN_OK;
}

imin_status_t imin_server_next(imin_server_t s, imin_query_t** done) {
    if (!s || !done) return IMIN_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->outstanding == 0) return IMIN_ERR_INVALID;
    s->done_cv.wait(lk, [&] { return !s->done.empty(); });
    *done = s->done.front();
    s->done.pop_front();
    --s->outstanding;
    return IMIN_OK;
}

imin_status_t imin_server_destroy(imin_server_t s) {
    if (!s) return IMIN_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->submitted_cv.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    delete s;
    return IMIN_OK;
}

}  // extern "C"
