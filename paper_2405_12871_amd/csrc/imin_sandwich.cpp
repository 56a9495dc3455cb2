// SandIMIN (Algorithm 1, Section 3.1) and its three solvers: LSBM (Algorithm
// 4, Section 5.1), GSBM (Section 5.2) and LHGA (Section 5.3).
//
// The drivers are host code: their decisions (the stopping rules' sample
// counts, the theta schedules, the ratio tests, the final choice) are a few
// scalars, while every world and every LRR set is drawn and reduced on the
// device by imin_reach_counts, imin_evaluate, imin_max_coverage,
// imin_coverage, imin_lrr_max_coverage and imin_lrr_coverage.
// Floating-point steps are written in the order the header states, in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "imin.h"
#include "imin_internal.hpp"

namespace {

constexpr uint64_t kPool2Xor = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSraXor = 0xC2B2AE3D27D4EB4Full;
constexpr uint64_t kLrr1Xor = 0x2545F4914F6CDD1Dull;
constexpr uint64_t kLrr2Xor = 0x9FB21C651E98DF25ull;
constexpr uint64_t kEvalXor = 0xD6E8FEB86659FD93ull;
constexpr double kE = 2.718281828459045;  // the double nearest e

#define SW_TRY_HIP(expr)                 \
    do {                                 \
        if ((expr) != hipSuccess) {      \
            (void)hipGetLastError();     \
            return IMIN_ERR_DEVICE;      \
        }                                \
    } while (0)
#define SW_TRY(expr)                      \
    do {                                  \
        const imin_status_t st_ = (expr); \
        if (st_ != IMIN_OK) return st_;   \
    } while (0)

// device buffer released on scope exit
template <class T>
struct DevBuf {
    T* p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) { return hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)); }
};

template <class T>
imin_status_t to_host(std::vector<T>& dst, const T* src, size_t count) {
    dst.resize(count);
    if (count && hipMemcpy(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return IMIN_ERR_DEVICE;
    }
    return IMIN_OK;
}

double ln_binom(int64_t N, int64_t k) {
    double s = 0.0;
    for (int64_t j = 1; j <= k; ++j) s += std::log((double)(N - k + j) / (double)j);
    return s;
}

// Upsilon_1 of the Stopping Rule Algorithm (Dagum, Karp, Luby, Ross):
// relative error eps, failure probability fail
double sra_upsilon1(double eps, double fail) {
    const double ups = 4.0 * (kE - 2.0) * std::log(2.0 / fail) / (eps * eps);
    return 1.0 + (1.0 + eps) * ups;
}

// What every solver of a query shares: the host seeds, ON, and the bound b.
struct Query {
    imin_graph_t g = nullptr;
    const imin::HostGraph* h = nullptr;
    const int32_t* seeds_dev = nullptr;
    int32_t n_seeds = 0;
    hipStream_t s = nullptr;
    std::vector<int32_t> seeds;
    std::vector<uint8_t> is_seed;
    std::vector<int32_t> on;  // ascending
    int64_t b = 0;            // |S| + |V'_s|
    std::vector<int32_t> vprime;
};

imin_status_t prepare(imin_graph_t g, const int32_t* seeds_dev, int32_t n_seeds, void* stream, Query& q) {
    q.g = g;
    q.seeds_dev = seeds_dev;
    q.n_seeds = n_seeds;
    q.s = (hipStream_t)stream;
    q.h = imin::graph_host(g);
    if (!q.h) return IMIN_ERR_DEVICE;
    const int32_t n = q.h->n;
    q.seeds.resize((size_t)n_seeds);
    SW_TRY_HIP(hipMemcpyAsync(q.seeds.data(), seeds_dev, (size_t)n_seeds * sizeof(int32_t), hipMemcpyDeviceToHost,
                              q.s));
    SW_TRY_HIP(hipStreamSynchronize(q.s));
    q.is_seed.assign((size_t)n, 0);
    for (int32_t v : q.seeds) {
        if (v < 0 || v >= n || q.is_seed[(size_t)v]) return IMIN_ERR_DATA;
        q.is_seed[(size_t)v] = 1;
    }
    std::vector<uint8_t> in_on((size_t)n, 0);
    for (int32_t u : q.seeds)
        for (int64_t e = q.h->row_ptr[(size_t)u]; e < q.h->row_ptr[(size_t)u + 1]; ++e) {
            const int32_t v = q.h->col[(size_t)e];
            if (q.h->thr[(size_t)e] != 0u && !q.is_seed[(size_t)v]) in_on[(size_t)v] = 1;
        }
    for (int32_t v = 0; v < n; ++v)
        if (in_on[(size_t)v]) q.on.push_back(v);
    q.vprime = imin::reachable_nonseeds(*q.h, q.seeds);
    q.b = (int64_t)q.seeds.size() + (int64_t)q.vprime.size();
    return IMIN_OK;
}

// The stopping-rule estimate of E[I_G(s)] (relative error beta, failure
// delta / 6) over the worlds of key_sra, and the reach counts of every node
// over the N worlds it drew.
struct Estimates {
    int64_t N = 0;
    double i_hat = 0.0;
    std::vector<int64_t> counts;
};

// One pass draws each batch's worlds once for both the sizes and the reach
// counts; the batch where the sum crosses the threshold is corrected to its
// first N - w0 worlds by drawing its shorter part again (the counts of
// disjoint world ranges add up).
imin_status_t spread_estimate(const Query& q, double beta, double delta, uint64_t key_sra, Estimates& est) {
    const double ups1 = sra_upsilon1(beta, delta / 6.0);
    const double need = (double)q.b * ups1;
    const int32_t n = q.h->n;
    DevBuf<int64_t> counts;
    DevBuf<int32_t> sizes;
    SW_TRY_HIP(counts.alloc((size_t)n));
    const int64_t kMaxBatch = (int64_t)1 << 22;
    SW_TRY_HIP(sizes.alloc((size_t)kMaxBatch));
    std::vector<int32_t> hs;
    std::vector<int64_t> hc;
    est.counts.assign((size_t)n, 0);
    auto add_counts = [&](int64_t sign) {
        const imin_status_t st = to_host(hc, counts.p, (size_t)n);
        if (st == IMIN_OK)
            for (size_t v = 0; v < (size_t)n; ++v) est.counts[v] += sign * hc[v];
        return st;
    };
    int64_t total = 0, w0 = 0, batch = 4096, N = 0;
    while (N == 0) {
        batch = std::min(batch, kMaxBatch);
        if (w0 + batch > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;  // world ids are 32-bit
        SW_TRY(imin_reach_counts(q.g, q.seeds_dev, q.n_seeds, w0, batch, key_sra, q.s, counts.p, sizes.p));
        SW_TRY(to_host(hs, sizes.p, (size_t)batch));
        for (int64_t i = 0; i < batch; ++i) {
            total += hs[(size_t)i];
            if ((double)total >= need) {
                N = w0 + i + 1;
                break;
            }
        }
        if (N == 0) {
            SW_TRY(add_counts(1));
        } else if (N - w0 <= w0 + batch - N) {
            // keep worlds [w0, N): draw them again
            SW_TRY(imin_reach_counts(q.g, q.seeds_dev, q.n_seeds, w0, N - w0, key_sra, q.s, counts.p, nullptr));
            SW_TRY(add_counts(1));
        } else {
            // drop worlds [N, w0 + batch) from the batch's counts
            SW_TRY(add_counts(1));
            if (w0 + batch > N) {
                SW_TRY(imin_reach_counts(q.g, q.seeds_dev, q.n_seeds, N, w0 + batch - N, key_sra, q.s, counts.p,
                                         nullptr));
                SW_TRY(add_counts(-1));
            }
        }
        w0 += batch;
        batch *= 2;
    }
    est.N = N;
    est.i_hat = (double)q.b * ups1 / (double)N;
    return IMIN_OK;
}

double opt_lower(const Query& q, const Estimates& est, int32_t k) {
    std::vector<int64_t> onc;
    onc.reserve(q.on.size());
    for (int32_t v : q.on) onc.push_back(est.counts[(size_t)v]);
    std::sort(onc.begin(), onc.end(), [](int64_t x, int64_t y) { return x > y; });
    int64_t top = 0;
    for (size_t i = 0; i < onc.size() && i < (size_t)k; ++i) top += onc[i];
    const double opt = (double)top / (double)est.N;
    return opt > 0.0 ? opt : 1.0 / (double)est.N;
}

imin_status_t return_on(const Query& q, int32_t* blockers, int32_t* n_selected) {
    const int32_t cnt = (int32_t)q.on.size();
    if (cnt > 0)
        SW_TRY_HIP(hipMemcpyAsync(blockers, q.on.data(), (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, q.s));
    SW_TRY_HIP(hipMemcpyAsync(n_selected, &cnt, sizeof(int32_t), hipMemcpyHostToDevice, q.s));
    SW_TRY_HIP(hipStreamSynchronize(q.s));
    return IMIN_OK;
}

// ------------------------------------------------------------------ LSBM
double lsbm_sigma_lower(int64_t cov2, int64_t theta2, double beta, double i_hat, double a1) {
    auto f = [&](double x) {
        const double d = std::sqrt(x + 2.0 * a1 / 9.0) - std::sqrt(a1 / 2.0);
        return (d * d - a1 / 18.0) / (double)theta2;
    };
    const double lo = (double)cov2 * (1.0 - beta) / i_hat;
    const double hi = (double)cov2 * (1.0 + beta) / i_hat;
    if (lo >= 5.0 * a1 / 18.0) return f(lo);
    if (hi <= 5.0 * a1 / 18.0) return f(hi);
    return 0.0;
}

double lsbm_sigma_upper(int64_t cov_u, int64_t theta1, double beta, double i_hat, double a2) {
    const double y = (double)cov_u * (1.0 + beta) / i_hat;
    const double d = std::sqrt(y + a2 / 2.0) + std::sqrt(a2 / 2.0);
    return d * d / (double)theta1;
}

// the doubling loop of Algorithm 4 (and GSBM): Max-Coverage on pool 1, the
// coverage of its answer on pool 2, the bounds and the ratio test
struct LoopOut {
    int32_t iterations = 0;
    int64_t theta = 0, cov1 = 0, cov2 = 0, cov_upper = 0;
    double sigma_l = 0.0, sigma_u = 0.0;
    int32_t n_selected = 0;
};

template <class MaxCov, class Cov, class Bounds>
imin_status_t doubling_loop(const Query& q, int32_t k, double eps, double theta_0, int32_t i_max, MaxCov max_cov,
                            Cov cov_of, Bounds bounds, int32_t* blockers, int32_t* n_selected, LoopOut& lo) {
    DevBuf<int64_t> gains, cov, cov_upper, cov2;
    DevBuf<int32_t> nsel;
    SW_TRY_HIP(gains.alloc((size_t)k));
    SW_TRY_HIP(cov.alloc((size_t)k + 1));
    SW_TRY_HIP(cov_upper.alloc((size_t)k + 1));
    SW_TRY_HIP(cov2.alloc(1));
    SW_TRY_HIP(nsel.alloc(1));
    const double target = 1.0 - 1.0 / kE - eps;
    int64_t theta = (int64_t)std::ceil(theta_0);
    for (int32_t i = 1; i <= i_max; ++i) {
        if (theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
        SW_TRY(max_cov(theta, blockers, gains.p, cov.p, cov_upper.p, nsel.p));
        int32_t r = 0;
        SW_TRY_HIP(hipMemcpy(&r, nsel.p, sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int64_t> hcov, hcu;
        SW_TRY(to_host(hcov, cov.p, (size_t)r + 1));
        SW_TRY(to_host(hcu, cov_upper.p, (size_t)r + 1));
        SW_TRY(cov_of(theta, blockers, r, cov2.p));
        int64_t c2 = 0;
        SW_TRY_HIP(hipMemcpy(&c2, cov2.p, sizeof(int64_t), hipMemcpyDeviceToHost));
        const int64_t cu = *std::min_element(hcu.begin(), hcu.end());
        double sl = 0.0, su = 1.0;
        bounds(c2, cu, theta, sl, su);
        lo.iterations = i;
        lo.theta = theta;
        lo.cov1 = hcov[(size_t)r];
        lo.cov2 = c2;
        lo.cov_upper = cu;
        lo.sigma_l = sl;
        lo.sigma_u = su;
        lo.n_selected = r;
        if (sl / su >= target || i == i_max) {
            SW_TRY_HIP(hipMemcpyAsync(n_selected, &r, sizeof(int32_t), hipMemcpyHostToDevice, q.s));
            SW_TRY_HIP(hipStreamSynchronize(q.s));
            return IMIN_OK;
        }
        theta *= 2;
    }
    return IMIN_ERR_INTERNAL;  // the last iteration returns
}

imin_status_t lsbm_core(const Query& q, const Estimates& est, int32_t k, double eps, double beta, double delta,
                        uint64_t rng_seed, int32_t* blockers, int32_t* n_selected, imin_lsbm_info_t& info) {
    const int32_t n = q.h->n;
    const double opt_l = opt_lower(q, est, k);
    const double i_hat = est.i_hat;
    info.reach_bound = q.b;
    info.sra_worlds = est.N;
    info.i_hat = i_hat;
    info.opt_l = opt_l;
    const double c = 1.0 - 1.0 / kE;
    const double l12 = std::log(12.0 / delta);
    const double root = c * std::sqrt(l12) + std::sqrt(c * (ln_binom((int64_t)n - q.n_seeds, k) + l12));
    const double theta_max = 2.0 * i_hat * root * root / ((1.0 - beta) * eps * eps * opt_l);
    const double theta_0 = theta_max * (1.0 - beta) * eps * eps * opt_l / i_hat;
    const int32_t i_max = std::max(1, (int32_t)std::ceil(std::log2(theta_max / theta_0)));
    const double a1 = std::log(3.0 * i_max / delta);
    info.theta_max = theta_max;
    info.theta_0 = theta_0;
    info.i_max = i_max;
    info.a1 = a1;
    const uint64_t key1 = rng_seed, key2 = rng_seed ^ kPool2Xor;
    auto max_cov = [&](int64_t theta, int32_t* bl, int64_t* gains, int64_t* cov, int64_t* cu, int32_t* ns) {
        return imin_max_coverage(q.g, q.seeds_dev, q.n_seeds, k, theta, key1, q.s, bl, gains, cov, cu, ns);
    };
    auto cov_of = [&](int64_t theta, const int32_t* bl, int32_t r, int64_t* out) {
        return imin_coverage(q.g, q.seeds_dev, q.n_seeds, bl, r, theta, key2, q.s, out);
    };
    auto bounds = [&](int64_t c2, int64_t cu, int64_t theta, double& sl, double& su) {
        sl = lsbm_sigma_lower(c2, theta, beta, i_hat, a1);
        su = lsbm_sigma_upper(cu, theta, beta, i_hat, a1);
    };
    LoopOut lo;
    SW_TRY(doubling_loop(q, k, eps, theta_0, i_max, max_cov, cov_of, bounds, blockers, n_selected, lo));
    info.iterations = lo.iterations;
    info.theta = lo.theta;
    info.cov1 = lo.cov1;
    info.cov2 = lo.cov2;
    info.cov_upper = lo.cov_upper;
    info.sigma_l = lo.sigma_l;
    info.sigma_u = lo.sigma_u;
    return IMIN_OK;
}

// ------------------------------------------------------------------ GSBM
imin_status_t gsbm_core(const Query& q, const Estimates& est, int32_t k, double eps, double delta, uint64_t rng_seed,
                        int32_t* blockers, int32_t* n_selected, imin_gsbm_info_t& info) {
    const int32_t n = q.h->n;
    const double nvp = (double)q.vprime.size();
    const double opt_l = opt_lower(q, est, k);
    info.nvp = (int64_t)q.vprime.size();
    info.sra_worlds = est.N;
    info.opt_l = opt_l;
    const double c = 1.0 - 1.0 / kE;
    const double l6 = std::log(6.0 / delta);
    const double root = c * std::sqrt(l6) + std::sqrt(c * (ln_binom((int64_t)n - q.n_seeds, k) + l6));
    const double theta_max = 2.0 * nvp * root * root / (eps * eps * opt_l);
    const double theta_0 = theta_max * eps * eps * opt_l / nvp;
    const int32_t i_max = std::max(1, (int32_t)std::ceil(std::log2(theta_max / theta_0)));
    const double a1 = std::log(3.0 * i_max / delta);
    info.theta_max = theta_max;
    info.theta_0 = theta_0;
    info.i_max = i_max;
    info.a1 = a1;
    const uint64_t key1 = rng_seed ^ kLrr1Xor, key2 = rng_seed ^ kLrr2Xor;
    auto max_cov = [&](int64_t theta, int32_t* bl, int64_t* gains, int64_t* cov, int64_t* cu, int32_t* ns) {
        return imin_lrr_max_coverage(q.g, q.seeds_dev, q.n_seeds, k, theta, key1, q.s, bl, gains, cov, cu, ns);
    };
    auto cov_of = [&](int64_t theta, const int32_t* bl, int32_t r, int64_t* out) {
        return imin_lrr_coverage(q.g, q.seeds_dev, q.n_seeds, bl, r, theta, key2, q.s, out);
    };
    auto bounds = [&](int64_t c2, int64_t cu, int64_t theta, double& sl, double& su) {
        const double dl = std::sqrt((double)c2 + 2.0 * a1 / 9.0) - std::sqrt(a1 / 2.0);
        sl = (dl * dl - a1 / 18.0) * nvp / (double)theta;
        const double du = std::sqrt((double)cu + a1 / 2.0) + std::sqrt(a1 / 2.0);
        su = du * du * nvp / (double)theta;
    };
    LoopOut lo;
    SW_TRY(doubling_loop(q, k, eps, theta_0, i_max, max_cov, cov_of, bounds, blockers, n_selected, lo));
    info.iterations = lo.iterations;
    info.theta = lo.theta;
    info.cov1 = lo.cov1;
    info.cov2 = lo.cov2;
    info.cov_upper = lo.cov_upper;
    info.sigma_l = lo.sigma_l;
    info.sigma_u = lo.sigma_u;
    return IMIN_OK;
}

// ------------------------------------------------------------------ LHGA
std::vector<int32_t> lhga_core(const Query& q, const Estimates& est, int32_t k) {
    std::vector<int32_t> order(q.on);
    auto score = [&](int32_t v) {
        const int64_t deg = q.h->row_ptr[(size_t)v + 1] - q.h->row_ptr[(size_t)v];
        return est.counts[(size_t)v] * deg;
    };
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int64_t sa = score(a), sb = score(b);
        return sa > sb || (sa == sb && a < b);
    });
    if ((int64_t)order.size() > (int64_t)k) order.resize((size_t)k);
    return order;
}

// ------------------------------------------------------------- SandIMIN
// (gamma, delta) estimate of E[I_{G[V \ B]}(s)]: the Stopping Rule Algorithm
// on |R_w(B)| / b over the worlds of key
imin_status_t blocked_spread(const Query& q, const int32_t* blocked_dev, int32_t nb, double gamma, double delta,
                             uint64_t key, double& estimate, int64_t& N_out) {
    const double ups1 = sra_upsilon1(gamma, delta);
    const double need = (double)q.b * ups1;
    const int64_t kMaxBatch = (int64_t)1 << 22;
    DevBuf<int32_t> sizes;
    SW_TRY_HIP(sizes.alloc((size_t)kMaxBatch));
    std::vector<int32_t> hs;
    int64_t total = 0, w0 = 0, batch = 4096, N = 0;
    while (N == 0) {
        batch = std::min(batch, kMaxBatch);
        if (w0 + batch > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;
        SW_TRY(imin_world_sizes(q.g, q.seeds_dev, q.n_seeds, blocked_dev, nb, w0, batch, key, q.s, sizes.p));
        SW_TRY(to_host(hs, sizes.p, (size_t)batch));
        for (int64_t i = 0; i < batch; ++i) {
            total += hs[(size_t)i];
            if ((double)total >= need) {
                N = w0 + i + 1;
                break;
            }
        }
        w0 += batch;
        batch *= 2;
    }
    estimate = (double)q.b * ups1 / (double)N;
    N_out = N;
    return IMIN_OK;
}

bool valid_params(int32_t k, double eps, double beta, double delta) {
    return k >= 1 && eps > 0.0 && eps < 1.0 && beta >= 0.0 && beta < 1.0 && delta > 0.0 && delta < 1.0;
}

imin_status_t lsbm_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps, double beta,
                        double delta, uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected,
                        imin_lsbm_info_t* info_out) {
    if (!g || !seeds || !blockers || !n_selected || !valid_params(k, eps, beta, delta)) return IMIN_ERR_INVALID;
    int32_t n = 0;
    SW_TRY(imin_graph_info(g, &n, nullptr));
    if (n_seeds < 1 || n_seeds > n || k > n) return IMIN_ERR_INVALID;
    Query q;
    SW_TRY(prepare(g, seeds, n_seeds, stream, q));
    imin_lsbm_info_t info{};
    info.on_size = (int32_t)q.on.size();
    if ((int64_t)q.on.size() <= (int64_t)k) {
        info.returned_on = 1;
        SW_TRY(return_on(q, blockers, n_selected));
    } else {
        Estimates est;
        SW_TRY(spread_estimate(q, beta, delta, rng_seed ^ kSraXor, est));
        SW_TRY(lsbm_core(q, est, k, eps, beta, delta, rng_seed, blockers, n_selected, info));
    }
    if (info_out) *info_out = info;
    return IMIN_OK;
}

imin_status_t gsbm_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps, double beta,
                        double delta, uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected,
                        imin_gsbm_info_t* info_out) {
    if (!g || !seeds || !blockers || !n_selected || !valid_params(k, eps, beta, delta)) return IMIN_ERR_INVALID;
    int32_t n = 0;
    SW_TRY(imin_graph_info(g, &n, nullptr));
    if (n_seeds < 1 || n_seeds > n || k > n) return IMIN_ERR_INVALID;
    Query q;
    SW_TRY(prepare(g, seeds, n_seeds, stream, q));
    imin_gsbm_info_t info{};
    info.on_size = (int32_t)q.on.size();
    if ((int64_t)q.on.size() <= (int64_t)k) {
        info.returned_on = 1;
        SW_TRY(return_on(q, blockers, n_selected));
    } else {
        Estimates est;
        SW_TRY(spread_estimate(q, beta, delta, rng_seed ^ kSraXor, est));
        SW_TRY(gsbm_core(q, est, k, eps, delta, rng_seed, blockers, n_selected, info));
    }
    if (info_out) *info_out = info;
    return IMIN_OK;
}

imin_status_t lhga_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double beta, double delta,
                        uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected) {
    if (!g || !seeds || !blockers || !n_selected || !valid_params(k, 0.5, beta, delta)) return IMIN_ERR_INVALID;
    int32_t n = 0;
    SW_TRY(imin_graph_info(g, &n, nullptr));
    if (n_seeds < 1 || n_seeds > n || k > n) return IMIN_ERR_INVALID;
    Query q;
    SW_TRY(prepare(g, seeds, n_seeds, stream, q));
    if ((int64_t)q.on.size() <= (int64_t)k) return return_on(q, blockers, n_selected);
    Estimates est;
    SW_TRY(spread_estimate(q, beta, delta, rng_seed ^ kSraXor, est));
    const std::vector<int32_t> br = lhga_core(q, est, k);
    const int32_t cnt = (int32_t)br.size();
    SW_TRY_HIP(hipMemcpyAsync(blockers, br.data(), (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, q.s));
    SW_TRY_HIP(hipMemcpyAsync(n_selected, &cnt, sizeof(int32_t), hipMemcpyHostToDevice, q.s));
    SW_TRY_HIP(hipStreamSynchronize(q.s));
    return IMIN_OK;
}

imin_status_t sandimin_impl(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps,
                            double beta, double gamma, double delta, uint64_t rng_seed, void* stream,
                            int32_t* blockers, int32_t* n_selected, int32_t* candidates,
                            imin_sandimin_info_t* info_out) {
    if (!g || !seeds || !blockers || !n_selected || !valid_params(k, eps, beta, delta) || !(gamma > 0.0 && gamma < 1.0))
        return IMIN_ERR_INVALID;
    int32_t n = 0;
    SW_TRY(imin_graph_info(g, &n, nullptr));
    if (n_seeds < 1 || n_seeds > n || k > n) return IMIN_ERR_INVALID;
    Query q;
    SW_TRY(prepare(g, seeds, n_seeds, stream, q));
    imin_sandimin_info_t info{};
    DevBuf<int32_t> cand, nsel;
    SW_TRY_HIP(cand.alloc((size_t)3 * k));
    SW_TRY_HIP(nsel.alloc(3));
    int32_t counts[3] = {0, 0, 0};
    if ((int64_t)q.on.size() <= (int64_t)k) {
        // every solver returns ON
        info.lsbm.returned_on = info.gsbm.returned_on = 1;
        info.lsbm.on_size = info.gsbm.on_size = (int32_t)q.on.size();
        for (int c = 0; c < 3; ++c) {
            SW_TRY(return_on(q, cand.p + (size_t)c * k, nsel.p + c));
            counts[c] = (int32_t)q.on.size();
        }
    } else {
        Estimates est;
        SW_TRY(spread_estimate(q, beta, delta, rng_seed ^ kSraXor, est));
        info.lsbm.on_size = info.gsbm.on_size = (int32_t)q.on.size();
        SW_TRY(lsbm_core(q, est, k, eps, beta, delta, rng_seed, cand.p, nsel.p, info.lsbm));
        SW_TRY(gsbm_core(q, est, k, eps, delta, rng_seed, cand.p + k, nsel.p + 1, info.gsbm));
        const std::vector<int32_t> br = lhga_core(q, est, k);
        const int32_t cnt = (int32_t)br.size();
        SW_TRY_HIP(hipMemcpy(cand.p + 2 * (size_t)k, br.data(), (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice));
        SW_TRY_HIP(hipMemcpy(nsel.p + 2, &cnt, sizeof(int32_t), hipMemcpyHostToDevice));
        SW_TRY_HIP(hipMemcpy(counts, nsel.p, 3 * sizeof(int32_t), hipMemcpyDeviceToHost));
    }
    const uint64_t key_eval = rng_seed ^ kEvalXor;
    int best = 0;
    for (int c = 0; c < 3; ++c) {
        double e = 0.0;
        int64_t N = 0;
        SW_TRY(blocked_spread(q, cand.p + (size_t)c * k, counts[c], gamma, delta, key_eval, e, N));
        info.estimate[c] = e;
        info.eval_worlds[c] = N;
        info.n_blockers[c] = counts[c];
        if (e < info.estimate[best]) best = c;  // ties keep the earlier of L, U, R
    }
    info.choice = best;
    SW_TRY_HIP(hipMemcpyAsync(blockers, cand.p + (size_t)best * k, (size_t)counts[best] * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, q.s));
    SW_TRY_HIP(hipMemcpyAsync(n_selected, &counts[best], sizeof(int32_t), hipMemcpyHostToDevice, q.s));
    if (candidates)
        SW_TRY_HIP(hipMemcpyAsync(candidates, cand.p, (size_t)3 * k * sizeof(int32_t), hipMemcpyDeviceToDevice, q.s));
    SW_TRY_HIP(hipStreamSynchronize(q.s));
    if (info_out) *info_out = info;
    return IMIN_OK;
}

template <class F>
imin_status_t guarded(F f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}

}  // namespace

extern "C" {

imin_status_t imin_lsbm(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps, double beta,
                        double delta, uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected,
                        imin_lsbm_info_t* info) {
    return guarded([&] {
        return lsbm_impl(g, seeds, n_seeds, k, eps, beta, delta, rng_seed, stream, blockers, n_selected, info);
    });
}

imin_status_t imin_gsbm(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps, double beta,
                        double delta, uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected,
                        imin_gsbm_info_t* info) {
    return guarded([&] {
        return gsbm_impl(g, seeds, n_seeds, k, eps, beta, delta, rng_seed, stream, blockers, n_selected, info);
    });
}

imin_status_t imin_lhga(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double beta, double delta,
                        uint64_t rng_seed, void* stream, int32_t* blockers, int32_t* n_selected) {
    return guarded([&] { return lhga_impl(g, seeds, n_seeds, k, beta, delta, rng_seed, stream, blockers, n_selected); });
}

imin_status_t imin_sandimin(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps, double beta,
                            double gamma, double delta, uint64_t rng_seed, void* stream, int32_t* blockers,
                            int32_t* n_selected, int32_t* candidates, imin_sandimin_info_t* info) {
    return guarded([&] {
        return sandimin_impl(g, seeds, n_seeds, k, eps, beta, gamma, delta, rng_seed, stream, blockers, n_selected,
                             candidates, info);
    });
}

}  // extern "C"
