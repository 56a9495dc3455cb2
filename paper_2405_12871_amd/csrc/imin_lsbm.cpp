// LSBM (Algorithm 4, Section 5.1) on the library's coverage primitives.
//
// The driver is host code: its decisions (the stopping rule's N, the theta
// schedule, the ratio test) are a few scalars per iteration, while every
// world is drawn and reduced on the device by imin_reach_counts,
// imin_max_coverage and imin_coverage.  Floating-point steps are written in
// the order the header states, in double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "imin.h"

namespace {

constexpr uint64_t kPool2Xor = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSraXor = 0xC2B2AE3D27D4EB4Full;
constexpr double kE = 2.718281828459045;  // the double nearest e

#define LSBM_TRY_HIP(expr)                                          \
    do {                                                            \
        if ((expr) != hipSuccess) {                                 \
            (void)hipGetLastError();                                \
            return IMIN_ERR_DEVICE;                                 \
        }                                                           \
    } while (0)
#define LSBM_TRY(expr)                        \
    do {                                      \
        const imin_status_t st_ = (expr);     \
        if (st_ != IMIN_OK) return st_;       \
    } while (0)

// device buffer released on scope exit
template <class T>
struct DevBuf {
    T* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) { return hipMalloc((void**)&p, std::max<size_t>(count, 1) * sizeof(T)); }
};

// The graph as the host sees it: CSR offsets, heads and thresholds.
struct HostGraph {
    int32_t n = 0;
    int64_t m = 0;
    std::vector<int64_t> row_ptr;
    std::vector<int32_t> col;
    std::vector<uint32_t> thr;
};

double ln_binom(int64_t N, int64_t k) {
    double s = 0.0;
    for (int64_t j = 1; j <= k; ++j) s += std::log((double)(N - k + j) / (double)j);
    return s;
}

// nodes reachable from S over edges that can be live (threshold > 0)
int64_t reach_bound(const HostGraph& h, const std::vector<int32_t>& seeds) {
    std::vector<uint8_t> seen((size_t)h.n, 0);
    std::vector<int32_t> queue;
    queue.reserve(seeds.size());
    for (int32_t v : seeds)
        if (!seen[(size_t)v]) {
            seen[(size_t)v] = 1;
            queue.push_back(v);
        }
    for (size_t head = 0; head < queue.size(); ++head) {
        const int32_t u = queue[head];
        for (int64_t e = h.row_ptr[(size_t)u]; e < h.row_ptr[(size_t)u + 1]; ++e) {
            const int32_t v = h.col[(size_t)e];
            if (h.thr[(size_t)e] == 0u || seen[(size_t)v]) continue;
            seen[(size_t)v] = 1;
            queue.push_back(v);
        }
    }
    return (int64_t)queue.size();
}

double sigma_lower(int64_t cov2, int64_t theta2, double beta, double i_hat, double a1) {
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

double sigma_upper(int64_t cov_u, int64_t theta1, double beta, double i_hat, double a2) {
    const double y = (double)cov_u * (1.0 + beta) / i_hat;
    const double d = std::sqrt(y + a2 / 2.0) + std::sqrt(a2 / 2.0);
    return d * d / (double)theta1;
}

imin_status_t lsbm_impl(imin_graph_t g, const int32_t* seeds_dev, int32_t n_seeds, int32_t k, double eps,
                        double beta, double delta, uint64_t rng_seed, void* stream, int32_t* blockers,
                        int32_t* n_selected, imin_lsbm_info_t* info_out) {
    if (!g || !seeds_dev || !blockers || !n_selected) return IMIN_ERR_INVALID;
    if (!(eps > 0.0 && eps < 1.0) || !(beta >= 0.0 && beta < 1.0) || !(delta > 0.0 && delta < 1.0) || k < 1)
        return IMIN_ERR_INVALID;
    int32_t n = 0;
    int64_t m = 0;
    LSBM_TRY(imin_graph_info(g, &n, &m));
    if (n_seeds < 1 || n_seeds > n || k > n) return IMIN_ERR_INVALID;
    const hipStream_t s = (hipStream_t)stream;
    imin_lsbm_info_t info{};

    HostGraph h;
    h.n = n;
    h.m = m;
    h.row_ptr.resize((size_t)n + 1);
    h.col.resize((size_t)std::max<int64_t>(m, 1));
    h.thr.resize((size_t)std::max<int64_t>(m, 1));
    LSBM_TRY(imin_graph_export(g, h.row_ptr.data(), h.col.data(), h.thr.data()));
    std::vector<int32_t> seeds((size_t)n_seeds);
    LSBM_TRY_HIP(hipMemcpyAsync(seeds.data(), seeds_dev, (size_t)n_seeds * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LSBM_TRY_HIP(hipStreamSynchronize(s));
    std::vector<uint8_t> is_seed((size_t)n, 0);
    for (int32_t v : seeds) {
        if (v < 0 || v >= n || is_seed[(size_t)v]) return IMIN_ERR_DATA;
        is_seed[(size_t)v] = 1;
    }

    // 1. ON
    std::vector<int32_t> on;
    {
        std::vector<uint8_t> in_on((size_t)n, 0);
        for (int32_t u : seeds)
            for (int64_t e = h.row_ptr[(size_t)u]; e < h.row_ptr[(size_t)u + 1]; ++e) {
                const int32_t v = h.col[(size_t)e];
                if (h.thr[(size_t)e] != 0u && !is_seed[(size_t)v]) in_on[(size_t)v] = 1;
            }
        for (int32_t v = 0; v < n; ++v)
            if (in_on[(size_t)v]) on.push_back(v);
    }
    info.on_size = (int32_t)on.size();
    if ((int64_t)on.size() <= (int64_t)k) {
        const int32_t cnt = (int32_t)on.size();
        if (cnt > 0)
            LSBM_TRY_HIP(hipMemcpyAsync(blockers, on.data(), (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, s));
        LSBM_TRY_HIP(hipMemcpyAsync(n_selected, &cnt, sizeof(int32_t), hipMemcpyHostToDevice, s));
        LSBM_TRY_HIP(hipStreamSynchronize(s));
        info.returned_on = 1;
        if (info_out) *info_out = info;
        return IMIN_OK;
    }

    const uint64_t key1 = rng_seed, key2 = rng_seed ^ kPool2Xor, key_sra = rng_seed ^ kSraXor;
    DevBuf<int64_t> counts;
    LSBM_TRY_HIP(counts.alloc((size_t)n));

    // 2. the stopping rule on |R_w| / b
    const int64_t b = reach_bound(h, seeds);
    info.reach_bound = b;
    const double ups = 4.0 * (kE - 2.0) * std::log(2.0 / (delta / 6.0)) / (beta * beta);
    const double ups1 = 1.0 + (1.0 + beta) * ups;
    const double need = (double)b * ups1;
    int64_t N = 0;
    {
        int64_t total = 0, w0 = 0, batch = 4096;
        DevBuf<int32_t> sizes;
        std::vector<int32_t> hs;
        while (N == 0) {
            if (w0 + batch > ((int64_t)1 << 32)) return IMIN_ERR_INVALID;  // world ids are 32-bit
            LSBM_TRY_HIP(sizes.p ? hipSuccess : sizes.alloc((size_t)1 << 22));
            batch = std::min<int64_t>(batch, (int64_t)1 << 22);
            LSBM_TRY(imin_reach_counts(g, seeds_dev, n_seeds, w0, batch, key_sra, stream, counts.p, sizes.p));
            hs.resize((size_t)batch);
            LSBM_TRY_HIP(hipMemcpy(hs.data(), sizes.p, (size_t)batch * sizeof(int32_t), hipMemcpyDeviceToHost));
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
    }
    info.sra_worlds = N;
    const double i_hat = (double)b * ups1 / (double)N;
    info.i_hat = i_hat;

    // 3. OPT^L from the reach counts of ON over the same N worlds
    LSBM_TRY(imin_reach_counts(g, seeds_dev, n_seeds, 0, N, key_sra, stream, counts.p, nullptr));
    std::vector<int64_t> hc((size_t)n);
    LSBM_TRY_HIP(hipMemcpy(hc.data(), counts.p, (size_t)n * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<int64_t> onc;
    onc.reserve(on.size());
    for (int32_t v : on) onc.push_back(hc[(size_t)v]);
    std::sort(onc.begin(), onc.end(), [](int64_t x, int64_t y) { return x > y; });
    int64_t top = 0;
    for (size_t i = 0; i < onc.size() && i < (size_t)k; ++i) top += onc[i];
    double opt_l = (double)top / (double)N;
    if (opt_l <= 0.0) opt_l = 1.0 / (double)N;
    info.opt_l = opt_l;

    // 4. the theta schedule
    const double c = 1.0 - 1.0 / kE;
    const double l12 = std::log(12.0 / delta);
    const double root = c * std::sqrt(l12) + std::sqrt(c * (ln_binom((int64_t)n - n_seeds, k) + l12));
    const double theta_max = 2.0 * i_hat * root * root / ((1.0 - beta) * eps * eps * opt_l);
    const double theta_0 = theta_max * (1.0 - beta) * eps * eps * opt_l / i_hat;
    const int32_t i_max = std::max(1, (int32_t)std::ceil(std::log2(theta_max / theta_0)));
    const double a1 = std::log(3.0 * i_max / delta);
    const double a2 = a1;
    info.theta_max = theta_max;
    info.theta_0 = theta_0;
    info.i_max = i_max;
    info.a1 = a1;
    const double target = 1.0 - 1.0 / kE - eps;

    // 5. the doubling loop
    DevBuf<int64_t> gains, cov, cov_upper, cov2;
    DevBuf<int32_t> nsel;
    LSBM_TRY_HIP(gains.alloc((size_t)k));
    LSBM_TRY_HIP(cov.alloc((size_t)k + 1));
    LSBM_TRY_HIP(cov_upper.alloc((size_t)k + 1));
    LSBM_TRY_HIP(cov2.alloc(1));
    LSBM_TRY_HIP(nsel.alloc(1));
    int64_t theta = (int64_t)std::ceil(theta_0);
    for (int32_t i = 1; i <= i_max; ++i) {
        if (theta > (int64_t)0xFFFFFFFFll) return IMIN_ERR_INVALID;
        LSBM_TRY(imin_max_coverage(g, seeds_dev, n_seeds, k, theta, key1, stream, blockers, gains.p, cov.p,
                                   cov_upper.p, nsel.p));
        int32_t r = 0;
        LSBM_TRY_HIP(hipMemcpy(&r, nsel.p, sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int64_t> hcov((size_t)r + 1), hcu((size_t)r + 1);
        LSBM_TRY_HIP(hipMemcpy(hcov.data(), cov.p, hcov.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        LSBM_TRY_HIP(hipMemcpy(hcu.data(), cov_upper.p, hcu.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        LSBM_TRY(imin_coverage(g, seeds_dev, n_seeds, blockers, r, theta, key2, stream, cov2.p));
        int64_t c2 = 0;
        LSBM_TRY_HIP(hipMemcpy(&c2, cov2.p, sizeof(int64_t), hipMemcpyDeviceToHost));
        const int64_t cu = *std::min_element(hcu.begin(), hcu.end());
        const double sl = sigma_lower(c2, theta, beta, i_hat, a1);
        const double su = sigma_upper(cu, theta, beta, i_hat, a2);
        info.iterations = i;
        info.theta = theta;
        info.cov1 = hcov[(size_t)r];
        info.cov2 = c2;
        info.cov_upper = cu;
        info.sigma_l = sl;
        info.sigma_u = su;
        if (sl / su >= target || i == i_max) {
            LSBM_TRY_HIP(hipMemcpyAsync(n_selected, &r, sizeof(int32_t), hipMemcpyHostToDevice, s));
            LSBM_TRY_HIP(hipStreamSynchronize(s));
            if (info_out) *info_out = info;
            return IMIN_OK;
        }
        theta *= 2;
    }
    return IMIN_ERR_INTERNAL;  // the last iteration returns
}

}  // namespace

extern "C" imin_status_t imin_lsbm(imin_graph_t g, const int32_t* seeds, int32_t n_seeds, int32_t k, double eps,
                                   double beta, double delta, uint64_t rng_seed, void* stream, int32_t* blockers,
                                   int32_t* n_selected, imin_lsbm_info_t* info) {
    try {
        return lsbm_impl(g, seeds, n_seeds, k, eps, beta, delta, rng_seed, stream, blockers, n_selected, info);
    } catch (const std::bad_alloc&) {
        return IMIN_ERR_NOMEM;
    } catch (...) {
        return IMIN_ERR_INTERNAL;
    }
}
