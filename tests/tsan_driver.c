/*
 * Drives the threaded entry points of the C oracle under ThreadSanitizer
 * (built with gcc -fsanitize=thread together with oracle/imin_oracle.c by
 * tests/test_oracle_tsan.py).  A small random graph, several threads per
 * call; exits 0 when every call succeeds.  The sanitizer reports any data
 * race on stderr.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_eval(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                const int32_t* seeds, int32_t n_seeds, const uint8_t* blocked, uint64_t rng_seed, uint64_t w0,
                uint64_t nw, int mode, int nthreads, int64_t* gain, int64_t* total, int32_t* rsize, int64_t* rsum);
int oracle_solve(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                 const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed, int mode,
                 int nthreads, int32_t* blockers, int64_t* gains, int64_t* totals, int32_t* n_selected);
int oracle_max_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, int32_t k, uint64_t theta, uint64_t rng_seed,
                        int nthreads, int32_t* blockers, int64_t* gains, int64_t* cov, int64_t* cov_upper,
                        int32_t* n_selected);
int oracle_coverage(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                    const int32_t* seeds, int32_t n_seeds, const int32_t* blockers, int32_t n_blockers,
                    uint64_t theta, uint64_t rng_seed, int nthreads, int64_t* cov);
int oracle_reach_counts(int32_t n, int64_t m, const int64_t* row_ptr, const int32_t* col, const uint32_t* thr,
                        const int32_t* seeds, int32_t n_seeds, uint64_t rng_seed, uint64_t w0, uint64_t nw,
                        int nthreads, int64_t* counts);

int main(void) {
    const int32_t n = 400;
    const int64_t m = 2400;
    int64_t* row_ptr = calloc((size_t)n + 1, sizeof(int64_t));
    int32_t* col = malloc((size_t)m * sizeof(int32_t));
    uint32_t* thr = malloc((size_t)m * sizeof(uint32_t));
    int64_t* gain = malloc((size_t)n * sizeof(int64_t));
    if (!row_ptr || !col || !thr || !gain) return 2;
    uint64_t x = 12345;
    for (int64_t e = 0; e < m; ++e) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        col[e] = (int32_t)((x >> 33) % (uint64_t)n);
        thr[e] = (uint32_t)(x >> 20) | 0x10000000u;
        row_ptr[(e * n) / m + 1] += 1;
    }
    for (int32_t v = 0; v < n; ++v) row_ptr[v + 1] += row_ptr[v];
    const int32_t seeds[3] = {1, 50, 300};
    int64_t total = 0;
    int32_t blockers[8], nsel = 0, set[4] = {7, 8, 9, 10};
    int64_t gains[8], totals[9], cov[9], cu[9], c = 0;
    int bad = 0;
    bad |= oracle_eval(n, m, row_ptr, col, thr, seeds, 3, NULL, 5, 0, 600, 0, 4, gain, &total, NULL, NULL);
    bad |= oracle_solve(n, m, row_ptr, col, thr, seeds, 3, 4, 300, 5, 0, 4, blockers, gains, totals, &nsel);
    bad |= oracle_max_coverage(n, m, row_ptr, col, thr, seeds, 3, 8, 500, 5, 4, blockers, gains, cov, cu, &nsel);
    bad |= oracle_coverage(n, m, row_ptr, col, thr, seeds, 3, set, 4, 500, 5, 4, &c);
    bad |= oracle_reach_counts(n, m, row_ptr, col, thr, seeds, 3, 5, 0, 700, 4, gain);
    printf("status %d total %lld selected %d coverage %lld\n", bad, (long long)total, nsel, (long long)c);
    free(row_ptr); free(col); free(thr); free(gain);
    return bad ? 1 : 0;
}
