/* Column-support sampler for the synthetic CSR inputs.
 *
 * Draws, for every row, a set of k_i DISTINCT columns whose ranks follow a
 * given discrete law (Zipf, or uniform), by successive sampling: i.i.d. draws
 * from the law, keeping the first k_i distinct values in draw order.  That is
 * exactly weighted sampling without replacement.  Ranks map to columns through
 * a caller-supplied permutation, and each row's columns are returned sorted
 * ascending (canonical CSR).
 *
 * This file only builds inputs; it holds none of the optimisation method's
 * arithmetic.  Each row draws from its own counter-based stream
 * (SplitMix64, Steele, Lea & Flood 2014, keyed by the row's seed), so the
 * output does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* smallest r with cdf[r] > u (cdf nondecreasing, cdf[m-1] == 1) */
static inline int64_t inv_cdf(const double* cdf, int64_t m, double u) {
    int64_t lo = 0, hi = m - 1;
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    return lo;
}

static void sort_i32(int32_t* a, int64_t k) {
    for (int64_t i = 1; i < k; ++i) {
        int32_t v = a[i];
        int64_t j = i - 1;
        while (j >= 0 && a[j] > v) { a[j + 1] = a[j]; --j; }
        a[j + 1] = v;
    }
}

/* Returns 0 on success, -1 if a row asks for more distinct columns than the
 * law's support can give, -2 on allocation failure. */
int datagen_distinct_rows(const uint64_t* row_seed, int64_t n, int64_t d,
                          const double* cdf, const int32_t* perm,
                          const int64_t* rowptr, int32_t* colidx) {
    int err = 0;
#pragma omp parallel
    {
        uint8_t* seen = (uint8_t*)calloc((size_t)d, 1);
        if (!seen) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            if (!seen) continue;
            int64_t k = rowptr[i + 1] - rowptr[i];
            if (k > d) {
#pragma omp atomic write
                err = -1;
                continue;
            }
            int32_t* out = colidx + rowptr[i];
            int64_t got = 0;
            uint64_t ctr = 0;
            while (got < k) {
                uint64_t r = mix64(row_seed[i] + (++ctr) * 0x9E3779B97F4A7C15ULL);
                double u = (double)(r >> 11) * 0x1.0p-53;
                int32_t c = perm[inv_cdf(cdf, d, u)];
                if (!seen[c]) { seen[c] = 1; out[got++] = c; }
            }
            for (int64_t j = 0; j < k; ++j) seen[out[j]] = 0;
            sort_i32(out, k);
        }
        free(seen);
    }
    return err;
}
