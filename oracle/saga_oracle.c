/* Sequential Sparse SAGA oracle -- plain C, FP64, one thread.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this code.  It shares no
 * code, header or table with the HIP library it checks.
 *
 * What it computes (paper: Leblond, Pedregosa & Lacoste-Julien, "ASAGA:
 * Asynchronous Parallel SAGA", AISTATS 2017):
 *
 *   problem   min_x f(x) = (1/n) sum_i f_i(x)                (Section 1, Eq. finiteSum)
 *             f_i(x) = phi(a_i . x; b_i) + (lambda/2) ||x||^2
 *             logistic phi(z; b) = log(1 + exp(-b z))         (Section 4.1, "Models")
 *             squared  phi(z; b) = (z - b)^2 / 2              (least squares; not in the
 *                                                              paper, reading of the ridge
 *                                                              closed form (A'A/n+lI)^-1 A'b/n)
 *   memory    alpha_i is one scalar per sample, the last phi' seen for row i,
 *             so f'_i - alpha_i = (phi'(a_i.x) - alpha_i) a_i  (Section 2 footnote on
 *                                                              linear models; App. G)
 *   update    x+ = x - gamma (f'_i(x) - alpha_i + D_i abar + lambda D_i x)
 *             with D = diag(1/p_v), p_v = #{i : v in S_i} / n, D_i = P_{S_i} D
 *                                                             (Section 2, Eq. SparseSAGA;
 *                                                              Section 4.2 "Exact regularization")
 *             abar += (delta/n) a_i,  alpha_i += delta         (Algorithm 2, shared-memory
 *                                                              updates; serial here)
 *
 *   async     (simulated, oracle_delayed_saga_run) each read lacks some
 *             coordinate writes of the last tau updates   (Section 3.3, Eq. async)
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - x0 = 0, alpha0 = 0, abar0 = 0 (the Section 2 footnote lets the memory
 *     start at any value; zero is the usual choice).
 *   - S_i is the structural support of row i (its stored entries); a column
 *     no row touches gets D_v = 0 and keeps x_v = 0, its optimum.
 *   - Within an update, x_v and abar_v are read before any write (Algorithm 2
 *     reads before it writes); the lambda term uses that same read of x_v.
 *   - L = c max_i ||a_i||^2 + lambda with c = 1/4 (logistic), 1 (squared);
 *     gamma = min(1/(3L), 1/(lambda max_v D_v)).
 *   - Samples i_t come from a counter-based stream: SplitMix64 (Steele, Lea &
 *     Flood 2014) of state seed + (t+1) * 0x9E3779B97F4A7C15, mapped to
 *     [0, n) by the high 64 bits of the 128-bit product with n (Lemire).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_LOGISTIC 0
#define ORACLE_SQUARED 1

/* ------------------------------------------------------------------ */
/* sample stream                                                       */
/* ------------------------------------------------------------------ */

uint64_t oracle_splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int64_t oracle_sample(uint64_t seed, uint64_t t, int64_t n) {
    unsigned __int128 prod = (unsigned __int128)oracle_splitmix64(seed, t) * (unsigned __int128)(uint64_t)n;
    return (int64_t)(uint64_t)(prod >> 64);
}

void oracle_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out) {
    for (int64_t s = 0; s < count; ++s) out[s] = oracle_sample(seed, t0 + (uint64_t)s, n);
}

/* ------------------------------------------------------------------ */
/* per-sample loss and its derivative in z = a_i . x                   */
/* ------------------------------------------------------------------ */

double oracle_phi(double z, double b, int loss) {
    if (loss == ORACLE_SQUARED) return 0.5 * (z - b) * (z - b);
    double m = b * z; /* log(1 + exp(-m)) */
    if (m > 0.0) return log1p(exp(-m));
    return -m + log1p(exp(m));
}

double oracle_dphi(double z, double b, int loss) {
    if (loss == ORACLE_SQUARED) return z - b;
    double m = b * z; /* d/dz log(1 + exp(-b z)) = -b / (1 + exp(b z)) */
    if (m > 0.0) {
        double e = exp(-m);
        return -b * e / (1.0 + e);
    }
    return -b / (1.0 + exp(m));
}

/* ------------------------------------------------------------------ */
/* p_v, D, L, gamma                                                    */
/* ------------------------------------------------------------------ */

/* cnt_v = #{i : v in S_i}  (so p_v = cnt_v / n; Section 2) */
void oracle_column_counts(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, int64_t* cnt) {
    memset(cnt, 0, (size_t)d * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) cnt[colidx[k]] += 1;
}

/* D_v = 1 / p_v = n / cnt_v, 0 for untouched columns (Section 2) */
void oracle_reweighting(int64_t n, int64_t d, const int64_t* cnt, double* D) {
    for (int64_t v = 0; v < d; ++v) D[v] = cnt[v] > 0 ? (double)n / (double)cnt[v] : 0.0;
}

double oracle_smoothness(int64_t n, const int64_t* rowptr, const double* val, int loss, double lambda) {
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * val[k];
        if (s > mx) mx = s;
    }
    return (loss == ORACLE_LOGISTIC ? 0.25 : 1.0) * mx + lambda;
}

double oracle_step_size(double L, double lambda, int64_t d, const double* D) {
    double dmax = 0.0;
    for (int64_t v = 0; v < d; ++v)
        if (D[v] > dmax) dmax = D[v];
    double g = 1.0 / (3.0 * L);
    if (lambda * dmax > 0.0 && 1.0 / (lambda * dmax) < g) g = 1.0 / (lambda * dmax);
    return g;
}

/* ------------------------------------------------------------------ */
/* the Sparse SAGA iteration                                           */
/* ------------------------------------------------------------------ */

/* One Sparse SAGA update on sample i, in place on (x, alpha, abar).
 * Returns delta = phi'(a_i . x) - alpha_i. */
static double sparse_saga_update(int64_t i, int64_t n, const int64_t* rowptr, const int32_t* colidx,
                                 const double* val, const double* b, int loss, double lambda,
                                 const double* D, double gamma, double* x, double* alpha, double* abar) {
    int64_t s = rowptr[i], e = rowptr[i + 1];
    /* read x on S_i, form the dot product */
    double z = 0.0;
    for (int64_t k = s; k < e; ++k) z += val[k] * x[colidx[k]];
    /* scalar gradient and its change against the stored memory */
    double delta = oracle_dphi(z, b[i], loss) - alpha[i];
    /* per-coordinate step and running-average update on S_i */
    for (int64_t k = s; k < e; ++k) {
        int32_t v = colidx[k];
        double xo = x[v];
        double ab = abar[v];
        x[v] = xo - gamma * (delta * val[k] + D[v] * (ab + lambda * xo));
        abar[v] = ab + delta * val[k] / (double)n;
    }
    alpha[i] = alpha[i] + delta;
    return delta;
}

/* Updates on an explicit list of samples idx[0..count). */
int oracle_saga_indices(int64_t n, const int64_t* rowptr, const int32_t* colidx, const double* val,
                        const double* b, int loss, double lambda, const double* D, double gamma,
                        const int64_t* idx, int64_t count, double* x, double* alpha, double* abar) {
    for (int64_t s = 0; s < count; ++s) {
        if (idx[s] < 0 || idx[s] >= n) return -1;
        sparse_saga_update(idx[s], n, rowptr, colidx, val, b, loss, lambda, D, gamma, x, alpha, abar);
    }
    return 0;
}

/* Updates t = t0 .. t0+count-1 of the seeded sample stream. */
int oracle_saga_run(int64_t n, const int64_t* rowptr, const int32_t* colidx, const double* val,
                    const double* b, int loss, double lambda, const double* D, double gamma,
                    uint64_t seed, uint64_t t0, int64_t count, double* x, double* alpha, double* abar) {
    for (int64_t s = 0; s < count; ++s) {
        int64_t i = oracle_sample(seed, t0 + (uint64_t)s, n);
        sparse_saga_update(i, n, rowptr, colidx, val, b, loss, lambda, D, gamma, x, alpha, abar);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Simulated asynchrony: inconsistent reads with bounded overlap        */
/* ------------------------------------------------------------------ */

/* The asynchronous iteration as the analysis models it (Section 3.3: the
 * bounded-overlap assumption and Eq. async).  Update t reads
 *     x^_t = x_t + gamma sum_{u=(t-tau)+}^{t-1} G_u^t g_u ,
 * the current iterate lacking some coordinate writes of the last tau
 * updates (G_u^t diagonal with entries in {0, 1}); the reads of abar and of
 * the memory alpha_i lack the same updates' writes.  The update is computed
 * from those reads and added to the shared state (atomic additions,
 * Property 3), in update order, so abar = (1/n) sum_i alpha_i a_i holds
 * whatever was missing from the reads.
 * Readings (not fixed by the paper): coordinate v of update u is missing
 * from read t independently with probability q, decided by SplitMix64
 * started from delay_seed at counter ((t (tau + 1) + (t - u)) (d + 1) + v),
 * t and u absolute update counters, v = d standing for the memory write
 * alpha_{i_u}.  q = 0 is Sparse SAGA exactly; q = 1 makes every read the
 * state of tau updates earlier.  The window starts empty at each call.
 * Samples come from the serial stream. */
static int delay_missing(uint64_t delay_seed, uint64_t t, uint64_t back, int64_t tau, int64_t d, int64_t v,
                         double q) {
    if (q <= 0.0) return 0;
    if (q >= 1.0) return 1;
    uint64_t key = ((t * (uint64_t)(tau + 1) + back) * (uint64_t)(d + 1)) + (uint64_t)v;
    double r = (double)(oracle_splitmix64(delay_seed, key) >> 11) * 0x1.0p-53;
    return r < q;
}

int oracle_delayed_saga_run(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                            const double* b, int loss, double lambda, const double* D, double gamma,
                            uint64_t seed, uint64_t t0, int64_t count, int64_t tau, double q, uint64_t delay_seed,
                            double* x, double* alpha, double* abar) {
    if (tau < 0 || count < 0) return -1;
    int64_t maxlen = 0;
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] - rowptr[i] > maxlen) maxlen = rowptr[i + 1] - rowptr[i];
    int64_t slots = tau > 0 ? tau : 1;
    int64_t* ring_i = calloc((size_t)slots, sizeof(int64_t));
    double* ring_dx = calloc((size_t)(slots * (maxlen > 0 ? maxlen : 1)), sizeof(double));
    double* ring_dab = calloc((size_t)(slots * (maxlen > 0 ? maxlen : 1)), sizeof(double));
    double* ring_da = calloc((size_t)slots, sizeof(double));
    double* miss_x = calloc((size_t)(d > 0 ? d : 1), sizeof(double));
    double* miss_ab = calloc((size_t)(d > 0 ? d : 1), sizeof(double));
    double* xh = calloc((size_t)(maxlen > 0 ? maxlen : 1), sizeof(double));
    double* abh = calloc((size_t)(maxlen > 0 ? maxlen : 1), sizeof(double));
    int rc = 0;
    if (!ring_i || !ring_dx || !ring_dab || !ring_da || !miss_x || !miss_ab || !xh || !abh) rc = -2;
    for (int64_t s = 0; s < count && rc == 0; ++s) {
        uint64_t t = t0 + (uint64_t)s;
        int64_t i = oracle_sample(seed, t, n);
        int64_t first = s - tau > 0 ? s - tau : 0;
        /* the writes of the window's updates that read t does not see */
        double miss_alpha = 0.0;
        for (int64_t u = first; u < s; ++u) {
            int64_t slot = u % slots, iu = ring_i[slot];
            uint64_t back = (uint64_t)(s - u);
            for (int64_t k = rowptr[iu]; k < rowptr[iu + 1]; ++k) {
                int32_t v = colidx[k];
                if (delay_missing(delay_seed, t, back, tau, d, v, q)) {
                    miss_x[v] += ring_dx[slot * maxlen + (k - rowptr[iu])];
                    miss_ab[v] += ring_dab[slot * maxlen + (k - rowptr[iu])];
                }
            }
            if (iu == i && delay_missing(delay_seed, t, back, tau, d, d, q)) miss_alpha += ring_da[slot];
        }
        /* inconsistent read of x, abar on S_i and of alpha_i */
        int64_t rs = rowptr[i], re = rowptr[i + 1];
        double z = 0.0;
        for (int64_t k = rs; k < re; ++k) {
            int32_t v = colidx[k];
            xh[k - rs] = x[v] - miss_x[v];
            abh[k - rs] = abar[v] - miss_ab[v];
            z += val[k] * xh[k - rs];
        }
        double delta = oracle_dphi(z, b[i], loss) - (alpha[i] - miss_alpha);
        /* clear the scratch for the next read */
        for (int64_t u = first; u < s; ++u) {
            int64_t iu = ring_i[u % slots];
            for (int64_t k = rowptr[iu]; k < rowptr[iu + 1]; ++k) {
                miss_x[colidx[k]] = 0.0;
                miss_ab[colidx[k]] = 0.0;
            }
        }
        /* the update, added to the shared state and kept for later reads */
        int64_t slot = tau > 0 ? s % slots : 0;
        for (int64_t k = rs; k < re; ++k) {
            int32_t v = colidx[k];
            double wx = -gamma * (delta * val[k] + D[v] * (abh[k - rs] + lambda * xh[k - rs]));
            double wab = delta * val[k] / (double)n;
            x[v] += wx;
            abar[v] += wab;
            ring_dx[slot * maxlen + (k - rs)] = wx;
            ring_dab[slot * maxlen + (k - rs)] = wab;
        }
        alpha[i] += delta;
        ring_i[slot] = i;
        ring_da[slot] = delta;
    }
    free(ring_i);
    free(ring_dx);
    free(ring_dab);
    free(ring_da);
    free(miss_x);
    free(miss_ab);
    free(xh);
    free(abh);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sparse SVRG with randomly timed full gradients (Appendix C)         */
/* ------------------------------------------------------------------ */

/* The SVRG variant the paper extends its analysis to (Appendix C,
 * "Extension to SVRG"): at the start of every iteration a binary U with
 * P(U = 1) = 1/n decides whether a full gradient is computed at the current
 * point (the snapshot x~) or an inner step is made.  For linear models the
 * snapshot's per-sample gradients are the scalars alpha_i = phi'(a_i . x~)
 * and its full gradient's data part is abar = (1/n) sum_i alpha_i a_i; the
 * sparse inner step (the Sparse SVRG that Section 2 builds Sparse SAGA from)
 * is
 *     x+ = x - gamma ((phi'(a_i . x) - alpha_i) a_i + D_i (abar + lambda x)),
 * i.e. Eq. SparseSAGA with the memory held at the snapshot.
 * Readings (not fixed by the paper):
 *   - U_t = 1 iff the sample-stream map of SplitMix64 started from
 *     seed XOR ORACLE_SVRG_TAG gives index 0 for counter t (probability 1/n);
 *   - an iteration with U_t = 1 computes the snapshot and makes no step;
 *   - a snapshot is taken at x0 before the first iteration. */
#define ORACLE_SVRG_TAG 0xA5A5A5A5A5A5A5A5ull

int oracle_svrg_full_gradient_due(uint64_t seed, uint64_t t, int64_t n) {
    return oracle_sample(seed ^ ORACLE_SVRG_TAG, t, n) == 0;
}

/* The snapshot at x: alpha_i = phi'(a_i . x; b_i), abar = (1/n) sum alpha_i a_i. */
void oracle_svrg_snapshot(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                          const double* b, int loss, const double* x, double* alpha, double* abar) {
    for (int64_t v = 0; v < d; ++v) abar[v] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double z = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) z += val[k] * x[colidx[k]];
        alpha[i] = oracle_dphi(z, b[i], loss);
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) abar[colidx[k]] += alpha[i] * val[k];
    }
    for (int64_t v = 0; v < d; ++v) abar[v] /= (double)n;
}

/* One sparse SVRG inner step on sample i: x only; alpha and abar stay. */
static void sparse_svrg_step(int64_t i, const int64_t* rowptr, const int32_t* colidx, const double* val,
                             const double* b, int loss, double lambda, const double* D, double gamma, double* x,
                             const double* alpha, const double* abar) {
    int64_t s = rowptr[i], e = rowptr[i + 1];
    double z = 0.0;
    for (int64_t k = s; k < e; ++k) z += val[k] * x[colidx[k]];
    double delta = oracle_dphi(z, b[i], loss) - alpha[i];
    for (int64_t k = s; k < e; ++k) {
        int32_t v = colidx[k];
        double xo = x[v];
        x[v] = xo - gamma * (delta * val[k] + D[v] * (abar[v] + lambda * xo));
    }
}

/* Inner steps on an explicit list of samples (no snapshot). */
int oracle_svrg_indices(const int64_t* rowptr, const int32_t* colidx, const double* val, const double* b, int loss,
                        double lambda, const double* D, double gamma, int64_t n, const int64_t* idx, int64_t count,
                        double* x, const double* alpha, const double* abar) {
    for (int64_t s = 0; s < count; ++s) {
        if (idx[s] < 0 || idx[s] >= n) return -1;
        sparse_svrg_step(idx[s], rowptr, colidx, val, b, loss, lambda, D, gamma, x, alpha, abar);
    }
    return 0;
}

/* Iterations t = t0 .. t0+count-1: snapshot where U_t = 1, otherwise an
 * inner step on sample i_t of the seeded stream. */
int oracle_svrg_run(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                    const double* b, int loss, double lambda, const double* D, double gamma, uint64_t seed,
                    uint64_t t0, int64_t count, double* x, double* alpha, double* abar) {
    for (int64_t s = 0; s < count; ++s) {
        uint64_t t = t0 + (uint64_t)s;
        if (oracle_svrg_full_gradient_due(seed, t, n))
            oracle_svrg_snapshot(n, d, rowptr, colidx, val, b, loss, x, alpha, abar);
        else
            sparse_svrg_step(oracle_sample(seed, t, n), rowptr, colidx, val, b, loss, lambda, D, gamma, x, alpha,
                             abar);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* dense and lagged SAGA (Appendix F), for the comparison with Sparse  */
/* SAGA; serial only                                                   */
/* ------------------------------------------------------------------ */

/* Dense SAGA with the linear-model memory (Eq. SAGAupdate of Section 2):
 *     x+ = x - gamma ((phi'(a_i . x) - alpha_i) a_i + abar + lambda x)
 * over every coordinate, then abar += (delta/n) a_i, alpha_i += delta. */
int oracle_dense_saga_run(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                          const double* b, int loss, double lambda, double gamma, uint64_t seed, uint64_t t0,
                          int64_t count, double* x, double* alpha, double* abar) {
    for (int64_t s = 0; s < count; ++s) {
        int64_t i = oracle_sample(seed, t0 + (uint64_t)s, n);
        double z = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) z += val[k] * x[colidx[k]];
        double delta = oracle_dphi(z, b[i], loss) - alpha[i];
        /* the memory average and the L2 term reach every coordinate (read before the write) */
        for (int64_t v = 0; v < d; ++v) x[v] = x[v] - gamma * (abar[v] + lambda * x[v]);
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            x[colidx[k]] -= gamma * delta * val[k];
            abar[colidx[k]] += delta * val[k] / (double)n;
        }
        alpha[i] += delta;
    }
    return 0;
}

/* Bring coordinate v from iteration last[v] to iteration t: each skipped
 * dense step was x_v <- (1 - gamma lambda) x_v - gamma abar_v with abar_v
 * unchanged (it changes only when v is in a sampled support), so after k
 * steps x_v = q (x_v + abar_v / lambda) - abar_v / lambda, q = (1 - gamma lambda)^k. */
static void lagged_catch_up(int64_t v, uint64_t t, double gamma, double lambda, double* x, const double* abar,
                            uint64_t* last) {
    uint64_t k = t - last[v];
    if (k == 0) return;
    double lq = (double)k * log1p(-gamma * lambda);
    double q = exp(lq);
    /* q x - (1 - q) abar / lambda, with 1 - q = -expm1(lq) free of cancellation */
    x[v] = q * x[v] + expm1(lq) * abar[v] / lambda;
    last[v] = t;
}

/* Lagged SAGA (the lagged-update implementation Appendix F compares with):
 * the dense part of each step is applied to a coordinate only when a
 * sampled support next reads it (last[v] holds the iteration x_v is current
 * at); the same iterates as dense SAGA, computed on the supports only.
 * All coordinates are brought up to date at the end of the call. */
int oracle_lagged_saga_run(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                           const double* b, int loss, double lambda, double gamma, uint64_t seed, uint64_t t0,
                           int64_t count, double* x, double* alpha, double* abar, uint64_t* last) {
    if (!(lambda > 0.0)) return -1;
    for (int64_t s = 0; s < count; ++s) {
        uint64_t t = t0 + (uint64_t)s;
        int64_t i = oracle_sample(seed, t, n);
        double z = 0.0;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            lagged_catch_up(colidx[k], t, gamma, lambda, x, abar, last);
            z += val[k] * x[colidx[k]];
        }
        double delta = oracle_dphi(z, b[i], loss) - alpha[i];
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int32_t v = colidx[k];
            double xo = x[v];
            x[v] = xo - gamma * (delta * val[k] + abar[v] + lambda * xo);
            abar[v] += delta * val[k] / (double)n;
            last[v] = t + 1;
        }
        alpha[i] += delta;
    }
    for (int64_t v = 0; v < d; ++v) lagged_catch_up(v, t0 + (uint64_t)count, gamma, lambda, x, abar, last);
    return 0;
}

/* ------------------------------------------------------------------ */
/* objective and gradient, Neumaier-compensated sums                   */
/* ------------------------------------------------------------------ */

typedef struct { double s, c; } ksum;

static inline void kadd(ksum* a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

/* f(x) = (1/n) sum_i phi(a_i . x; b_i) + (lambda/2) ||x||^2   (Section 4.1) */
double oracle_objective(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                        const double* b, int loss, double lambda, const double* x) {
    ksum data = {0.0, 0.0}, reg = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        ksum z = {0.0, 0.0};
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) kadd(&z, val[k] * x[colidx[k]]);
        kadd(&data, oracle_phi(z.s + z.c, b[i], loss));
    }
    for (int64_t v = 0; v < d; ++v) kadd(&reg, x[v] * x[v]);
    return (data.s + data.c) / (double)n + 0.5 * lambda * (reg.s + reg.c);
}

/* grad f(x) = (1/n) sum_i phi'(a_i . x; b_i) a_i + lambda x */
int oracle_gradient(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx, const double* val,
                    const double* b, int loss, double lambda, const double* x, double* g) {
    ksum* acc = (ksum*)calloc((size_t)d, sizeof(ksum));
    if (!acc) return -2;
    for (int64_t i = 0; i < n; ++i) {
        ksum z = {0.0, 0.0};
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) kadd(&z, val[k] * x[colidx[k]]);
        double gi = oracle_dphi(z.s + z.c, b[i], loss);
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) kadd(&acc[colidx[k]], gi * val[k]);
    }
    for (int64_t v = 0; v < d; ++v) g[v] = (acc[v].s + acc[v].c) / (double)n + lambda * x[v];
    free(acc);
    return 0;
}

/* (1/n) sum_i alpha_i a_i, compensated: what abar must equal at all times. */
int oracle_memory_average(int64_t n, int64_t d, const int64_t* rowptr, const int32_t* colidx,
                          const double* val, const double* alpha, double* out) {
    ksum* acc = (ksum*)calloc((size_t)d, sizeof(ksum));
    if (!acc) return -2;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) kadd(&acc[colidx[k]], alpha[i] * val[k]);
    for (int64_t v = 0; v < d; ++v) out[v] = (acc[v].s + acc[v].c) / (double)n;
    free(acc);
    return 0;
}
