/* asaga.h -- C ABI of the MI355X (gfx950) Sparse SAGA / ASAGA library.
 *
 * Method: Leblond, Pedregosa & Lacoste-Julien, "ASAGA: Asynchronous Parallel
 * SAGA", AISTATS 2017.
 *
 * Problem (Section 1, Eq. finiteSum; models of Section 4.1):
 *     min_x f(x) = (1/n) sum_i phi(a_i . x; b_i) + (lambda/2) ||x||^2
 *     logistic: phi(z; b) = log(1 + exp(-b z)),  b in {-1, +1}
 *     squared:  phi(z; b) = (z - b)^2 / 2
 * a_i is row i of an n x d CSR matrix A.
 *
 * Update (Section 2, Eq. SparseSAGA, with the projected L2 term of Section
 * 4.2), for a sample i drawn uniformly with replacement:
 *     z      = a_i . x_hat                        (x_hat: read of x on S_i)
 *     delta  = phi'(z; b_i) - alpha_i             (alpha_i: scalar memory)
 *     x_v   += -gamma (delta a_iv + D_v (abar_v + lambda x_hat_v))   v in S_i
 *     abar_v += delta a_iv / n                                         v in S_i
 *     alpha_i += delta
 * S_i is the set of stored entries of row i, D_v = n / #{i : v in S_i}
 * (0 for an empty column).  x, alpha and abar start at 0.
 *
 * Modes:
 *   ASAGA_MODE_SERIAL  one wavefront applies the updates one after another in
 *                      the order of the seeded sample stream (deterministic;
 *                      the sequential Sparse SAGA of Section 2).
 *   ASAGA_MODE_ASYNC   many wavefronts apply updates concurrently, lock-free,
 *                      with inconsistent reads and atomic additions (the
 *                      ASAGA implementation of Algorithm 2; atomicity as in
 *                      Section 3.3, Property 3).  The multiset of samples is
 *                      the same stream as in serial mode.
 *
 * Sample stream: sample t (t = 0, 1, 2, ... counted across calls) is
 *     i_t = floor(n * SplitMix64(seed, t) / 2^64)
 * with SplitMix64(seed, t) the (t+1)-th output of the SplitMix64 generator of
 * Steele, Lea & Flood (2014) started from state `seed`.  One epoch = n samples.
 *
 * Step size: when opts.step <= 0, gamma = min(1/(3L), 1/(lambda max_v D_v))
 * with L = c max_i ||a_i||^2 + lambda, c = 1/4 (logistic) or 1 (squared);
 * in ASAGA_MODE_ASYNC that value is divided by 4.  With many samples in
 * flight, updates read state that is older by up to tau samples (Section
 * 3.3, Assumption 1), and the stable step shrinks as tau grows along the
 * directions many rows share (Theorem 2); asaga_autotune measures the step
 * and launch shape that reach a target accuracy soonest.
 *
 * Columns are relabelled internally by descending count; every vector that
 * crosses this interface (x, gradients, abar) is in the caller's order.
 *
 * Conventions:
 *   - Every function returns ASAGA_OK (0) or a negative ASAGA_E_* code; the
 *     message of the last failure is available from asaga_last_error().
 *     No exception and no abort crosses this interface.
 *   - Pointers named *_host are host memory owned by the caller; outputs are
 *     always written into caller-owned host buffers.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Work is enqueued on opts.stream (a hipStream_t; NULL = null stream).
 *     asaga_epochs returns without waiting; every call that returns data
 *     waits for the stream.
 *   - `inst` selects an instance of a batched context (0 for a single solve).
 */
#ifndef ASAGA_H
#define ASAGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define ASAGA_OK 0
#define ASAGA_E_ARG (-1)      /* bad argument (NULL, out of range, bad enum)          */
#define ASAGA_E_CSR (-2)      /* malformed CSR / labels / values (see asaga_init)     */
#define ASAGA_E_OOM (-3)      /* device or host allocation failed                     */
#define ASAGA_E_HIP (-4)      /* a HIP runtime call or kernel launch failed           */
#define ASAGA_E_DIVERGED (-5) /* a non-finite value appeared in the iterate/objective */
#define ASAGA_E_STATE (-6)    /* call not valid in the context's current state        */

/* losses */
#define ASAGA_LOSS_LOGISTIC 0
#define ASAGA_LOSS_SQUARED 1

/* element type of the CSR values */
#define ASAGA_VAL_F64 0
#define ASAGA_VAL_F32 1
#define ASAGA_VAL_BF16 2 /* raw bfloat16 bit patterns (uint16) */

/* where the problem arrays live */
#define ASAGA_MEM_HOST 0   /* copied to the device by asaga_init                   */
#define ASAGA_MEM_DEVICE 1 /* borrowed: must stay alive and unchanged until free  */

/* execution mode */
#define ASAGA_MODE_SERIAL 0
#define ASAGA_MODE_ASYNC 1

/* precision of the state */
#define ASAGA_PREC_F64 0   /* x, alpha, abar in FP64                               */
#define ASAGA_PREC_MIXED 1 /* x, alpha in FP32 (phi' rounded to FP32 before delta
                              is formed); abar and D in FP64                       */

typedef struct asaga_ctx asaga_ctx;

/* The data of the problem.  CSR requirements (checked by asaga_init):
 * rowptr[0] = 0, rowptr nondecreasing, every row non-empty, rowptr[n] = nnz,
 * 0 <= colidx < d and strictly increasing within each row, values finite,
 * b finite and, for the logistic loss, in {-1, +1}; 1 <= n < 2^31,
 * 1 <= d < 2^27, lambda > 0 and finite.  Layout: rowptr int64[n+1], colidx int32[nnz],
 * val[nnz] of type val_dtype, b double[n]. */
typedef struct asaga_problem {
    int64_t n;
    int64_t d;
    const int64_t* rowptr;
    const int32_t* colidx;
    const void* val;
    const double* b;
    double lambda;
    int32_t val_dtype; /* ASAGA_VAL_* */
    int32_t loss;      /* ASAGA_LOSS_* */
    int32_t mem;       /* ASAGA_MEM_* (applies to rowptr, colidx, val and b)  */
    int32_t reserved;  /* must be 0 */
} asaga_problem;

/* Solver options.  Zero-initialised options are valid: serial FP64, the
 * step-size rule, seed 0, automatic launch shape, null stream. */
typedef struct asaga_opts {
    double step;              /* gamma; <= 0 selects the rule above               */
    uint64_t seed;            /* sample-stream seed                                */
    int32_t mode;             /* ASAGA_MODE_*                                      */
    int32_t precision;        /* ASAGA_PREC_*                                      */
    int32_t waves;            /* async: wavefronts in flight, per instance in a
                                 batch (0 = automatic: 8 per compute unit, or
                                 64 per instance in a batch)                      */
    int32_t lanes_per_sample; /* async: 64, 32, 16 or 8 lanes per sample
                                 (0 = automatic from the mean row length)          */
    int32_t racy;             /* 1: plain read-modify-write instead of atomic adds
                                 (the non-thread-safe variant of App. G; a
                                 negative control, async only)                    */
    int32_t hot_columns;      /* async: the H most-used columns whose writes each
                                 workgroup combines in LDS before adding them to
                                 the shared state (0 = automatic, -1 = none;
                                 at most 4096)                                    */
    int32_t flush_every;      /* async: samples each lane group applies between
                                 two flushes of those combined writes
                                 (0 = automatic)                                  */
    int32_t threads_per_block;/* async: workgroup size, a multiple of 64 up to
                                 512 (0 = automatic)                              */
    int32_t hot_tier_columns; /* async: the first hot columns, flushed after every
                                 round of flush_every samples; the others are
                                 flushed every hot_tier_every rounds
                                 (0 = automatic, -1 = all hot columns every round) */
    int32_t hot_tier_every;   /* async: see hot_tier_columns (0 = automatic)      */
    int32_t plain_launch;     /* batched: 1 launches each epoch's kernel directly;
                                 0 (default) replays the epochs of one
                                 asaga_epochs call as a captured hipGraph        */
    int32_t reserved;         /* must be 0                                         */
    void* stream;             /* hipStream_t */
} asaga_opts;

/* Many solves over one shared matrix (a regularisation path times
 * cross-validation folds).  Instance k minimises
 *     f_k(x) = (1/n_k) sum_{i : row_fold[i] != inst_fold[k]} phi(a_i . x; b_i)
 *              + (inst_lambda[k]/2) ||x||^2
 * over its n_k training rows (inst_fold[k] = -1 trains on every row), with
 * its own D (column counts over its training rows), step size and sample
 * stream (seed + k).  All arrays are host memory. */
typedef struct asaga_batch {
    int32_t n_inst;
    int32_t reserved;
    const int8_t* row_fold;     /* [n]      fold id of each row, or NULL if every inst_fold is -1 */
    const int32_t* inst_fold;   /* [n_inst] held-out fold of each instance, or -1             */
    const double* inst_lambda;  /* [n_inst] lambda of each instance (> 0)                    */
} asaga_batch;

/* Numbers the library derived at initialisation. */
typedef struct asaga_info {
    int64_t n, d, nnz;
    int64_t delta_r;   /* max_v #{i : v in S_i} (Section 3.4, sparsity definition) */
    int64_t t;         /* samples applied so far (instance 0)                        */
    double L;          /* smoothness constant used by the step-size rule            */
    double gamma;      /* step size in use (instance 0)                             */
    double lambda;     /* instance 0                                                */
    int32_t waves;     /* async launch: wavefronts in flight (per instance if batched) */
    int32_t lanes_per_sample;
    int32_t n_inst;
    int32_t hot_columns;
    int32_t flush_every;
    int32_t threads_per_block;
    int32_t hot_tier_columns;
    int32_t hot_tier_every;
    int32_t reserved;
} asaga_info;

/* What asaga_autotune measured and chose. */
typedef struct asaga_tune_report {
    int32_t candidates;       /* (launch shape, step) pairs probed                  */
    int32_t waves;            /* chosen launch shape                                */
    int32_t hot_columns;
    int32_t hot_tier_columns;
    double gamma;             /* chosen step                                        */
    double ms_per_epoch;      /* measured kernel time per epoch at the choice       */
    double est_epochs;        /* estimated epochs from a cold start to the target   */
    double est_seconds;       /* estimated kernel seconds to the target             */
} asaga_tune_report;

/* Create a context: validate the problem, copy host arrays to the device
 * (device arrays are borrowed), count columns (D, Delta_r), compute L and
 * gamma, zero x, alpha and abar.  On failure *out is NULL and the message is
 * available from asaga_last_error(NULL). */
int asaga_init(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts);

/* As asaga_init, for a batch of instances sharing the matrix. */
int asaga_init_batched(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts,
                       const asaga_batch* batch);

/* Apply n_epochs * n samples (n_k per instance in a batch), continuing the
 * sample stream.  Enqueued on the context's stream; returns without waiting
 * for single-instance contexts.  A batched context runs one persistent
 * kernel per epoch over every active instance; the n_epochs launches are
 * captured once per distinct n_epochs (up to 64; larger counts run in pieces)
 * into a hipGraph on a private stream and replayed on the context's stream
 * (unless opts.plain_launch).  It waits for the previous call's work before
 * rewriting the per-instance descriptors the kernels read. */
int asaga_epochs(asaga_ctx* ctx, int64_t n_epochs);

/* Batched contexts: switch instances on (1) or off (0) for later
 * asaga_epochs calls (active is uint8_t[n_inst]).  An instance that is off
 * keeps its state and sample counter unchanged; every instance starts on.
 * The usual use: switch off each instance once its certificate or
 * validation check has met the tolerance. */
int asaga_set_active(asaga_ctx* ctx, const uint8_t* active);

/* Apply `count` samples (single-instance contexts only). */
int asaga_updates(asaga_ctx* ctx, int64_t count);

/* f(x) in FP64 (Section 4.1 objective, pairwise-summed).  x_host = NULL
 * evaluates the instance's current iterate; otherwise x_host is double[d].
 * Returns ASAGA_E_DIVERGED if the value is not finite. */
int asaga_objective(asaga_ctx* ctx, int32_t inst, const double* x_host, double* f_out);

/* grad f(x) = (1/n) sum_i phi'(a_i . x; b_i) a_i + lambda x in FP64 into
 * g_host (double[d]).  x_host as for asaga_objective. */
int asaga_full_grad(asaga_ctx* ctx, int32_t inst, const double* x_host, double* g_host);

/* Copy the instance's iterate x (widened to FP64) into x_host (double[d]). */
int asaga_get_x(asaga_ctx* ctx, int32_t inst, double* x_host);

/* Copy / overwrite the instance's whole state: x, abar (double[d]), alpha
 * (double[n_k], in the order of the instance's training rows) and the sample
 * counter t.  Any pointer may be NULL to skip that part (get) or to leave it
 * unchanged (set).  A serial run resumed from a saved state reproduces the
 * uninterrupted run. */
int asaga_get_state(asaga_ctx* ctx, int32_t inst, double* x_host, double* alpha_host, double* abar_host,
                    int64_t* t_out);
int asaga_set_state(asaga_ctx* ctx, int32_t inst, const double* x_host, const double* alpha_host,
                    const double* abar_host, const int64_t* t_in);

/* Recompute abar = (1/n_k) sum_i alpha_i a_i exactly (FP64) from the stored
 * memory, removing the drift that concurrent or reduced-precision additions
 * leave in the running average (every instance). */
int asaga_reanchor(asaga_ctx* ctx);

/* Choose the number of wavefronts in flight and the step that reach
 * relative suboptimality `target` soonest on this problem (async contexts;
 * the other shape parameters stay as the context has them, except as said
 * for batches below).
 * Fewer samples in flight tolerate a larger step (Theorem 2) but take longer
 * per epoch, so wavefront counts are tried from 8 per compute unit down to
 * 1/8 per compute unit, halving.  For each count it times one epoch, then,
 * for steps from the serial rule downwards by halves (to 1/64 of it), runs
 * `probe_epochs` epochs from x = 0, measures the decay rate of ||grad f||
 * (FP64 full gradients at three checkpoints; a step whose gradient norm does
 * not decrease at every checkpoint is rejected as unstable) and extrapolates
 * to ||grad f||^2 <= 2 lambda target f, which bounds (f - f*)/f by `target`
 * (f is lambda-strongly convex).  Smaller steps are probed while the
 * estimate improves; a count whose probe alone would take longer than the
 * best estimate so far ends the search.  The best pair is kept, the state is
 * reset to x = alpha = abar = 0, t = 0.  Returns ASAGA_E_DIVERGED if no pair
 * was stable.
 * Batched contexts: the candidates are wavefronts per instance (64 down to
 * the workgroup's wave count, halving) times hot-set sizes (4096 and 1024
 * columns), ordered by their measured time per epoch of the whole batch; a
 * step is a common fraction of every instance's own rule; a pair is stable
 * if every active instance's gradient norm decreases at every checkpoint,
 * and its estimate is the slowest instance's epochs times the batch's time
 * per epoch.  `waves` in the report is per instance. */
int asaga_autotune(asaga_ctx* ctx, double target, int32_t probe_epochs, asaga_tune_report* report);

/* Derived numbers (instance 0, plus launch shape). */
int asaga_info_get(asaga_ctx* ctx, asaga_info* out);

/* Wait until all work enqueued by the context has finished. */
int asaga_sync(asaga_ctx* ctx);

/* The sample indices i_t, t = t0 .. t0+count-1, as generated on the device
 * (for cross-checking the stream; needs a GPU). */
int asaga_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out_host);

/* Message of the last failure of ctx (or of the last failed asaga_init* when
 * ctx is NULL).  Never NULL; the pointer is valid until the next call. */
const char* asaga_last_error(const asaga_ctx* ctx);

/* Release the context and its device memory.  NULL is a no-op. */
void asaga_free(asaga_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ASAGA_H */
