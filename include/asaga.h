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
 *   ASAGA_MODE_SERIAL  one lane group applies the updates one after another
 *                      in the order of the seeded sample stream
 *                      (deterministic; the sequential Sparse SAGA of Section
 *                      2).  It runs the asynchronous kernel's code with a
 *                      single active lane group: lanes_per_sample,
 *                      threads_per_block, hot_columns, flush_every and the
 *                      hot_tier and hot_reload options select the same
 *                      paths (LDS hot set, tiered flush, view reload,
 *                      long-row chunks) as in ASAGA_MODE_ASYNC, and the
 *                      iterates do not depend on them beyond rounding.
 *                      Defaults: 64 lanes, one 64-thread workgroup, no hot
 *                      set.  A batch in this mode runs every instance
 *                      sequentially on one workgroup of its own, all
 *                      instances concurrently.
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
 * in ASAGA_MODE_ASYNC that value is multiplied by min(1, 512 / G), G the
 * samples in flight (lane groups of the launch).  With many samples in
 * flight, updates read state that is older by up to tau samples (Section
 * 3.3, Assumption 1), and the stable step shrinks like 1/tau along the
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
                              is formed); abar and D in FP64.  abar receives the
                              change the FP32 memory entry actually takes,
                              fl32(alpha_i + fl32(delta)) - alpha_i, so that it
                              stays the average of the stored memory            */
#define ASAGA_PREC_F32 2   /* x, alpha and abar in FP32 (phi' rounded as above).
                              A column's x and abar share 8 bytes, so the two
                              lanes that add to them issue one memory request
                              (the mixed layout's FP32 x and FP64 abar take two)
                              and the LDS hot set holds up to 10240 columns.
                              The hot columns' FP32 sums are compensated: each
                              flush's rounding error (known exactly from the
                              returning atomic) stays pending in the
                              workgroup and is added with its next flush of
                              the slot; at most half a unit in the last place
                              per slot and workgroup is dropped per launch.
                              abar receives the change the FP32 memory entry
                              takes, as above.  asaga_reanchor recomputes abar
                              in FP64 (then rounds it once); asaga_widen
                              switches to FP64 for the final polish          */

/* method (single-instance contexts) */
#define ASAGA_METHOD_SAGA 0 /* Sparse SAGA (Eq. SparseSAGA), the memory updated by every step */
#define ASAGA_METHOD_SVRG 1 /* sparse SVRG with randomly timed full gradients (Appendix C):
                               at iteration t, with probability 1/n (U_t = 1 iff
                               floor(n * SplitMix64(seed XOR 0xA5A5A5A5A5A5A5A5, t) / 2^64)
                               == 0) the memory is reset to the snapshot of the current x,
                               alpha_i = phi'(a_i . x), abar = (1/n) sum alpha_i a_i, and no
                               step is made; otherwise sample i_t takes the Sparse SAGA step
                               with the memory held fixed.  A snapshot is also taken at x0.
                               Snapshots are synchronised (between launches)           */

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
    int32_t waves;            /* async: wavefronts in flight (0 = automatic: one
                                 workgroup per compute unit, and at most n/64
                                 samples in flight).  Batches: wavefronts per
                                 instance, fixed; 0 shares the device's
                                 resident workgroups equally among the
                                 instances still active (see asaga_epochs)       */
    int32_t lanes_per_sample; /* async: 64, 32, 16 or 8 lanes per sample
                                 (0 = automatic from the mean row length)          */
    int32_t racy;             /* 1: plain read-modify-write instead of atomic adds
                                 (the non-thread-safe variant of App. G; a
                                 negative control, async only)                    */
    int32_t hot_columns;      /* async: the H most-used columns whose writes each
                                 workgroup combines in LDS before adding them to
                                 the shared state (0 = automatic, -1 = none;
                                 at most 5120, or 10240 with ASAGA_PREC_F32).
                                 Automatic: that maximum, less the
                                 columns v with gamma lambda D_v W > 0.2 (W the
                                 workgroups serving the instance): a hot
                                 column's LDS view is refreshed only when the
                                 workgroup next writes it, which delays its
                                 regulariser step by about W of its updates.
                                 Where gamma 3L W D_v exceeds 4.8e4, the view
                                 is also reloaded at every full flush
                                 (asaga_info.hot_reload_from)                 */
    int32_t flush_every;      /* async: samples each lane group applies between
                                 two flushes of those combined writes
                                 (0 = automatic)                                  */
    int32_t threads_per_block;/* async: workgroup size, a multiple of 64 up to
                                 1024 (0 = automatic: 512, batches 1024).  A
                                 workgroup shares one hot set, so larger ones
                                 need fewer flush requests per sample, but one
                                 workgroup per compute unit then puts more
                                 samples in flight, which lowers the stable
                                 step                                          */
    int32_t hot_tier_columns; /* async: the first hot columns, flushed after every
                                 round of flush_every samples; the others are
                                 flushed every hot_tier_every rounds
                                 (0 = automatic, -1 = all hot columns every round) */
    int32_t hot_tier_every;   /* async: see hot_tier_columns (0 = automatic: 16,
                                 fewer when gamma * lambda * lane groups in
                                 flight is large, since that tier's columns
                                 are seen late by the other workgroups and
                                 their regulariser step then lags)           */
    int32_t plain_launch;     /* batched: 1 launches each epoch's kernel directly;
                                 0 (default) replays the epochs of one
                                 asaga_epochs call as a captured hipGraph        */
    int32_t method;           /* ASAGA_METHOD_* (SVRG: single-instance contexts,
                                 not racy)                                        */
    void* stream;             /* hipStream_t */
    int32_t hot_reload_from;  /* first hot column whose LDS view a workgroup
                                 reloads from the shared state at every full
                                 flush when it wrote nothing to it since the
                                 last one (0 = automatic: see hot_columns;
                                 serial mode none; -1 = none; c >= 1: columns
                                 [c, hot_columns))                              */
    int32_t reserved;         /* must be 0 */
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
    int32_t hot_reload_from; /* first hot column whose LDS view each workgroup
                                reloads at every full flush (hot_columns: none);
                                instance 0, at the launch shape of the next
                                asaga_epochs call (batched: of the last one)   */
} asaga_info;

/* What asaga_autotune measured and chose. */
typedef struct asaga_tune_report {
    int32_t candidates;       /* (launch shape, step) pairs probed                  */
    int32_t waves;            /* chosen launch shape                                */
    int32_t hot_columns;
    int32_t hot_tier_columns;
    double gamma;             /* chosen step                                        */
    double ms_per_epoch;      /* measured kernel time per epoch at the choice
                                 (batches: one epoch of every active instance)    */
    double est_epochs;        /* estimated epochs from a cold start to the target   */
    double est_seconds;       /* estimated kernel seconds to the target             */
    double step_groups;       /* batches: the step law gamma_k = rule_k * min(step_cap,
                                 step_groups / G_k), G_k the lane groups serving
                                 instance k (at most step_groups / step_cap);
                                 one solve: 0                                      */
    double step_cap;
    double widen_gamma;       /* the step asaga_widen switches to: gamma, or with
                                 FP32 x, when gamma is the largest stable step
                                 probed at its wavefront count, the next smaller
                                 one (gamma * 2^(-1/3)); batches: gamma         */
    int32_t threads_per_block; /* chosen workgroup size                             */
    int32_t reserved;
} asaga_tune_report;

/* Create a context for the problem of Section 1 (Eq. finiteSum with the
 * L2-regularised models of Section 4.1): validate the problem, copy host
 * arrays to the device (device arrays are borrowed), count each column's
 * rows to form p_v = #{i : v in S_i}/n and D_v = 1/p_v (Section 2, the
 * reweighting of Eq. SparseSAGA) and Delta_r = max_v #{i : v in S_i} (the
 * sparsity measure of Section 3.4), compute L and gamma, and set x, alpha
 * and abar to 0 (the initial memory of Section 2).
 * *out: receives the context (owned by the caller, released by asaga_free);
 * prob, opts: read during the call only.  Errors: ASAGA_E_ARG (NULL or out
 * of range arguments), ASAGA_E_CSR (malformed problem, see asaga_problem),
 * ASAGA_E_OOM, ASAGA_E_HIP.  On failure *out is NULL and the message is
 * available from asaga_last_error(NULL). */
int asaga_init(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts);

/* As asaga_init, for a batch of instances sharing the matrix. */
int asaga_init_batched(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts,
                       const asaga_batch* batch);

/* Apply n_epochs * n samples, continuing the sample stream.  Enqueued on the
 * context's stream; returns without waiting for single-instance contexts.
 * A batch makes n_epochs launches; in each, instance k applies n_k samples
 * with opts.waves set, and with automatic waves max(n_k, W_k P) samples, W_k
 * its workgroups and P the largest ceil(n_j / W_j): every workgroup stays
 * busy for the whole launch, so an instance holding more workgroups per
 * sample than others applies more than one epoch (the sample counter t of
 * each instance, asaga_get_state, says how many).
 * A batched context runs one persistent kernel per epoch over every active
 * instance.  With opts.waves = 0 the workgroups the device holds at once
 * are shared equally among the active instances (each at least one, and at
 * most n_k/64 samples in flight), so the instances still running take over
 * the workgroups of those switched off; without opts.step, instance k then
 * steps with
 *     gamma_k = rule_k * min(cap, c / G_k),
 * G_k the lane groups (samples in flight) serving it: the stable step
 * shrinks with the delay (Theorem 2), and an instance gets at most c / cap
 * lane groups, past which more of them only shrink its step.  c and cap come
 * from asaga_autotune; before it, c = 512 (the single-instance default) and
 * cap = 1.  The n_epochs launches are captured once per distinct n_epochs
 * (up to 64; larger counts run in pieces) into a hipGraph on a private
 * stream and replayed on the context's stream (unless opts.plain_launch).  It waits for the previous call's work before
 * rewriting the per-instance descriptors and the workgroup map the kernels
 * read.  With the stop test armed (asaga_set_stop) each epoch's launch is
 * followed by the test, and the call waits for its launches before it
 * returns: the instances the test switched off are then off
 * (asaga_instance_get), and their sample counters count the epochs they
 * ran.  Pieces of a call past 64 epochs share the running instances'
 * workgroups anew. */
int asaga_epochs(asaga_ctx* ctx, int64_t n_epochs);

/* Batched contexts: switch instances on (1) or off (0) for later
 * asaga_epochs calls (active is uint8_t[n_inst]).  An instance that is off
 * keeps its state and sample counter unchanged; every instance starts on.
 * The usual use: switch off each instance once its certificate or
 * validation check has met the tolerance. */
int asaga_set_active(asaga_ctx* ctx, const uint8_t* active);

/* Batched contexts: arm the stop test of asaga_epochs with one threshold
 * per instance (thresholds is double[n_inst], each >= 0; +infinity stops an
 * instance after its first epoch), or disarm it (thresholds = NULL).  After
 * every epoch of a call, a kernel on the same stream computes for each
 * instance still running
 *     r_k = || abar_k + lambda_k x_k ||^2,
 * in FP64 over all d columns: abar is the average of the memory (Section 2,
 * the running average of Eq. SparseSAGA, a_j scaled by each row's stored
 * derivative alpha_j), so abar + lambda x is the objective's full gradient
 * (the Section 4.1 objective) with every alpha_j taken from when row j was
 * last sampled instead of at the current x.  It costs O(d) per instance,
 * not a pass over the rows.  An instance with r_k <= thresholds[k] applies
 * no more samples in that call and is switched off when it returns.  The
 * proxy is not the gradient: a threshold 2 lambda_k eps f_k (f_k at or
 * below the optimum's value) would certify (f - f*)/f* <= eps through strong
 * convexity only for the exact gradient (asaga_full_grad), so a caller
 * confirms a switched-off instance with the exact FP64 objective or
 * gradient and switches it on again if the check fails.  The thresholds
 * are copied; the call waits for the context's stream.  The autotuner runs
 * without the test.  Errors: ASAGA_E_STATE (not batched), ASAGA_E_ARG (a
 * threshold below 0 or NaN), ASAGA_E_OOM (first call: three arrays of
 * n_inst entries). */
int asaga_set_stop(asaga_ctx* ctx, const double* thresholds);

/* Batched contexts: what the stop test saw in the last asaga_epochs call
 * with it armed (the proxy of asaga_set_stop: the Section 4.1 objective's
 * gradient with the derivatives held in the memory of Section 2).
 * proxy_out (double[n_inst], or NULL): r_k after the last
 * epoch instance k ran in that call (NaN if it ran none); epochs_out
 * (int64_t[n_inst], or NULL): the epochs (launches) it ran, fewer than the
 * call's where the test switched it off.  Before any such call: NaN and 0. */
int asaga_stop_report(asaga_ctx* ctx, double* proxy_out, int64_t* epochs_out);

/* Apply `count` samples (single-instance contexts only).  With
 * ASAGA_METHOD_SVRG, `count` iterations, the full-gradient ones included
 * (an epoch is n iterations either way). */
int asaga_updates(asaga_ctx* ctx, int64_t count);

/* f(x) in FP64 (Section 4.1 objective, pairwise-summed).  x_host = NULL
 * evaluates the instance's current iterate; otherwise x_host is double[d].
 * Returns ASAGA_E_DIVERGED if the value is not finite. */
int asaga_objective(asaga_ctx* ctx, int32_t inst, const double* x_host, double* f_out);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * objective of asaga_objective, for a problem held in device memory, with
 * no context and no allocation of any kind.
 *     f(x) = (1/n) sum_i phi(a_i . x; b_i) + (lambda/2) ||x||^2
 * prob: its arrays in device memory (mem = ASAGA_MEM_DEVICE), in the
 *   caller's column order, laid out as asaga_problem says and meeting its
 *   requirements (they are read, not checked: validate them once with
 *   asaga_init if they come from elsewhere); 1 <= n <= ASAGA_NOALLOC_MAX_ROWS.
 * x_dev: double[d] in device memory.  f_dev: one double in device memory,
 *   written by the last kernel (not checked for being finite).
 * stream: a hipStream_t (NULL = null stream); the work is enqueued there and
 *   the call returns without waiting.
 * Scratch: the per-row terms and partial sums go to a static device array
 * of ASAGA_NOALLOC_MAX_ROWS + 1026 doubles (32 MiB), one copy on each GPU
 * the library runs on, held until the process ends and located at the
 * first call on each device.  Every call on a GPU uses that GPU's copy:
 * calls that overlap on one GPU (other streams, other threads) race and
 * must be ordered by the caller.  Nothing in it needs clearing.
 * Errors (nothing enqueued): ASAGA_E_ARG (NULL pointers, mem not DEVICE, n
 * or d out of range, bad enum, lambda not > 0, reserved not 0), ASAGA_E_HIP;
 * the message is available from asaga_last_error(NULL). */
#define ASAGA_NOALLOC_MAX_ROWS 4194304
int asaga_objective_noalloc(const asaga_problem* prob, const double* x_dev, double* f_dev, void* stream);

/* The gradient of the finite sum (Section 1, Eq. finiteSum, with the
 * L2-regularised models of Section 4.1):
 *     grad f(x) = (1/n) sum_i phi'(a_i . x; b_i) a_i + lambda x
 * in FP64 (per-coordinate sums over the rows) into g_host (double[d],
 * caller-owned, in the caller's column order).  x_host as for
 * asaga_objective.  Errors: ASAGA_E_ARG (NULL g_host, inst out of range),
 * ASAGA_E_HIP. */
int asaga_full_grad(asaga_ctx* ctx, int32_t inst, const double* x_host, double* g_host);

/* Copy the instance's iterate x (the x_t of Algorithm 2 after the samples
 * applied so far, read once every enqueued update has finished; FP32 x
 * widened to FP64) into x_host (double[d], caller-owned, in the caller's
 * column order).  Waits for the context's stream.  Errors: ASAGA_E_ARG
 * (NULL x_host, inst out of range), ASAGA_E_HIP, ASAGA_E_DIVERGED (a
 * non-finite gradient change appeared during the updates). */
int asaga_get_x(asaga_ctx* ctx, int32_t inst, double* x_host);

/* What an instance of a context is: its own finite sum of Section 1 over
 * its m training rows, with its lambda and step. */
typedef struct asaga_instance {
    int64_t m;        /* training rows n_k (the length of its alpha)           */
    int64_t t;        /* samples applied so far                                 */
    double lambda;
    double gamma;     /* step size of the next asaga_epochs call (batches: of
                         the last one)                                          */
    double L;         /* smoothness constant of the step-size rule              */
    int32_t fold;     /* held-out fold, -1 for none                             */
    int32_t active;   /* 1 if it takes part in asaga_epochs                     */
} asaga_instance;

/* Fill *out for instance `inst` (host memory, caller-owned).  Errors:
 * ASAGA_E_ARG (NULL context or out, inst out of range). */
int asaga_instance_get(asaga_ctx* ctx, int32_t inst, asaga_instance* out);

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

/* ASAGA_PREC_MIXED and ASAGA_PREC_F32 contexts: widen every instance's
 * state to FP64 (x carried over exactly, alpha into a new FP64 array),
 * recompute abar from alpha as asaga_reanchor does, and continue in FP64
 * from there: the final polish, since FP32 x cannot hold the optimum more
 * closely than its own rounding (and FP32 atomic additions smaller than
 * half an ulp are lost).  The hot set keeps at most the FP64 layout's 5120
 * columns.  The launch shape and the step are kept, except after
 * asaga_autotune chose the largest stable step it probed at its wavefront
 * count: then the polish takes the next smaller step of the tuner's ladder
 * (report.widen_gamma).  The FP64 kernel serves its atomics faster than the
 * FP32 state's, so at the same launch more updates are in flight, and the
 * largest stable step shrinks with them (Theorem 2).  The context stays FP64
 * afterwards; no-op on FP64 contexts. */
int asaga_widen(asaga_ctx* ctx);

/* Choose the number of wavefronts in flight and the step that reach
 * relative suboptimality `target` soonest on this problem (async contexts;
 * the other shape parameters stay as the context has them, except the
 * workgroup size as said below and for batches).
 * Fewer samples in flight tolerate a larger step (Theorem 2) but take longer
 * per epoch, so wavefront counts are tried from one workgroup per compute
 * unit (at most n/64 samples in flight) down to 1/8 wavefront per compute
 * unit, halving.  For each count it times one epoch, then, for steps from
 * the serial rule downwards by factors of 2^(1/3) (to 1/64 of it), runs
 * `probe_epochs` epochs from x = 0 with FP64 objectives and full gradients
 * at three equally spaced checkpoints (a step whose gradient norm does not
 * fall, or whose objective rises, between checkpoints is rejected as
 * unstable, unless the run is already certified), and estimates the epochs to
 * (f - f*)/f* <= `target` by Aitken's extrapolation of the objective (f* and
 * the contraction per epoch from the three values); where the objective
 * gives no estimate, it extrapolates the gradient norm's decay to
 * ||grad f||^2 <= 2 lambda target f, which bounds (f - f*)/f by `target`
 * (f is lambda-strongly convex).  Smaller steps are probed while the
 * estimate improves (a step that fails does not end the search: above the
 * stable steps a short probe can pass by chance); the search ends once a
 * count's probe alone would take four times the best estimate.  Short
 * probes from x = 0 see mostly the early decrease: a step too large for its
 * delay converges fastest there and then hovers at a noise floor, and with
 * FP32 x a small step stalls at the floor FP32 additions leave.  So the
 * finalists (per count its largest and next smaller stable steps and its
 * best-estimated one, at most eight) race from x = 0, checked every
 * probe_epochs / 3 epochs: a finalist finishes when the strong-convexity
 * certificate holds (not the FP32 floor) or, at three checks in a row that
 * agree on it, Aitken's limit of its last three objectives (after three
 * falls of the objective and of the gradient norm, which a run hovering at a
 * noise floor does not show) is within `target` of the last one (with FP32 x: a tenth of `target`, so
 * that a run stalling at its FP32 floor just above it does not count), and
 * drops out once its kernel time reaches the best finished one's, once it
 * makes no new minimum for three checks, or after 40 * probe_epochs epochs.
 * The one finished in the least kernel
 * time is kept, and the report's est_epochs and est_seconds are its
 * measured epochs and kernel time to finish; if none finishes, the one
 * that got lowest is kept, with the epochs it ran and their kernel time.
 * Unless opts.threads_per_block is set, a finished winner then runs once
 * more in workgroups half as large (at least 256 threads: the same
 * wavefronts over twice the compute units, a shorter latency per sample but
 * fewer samples per hot set), timed for one epoch first, and replaces it if
 * it finishes in less kernel time.
 * In the probes, with FP32 x (ASAGA_PREC_MIXED, ASAGA_PREC_F32), a gradient
 * norm at the floor FP32 rounding leaves (8 * 2^-24 * L * ||x||) no longer
 * has to fall, so that stalling there is not taken for instability; it
 * certifies nothing (the objective then decides the estimate); if the pair
 * kept has the largest stable step probed at its count, asaga_widen lowers
 * it one rung (report.widen_gamma).  The best pair is kept, the state is
 * reset to x = alpha = abar = 0, t = 0.  Returns ASAGA_E_DIVERGED if no pair
 * was stable.
 * Batched contexts (opts.step and opts.waves must be 0) get the step law of
 * asaga_epochs, gamma_k = rule_k * min(cap, c / G_k) with at most c / cap
 * lane groups per instance, and the hot-set size (5120 or 1024 columns).
 * c is calibrated on the active instance with the smallest lambda (the
 * slowest, the last one running) alone on the device, running on c lane
 * groups at the full step: c from 512 (the single solve's default law) down
 * the same ladder with the single solve's stability test (with FP32 x, whose
 * rounding floor is reached within a short probe, the largest stable c),
 * then the choice again three times longer, down the ladder until one
 * passes.  The hot-set sizes are ranked by those estimated epochs times one
 * epoch of every active instance under their law.  cap is then the largest of 1, 1/2,
 * 1/4, 1/8 with which no active instance is unstable with all of them
 * running (1 with one active instance: the calibration has run it so), where among many instances unstable means a squared gradient
 * norm that more than doubles between checkpoints or does not decrease from
 * the first to the last (single checkpoints without decrease are noise of
 * the asynchronous updates).  `waves` in the report is per instance with all
 * active instances running, `gamma` instance 0's step then, `step_groups`
 * and `step_cap` the law. */
int asaga_autotune(asaga_ctx* ctx, double target, int32_t probe_epochs, asaga_tune_report* report);

/* Overlap of the asynchronous updates: an estimate of the delay tau of
 * Section 3 (Assumption 1: a read may miss the updates still in flight). */
typedef struct asaga_overlap_report {
    int64_t logged;          /* updates sampled (one in every `every`)                */
    int64_t every;           /* sampling interval                                     */
    double tau_mean;         /* updates in flight at a sampled update's read: mean,   */
    double tau_p50;          /*   median,                                             */
    double tau_p99;          /*   99th percentile                                     */
    double tau_max;          /*   and largest (each a count of sampled updates in     */
                             /*   flight times `every`)                               */
    double latency_mean_us;  /* read to writes visible device-wide, mean              */
    double latency_p99_us;   /*   and 99th percentile                                 */
    double updates_per_s;    /* throughput over the sampled epochs                    */
    double little;           /* updates_per_s * latency_mean: the mean in flight by   */
                             /*   Little's law, a cross-check of tau_mean             */
} asaga_overlap_report;

/* Single-instance async contexts: apply n_epochs epochs (they count as
 * ordinary epochs of the solve) while about one update in 1024, chosen by a
 * hash of its sample counter (independently of which wavefront runs it and
 * when), records the device clock at its read and once its global writes
 * are visible device-wide, then estimate the overlap from those intervals
 * with asaga_overlap_estimate.  Writes combined in a workgroup's LDS become
 * visible at its next flush, later than this clock says: tau counts updates
 * in flight, not that extra delay of hot columns. */
int asaga_overlap(asaga_ctx* ctx, int64_t n_epochs, asaga_overlap_report* report);

/* The estimator of asaga_overlap, on host memory (no device use): `log` holds
 * n_logged (start, end) clock pairs (int64, start <= end) of updates sampled
 * one in `every` from non-overlapping launches; clock_hz is the clock's rate,
 * updates_per_s the throughput.  For each sampled update, the sampled
 * updates that started before its start and end after it are in flight at
 * its read; times `every` that estimates all updates in flight.  Pairs with
 * start = 0 (not written) are skipped. */
int asaga_overlap_estimate(const int64_t* log, int64_t n_logged, int64_t every, double clock_hz,
                           double updates_per_s, asaga_overlap_report* report);

/* Derived numbers (instance 0, plus launch shape). */
int asaga_info_get(asaga_ctx* ctx, asaga_info* out);

/* Wait until all work enqueued by the context has finished. */
int asaga_sync(asaga_ctx* ctx);

/* The sample indices i_t, t = t0 .. t0+count-1, as generated on the device
 * (for cross-checking the stream; needs a GPU). */
int asaga_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out_host);

/* The device's memory-side request ceilings, measured now: the bound on the
 * atomic scatter that Property 3's atomic additions put on the update (the
 * second roofline of the hot path, next to the HBM stream).  Lane pairs add
 * to (mode 1: and read, device-coherently) pseudo-random 16-byte (x, abar)
 * slots of a state of `columns` columns, one memory request per pair and
 * operation, as the update's cold columns do.  *atomic_per_s: requests per
 * second with atomic additions only; *mixed_per_s: with one coherent read
 * and one atomic addition per iteration (the update's mix).  Allocates,
 * uses and frees a device buffer of 16 * columns bytes on a private stream;
 * takes tens of milliseconds.  ASAGA_E_ARG for columns outside
 * [1, 2^27 - 1] or NULL outputs, ASAGA_E_OOM, ASAGA_E_HIP. */
int asaga_request_ceiling(int64_t columns, double* atomic_per_s, double* mixed_per_s);

/* Message of the last failure of ctx (or of the last failed asaga_init* when
 * ctx is NULL).  Never NULL; the pointer is valid until the next call. */
const char* asaga_last_error(const asaga_ctx* ctx);

/* Release the context and its device memory.  NULL is a no-op. */
void asaga_free(asaga_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* ASAGA_H */
