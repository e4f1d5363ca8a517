// C ABI of the gfx950 Sparse SAGA / ASAGA library (declared in asaga.h):
// validation, column relabelling, device memory, the step-size rule,
// launches, read-back in the caller's column order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "asaga.h"
#include "internal.hpp"

using namespace asaga;

namespace {

thread_local std::string g_init_error = "no error";

constexpr int64_t kMaxD = ((int64_t)1 << 27) - 1;
// 32 bytes of LDS per hot column and workgroup: at most 160 KiB, all of a CU's
// LDS (on the RCV1-shaped instance 5120 columns run 6% faster than 4096: 13.6
// instead of 15 cold columns per row)
constexpr int kMaxHot = 5120;
// the FP32 layout keeps 16 bytes per hot column: twice the columns
constexpr int kMaxHotF32 = 10240;
constexpr int kMaxBlock = 1024;  // the update kernels are compiled for at most 1024 threads per workgroup
// Default workgroup (default_block): 512 threads for one solve, 1024 for a
// batch.  1024-thread workgroups share one hot set among twice the samples
// (fewer flush requests per sample: 400 vs 267 M updates/s on the
// RCV1-shaped instance at one workgroup per compute unit) but double the
// samples in flight, which halves the stable step; on a single instance
// whose convergence is step-limited (small lambda) that costs more epochs
// than it saves time, while an instance of a batch only gets the lane
// groups its step law uses at the full step.
// Default asynchronous step: rule * min(1, kStepGroups / G) with G the lane
// groups (samples) in flight.  The stable step falls like 1/G (Theorem 2);
// on the RCV1-shaped instance the edge is near 700 / G (2048 in flight:
// stable at 0.35, 4096: at 0.15, not at 0.19), and 512 / G leaves a margin.
constexpr double kStepGroups = 512.0;
constexpr int64_t kMaxGraphEpochs = 64;  // epochs captured in one hipGraph

struct Inst {
    int fold = -1;            // held-out fold (-1: trains on every row)
    int64_t m = 0;
    int32_t* rows = nullptr;  // device, nullptr = identity
    double lambda = 0.0, gamma = 0.0, L = 0.0;
    double rule = 0.0;        // the serial step rule (or the caller's step)
    bool active = true;       // batched: takes part in asaga_epochs
    int64_t delta_r = 0;
    int32_t cnt_min = 0;
    int32_t* cnt = nullptr;   // relabelled order
    // host: running minimum of cnt over the relabelled order (non-increasing)
    std::shared_ptr<std::vector<int32_t>> cnt_pmin;
    double* D = nullptr;      // relabelled order
    double* xa = nullptr;     // [2d] interleaved x / abar, relabelled order
    void* alpha = nullptr;    // [m]
    uint64_t seed = 0;
    int64_t t = 0;
};

}  // namespace

struct asaga_ctx {
    int64_t n = 0, d = 0, nnz = 0;
    int32_t loss = 0, val_dtype = 0;
    int64_t* rowptr = nullptr;
    const int32_t* colidx_in = nullptr;  // caller's column indices (device)
    int32_t* colidx = nullptr;           // relabelled copy (device, owned)
    int32_t* rank = nullptr;             // [d] caller's column -> internal column
    void* val = nullptr;
    double* b = nullptr;
    asaga_opts o{};
    hipStream_t st = nullptr;
    bool mixed = false;          // FP32 x and alpha (mixed and FP32 layouts)
    int layout = kLayF64;        // kLay*: the state layout of ASAGA_PREC_*
    double widen_gamma = 0.0;    // step asaga_widen switches to (0: keep the step)
    bool svrg = false;           // ASAGA_METHOD_SVRG
    UpdateShape shape{};
    std::vector<Inst> inst;
    InstArgs* d_insts = nullptr;
    BlockMap* d_map = nullptr;   // batched: workgroup -> (instance, rank)
    int64_t map_cap = 0;
    // host copies of the last batched plan (kept until the next call, which
    // first waits for the stream, so that the copies from them have ended)
    std::vector<InstArgs> plan_h;
    std::vector<BlockMap> plan_map;
    // batched step law: gamma_k = rule_k * min(step_cap, step_groups / G_k),
    // G_k the lane groups serving instance k (0: not calibrated, use
    // kStepGroups, the single-instance default)
    double step_groups = 0.0, step_cap = 1.0;
    // batched stop test (asaga_set_stop): per-instance thresholds, the proxy
    // after the last epoch each instance ran, the epochs each ran in a call
    // (device), and the last call's copies (host)
    bool stop_on = false;
    double* d_stop_thr = nullptr;
    double* d_proxy = nullptr;
    int32_t* d_ran = nullptr;
    std::vector<double> proxy_h;
    std::vector<int64_t> ran_h;
    // batched: captured epochs, keyed by epochs per replay, tier interval,
    // grid and whether the stop test follows each epoch
    hipStream_t cap = nullptr;
    struct Captured {
        int64_t epochs;
        int tier_every, hot, tier;
        int n_blocks;
        const void* map;
        bool stop;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Captured> graphs;
    std::vector<void*> allocs;
    // scratch
    double* z = nullptr;      // [n]
    double* tmp = nullptr;    // [n]
    double* vec1 = nullptr;   // [d]
    double* vec2 = nullptr;   // [d]
    long long* d_tau = nullptr;  // single instance: overlap log of (start, end) tick pairs
    unsigned long long* d_tau_count = nullptr;
    int64_t tau_cap = 0;         // pairs d_tau holds: twice the expected number per epoch, plus 64
    bool tau_on = false;         // asaga_overlap is logging
    double* part = nullptr;   // [kSumParts]
    double* scal = nullptr;   // [4]
    int* flag = nullptr;      // [1]
    int32_t* stats = nullptr; // [2]
    unsigned long long* maxbits = nullptr;
    std::string err = "no error";
};

namespace {

int fail(asaga_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

// On failure the runtime's last-error state is cleared too, so that a later
// launch does not report this failure as its own.
#define HIPCHK(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? ASAGA_E_OOM : ASAGA_E_HIP,              \
                        std::string(#call) + ": " + hipGetErrorString(e_));                        \
        }                                                                                          \
    } while (0)

template <typename T>
int dalloc(asaga_ctx* c, T** p, int64_t count) {
    void* q = nullptr;
    const size_t bytes = (size_t)(count > 0 ? count : 1) * sizeof(T);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, e == hipErrorOutOfMemory ? ASAGA_E_OOM : ASAGA_E_HIP,
                    "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    c->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return ASAGA_OK;
}

size_t val_size(int32_t dt) { return dt == ASAGA_VAL_F64 ? 8 : dt == ASAGA_VAL_F32 ? 4 : 2; }

double host_val(const void* v, int32_t dt, int64_t k) {
    if (dt == ASAGA_VAL_F64) return static_cast<const double*>(v)[k];
    if (dt == ASAGA_VAL_F32) return static_cast<const float*>(v)[k];
    uint32_t bits = (uint32_t) static_cast<const uint16_t*>(v)[k] << 16;
    float f;
    std::memcpy(&f, &bits, 4);
    return f;
}

// Host-side checks of a problem in host memory (before any device work).
int validate_host(const asaga_problem* p) {
    const int64_t n = p->n, d = p->d;
    if (p->rowptr[0] != 0) return fail(nullptr, ASAGA_E_CSR, "rowptr[0] != 0");
    const int64_t nnz = p->rowptr[n];
    if (nnz < n) return fail(nullptr, ASAGA_E_CSR, "rowptr[n] < n: some row is empty");
    if (nnz > (int64_t)1 << 40) return fail(nullptr, ASAGA_E_CSR, "nnz too large");
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s = p->rowptr[i], e = p->rowptr[i + 1];
        if (e < s || e > nnz) return fail(nullptr, ASAGA_E_CSR, "rowptr decreasing at row " + std::to_string(i));
        if (e == s) return fail(nullptr, ASAGA_E_CSR, "row " + std::to_string(i) + " is empty");
        int64_t prev = -1;
        for (int64_t k = s; k < e; ++k) {
            const int64_t c = p->colidx[k];
            if (c < 0 || c >= d) return fail(nullptr, ASAGA_E_CSR, "column index out of range in row " + std::to_string(i));
            if (c <= prev)
                return fail(nullptr, ASAGA_E_CSR, "columns not strictly increasing in row " + std::to_string(i));
            prev = c;
            if (!std::isfinite(host_val(p->val, p->val_dtype, k)))
                return fail(nullptr, ASAGA_E_CSR, "non-finite value in row " + std::to_string(i));
        }
        const double b = p->b[i];
        if (!std::isfinite(b)) return fail(nullptr, ASAGA_E_CSR, "non-finite label at row " + std::to_string(i));
        if (p->loss == ASAGA_LOSS_LOGISTIC && b != 1.0 && b != -1.0)
            return fail(nullptr, ASAGA_E_CSR, "logistic label not in {-1,+1} at row " + std::to_string(i));
    }
    return ASAGA_OK;
}

int check_args(const asaga_problem* p, const asaga_opts* o) {
    if (!p || !o) return fail(nullptr, ASAGA_E_ARG, "NULL problem or options");
    if (p->n < 1 || p->d < 1 || p->n > INT32_MAX)
        return fail(nullptr, ASAGA_E_ARG, "n must be in [1, 2^31) and d >= 1");
    if (p->d > kMaxD) return fail(nullptr, ASAGA_E_ARG, "d must be at most 2^27 - 1 (16-byte state slots, 32-bit offsets)");
    if (!p->rowptr || !p->colidx || !p->val || !p->b) return fail(nullptr, ASAGA_E_ARG, "NULL problem array");
    if (p->val_dtype < ASAGA_VAL_F64 || p->val_dtype > ASAGA_VAL_BF16)
        return fail(nullptr, ASAGA_E_ARG, "bad val_dtype");
    if (p->loss != ASAGA_LOSS_LOGISTIC && p->loss != ASAGA_LOSS_SQUARED) return fail(nullptr, ASAGA_E_ARG, "bad loss");
    if (p->mem != ASAGA_MEM_HOST && p->mem != ASAGA_MEM_DEVICE) return fail(nullptr, ASAGA_E_ARG, "bad mem");
    if (p->reserved != 0) return fail(nullptr, ASAGA_E_ARG, "problem.reserved must be 0");
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return fail(nullptr, ASAGA_E_ARG, "lambda must be > 0 and finite");
    if (o->mode != ASAGA_MODE_SERIAL && o->mode != ASAGA_MODE_ASYNC) return fail(nullptr, ASAGA_E_ARG, "bad mode");
    if (o->precision != ASAGA_PREC_F64 && o->precision != ASAGA_PREC_MIXED && o->precision != ASAGA_PREC_F32)
        return fail(nullptr, ASAGA_E_ARG, "bad precision");
    const int max_hot = o->precision == ASAGA_PREC_F32 ? kMaxHotF32 : kMaxHot;
    const std::string hot_range = "-1, 0 or in [1, " + std::to_string(max_hot) + "]";
    if (!std::isfinite(o->step)) return fail(nullptr, ASAGA_E_ARG, "step must be finite");
    if (o->waves < 0 || o->waves > (1 << 20)) return fail(nullptr, ASAGA_E_ARG, "waves out of range");
    if (o->lanes_per_sample != 0 && o->lanes_per_sample != 8 && o->lanes_per_sample != 16 &&
        o->lanes_per_sample != 32 && o->lanes_per_sample != 64)
        return fail(nullptr, ASAGA_E_ARG, "lanes_per_sample must be 0, 8, 16, 32 or 64");
    if (o->racy != 0 && o->racy != 1) return fail(nullptr, ASAGA_E_ARG, "racy must be 0 or 1");
    if (o->racy && o->mode != ASAGA_MODE_ASYNC) return fail(nullptr, ASAGA_E_ARG, "racy applies to async mode only");
    if (o->hot_columns < -1 || o->hot_columns > max_hot)
        return fail(nullptr, ASAGA_E_ARG, "hot_columns must be " + hot_range);
    if (o->flush_every < 0 || o->flush_every > (1 << 20)) return fail(nullptr, ASAGA_E_ARG, "flush_every out of range");
    if (o->hot_tier_columns < -1 || o->hot_tier_columns > max_hot)
        return fail(nullptr, ASAGA_E_ARG, "hot_tier_columns must be " + hot_range);
    if (o->hot_tier_every < 0 || o->hot_tier_every > (1 << 16))
        return fail(nullptr, ASAGA_E_ARG, "hot_tier_every out of range");
    if (o->threads_per_block < 0 || o->threads_per_block > kMaxBlock || o->threads_per_block % 64 != 0)
        return fail(nullptr, ASAGA_E_ARG, "threads_per_block must be 0 or a multiple of 64 up to 1024");
    if (o->plain_launch != 0 && o->plain_launch != 1) return fail(nullptr, ASAGA_E_ARG, "plain_launch must be 0 or 1");
    if (o->method != ASAGA_METHOD_SAGA && o->method != ASAGA_METHOD_SVRG)
        return fail(nullptr, ASAGA_E_ARG, "bad method");
    if (o->method == ASAGA_METHOD_SVRG && o->racy) return fail(nullptr, ASAGA_E_ARG, "racy applies to SAGA only");
    if (o->hot_reload_from < -1 || o->hot_reload_from > max_hot)
        return fail(nullptr, ASAGA_E_ARG, "hot_reload_from must be " + hot_range);
    if (o->reserved != 0) return fail(nullptr, ASAGA_E_ARG, "opts.reserved must be 0");
    return ASAGA_OK;
}

MatArgs mat(const asaga_ctx* c, bool relabelled = true) {
    MatArgs A;
    A.rowptr = c->rowptr;
    A.colidx = relabelled ? c->colidx : c->colidx_in;
    A.val = c->val;
    A.b = c->b;
    A.n = c->n;
    A.d = c->d;
    A.val_dtype = c->val_dtype;
    A.loss = c->loss;
    return A;
}

InstArgs inst_args(const Inst& I, uint64_t t0, uint64_t count) {
    InstArgs a;
    a.rows = I.rows;
    a.xa = I.xa;
    a.alpha = I.alpha;
    a.D = I.D;
    a.m = I.m;
    a.gamma = I.gamma;
    a.lambda = I.lambda;
    a.inv_m = 1.0 / (double)I.m;
    a.seed = I.seed;
    a.t0 = t0;
    a.count = count;
    a.blocks = 0;
    a.frozen = 0;
    a.reload_from = kNoReload;
    a.tau_log = nullptr;
    a.tau_count = nullptr;
    a.tau_cap = 0;
    return a;
}

// views of an instance's state in the relabelled order
XView x_view(const asaga_ctx* c, const Inst& I) {
    if (c->layout == kLayF32) return XView{I.xa, 2, 1};
    return c->layout == kLayMixed ? XView{I.xa, 4, 1} : XView{I.xa, 2, 0};
}
XView abar_view(const asaga_ctx* c, const Inst& I) {
    if (c->layout == kLayF32) return XView{reinterpret_cast<float*>(I.xa) + 1, 2, 1};
    return XView{I.xa + 1, 2, 0};
}

int max_hot(const asaga_ctx* c) { return c->layout == kLayF32 ? kMaxHotF32 : kMaxHot; }

// abar = (1/m) sum_j alpha_j a_j from the stored memory, in FP64 (rounded
// once to FP32 in the FP32 layout)
int recompute_abar(asaga_ctx* c, const Inst& I) {
    const MatArgs A = mat(c);
    HIPCHK(c, launch_alpha_coef(I.alpha, c->mixed, I.m, 1.0 / (double)I.m, c->tmp, c->st));
    if (c->layout == kLayF32) {
        HIPCHK(c, launch_fill_f64(c->vec2, 0.0, c->d, 1, c->st));
        HIPCHK(c, launch_scatter(A, I.rows, I.m, c->tmp, c->vec2, 1, c->st));
        HIPCHK(c, launch_store_slots(c->vec2, c->d, reinterpret_cast<float*>(I.xa) + 1, 2, true, c->st));
    } else {
        HIPCHK(c, launch_fill_f64(I.xa + 1, 0.0, c->d, 2, c->st));
        HIPCHK(c, launch_scatter(A, I.rows, I.m, c->tmp, I.xa + 1, 2, c->st));
    }
    return ASAGA_OK;
}

// ---- sparse SVRG (Appendix C): randomly timed, synchronised snapshots ----

// host copy of the sample-stream map (SplitMix64 of Steele, Lea & Flood
// 2014, Lemire's multiply-high to [0, n)), for the full-gradient decisions
uint64_t host_splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint64_t kSvrgTag = 0xA5A5A5A5A5A5A5A5ull;

// U_t: whether iteration t of an SVRG run takes a full gradient
bool svrg_full_gradient_due(uint64_t seed, uint64_t t, int64_t m) {
    return (uint64_t)(((unsigned __int128)host_splitmix64(seed ^ kSvrgTag, t) * (uint64_t)m) >> 64) == 0;
}

// The snapshot at the current x: alpha_j = phi'(a_j . x), abar = (1/m) sum alpha_j a_j.
int svrg_snapshot(asaga_ctx* c, Inst& I) {
    const MatArgs A = mat(c);
    HIPCHK(c, launch_rowdot(A, I.rows, I.m, x_view(c, I), c->z, c->st));
    if (c->mixed) {
        HIPCHK(c, launch_dphi_coef(A, I.rows, I.m, c->z, 1.0, c->tmp, c->st));
        HIPCHK(c, launch_narrow_f64(c->tmp, I.m, static_cast<float*>(I.alpha), c->st));
    } else {
        HIPCHK(c, launch_dphi_coef(A, I.rows, I.m, c->z, 1.0, static_cast<double*>(I.alpha), c->st));
    }
    // abar from the stored memory (so that it is the exact average of what steps read)
    return recompute_abar(c, I);
}

int zero_state(asaga_ctx* c, Inst& I) {
    HIPCHK(c, launch_fill_f64(I.xa, 0.0, 2 * c->d, 1, c->st));
    if (c->mixed) HIPCHK(c, launch_fill_f32(static_cast<float*>(I.alpha), 0.0f, I.m, c->st));
    else HIPCHK(c, launch_fill_f64(static_cast<double*>(I.alpha), 0.0, I.m, 1, c->st));
    I.t = 0;
    // SVRG starts from a snapshot at x0 = 0
    if (c->svrg) return svrg_snapshot(c, I);
    return ASAGA_OK;
}

// Relabel columns by descending count over all rows (ties: lower index first).
int relabel_columns(asaga_ctx* c) {
    int rc;
    int32_t* cnt = nullptr;
    if ((rc = dalloc(c, &cnt, c->d))) return rc;
    if ((rc = dalloc(c, &c->rank, c->d))) return rc;
    if ((rc = dalloc(c, &c->colidx, c->nnz))) return rc;
    HIPCHK(c, launch_fill_i32(cnt, 0, c->d, c->st));
    HIPCHK(c, launch_colcount(mat(c, false), nullptr, c->n, cnt, false, c->st));
    std::vector<int32_t> h(c->d);
    HIPCHK(c, hipMemcpyAsync(h.data(), cnt, c->d * 4, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<int32_t> order(c->d);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return h[a] > h[b]; });
    // Past the largest hot set the layout allows, the cold columns follow in
    // a fixed pseudo-random order (Fisher-Yates with a 64-bit LCG): sorted,
    // the most-used cold columns would share a few stretches of the state,
    // and their memory-side requests spread better scattered (3.6% shorter
    // epochs on the RCV1-shaped instance).  The hot-set prefix stays sorted
    // by count, as the hot-set size rules assume.
    const int64_t keep = max_hot(c);
    uint64_t lcg = 0x243F6A8885A308D3ull;
    for (int64_t r = c->d - 1; r > keep; --r) {
        lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
        const int64_t j = keep + (int64_t)((lcg >> 33) % (uint64_t)(r - keep + 1));
        std::swap(order[r], order[j]);
    }
    std::vector<int32_t> rank(c->d);
    for (int64_t r = 0; r < c->d; ++r) rank[order[r]] = (int32_t)r;
    HIPCHK(c, hipMemcpyAsync(c->rank, rank.data(), c->d * 4, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, launch_relabel(c->colidx_in, c->nnz, c->rank, c->colidx, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return ASAGA_OK;
}

// Column counts, D, Delta_r, L and gamma of one instance; zero its state.
// An instance that trains on the same rows as an earlier one (same held-out
// fold) shares that instance's counts, D and L.
int setup_instance(asaga_ctx* c, Inst& I, const Inst* same_rows) {
    int rc;
    if ((rc = dalloc(c, &I.xa, 2 * c->d))) return rc;
    char* ap = nullptr;
    if ((rc = dalloc(c, &ap, I.m * (int64_t)(c->mixed ? 4 : 8)))) return rc;
    I.alpha = ap;
    int32_t stats[2] = {0, 0x7fffffff};
    if (same_rows) {
        I.cnt = same_rows->cnt;
        I.cnt_pmin = same_rows->cnt_pmin;
        I.D = same_rows->D;
        I.delta_r = same_rows->delta_r;
        I.cnt_min = same_rows->cnt_min;
        I.L = same_rows->L - same_rows->lambda + I.lambda;
        stats[0] = (int32_t)I.delta_r;
        stats[1] = I.cnt_min;
    } else {
        if ((rc = dalloc(c, &I.cnt, c->d))) return rc;
        if ((rc = dalloc(c, &I.D, c->d))) return rc;
        const MatArgs A = mat(c);
        HIPCHK(c, launch_fill_i32(I.cnt, 0, c->d, c->st));
        HIPCHK(c, launch_colcount(A, I.rows, I.m, I.cnt, true, c->st));
        HIPCHK(c, hipMemcpyAsync(c->stats, stats, sizeof(stats), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, launch_reweight(I.cnt, c->d, I.m, I.D, c->stats, c->st));
        unsigned long long bits = 0;
        HIPCHK(c, hipMemcpyAsync(c->maxbits, &bits, sizeof(bits), hipMemcpyHostToDevice, c->st));
        HIPCHK(c, launch_rownorm_max(A, I.rows, I.m, c->maxbits, c->st));
        HIPCHK(c, hipMemcpyAsync(stats, c->stats, sizeof(stats), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipMemcpyAsync(&bits, c->maxbits, sizeof(bits), hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        double maxnorm;
        std::memcpy(&maxnorm, &bits, 8);
        auto pm = std::make_shared<std::vector<int32_t>>(c->d);
        HIPCHK(c, hipMemcpy(pm->data(), I.cnt, c->d * 4, hipMemcpyDeviceToHost));
        for (int64_t v = 1; v < c->d; ++v) (*pm)[v] = std::min((*pm)[v], (*pm)[v - 1]);
        I.cnt_pmin = pm;
        I.delta_r = stats[0];
        I.cnt_min = stats[1];
        I.L = (c->loss == ASAGA_LOSS_LOGISTIC ? 0.25 : 1.0) * maxnorm + I.lambda;
    }
    if (c->o.step > 0.0) {
        I.gamma = c->o.step;
        I.rule = c->o.step;
    } else {
        // gamma = min(1/(3L), 1/(lambda max_v D_v)); max_v D_v = m / min positive count
        const double dmax = stats[1] > 0 && stats[1] != 0x7fffffff ? (double)I.m / (double)stats[1] : 0.0;
        double g = 1.0 / (3.0 * I.L);
        if (I.lambda * dmax > 0.0 && 1.0 / (I.lambda * dmax) < g) g = 1.0 / (I.lambda * dmax);
        I.rule = g;
        // asynchronous: scaled to the samples in flight once the launch
        // shape is known (default_async_steps)
        I.gamma = g;
    }
    return zero_state(c, I);
}

// Automatic launch shapes keep the samples in flight for an instance at
// most m/64 (at least one workgroup): the analysis of Section 3 assumes a
// delay small against the number of samples, and well beyond that a short
// probe can no longer tell a stable step from a slowly diverging one.
int64_t max_groups_for(int64_t m) { return std::max<int64_t>(1, m / 64); }

// Automatic workgroup size.  One solve: 512 threads (a 1024-thread workgroup
// shares one hot set and one flush among twice the samples, +52% updates/s
// on the RCV1-shaped matrix, but doubles the samples in flight, and on the
// lambda path the halved stable step costs more epochs than that saves).  A
// batch: 1024, since each instance gets only the lane groups its step law
// can use at the full step (the lambda path x folds batch of 160 instances
// reaches 1e-9 in 6.3-6.6 s instead of 8.3-9.7 s with 512).
int default_block(const asaga_opts& o, bool batched) {
    if (o.threads_per_block > 0) return o.threads_per_block;
    return batched ? 1024 : 512;
}

// A workgroup's LDS view of hot column v is refreshed when the workgroup
// next writes v, so the column's regulariser step gamma lambda D_v x_v reads
// a value about one of v's own updates old per workgroup serving the
// instance (whatever v's count).  The hot set keeps only the leading columns
// with gamma lambda D_v * workgroups <= 0.2 (D_v = m / cnt_v); the others
// are read and written in global memory, where they are current.  (Measured
// on the 560,000-row lambda-path instance at lambda = 4.8e-5 with 256
// workgroups: 0.25 converges as fast as no hot set, 0.52 oscillates at
// 1e-4.)  The caller's explicit hot_columns is kept as given.
int stable_hot(const asaga_ctx* c, const Inst& I, int hot, double workgroups) {
    if (c->o.hot_columns != 0 || hot <= 0 || !I.cnt_pmin) return hot;
    const double gl = I.gamma * I.lambda * workgroups;
    if (!(gl > 0.0)) return hot;
    const double need = (double)I.m * gl / 0.2;  // cnt_v >= m gamma lambda W / 0.2
    const auto& pm = *I.cnt_pmin;
    // pm is non-increasing: count the leading columns with pm[v] >= need
    int64_t lo = 0, hi = std::min<int64_t>(hot, (int64_t)pm.size());
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((double)pm[mid] >= need) lo = mid + 1;
        else hi = mid;
    }
    return (int)lo;
}

// The first hot column whose LDS view a workgroup reloads at each full
// flush.  A workgroup refreshes its view of a hot column when it writes the
// column, about once in 1/(p_v s) rounds for a column of probability p_v (s
// samples per round), while the W workgroups serving the instance apply
// about W of its updates: the view lags by about W D_v samples (D_v = m /
// cnt_v), and the data term's step reads it.  Measured on the RCV1-shaped
// matrix, hot set of 4096 columns (D_v up to about 600), with rule = 1/(3L):
// (gamma / rule) W D_v = 0.25 * 256 * 593 = 3.8e4 converges like no hot set;
// 1.0 * 128 * 593 = 7.6e4 (a lambda = 1e-8 instance of the lambda path)
// stalls near 2e-3 until those views are reloaded.  Columns with
// (gamma / rule) W D_v above 4.8e4 are reloaded; the reload costs one memory
// request per 4 columns and flush.
constexpr double kViewLag = 49152.0;

int view_reload_from(const asaga_ctx* c, const Inst& I, int hot, double workgroups) {
    if (hot <= 0) return kNoReload;
    if (c->o.hot_reload_from > 0) return c->o.hot_reload_from < hot ? c->o.hot_reload_from : kNoReload;
    // serial mode: the only workgroup's views never lag
    if (c->o.hot_reload_from < 0 || c->shape.serial) return kNoReload;
    if (!I.cnt_pmin || !(I.L > 0.0)) return kNoReload;
    const double s = I.gamma * 3.0 * I.L * workgroups;  // (gamma / (1 / 3L)) W
    if (!(s > 0.0)) return kNoReload;
    const double need = (double)I.m * s / kViewLag;  // reload the columns with cnt_v < need
    const auto& pm = *I.cnt_pmin;
    int64_t lo = 0, hi = std::min<int64_t>(hot, (int64_t)pm.size());
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if ((double)pm[mid] >= need) lo = mid + 1;
        else hi = mid;
    }
    return lo < hot ? (int)lo : kNoReload;
}

// Rounds between flushes of the second hot tier.  A column of that tier is
// seen by other workgroups up to tier_every * G samples late (G lane groups
// in flight), and its regulariser step gamma lambda D_v x_v, applied on
// 1/D_v of the samples, then lags by gamma lambda tier_every G in units of
// its own decay: kept below 0.05 here, so that large-lambda instances
// flush that tier more often (the caller's hot_tier_every, if set, wins).
int tier_every_from(const asaga_ctx* c, double gamma_lambda_groups) {
    if (c->o.hot_tier_every > 0) return c->o.hot_tier_every;
    const double v = gamma_lambda_groups > 0.0 ? 0.05 / gamma_lambda_groups : 16.0;
    return (int)std::max(1.0, std::min(16.0, std::floor(v)));
}

int tier_every_for(const asaga_ctx* c, const UpdateShape& S) {
    double gl = 0.0;
    for (const Inst& I : c->inst)
        if (I.active) gl = std::max(gl, I.gamma * I.lambda);
    return tier_every_from(c, gl * (double)S.waves * (64.0 / (double)S.lanes));
}

// lane groups (samples) in flight of a single-instance launch shape
double groups_in_flight(const UpdateShape& S) { return (double)S.waves * (64.0 / (double)S.lanes); }

// Without opts.step, an asynchronous single instance starts from
// rule * min(1, kStepGroups / G); batches get theirs per launch.
void default_async_steps(asaga_ctx* c) {
    if (c->o.step > 0.0 || c->shape.serial || c->d_insts) return;
    for (Inst& I : c->inst) I.gamma = I.rule * std::min(1.0, kStepGroups / groups_in_flight(c->shape));
}

void pick_shape(asaga_ctx* c) {
    UpdateShape& S = c->shape;
    S.serial = c->o.mode == ASAGA_MODE_SERIAL;
    S.racy = c->o.racy != 0;
    S.layout = c->layout;
    if (S.serial) {
        // one lane group applies the samples in order; the options choose
        // which of the asynchronous kernel's paths it runs through
        S.lanes = c->o.lanes_per_sample > 0 ? c->o.lanes_per_sample : 64;
        S.block = c->o.threads_per_block > 0 ? c->o.threads_per_block : 64;
        S.block = std::max(S.block, S.lanes);
        S.waves = S.block / 64;
        S.hot = c->o.hot_columns > 0 ? (int)std::min<int64_t>(c->o.hot_columns, c->d) : 0;
        S.flush = c->o.flush_every > 0 ? c->o.flush_every : 1;
        const int tier = c->o.hot_tier_columns == 0 ? 256 : c->o.hot_tier_columns < 0 ? S.hot : c->o.hot_tier_columns;
        S.tier = std::min(tier, S.hot);
        S.tier_every = c->o.hot_tier_every > 0 ? c->o.hot_tier_every : 16;
        return;
    }
    const double mean = (double)c->nnz / (double)c->n;
    int lanes = c->o.lanes_per_sample;
    if (lanes == 0) {
        // about one lane pair per row entry, within [8, 64] lanes
        int p = 8;
        while (p < 64 && p < mean) p *= 2;
        lanes = p;
    }
    S.lanes = lanes;
    S.block = default_block(c->o, c->d_insts != nullptr);
    int waves = c->o.waves;
    if (waves == 0) {
        int cus = device_cu_count();
        if (cus <= 0) cus = 256;
        // one instance: one 16-wavefront workgroup per compute unit, within
        // the bound on samples in flight; a batch: planned per launch (64 per
        // instance is only reported until then)
        waves = c->d_insts ? 64
                           : (int)std::min<int64_t>(cus * (S.block / 64),
                                                    std::max<int64_t>(1, max_groups_for(c->n) * lanes / 64));
    }
    const int wpb = S.block / 64;
    S.waves = ((waves + wpb - 1) / wpb) * wpb;
    int hot = c->o.hot_columns;
    if (hot == 0) hot = max_hot(c);
    if (hot < 0 || S.racy) hot = 0;
    S.hot = (int)std::min<int64_t>(hot, c->d);
    S.flush = c->o.flush_every > 0 ? c->o.flush_every : 1;
    // first tier: the 256 most-used columns, flushed every round; the rest of
    // the hot set every 16 rounds
    const int tier = c->o.hot_tier_columns == 0 ? 256 : c->o.hot_tier_columns < 0 ? S.hot : c->o.hot_tier_columns;
    S.tier = std::min(tier, S.hot);
    S.tier_every = tier_every_for(c, S);
}

void drop_graphs(asaga_ctx* c) {
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

int free_all(asaga_ctx* c) {
    if (!c) return ASAGA_OK;
    if (c->st) (void)hipStreamSynchronize(c->st);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    c->cap = nullptr;
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    return ASAGA_OK;
}

int check_flag(asaga_ctx* c) {
    int f = 0;
    HIPCHK(c, hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (f) return fail(c, ASAGA_E_DIVERGED, "a non-finite gradient change appeared during the updates");
    return ASAGA_OK;
}

int init_common(asaga_ctx** out, const asaga_problem* p, const asaga_opts* o, const asaga_batch* bt) {
    if (!out) return fail(nullptr, ASAGA_E_ARG, "NULL output pointer");
    *out = nullptr;
    int rc = check_args(p, o);
    if (rc) return rc;
    if (bt) {
        if (bt->n_inst < 1 || bt->n_inst > 65536 || !bt->inst_fold || !bt->inst_lambda || bt->reserved != 0)
            return fail(nullptr, ASAGA_E_ARG, "bad batch descriptor");
        if (o->racy) return fail(nullptr, ASAGA_E_ARG, "racy is not available for batched solves");
        if (o->method != ASAGA_METHOD_SAGA) return fail(nullptr, ASAGA_E_ARG, "batched solves run Sparse SAGA");
        for (int k = 0; k < bt->n_inst; ++k) {
            if (!(bt->inst_lambda[k] > 0.0) || !std::isfinite(bt->inst_lambda[k]))
                return fail(nullptr, ASAGA_E_ARG, "instance lambda must be > 0 and finite");
            if (bt->inst_fold[k] < -1 || bt->inst_fold[k] > 127) return fail(nullptr, ASAGA_E_ARG, "bad inst_fold");
            if (bt->inst_fold[k] >= 0 && !bt->row_fold) return fail(nullptr, ASAGA_E_ARG, "row_fold is NULL");
        }
    }
    if (p->mem == ASAGA_MEM_HOST) {
        rc = validate_host(p);
        if (rc) return rc;
    }

    asaga_ctx* c = new (std::nothrow) asaga_ctx();
    if (!c) return fail(nullptr, ASAGA_E_OOM, "host allocation failed");
    c->o = *o;
    c->st = static_cast<hipStream_t>(o->stream);
    c->n = p->n;
    c->d = p->d;
    c->loss = p->loss;
    c->val_dtype = p->val_dtype;
    c->layout = o->precision == ASAGA_PREC_MIXED ? kLayMixed : o->precision == ASAGA_PREC_F32 ? kLayF32 : kLayF64;
    c->mixed = c->layout != kLayF64;
    c->svrg = o->method == ASAGA_METHOD_SVRG;

    auto bail = [&](int code) {
        std::string msg = c->err;
        free_all(c);
        delete c;
        g_init_error = msg;
        return code;
    };
    auto step = [&](auto&& fn) -> int { return fn(); };

    // problem arrays
    if (p->mem == ASAGA_MEM_HOST) {
        c->nnz = p->rowptr[p->n];
        int32_t* ci = nullptr;
        if ((rc = dalloc(c, &c->rowptr, c->n + 1))) return bail(rc);
        if ((rc = dalloc(c, &ci, c->nnz))) return bail(rc);
        c->colidx_in = ci;
        char* vp = nullptr;
        if ((rc = dalloc(c, &vp, c->nnz * (int64_t)val_size(c->val_dtype)))) return bail(rc);
        c->val = vp;
        if ((rc = dalloc(c, &c->b, c->n))) return bail(rc);
        if ((rc = step([&]() -> int {
                 HIPCHK(c, hipMemcpyAsync(c->rowptr, p->rowptr, (c->n + 1) * 8, hipMemcpyHostToDevice, c->st));
                 HIPCHK(c, hipMemcpyAsync(ci, p->colidx, c->nnz * 4, hipMemcpyHostToDevice, c->st));
                 HIPCHK(c, hipMemcpyAsync(c->val, p->val, c->nnz * val_size(c->val_dtype), hipMemcpyHostToDevice, c->st));
                 HIPCHK(c, hipMemcpyAsync(c->b, p->b, c->n * 8, hipMemcpyHostToDevice, c->st));
                 HIPCHK(c, hipStreamSynchronize(c->st));
                 return ASAGA_OK;
             })))
            return bail(rc);
    } else {
        c->rowptr = const_cast<int64_t*>(p->rowptr);
        c->colidx_in = p->colidx;
        c->val = const_cast<void*>(p->val);
        c->b = const_cast<double*>(p->b);
    }

    // scratch
    if ((rc = dalloc(c, &c->flag, 1))) return bail(rc);
    if ((rc = dalloc(c, &c->stats, 2))) return bail(rc);
    if ((rc = dalloc(c, &c->maxbits, 1))) return bail(rc);
    if ((rc = dalloc(c, &c->part, kSumParts))) return bail(rc);
    if ((rc = dalloc(c, &c->scal, 4))) return bail(rc);
    if ((rc = dalloc(c, &c->z, c->n))) return bail(rc);
    if ((rc = dalloc(c, &c->tmp, c->n))) return bail(rc);
    if ((rc = dalloc(c, &c->vec1, c->d))) return bail(rc);
    if ((rc = dalloc(c, &c->vec2, c->d))) return bail(rc);
    if ((rc = step([&]() -> int {
             HIPCHK(c, launch_fill_i32(c->flag, 0, 1, c->st));
             return ASAGA_OK;
         })))
        return bail(rc);

    if (p->mem == ASAGA_MEM_DEVICE) {
        // nnz from the device rowptr, then a device-side validation pass
        int64_t ends[2];
        if ((rc = step([&]() -> int {
                 HIPCHK(c, hipMemcpyAsync(&ends[0], c->rowptr, 8, hipMemcpyDeviceToHost, c->st));
                 HIPCHK(c, hipMemcpyAsync(&ends[1], c->rowptr + c->n, 8, hipMemcpyDeviceToHost, c->st));
                 HIPCHK(c, hipStreamSynchronize(c->st));
                 return ASAGA_OK;
             })))
            return bail(rc);
        if (ends[0] != 0 || ends[1] < c->n || ends[1] > ((int64_t)1 << 40)) {
            c->err = "rowptr[0] != 0 or rowptr[n] out of range";
            return bail(ASAGA_E_CSR);
        }
        c->nnz = ends[1];
        int32_t bad = 0;
        if ((rc = step([&]() -> int {
                 HIPCHK(c, launch_fill_i32(c->stats, 0, 1, c->st));
                 HIPCHK(c, launch_validate(mat(c, false), c->nnz, c->stats, c->st));
                 HIPCHK(c, hipMemcpyAsync(&bad, c->stats, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
                 HIPCHK(c, hipStreamSynchronize(c->st));
                 return ASAGA_OK;
             })))
            return bail(rc);
        if (bad) {
            c->err = "device CSR validation failed (flags " + std::to_string(bad) +
                     ": 1 rowptr, 2 empty row, 4 column range, 8 column order, 16 value, 32 label)";
            return bail(ASAGA_E_CSR);
        }
    }

    if ((rc = relabel_columns(c))) return bail(rc);

    // instances
    if (!bt) {
        Inst I;
        I.m = c->n;
        I.lambda = p->lambda;
        I.seed = o->seed;
        c->inst.push_back(I);
    } else {
        std::vector<int32_t> rows;
        for (int k = 0; k < bt->n_inst; ++k) {
            Inst I;
            I.lambda = bt->inst_lambda[k];
            I.seed = o->seed + (uint64_t)k;
            const int f = bt->inst_fold[k];
            I.fold = f;
            const Inst* same = nullptr;
            for (const Inst& J : c->inst)
                if (J.fold == f) same = &J;
            if (same) {
                I.m = same->m;
                I.rows = same->rows;
            } else if (f < 0) {
                I.m = c->n;
            } else {
                rows.clear();
                for (int64_t i = 0; i < c->n; ++i)
                    if (bt->row_fold[i] != f) rows.push_back((int32_t)i);
                I.m = (int64_t)rows.size();
                if (I.m == 0) {
                    c->err = "an instance has no training rows";
                    return bail(ASAGA_E_ARG);
                }
                if ((rc = dalloc(c, &I.rows, I.m))) return bail(rc);
                if ((rc = step([&]() -> int {
                         HIPCHK(c, hipMemcpyAsync(I.rows, rows.data(), I.m * 4, hipMemcpyHostToDevice, c->st));
                         HIPCHK(c, hipStreamSynchronize(c->st));
                         return ASAGA_OK;
                     })))
                    return bail(rc);
            }
            c->inst.push_back(I);
        }
        if ((rc = dalloc(c, &c->d_insts, (int64_t)c->inst.size()))) return bail(rc);
        // workgroup map: fixed waves per instance, or at most the device's
        // resident workgroups (no more than 2048 threads per compute unit),
        // and at least one per instance
        {
            int cus = device_cu_count();
            if (cus <= 0) cus = 256;
            const int block = default_block(*o, true);
            const int64_t bpi = o->waves > 0 ? ((int64_t)o->waves * 64 + block - 1) / block : 1;
            c->map_cap = std::max<int64_t>({(int64_t)c->inst.size() * bpi, (int64_t)cus * (2048 / block),
                                            (int64_t)c->inst.size()});
            if ((rc = dalloc(c, &c->d_map, c->map_cap))) return bail(rc);
        }
        if ((rc = step([&]() -> int {
                 HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
                 return ASAGA_OK;
             })))
            return bail(rc);
    }
    for (size_t k = 0; k < c->inst.size(); ++k) {
        const Inst* same = nullptr;
        for (size_t q = 0; q < k && !same; ++q)
            if (c->inst[q].fold == c->inst[k].fold) same = &c->inst[q];
        if ((rc = setup_instance(c, c->inst[k], same))) return bail(rc);
    }
    pick_shape(c);
    default_async_steps(c);
    if (!bt) {
        c->tau_cap = 2 * (c->n / (int64_t)kTauEvery) + 64;
        if ((rc = dalloc(c, &c->d_tau, 2 * c->tau_cap))) return bail(rc);
        if ((rc = dalloc(c, &c->d_tau_count, 1))) return bail(rc);
    }
    if ((rc = step([&]() -> int {
             HIPCHK(c, hipStreamSynchronize(c->st));
             return ASAGA_OK;
         })))
        return bail(rc);
    *out = c;
    return ASAGA_OK;
}

int check_inst(asaga_ctx* c, int32_t inst) {
    if (inst < 0 || inst >= (int32_t)c->inst.size()) return fail(c, ASAGA_E_ARG, "instance out of range");
    return ASAGA_OK;
}

// x of instance `inst`, or the caller's vector moved into the relabelled
// order, as a view for evaluation
int eval_x(asaga_ctx* c, int32_t inst, const double* x_host, XView* x) {
    if (x_host) {
        HIPCHK(c, hipMemcpyAsync(c->vec2, x_host, c->d * 8, hipMemcpyHostToDevice, c->st));
        HIPCHK(c, launch_scatter_slots(c->vec2, c->rank, c->d, c->vec1, 1, false, c->st));
        *x = XView{c->vec1, 1, 0};
    } else {
        *x = x_view(c, c->inst[inst]);
    }
    return ASAGA_OK;
}

// workgroups an instance of a batch can use under the step law (no limit
// with a fixed step)
int64_t useful_blocks(const asaga_ctx* c, const UpdateShape& S) {
    if (c->o.step > 0.0) return INT64_MAX;
    const double sg = c->step_groups > 0.0 ? c->step_groups : kStepGroups;
    const double gpb = (double)(S.block / S.lanes);
    return std::max<int64_t>(1, (int64_t)std::ceil(sg / (c->step_cap * gpb)));
}

// workgroups per instance of a batch with automatic waves when n_act
// instances are active (the plan's equal share, before the m/64 bound)
int64_t batched_share(const asaga_ctx* c, const UpdateShape& S, int n_act) {
    int res = batched_resident_blocks(S, c->val_dtype);
    if (res <= 0) res = std::max(1, device_cu_count());
    return std::min<int64_t>(useful_blocks(c, S), std::max(1, res / std::max(1, n_act)));
}

// Work plan of one batched launch: which workgroups serve which instance,
// each instance's step, and the tier interval.  With opts.waves set, every
// instance keeps waves / (waves per workgroup) workgroups.  Otherwise the
// grid is the device's resident capacity, shared equally among the active
// instances (each at least one workgroup), so that instances that are
// still running take over the workgroups of those switched off.  The step
// of instance k without opts.step is rule_k * min(step_cap, step_groups /
// G_k): samples in flight for an instance grow with its workgroups, and the
// stable step shrinks in proportion (Theorem 2).  An instance therefore gets
// at most step_groups / step_cap lane groups: beyond that its step shrinks
// as fast as its samples in flight grow, while the throughput they add grows
// more slowly (measured on the RCV1-shaped matrix), so an instance whose
// epochs grow like 1/step (the small-lambda instances of a lambda path, the
// last ones running) would reach a given accuracy later.
int plan_batched(asaga_ctx* c, UpdateShape* Sout) {
    const size_t ni = c->inst.size();
    UpdateShape S = c->shape;
    const int wpb = S.block / 64;
    std::vector<int> blocks(ni, 0);
    std::vector<size_t> act;
    for (size_t k = 0; k < ni; ++k)
        if (c->inst[k].active) act.push_back(k);
    int n_blocks = 0;
    if (S.serial) {
        // ordered: each active instance on one workgroup of its own
        for (size_t k : act) blocks[k] = 1;
        n_blocks = (int)act.size();
    } else if (c->o.waves > 0) {
        const int bpi = std::max(1, (S.waves + wpb - 1) / wpb);
        n_blocks = (int)ni * bpi;
        for (size_t k = 0; k < ni; ++k) blocks[k] = bpi;
    } else if (!act.empty()) {
        int res = batched_resident_blocks(S, c->val_dtype);
        if (res <= 0) res = std::max(1, device_cu_count());
        const int share = std::max<int>(res, (int)act.size());
        const int q = share / (int)act.size(), r = share % (int)act.size();
        const int64_t gpb = S.block / S.lanes;  // lane groups per workgroup
        const int64_t useful = useful_blocks(c, S);
        for (size_t a = 0; a < act.size(); ++a) {
            const int64_t cap = std::min(useful, std::max<int64_t>(1, max_groups_for(c->inst[act[a]].m) / gpb));
            blocks[act[a]] = (int)std::min<int64_t>(cap, q + ((int)a < r ? 1 : 0));
            n_blocks += blocks[act[a]];
        }
    }
    std::vector<BlockMap>& map = c->plan_map;
    map.assign(n_blocks, BlockMap{-1, 0});
    if (c->o.waves > 0 && !S.serial) {
        for (int b = 0; b < n_blocks; ++b) map[b] = BlockMap{b / blocks[0], b % blocks[0]};
    } else {
        int b = 0;
        for (size_t k : act)
            for (int r = 0; r < blocks[k]; ++r) map[b++] = BlockMap{(int32_t)k, r};
    }
    const double sg = c->step_groups > 0.0 ? c->step_groups : kStepGroups;
    double glg = 0.0;
    std::vector<InstArgs>& h = c->plan_h;
    h.resize(ni);
    for (size_t k = 0; k < ni; ++k) {
        Inst& I = c->inst[k];
        const double groups = (double)blocks[k] * (double)S.block / (double)S.lanes;
        if (c->o.step <= 0.0 && blocks[k] > 0 && !S.serial) I.gamma = I.rule * std::min(c->step_cap, sg / groups);
        h[k] = inst_args(I, (uint64_t)I.t, I.active ? (uint64_t)I.m : 0);
        h[k].blocks = blocks[k];
        if (I.active) glg = std::max(glg, I.gamma * I.lambda * groups);
    }
    // With automatic waves the instances hold unequal numbers of workgroups
    // (160 instances on 256 workgroups: 96 hold two); one epoch each would
    // leave the extra workgroups idle for half the launch.  Every workgroup
    // is kept busy instead: instance k applies max(m_k, blocks_k * P)
    // samples, P = max_j ceil(m_j / blocks_j) the samples per workgroup of
    // the instance that sets the launch's length: at least one epoch, more
    // where it holds more workgroups per sample.
    if (c->o.waves == 0 && !act.empty() && !S.serial) {
        int64_t per_block = 0;
        for (size_t k : act) per_block = std::max(per_block, (c->inst[k].m + blocks[k] - 1) / blocks[k]);
        for (size_t k : act) h[k].count = (uint64_t)std::max(c->inst[k].m, per_block * blocks[k]);
    }
    if (!S.serial) {
        S.tier_every = tier_every_from(c, glg);
        for (size_t k : act) S.hot = stable_hot(c, c->inst[k], S.hot, (double)blocks[k]);
        S.tier = std::min(S.tier, S.hot);
    }
    for (size_t k : act) h[k].reload_from = view_reload_from(c, c->inst[k], S.hot, (double)blocks[k]);
    *Sout = S;
    if ((int64_t)n_blocks > c->map_cap)
        return fail(c, ASAGA_E_STATE, "batched launch needs " + std::to_string(n_blocks) +
                                          " workgroups, more than the map allocated at initialisation");
    return ASAGA_OK;
}

// The hipGraph that applies `epochs` epochs of the planned launch: one
// batched launch per epoch, epoch index e in 0..epochs-1 baked into each
// node, each followed by the stop test when it is armed.  The descriptors
// and block map it reads are rewritten before each replay.
int epochs_graph(asaga_ctx* c, int64_t epochs, const UpdateShape& S, int n_blocks, hipGraphExec_t* out) {
    for (const auto& g : c->graphs)
        if (g.epochs == epochs && g.tier_every == S.tier_every && g.hot == S.hot && g.tier == S.tier &&
            g.n_blocks == n_blocks && g.map == c->d_map && g.stop == c->stop_on) {
            *out = g.exec;
            return ASAGA_OK;
        }
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
    hipError_t le = hipSuccess;
    for (int64_t e = 0; e < epochs && le == hipSuccess; ++e) {
        le = launch_updates_batched(mat(c), c->d_insts, c->d_map, n_blocks, (uint64_t)e, S, c->flag, c->cap);
        if (le == hipSuccess && c->stop_on)
            le = launch_batch_proxy(c->d_insts, (int)c->inst.size(), c->d, S.layout, c->d_stop_thr, c->d_proxy,
                                    c->d_ran, (int32_t)e, c->cap);
    }
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(c->cap, &graph);
    if (le != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(c, ASAGA_E_HIP, std::string("capturing the epochs graph: ") +
                                        hipGetErrorString(le != hipSuccess ? le : ee));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(c, ASAGA_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    c->graphs.push_back({epochs, S.tier_every, S.hot, S.tier, n_blocks, c->d_map, c->stop_on, graph, exec});
    *out = exec;
    return ASAGA_OK;
}

// `epochs` epochs of every active instance of a batch
int batched_piece(asaga_ctx* c, int64_t epochs) {
    // the previous call's launches read the descriptors: wait before overwriting them
    HIPCHK(c, hipStreamSynchronize(c->st));
    UpdateShape S;
    int rc = plan_batched(c, &S);
    if (rc) return rc;
    const int n_blocks = (int)c->plan_map.size();
    if (n_blocks == 0) return ASAGA_OK;
    HIPCHK(c, hipMemcpyAsync(c->d_insts, c->plan_h.data(), c->plan_h.size() * sizeof(InstArgs),
                             hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->d_map, c->plan_map.data(), c->plan_map.size() * sizeof(BlockMap),
                             hipMemcpyHostToDevice, c->st));
    const int ni = (int)c->inst.size();
    if (c->stop_on) {
        HIPCHK(c, launch_fill_i32(c->d_ran, 0, ni, c->st));
        HIPCHK(c, launch_fill_f64(c->d_proxy, std::nan(""), ni, 1, c->st));
    }
    if (c->o.plain_launch) {
        for (int64_t e = 0; e < epochs; ++e) {
            HIPCHK(c, launch_updates_batched(mat(c), c->d_insts, c->d_map, n_blocks, (uint64_t)e, S, c->flag, c->st));
            if (c->stop_on)
                HIPCHK(c, launch_batch_proxy(c->d_insts, ni, c->d, S.layout, c->d_stop_thr, c->d_proxy, c->d_ran,
                                             (int32_t)e, c->st));
        }
    } else {
        hipGraphExec_t exec = nullptr;
        if ((rc = epochs_graph(c, epochs, S, n_blocks, &exec))) return rc;
        HIPCHK(c, hipGraphLaunch(exec, c->st));
    }
    if (!c->stop_on) {
        for (int k = 0; k < ni; ++k)
            if (c->inst[k].active) c->inst[k].t += epochs * (int64_t)c->plan_h[k].count;
        return ASAGA_OK;
    }
    // the stop test: wait for the launches, then take the instances it
    // switched off out of the plan and count the epochs each one ran
    std::vector<int32_t> ran(ni);
    std::vector<double> proxy(ni);
    HIPCHK(c, hipMemcpyAsync(ran.data(), c->d_ran, ni * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(proxy.data(), c->d_proxy, ni * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (int k = 0; k < ni; ++k) {
        if (!c->inst[k].active || c->plan_h[k].count == 0) continue;
        const int64_t e = ran[k] > 0 ? (int64_t)ran[k] : epochs;
        c->inst[k].t += e * (int64_t)c->plan_h[k].count;
        c->ran_h[k] += e;
        c->proxy_h[k] = proxy[k];
        if (ran[k] > 0) c->inst[k].active = false;
    }
    return ASAGA_OK;
}

}  // namespace

// Scratch of asaga_objective_noalloc, one copy per device for the life of
// the process: the per-row terms phi(a_i . x; b_i) (computed in place over
// the row dots), then the partial and final sums.  The name is a host-side
// stand-in in host code: kernels get the device address that
// hipGetSymbolAddress reports for the current device.
constexpr int64_t kNoAllocRows = (int64_t)1 << 22;
constexpr int64_t kNoAllocScratch = kNoAllocRows + kSumParts + 2;
static __device__ __align__(256) double scratch[kNoAllocScratch];

namespace {

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_dev;  // by device ordinal; nullptr until first looked up

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int scratch_on_current_device(double** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, ASAGA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_dev[dev];
    return ASAGA_OK;
}

}  // namespace

extern "C" {

int asaga_set_active(asaga_ctx* c, const uint8_t* active) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!active) return fail(c, ASAGA_E_ARG, "NULL active mask");
    if (!c->d_insts) return fail(c, ASAGA_E_STATE, "asaga_set_active needs a batched context");
    for (size_t k = 0; k < c->inst.size(); ++k)
        if (active[k] > 1) return fail(c, ASAGA_E_ARG, "active entries must be 0 or 1");
    for (size_t k = 0; k < c->inst.size(); ++k) c->inst[k].active = active[k] != 0;
    return ASAGA_OK;
}

int asaga_set_stop(asaga_ctx* c, const double* thresholds) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!c->d_insts) return fail(c, ASAGA_E_STATE, "asaga_set_stop needs a batched context");
    if (!thresholds) {
        c->stop_on = false;
        return ASAGA_OK;
    }
    const int64_t ni = (int64_t)c->inst.size();
    for (int64_t k = 0; k < ni; ++k)
        if (!(thresholds[k] >= 0.0)) return fail(c, ASAGA_E_ARG, "stop thresholds must be >= 0");
    int rc = ASAGA_OK;
    if (!c->d_stop_thr) {
        if ((rc = dalloc(c, &c->d_stop_thr, ni)) || (rc = dalloc(c, &c->d_proxy, ni)) ||
            (rc = dalloc(c, &c->d_ran, ni)))
            return rc;
    }
    // a call still running may read the thresholds
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, hipMemcpyAsync(c->d_stop_thr, thresholds, ni * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (c->proxy_h.size() != (size_t)ni) {
        c->proxy_h.assign(ni, std::nan(""));
        c->ran_h.assign(ni, 0);
    }
    c->stop_on = true;
    return ASAGA_OK;
}

int asaga_stop_report(asaga_ctx* c, double* proxy_out, int64_t* epochs_out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!c->d_insts) return fail(c, ASAGA_E_STATE, "asaga_stop_report needs a batched context");
    const size_t ni = c->inst.size();
    for (size_t k = 0; k < ni; ++k) {
        if (proxy_out) proxy_out[k] = k < c->proxy_h.size() ? c->proxy_h[k] : std::nan("");
        if (epochs_out) epochs_out[k] = k < c->ran_h.size() ? c->ran_h[k] : 0;
    }
    return ASAGA_OK;
}

int asaga_init(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts) {
    return init_common(out, prob, opts, nullptr);
}

int asaga_init_batched(asaga_ctx** out, const asaga_problem* prob, const asaga_opts* opts, const asaga_batch* batch) {
    if (!batch) return fail(nullptr, ASAGA_E_ARG, "NULL batch descriptor");
    return init_common(out, prob, opts, batch);
}

int asaga_updates(asaga_ctx* c, int64_t count) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (count < 0) return fail(c, ASAGA_E_ARG, "negative update count");
    if (c->d_insts) return fail(c, ASAGA_E_STATE, "asaga_updates needs a single-instance context");
    Inst& I = c->inst[0];
    UpdateShape S = c->shape;
    if (!S.serial) {
        S.hot = stable_hot(c, I, S.hot, (double)((S.waves * 64 + S.block - 1) / S.block));
        S.tier = std::min(S.tier, S.hot);
        S.tier_every = tier_every_for(c, S);
    }
    // serial launches are cut into pieces of at most 2^18 updates
    const int64_t piece = S.serial ? ((int64_t)1 << 18) : count;
    for (int64_t done = 0; done < count;) {
        int64_t k = count - done < piece ? count - done : piece;
        if (c->svrg) {
            // a full gradient at iteration I.t, else inner steps up to the next one
            if (svrg_full_gradient_due(I.seed, (uint64_t)I.t, I.m)) {
                int rc = svrg_snapshot(c, I);
                if (rc) return rc;
                I.t += 1;
                done += 1;
                continue;
            }
            int64_t run = 1;
            while (run < k && !svrg_full_gradient_due(I.seed, (uint64_t)(I.t + run), I.m)) ++run;
            k = run;
        }
        InstArgs a = inst_args(I, (uint64_t)I.t, (uint64_t)k);
        a.frozen = c->svrg ? 1 : 0;
        a.reload_from = view_reload_from(c, I, S.hot, (double)((S.waves * 64 + S.block - 1) / S.block));
        if (c->tau_on) {
            a.tau_log = c->d_tau;
            a.tau_count = c->d_tau_count;
            a.tau_cap = (uint64_t)c->tau_cap;
        }
        HIPCHK(c, launch_updates(mat(c), a, S, c->flag, c->st));
        I.t += k;
        done += k;
    }
    return ASAGA_OK;
}

int asaga_epochs(asaga_ctx* c, int64_t n_epochs) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (n_epochs < 0) return fail(c, ASAGA_E_ARG, "negative epoch count");
    if (!c->d_insts) {
        for (int64_t e = 0; e < n_epochs; ++e) {
            int rc = asaga_updates(c, c->inst[0].m);
            if (rc) return rc;
        }
        return ASAGA_OK;
    }
    if (c->stop_on) {
        c->proxy_h.assign(c->inst.size(), std::nan(""));
        c->ran_h.assign(c->inst.size(), 0);
    }
    for (int64_t done = 0; done < n_epochs;) {
        const int64_t e = std::min(n_epochs - done, kMaxGraphEpochs);
        int rc = batched_piece(c, e);
        if (rc) return rc;
        done += e;
    }
    return ASAGA_OK;
}

int asaga_objective(asaga_ctx* c, int32_t inst, const double* x_host, double* f_out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!f_out) return fail(c, ASAGA_E_ARG, "NULL f_out");
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst];
    XView x;
    if ((rc = eval_x(c, inst, x_host, &x))) return rc;
    const MatArgs A = mat(c);
    HIPCHK(c, launch_rowdot(A, I.rows, I.m, x, c->z, c->st));
    HIPCHK(c, launch_phi_terms(A, I.rows, I.m, c->z, c->tmp, c->st));
    HIPCHK(c, launch_sum(c->tmp, I.m, c->part, c->scal + 0, c->st));
    HIPCHK(c, launch_sum_x2(x, c->d, c->part, c->scal + 1, c->st));
    double s[2];
    HIPCHK(c, hipMemcpyAsync(s, c->scal, sizeof(s), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    const double f = s[0] / (double)I.m + 0.5 * I.lambda * s[1];
    *f_out = f;
    if (!std::isfinite(f)) return fail(c, ASAGA_E_DIVERGED, "objective is not finite");
    return ASAGA_OK;
}

int asaga_objective_noalloc(const asaga_problem* p, const double* x_dev, double* f_dev, void* stream) {
    if (!p || !x_dev || !f_dev) return fail(nullptr, ASAGA_E_ARG, "NULL problem, x_dev or f_dev");
    if (p->mem != ASAGA_MEM_DEVICE) return fail(nullptr, ASAGA_E_ARG, "problem arrays must be in device memory");
    if (p->reserved != 0) return fail(nullptr, ASAGA_E_ARG, "reserved field must be 0");
    if (p->n < 1 || p->n > kNoAllocRows)
        return fail(nullptr, ASAGA_E_ARG,
                    "n = " + std::to_string(p->n) + " outside [1, " + std::to_string(kNoAllocRows) +
                        "]: the allocation-free objective holds one term per row in a fixed scratch array");
    if (p->d < 1 || p->d > kMaxD) return fail(nullptr, ASAGA_E_ARG, "d must be in [1, 2^27 - 1]");
    if (!p->rowptr || !p->colidx || !p->val || !p->b) return fail(nullptr, ASAGA_E_ARG, "NULL problem array");
    if (p->val_dtype < ASAGA_VAL_F64 || p->val_dtype > ASAGA_VAL_BF16)
        return fail(nullptr, ASAGA_E_ARG, "bad val_dtype");
    if (p->loss != ASAGA_LOSS_LOGISTIC && p->loss != ASAGA_LOSS_SQUARED) return fail(nullptr, ASAGA_E_ARG, "bad loss");
    if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return fail(nullptr, ASAGA_E_ARG, "lambda must be > 0 and finite");
    double* sc = nullptr;
    int rc = scratch_on_current_device(&sc);
    if (rc) return rc;
    double* terms = sc;                       // [n]
    double* part = sc + kNoAllocRows;         // [kSumParts]
    double* sums = part + kSumParts;          // [2]
    hipStream_t st = static_cast<hipStream_t>(stream);
    const MatArgs A{p->rowptr, p->colidx, p->val, p->b, p->n, p->d, p->val_dtype, p->loss};
    const XView x{x_dev, 1, 0};
    hipError_t e = launch_rowdot(A, nullptr, p->n, x, terms, st);
    if (e == hipSuccess) e = launch_phi_terms(A, nullptr, p->n, terms, terms, st);
    if (e == hipSuccess) e = launch_sum(terms, p->n, part, sums + 0, st);
    if (e == hipSuccess) e = launch_sum_x2(x, p->d, part, sums + 1, st);
    if (e == hipSuccess) e = launch_objective_finish(sums, (double)p->n, p->lambda, f_dev, st);
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_HIP, std::string("objective launch: ") + hipGetErrorString(e));
    return ASAGA_OK;
}

int asaga_full_grad(asaga_ctx* c, int32_t inst, const double* x_host, double* g_host) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!g_host) return fail(c, ASAGA_E_ARG, "NULL g_host");
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst];
    XView x;
    if ((rc = eval_x(c, inst, x_host, &x))) return rc;
    const MatArgs A = mat(c);
    HIPCHK(c, launch_rowdot(A, I.rows, I.m, x, c->z, c->st));
    HIPCHK(c, launch_dphi_coef(A, I.rows, I.m, c->z, 1.0 / (double)I.m, c->tmp, c->st));
    HIPCHK(c, launch_fill_f64(c->vec2, 0.0, c->d, 1, c->st));
    HIPCHK(c, launch_scatter(A, I.rows, I.m, c->tmp, c->vec2, 1, c->st));
    HIPCHK(c, launch_axpy_x(x, c->d, I.lambda, c->vec2, c->st));
    // back to the caller's column order
    HIPCHK(c, launch_gather_view(XView{c->vec2, 1, 0}, c->rank, c->d, c->vec1, c->st));
    HIPCHK(c, hipMemcpyAsync(g_host, c->vec1, c->d * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return ASAGA_OK;
}

int asaga_get_state(asaga_ctx* c, int32_t inst, double* x_host, double* alpha_host, double* abar_host, int64_t* t_out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst];
    if (x_host) {
        HIPCHK(c, launch_gather_view(x_view(c, I), c->rank, c->d, c->vec1, c->st));
        HIPCHK(c, hipMemcpyAsync(x_host, c->vec1, c->d * 8, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    if (abar_host) {
        HIPCHK(c, launch_gather_view(abar_view(c, I), c->rank, c->d, c->vec1, c->st));
        HIPCHK(c, hipMemcpyAsync(abar_host, c->vec1, c->d * 8, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    if (alpha_host) {
        if (c->mixed) {
            HIPCHK(c, launch_widen_f32(static_cast<const float*>(I.alpha), I.m, c->tmp, c->st));
            HIPCHK(c, hipMemcpyAsync(alpha_host, c->tmp, I.m * 8, hipMemcpyDeviceToHost, c->st));
        } else {
            HIPCHK(c, hipMemcpyAsync(alpha_host, I.alpha, I.m * 8, hipMemcpyDeviceToHost, c->st));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (t_out) *t_out = I.t;
    return check_flag(c);
}

int asaga_get_x(asaga_ctx* c, int32_t inst, double* x_host) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!x_host) return fail(c, ASAGA_E_ARG, "NULL x_host");
    return asaga_get_state(c, inst, x_host, nullptr, nullptr, nullptr);
}

int asaga_set_state(asaga_ctx* c, int32_t inst, const double* x_host, const double* alpha_host, const double* abar_host,
                    const int64_t* t_in) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    int rc = check_inst(c, inst);
    if (rc) return rc;
    Inst& I = c->inst[inst];
    if (t_in && *t_in < 0) return fail(c, ASAGA_E_ARG, "negative sample counter");
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (x_host) {
        HIPCHK(c, hipMemcpyAsync(c->vec1, x_host, c->d * 8, hipMemcpyHostToDevice, c->st));
        if (c->layout == kLayF32) HIPCHK(c, launch_scatter_slots(c->vec1, c->rank, c->d, I.xa, 2, true, c->st));
        else if (c->mixed) HIPCHK(c, launch_scatter_slots(c->vec1, c->rank, c->d, I.xa, 4, true, c->st));
        else HIPCHK(c, launch_scatter_slots(c->vec1, c->rank, c->d, I.xa, 2, false, c->st));
    }
    if (abar_host) {
        HIPCHK(c, hipMemcpyAsync(c->vec2, abar_host, c->d * 8, hipMemcpyHostToDevice, c->st));
        if (c->layout == kLayF32)
            HIPCHK(c, launch_scatter_slots(c->vec2, c->rank, c->d, reinterpret_cast<float*>(I.xa) + 1, 2, true, c->st));
        else
            HIPCHK(c, launch_scatter_slots(c->vec2, c->rank, c->d, I.xa + 1, 2, false, c->st));
    }
    if (alpha_host) {
        if (c->mixed) {
            HIPCHK(c, hipMemcpyAsync(c->tmp, alpha_host, I.m * 8, hipMemcpyHostToDevice, c->st));
            HIPCHK(c, launch_narrow_f64(c->tmp, I.m, static_cast<float*>(I.alpha), c->st));
        } else {
            HIPCHK(c, hipMemcpyAsync(I.alpha, alpha_host, I.m * 8, hipMemcpyHostToDevice, c->st));
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (t_in) I.t = *t_in;
    return ASAGA_OK;
}

int asaga_reanchor(asaga_ctx* c) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    for (auto& I : c->inst) {
        int rc = recompute_abar(c, I);
        if (rc) return rc;
    }
    return ASAGA_OK;
}

int asaga_widen(asaga_ctx* c) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!c->mixed) return ASAGA_OK;
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<void*> wide(c->inst.size());
    for (size_t k = 0; k < c->inst.size(); ++k) {
        double* a = nullptr;
        int rc = dalloc(c, &a, c->inst[k].m);
        if (rc) return rc;
        wide[k] = a;
    }
    for (size_t k = 0; k < c->inst.size(); ++k) {
        Inst& I = c->inst[k];
        if (c->layout == kLayF32) {
            // x out of the 8-byte slots, then back as FP64 pairs (abar: below)
            HIPCHK(c, launch_copy_view(x_view(c, I), c->d, c->vec1, 1, c->st));
            HIPCHK(c, launch_fill_f64(I.xa, 0.0, 2 * c->d, 1, c->st));
            HIPCHK(c, launch_copy_view(XView{c->vec1, 1, 0}, c->d, I.xa, 2, c->st));
        } else {
            HIPCHK(c, launch_widen_x_slots(I.xa, c->d, c->st));
        }
        HIPCHK(c, launch_widen_f32(static_cast<const float*>(I.alpha), I.m, static_cast<double*>(wide[k]), c->st));
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (size_t k = 0; k < c->inst.size(); ++k) c->inst[k].alpha = wide[k];
    c->mixed = false;
    c->layout = kLayF64;
    c->shape.layout = kLayF64;
    if (c->widen_gamma > 0.0 && !c->d_insts) c->inst[0].gamma = c->widen_gamma;
    c->widen_gamma = 0.0;
    // the FP64 layout's LDS holds at most kMaxHot hot columns
    c->shape.hot = std::min(c->shape.hot, kMaxHot);
    c->shape.tier = std::min(c->shape.tier, c->shape.hot);
    drop_graphs(c);
    // abar from the memory it averages, in FP64
    return asaga_reanchor(c);
}

namespace {

// ||grad f(x)||^2 and f(x) at an instance's current iterate (FP64)
int grad_norm2(asaga_ctx* c, int inst, double* g2, double* f, double* x2 = nullptr) {
    const Inst& I = c->inst[inst];
    const XView x = x_view(c, I);
    const MatArgs A = mat(c);
    HIPCHK(c, launch_rowdot(A, I.rows, I.m, x, c->z, c->st));
    HIPCHK(c, launch_phi_terms(A, I.rows, I.m, c->z, c->tmp, c->st));
    HIPCHK(c, launch_sum(c->tmp, I.m, c->part, c->scal + 0, c->st));
    HIPCHK(c, launch_sum_x2(x, c->d, c->part, c->scal + 1, c->st));
    HIPCHK(c, launch_dphi_coef(A, I.rows, I.m, c->z, 1.0 / (double)I.m, c->tmp, c->st));
    HIPCHK(c, launch_fill_f64(c->vec2, 0.0, c->d, 1, c->st));
    HIPCHK(c, launch_scatter(A, I.rows, I.m, c->tmp, c->vec2, 1, c->st));
    HIPCHK(c, launch_axpy_x(x, c->d, I.lambda, c->vec2, c->st));
    HIPCHK(c, launch_sum_x2(XView{c->vec2, 1, 0}, c->d, c->part, c->scal + 2, c->st));
    double s[3];
    HIPCHK(c, hipMemcpyAsync(s, c->scal, sizeof(s), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    *f = s[0] / (double)I.m + 0.5 * I.lambda * s[1];
    *g2 = s[2];
    if (x2) *x2 = s[1];
    return ASAGA_OK;
}

// A probe's run is unstable if ||grad f||^2 more than doubles between two
// checkpoints or shows no net decrease from the first to the last; single
// steps without decrease are noise of the asynchronous updates.
bool probe_unstable(const double* g2, int k) {
    if (k == 0) return false;
    return g2[k] > 2.0 * g2[k - 1] || (k == 2 && !(g2[2] < g2[0]));
}

// decay rate per epoch of ||grad f|| over the last two checkpoints, else
// over the whole probe (0 if there was none)
double probe_rate(const double* g2, const int* cps) {
    double r = 0.5 * std::log(g2[1] / g2[2]) / (double)(cps[2] - cps[1]);
    if (!(r > 0.0)) r = 0.5 * std::log(g2[0] / g2[2]) / (double)(cps[2] - cps[0]);
    return r > 0.0 ? r : 0.0;
}

// Epochs until (f - f*)/f* <= target, from the objective at three equally
// spaced checkpoints: the differences of a linearly converging sequence
// shrink geometrically, so Aitken's extrapolation estimates f* and the
// contraction per epoch.  Returns the checkpoint epoch if the last
// difference is already below the target, and a negative value if the
// differences do not shrink (no estimate).
double aitken_epochs(const double* f, const int* cps, double target) {
    const double d1 = f[1] - f[0], d2 = f[2] - f[1];
    if (std::fabs(d2) <= target * std::fabs(f[2])) return (double)cps[2];
    if (!(d1 < 0.0 && d2 < 0.0)) return -1.0;
    const double r = d2 / d1;
    if (!(r > 0.0 && r < 1.0)) return -1.0;
    const double fstar = f[2] - d2 * d2 / (d2 - d1);
    const double gap = f[2] - fstar;
    if (!(gap > 0.0) || gap <= target * std::fabs(fstar)) return (double)cps[2];
    const double per_epoch = std::log(r) / (double)(cps[2] - cps[1]);  // log contraction per epoch (< 0)
    return (double)cps[2] + std::log(target * std::fabs(fstar) / gap) / per_epoch;
}

// ||grad f||^2 an autotuning probe accepts as converged: the strong-convexity
// certificate of relative suboptimality `target`, or, with FP32 x, the floor
// its rounding leaves (a gradient error of about 8 * 2^-24 * L * ||x||).
double probe_goal(const asaga_ctx* c, const Inst& I, double target, double f, double x2) {
    const double cert = 2.0 * I.lambda * target * f;
    if (!c->mixed) return cert;
    const double e = 8.0 * 0x1p-24 * I.L;
    return std::max(cert, e * e * x2);
}

int reset_state(asaga_ctx* c) {
    for (auto& I : c->inst) {
        int rc = zero_state(c, I);
        if (rc) return rc;
    }
    HIPCHK(c, launch_fill_i32(c->flag, 0, 1, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return ASAGA_OK;
}

}  // namespace

namespace {

// asaga_autotune for a batch: the hot-set size and the step law.  The law
// gamma_k = rule_k * min(step_cap, step_groups / G_k) is calibrated where it
// matters most, on the instance with the smallest lambda (the slowest, the
// last one running) given the whole device, as a single-instance step
// ladder (from the single solve's default law down) with the single solve's
// stability test, and a three times longer run of the choice; then step_cap
// is checked with every instance running.
int autotune_batched(asaga_ctx* c, double target, int32_t probe_epochs, asaga_tune_report* rep) {
    if (c->o.step > 0.0) return fail(c, ASAGA_E_STATE, "batched autotuning chooses the steps: opts.step must be 0");
    if (c->o.waves > 0)
        return fail(c, ASAGA_E_STATE, "batched autotuning shares the device among the instances: opts.waves must be 0");
    const size_t ni = c->inst.size();
    std::vector<bool> was_active(ni);
    size_t cal = ni;
    for (size_t k = 0; k < ni; ++k) {
        was_active[k] = c->inst[k].active;
        if (was_active[k] && (cal == ni || c->inst[k].lambda < c->inst[cal].lambda)) cal = k;
    }
    if (cal == ni) return fail(c, ASAGA_E_STATE, "no active instance to tune on");
    const UpdateShape base = c->shape;
    const double base_groups = c->step_groups, base_cap = c->step_cap;
    auto set_active = [&](bool solo) {
        for (size_t k = 0; k < ni; ++k) c->inst[k].active = solo ? k == cal : (bool)was_active[k];
    };
    auto restore = [&]() {
        c->shape = base;
        c->step_groups = base_groups;
        c->step_cap = base_cap;
        set_active(false);
        drop_graphs(c);
        (void)reset_state(c);
    };
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int rc = ASAGA_OK, tried = 0;
    const int cps[3] = {probe_epochs / 3, 2 * probe_epochs / 3, probe_epochs};
    const int cps3[3] = {probe_epochs, 2 * probe_epochs, 3 * probe_epochs};
    // Run from zero with checkpoints cp; false if some active instance was
    // unstable before it was already certified: with `strict` (one instance
    // alone), unless its ||grad f|| fell and its objective did not rise at
    // every checkpoint, as for a single solve; otherwise unless ||grad f||
    // never doubled and ended below its first value.  *est_e: epochs until
    // the slowest one reaches ||g||^2 <= 2 lambda target f at its last
    // measured rate.
    auto probe = [&](const int* cp, bool strict, double* est_e) -> bool {
        if ((rc = reset_state(c))) return false;
        std::vector<double> g2(3 * ni, 0.0), f(3 * ni, 0.0), goal(ni, 0.0);
        std::vector<int> reached(ni, -1);
        int done = 0;
        for (int k = 0; k < 3; ++k) {
            if ((rc = asaga_epochs(c, cp[k] - done))) return false;
            done = cp[k];
            for (size_t j = 0; j < ni; ++j) {
                if (!c->inst[j].active || reached[j] >= 0) continue;
                double* gj = &g2[3 * j];
                double x2 = 0.0;
                if ((rc = grad_norm2(c, (int)j, &gj[k], &f[3 * j + k], &x2))) return false;
                if (!(std::isfinite(gj[k]) && std::isfinite(f[3 * j + k]))) return false;
                goal[j] = probe_goal(c, c->inst[j], target, f[3 * j + k], x2);
                if (gj[k] <= goal[j]) reached[j] = k;
                else if (strict ? k > 0 && !(gj[k] < gj[k - 1] && f[3 * j + k] <= f[3 * j + k - 1])
                                : probe_unstable(gj, k))
                    return false;
            }
        }
        int flag = 0;
        const hipError_t he = hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost);
        if (he != hipSuccess) {
            rc = fail(c, ASAGA_E_HIP, std::string("autotune flag: ") + hipGetErrorString(he));
            return false;
        }
        if (flag) return false;
        double e = (double)cp[2];
        for (size_t j = 0; j < ni; ++j) {
            if (!c->inst[j].active || reached[j] >= 0) continue;
            const double* gj = &g2[3 * j];
            const double ea = aitken_epochs(&f[3 * j], cp, target);
            if (ea >= 0.0) {
                e = std::max(e, ea);
                continue;
            }
            const double r = probe_rate(gj, cp);
            if (r == 0.0) return false;
            e = std::max(e, (double)cp[2] + (gj[2] > goal[j] ? 0.5 * std::log(gj[2] / goal[j]) / r : 0.0));
        }
        *est_e = e;
        return true;
    };
    struct Best {
        double est_s = INFINITY, est_e = 0, ms = 0, groups = 0;
        UpdateShape S{};
    } best;
    // 1. the calibration instance alone on the device, per hot-set size
    set_active(true);
    std::vector<int> hots;
    for (int h : {max_hot(c), kMaxHot, 1024}) {
        const int hot = (int)std::min<int64_t>(h, c->d);
        if (std::find(hots.begin(), hots.end(), hot) == hots.end()) hots.push_back(hot);
    }
    std::vector<double> scales;
    for (int k = 0; k <= 18; ++k) scales.push_back(std::exp2(-(double)k / 3.0));
    for (int hot : hots) {
        UpdateShape S = base;
        S.hot = hot;
        S.tier = std::min(256, hot);
        c->shape = S;
        drop_graphs(c);
        int res = batched_resident_blocks(S, c->val_dtype);
        if (res <= 0) res = std::max(1, device_cu_count());
        const int64_t gpb = S.block / S.lanes;
        const int64_t cal_blocks = std::min<int64_t>(res, std::max<int64_t>(1, max_groups_for(c->inst[cal].m) / gpb));
        const double groups = (double)(cal_blocks * gpb);
        // the ladder starts from the single solve's default law (measured
        // stable on the RCV1-shaped matrix up to 4096 samples in flight):
        // short probes from zero cannot certify a larger one, whose
        // instability may grow only near the optimum
        const double top = std::min(groups, kStepGroups);
        double shape_best = INFINITY;
        Best hb;  // this hot-set size's best law
        for (double sc : scales) {
            ++tried;
            c->step_groups = sc * top;
            c->step_cap = 1.0;
            // kernel time per epoch under this law (it sets the workgroups)
            float ms = 0.0f;
            if ((rc = reset_state(c))) break;
            hipError_t he = hipEventRecord(e0, c->st);
            if (he == hipSuccess && (rc = batched_piece(c, 1))) break;
            if (he == hipSuccess) he = hipEventRecord(e1, c->st);
            if (he == hipSuccess) he = hipEventSynchronize(e1);
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            if (he != hipSuccess) {
                rc = fail(c, ASAGA_E_HIP, std::string("autotune timing: ") + hipGetErrorString(he));
                break;
            }
            double est_e = 0.0;
            const bool ok = probe(cps, true, &est_e);
            if (rc) break;
            if (!ok) continue;  // as for one solve, a failure does not end the ladder
            const double est_s = est_e * (double)ms * 1e-3;
            if (est_s < hb.est_s) hb = Best{est_s, est_e, (double)ms, sc * top, S};
            // FP32 x reaches its rounding floor within a short probe whatever
            // the step, so the rates cannot rank the steps: the largest stable
            // one is kept (in the step-limited regime it converges fastest)
            if (c->mixed || est_s >= shape_best) break;
            shape_best = est_s;
        }
        if (rc) break;
        if (!std::isfinite(hb.est_s)) continue;
        // The hot-set sizes are ranked by one epoch of the whole batch under
        // their law: the calibration instance alone on its few workgroups
        // hardly feels the hot set's size, the batch (most of the time, every
        // instance on one or two workgroups) does.  Its epochs to the target
        // are not part of the ranking: at the full step they do not depend on
        // the hot set, and their estimates vary by some 10% from run to run,
        // more than the epoch times differ.
        set_active(false);
        c->step_groups = hb.groups;
        float ms_all = 0.0f;
        if ((rc = reset_state(c))) break;
        hipError_t he = hipEventRecord(e0, c->st);
        if (he == hipSuccess && (rc = batched_piece(c, 1))) break;
        if (he == hipSuccess) he = hipEventRecord(e1, c->st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms_all, e0, e1);
        if (he != hipSuccess) {
            rc = fail(c, ASAGA_E_HIP, std::string("autotune timing: ") + hipGetErrorString(he));
            break;
        }
        set_active(true);
        hb.ms = (double)ms_all;
        hb.est_s = hb.est_e * hb.ms * 1e-3;
        if (!std::isfinite(best.est_s) || hb.ms < best.ms) best = hb;
    }
    // The short probes see mostly the fast early decrease, which a step at
    // the edge of stability can still show (or not, from one run to the
    // next): from the chosen law down the ladder, the calibration instance
    // runs three times longer until a law passes that too.  (The instance
    // runs on step_groups lane groups at the full step, so of two stable
    // laws the larger is the faster.)
    if (!rc && std::isfinite(best.est_s)) {
        c->shape = best.S;
        c->step_cap = 1.0;
        drop_graphs(c);
        const double g0 = best.groups;
        bool ok = false;
        for (int down = 0; down < 12 && !ok && !rc; ++down) {
            ++tried;
            c->step_groups = g0 * std::exp2(-(double)down / 3.0);
            double est_e = 0.0;
            ok = probe(cps3, true, &est_e);
            if (ok) {
                best.groups = c->step_groups;
                best.est_e = est_e;
            }
        }
        if (!ok && !rc) best.est_s = INFINITY;
    }
    // 2. every instance running: the largest stable cap.  With one active
    // instance cap 1 is the run the calibration has just verified (that
    // instance alone on step_groups lane groups at the full step, three
    // times longer than a probe).  A short probe repeating it at a law on
    // the edge of stability can fail by chance, and a smaller cap gives the
    // lone instance more lane groups at a proportionally smaller step: on
    // the URL-shaped instance cap 1/8 (416 wavefronts) hovered near 3e-4
    // where cap 1 (64 wavefronts) reached 1e-9 in 30 epochs.
    double cap = 0.0;
    int n_was = 0;  // instances the caller has switched on
    for (size_t k = 0; k < ni; ++k) n_was += was_active[k] ? 1 : 0;
    if (!rc && std::isfinite(best.est_s) && n_was == 1) cap = 1.0;
    if (!rc && std::isfinite(best.est_s) && n_was > 1) {
        set_active(false);
        c->shape = best.S;
        c->step_groups = best.groups;
        drop_graphs(c);
        for (double cp : {1.0, 0.5, 0.25, 0.125}) {
            ++tried;
            c->step_cap = cp;
            double est_e = 0.0;
            const bool ok = probe(cps, false, &est_e);
            if (rc) break;
            if (ok) {
                cap = cp;
                break;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        restore();
        return rc;
    }
    if (!std::isfinite(best.est_s) || cap == 0.0) {
        restore();
        return fail(c, ASAGA_E_DIVERGED, "no probed hot-set size and step law reduced every gradient norm steadily");
    }
    c->step_cap = cap;
    set_active(false);
    drop_graphs(c);
    if ((rc = reset_state(c))) return rc;
    UpdateShape S;
    if ((rc = plan_batched(c, &S))) return rc;  // sets every instance's step for the full batch
    if (rep) {
        int n_act = 0;
        for (size_t k = 0; k < ni; ++k) n_act += c->inst[k].active ? 1 : 0;
        rep->candidates = tried;
        rep->waves = (int32_t)batched_share(c, S, n_act) * (S.block / 64);
        rep->hot_columns = S.hot;
        rep->hot_tier_columns = S.tier;
        rep->gamma = c->inst[0].gamma;
        rep->ms_per_epoch = best.ms;
        rep->est_epochs = best.est_e;
        rep->est_seconds = best.est_s;
        rep->step_groups = c->step_groups;
        rep->step_cap = c->step_cap;
        rep->widen_gamma = c->inst[0].gamma;
        rep->threads_per_block = S.block;
    }
    return ASAGA_OK;
}

}  // namespace

int asaga_autotune(asaga_ctx* c, double target, int32_t probe_epochs, asaga_tune_report* rep) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (c->shape.serial) return fail(c, ASAGA_E_STATE, "autotuning needs an async context");
    if (!(target > 0.0 && target < 1.0)) return fail(c, ASAGA_E_ARG, "target must be in (0, 1)");
    if (probe_epochs < 3 || probe_epochs > 1000) return fail(c, ASAGA_E_ARG, "probe_epochs must be in [3, 1000]");
    c->widen_gamma = 0.0;
    if (c->d_insts) {
        // the tuner's probes run whole epochs: no stop test meanwhile
        const bool stop = c->stop_on;
        c->stop_on = false;
        const int rc = autotune_batched(c, target, probe_epochs, rep);
        c->stop_on = stop;
        return rc;
    }
    Inst& I = c->inst[0];
    const UpdateShape base = c->shape;
    const double serial_rule = c->o.step > 0.0 ? c->o.step : I.rule;
    int cus = device_cu_count();
    if (cus <= 0) cus = 256;
    const int wpb = base.block / 64;
    auto round_waves = [&](int w) { return std::max(wpb, ((w + wpb - 1) / wpb) * wpb); };
    // wavefront counts from the fastest epoch (most samples in flight) to the
    // slowest; fewer samples in flight tolerate a larger step (Theorem 2)
    std::vector<UpdateShape> shapes;
    const int wmax = (int)std::min<int64_t>(cus * wpb, std::max<int64_t>(1, max_groups_for(I.m) * base.lanes / 64));
    for (int w = wmax; w >= std::max(wpb, std::min(wmax, cus / 8)); w /= 2) {
        UpdateShape S = base;
        S.waves = round_waves(w);
        if (!shapes.empty() && shapes.back().waves == S.waves) continue;
        shapes.push_back(S);
    }
    // steps from the serial rule down to 1/64 of it, three per halving
    std::vector<double> scales;
    for (int k = 0; k <= 18; ++k) scales.push_back(std::exp2(-(double)k / 3.0));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    struct Cand {
        double est_s = INFINITY, est_e = 0, ms = 0, gamma = 0;
        UpdateShape S{};
    } best;
    std::vector<Cand> stable_cands;
    int tried = 0, rc = ASAGA_OK;
    // Run from x = 0 at step I.gamma with checkpoints cps[0..2]: false if
    // ||grad f|| did not decrease at every checkpoint; else the estimated
    // epochs to the target by Aitken's extrapolation of the objective (else
    // with ||g|| taken to decay like exp(-r t) at the rate r of the last two
    // checkpoints, to ||g||^2 <= 2 lambda target f).
    auto probe = [&](const int* cps, double* est_e) -> bool {
        if ((rc = reset_state(c))) return false;
        double g2[3], f[3], x2 = 0.0;
        int done = 0;
        bool at_floor = false;  // FP32 x: the gradient reached its rounding floor
        for (int k = 0; k < 3; ++k) {
            if ((rc = asaga_updates(c, (int64_t)(cps[k] - done) * I.m))) return false;
            done = cps[k];
            if ((rc = grad_norm2(c, 0, &g2[k], &f[k], &x2))) return false;
            if (!(std::isfinite(g2[k]) && std::isfinite(f[k]))) return false;
            // already certified: later checkpoints would only see the noise
            // floor; the crossing is interpolated on log ||g||^2
            const double cert = 2.0 * I.lambda * target * f[k];
            if (g2[k] <= cert) {
                *est_e = (double)cps[k];
                if (k > 0 && g2[k - 1] > cert && g2[k] > 0.0)
                    *est_e = (double)cps[k - 1] +
                             (double)(cps[k] - cps[k - 1]) * std::log(g2[k - 1] / cert) / std::log(g2[k - 1] / g2[k]);
                return true;
            }
            // With FP32 x a gradient at the floor its rounding leaves need no
            // longer fall; it certifies nothing (on strongly ill-conditioned
            // data that floor is reached far from the optimum), so the
            // objective then decides the estimate.
            if (g2[k] <= probe_goal(c, I, target, f[k], x2)) at_floor = true;
            // one instance: the gradient norm must fall and the objective
            // must not rise at every checkpoint (slow instabilities pass a
            // looser test within a short probe)
            if (k > 0 && !((at_floor || g2[k] < g2[k - 1]) && f[k] <= f[k - 1])) return false;
        }
        int flag = 0;
        const hipError_t he = hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost);
        if (he != hipSuccess) {
            rc = fail(c, ASAGA_E_HIP, std::string("autotune flag: ") + hipGetErrorString(he));
            return false;
        }
        if (flag) return false;
        // ranked on the objective (Aitken), which the target is about; the
        // gradient-norm rate only when the objective gives no estimate
        const double ea = aitken_epochs(f, cps, target);
        if (ea >= 0.0) {
            *est_e = ea;
            return true;
        }
        if (at_floor) {
            // no estimate from the objective: twice the probe, for the race
            *est_e = 2.0 * (double)cps[2];
            return true;
        }
        const double r = probe_rate(g2, cps);
        if (r == 0.0) return false;
        const double goal = probe_goal(c, I, target, f[2], x2);
        const double more = g2[2] > goal ? 0.5 * std::log(g2[2] / goal) / r : 0.0;
        *est_e = (double)cps[2] + more;
        return true;
    };
    const int cps[3] = {probe_epochs / 3, 2 * probe_epochs / 3, probe_epochs};
    for (const UpdateShape& S : shapes) {
        c->shape = S;
        // kernel time per epoch at this shape
        if ((rc = reset_state(c))) break;
        hipError_t he = hipEventRecord(e0, c->st);
        if (he == hipSuccess && (rc = asaga_updates(c, I.m)) != ASAGA_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, c->st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
            rc = fail(c, ASAGA_E_HIP, std::string("autotune timing: ") + hipGetErrorString(he));
            break;
        }
        // Every later shape is slower per epoch.  A short probe's estimate is
        // too rough to rule the slower counts out (they tolerate larger
        // steps), so the search ends only once the probe alone takes four
        // times the best estimate so far.
        if ((double)probe_epochs * (double)ms * 1e-3 >= 4.0 * best.est_s) break;
        // steps from the largest down, while the estimate improves: past the
        // best stable step, smaller steps only converge more slowly
        double shape_best = INFINITY;
        for (double sc : scales) {
            ++tried;
            I.gamma = serial_rule * sc;
            double est_e = 0.0;
            const bool ok = probe(cps, &est_e);
            if (rc) break;
            // A failure does not end the ladder: above the stable steps a probe
            // can pass by chance (4096 wavefronts on the RCV1-shaped matrix:
            // even the serial rule, estimated at 100-200 epochs, now and then),
            // and the steps that work lie further down.  The ladder ends once
            // a passing step estimates worse than the best one of this shape.
            if (!ok) continue;
            const double est_s = est_e * (double)ms * 1e-3;
            stable_cands.push_back({est_s, est_e, (double)ms, I.gamma, S});
            if (est_s < best.est_s) best = stable_cands.back();
            if (est_s >= shape_best) break;
            shape_best = est_s;
        }
        if (rc) break;
    }
    // The short probes from x = 0 see mostly the fast early decrease.  A
    // step too large for its delay converges fastest there and then hovers
    // at a noise floor; with FP32 x a small step stalls at the floor FP32
    // additions leave.  Neither shows within a probe, so the finalists (per
    // wavefront count its largest stable step, the next smaller one and its
    // best-estimated one; at most eight, in order of their estimates) race
    // from x = 0 with a check every probe_epochs / 3 epochs: a finalist
    // finishes when the strong-convexity certificate holds or when Aitken's
    // limit of its last three objectives is within the target of the last
    // one at three checks in a row that agree on it, after falls of the
    // objective and of the gradient norm (below); it drops out once its
    // kernel time reaches the best finished one's, once it stops reaching
    // new minima for three checks (the noise floor), when a value turns
    // non-finite, or after 40 * probe_epochs epochs.  The finalist finished
    // in the least kernel time wins; if none finishes, the one that got
    // lowest.
    if (!rc && stable_cands.size() > 1) {
        std::vector<Cand> by_est = stable_cands;
        std::sort(by_est.begin(), by_est.end(), [](const Cand& a, const Cand& b) { return a.est_s < b.est_s; });
        std::vector<Cand> fin;
        auto add = [&](const Cand& k) {
            for (const Cand& q : fin)
                if (q.S.waves == k.S.waves && q.gamma == k.gamma) return;
            if (fin.size() < 8) fin.push_back(k);
        };
        for (const Cand& k : by_est) {
            // this count's largest and next smaller stable steps (candidates
            // were recorded from the largest step down)
            int taken = 0;
            for (const Cand& q : stable_cands)
                if (q.S.waves == k.S.waves && taken < 2) {
                    add(q);
                    ++taken;
                }
            add(k);
        }
        std::sort(fin.begin(), fin.end(), [](const Cand& a, const Cand& b) { return a.est_s < b.est_s; });
        // without a finisher: the finalist that got lowest while staying finite
        Cand lowest;
        double lowest_f = INFINITY;
        // with FP32 x, a tenth of the target, so that a run stalling at its
        // FP32 floor just above the target does not count as finished
        const double tgt = c->mixed ? 0.1 * target : target;
        best = Cand{};
        const int chk = std::max(1, probe_epochs / 3);
        const int max_e = 40 * probe_epochs;
        // one finalist's run from x = 0, up to the kernel time `bound`: true
        // if it finished, with its epochs in *e_out; *fmin_out the lowest
        // objective it reached
        auto race = [&](const Cand& k, double bound, int* e_out, double* fmin_out) -> bool {
            c->shape = k.S;
            I.gamma = k.gamma;
            *e_out = 0;
            *fmin_out = INFINITY;
            if ((rc = reset_state(c))) return false;
            std::vector<double> fs, gs;
            double fmin = INFINITY, prev_lim = NAN;
            int since_min = 0, e = 0, agreed = 0;
            bool finished = false;
            while (e < max_e && !finished) {
                if ((double)(e + chk) * k.ms * 1e-3 >= bound) break;  // cannot beat the best
                if ((rc = asaga_updates(c, (int64_t)chk * I.m))) break;
                e += chk;
                double g2 = 0.0, f = 0.0;
                if ((rc = grad_norm2(c, 0, &g2, &f))) break;
                if (!(std::isfinite(g2) && std::isfinite(f))) break;
                // the strong-convexity certificate alone (the FP32 gradient
                // floor of the probes holds long before the objective does)
                if (g2 <= 2.0 * I.lambda * tgt * f) finished = true;
                fs.push_back(f);
                gs.push_back(g2);
                if (f < fmin) {
                    fmin = f;
                    since_min = 0;
                } else if (++since_min >= 3) {
                    break;  // hovering: no new minimum for three checks
                }
                // Aitken's limit of the last three objectives (after three
                // falls of the objective and of the gradient norm): finished
                // when it is within tgt of the last objective at three checks
                // in a row that agree on it.  A run converging to a noise
                // floor instead of the optimum looks the same in the
                // objective, but there the gradient norm stops falling.
                const size_t n = fs.size();
                double lim = NAN;
                if (n >= 4 && fs[n - 1] < fs[n - 2] && fs[n - 2] < fs[n - 3] && fs[n - 3] < fs[n - 4] &&
                    gs[n - 1] < gs[n - 2] && gs[n - 2] < gs[n - 3] && gs[n - 3] < gs[n - 4]) {
                    const double d1 = fs[n - 2] - fs[n - 3], d2 = fs[n - 1] - fs[n - 2];
                    if (d2 / d1 > 0.0 && d2 / d1 < 1.0) lim = fs[n - 1] - d2 * d2 / (d2 - d1);
                }
                const bool near = std::isfinite(lim) && fs[n - 1] - lim <= tgt * std::fabs(lim);
                if (near && std::isfinite(prev_lim) && std::fabs(lim - prev_lim) <= tgt * std::fabs(lim))
                    ++agreed;
                else
                    agreed = 0;
                if (agreed >= 2) finished = true;
                prev_lim = near ? lim : NAN;
            }
            *e_out = e;
            *fmin_out = fmin;
            return finished && !rc;
        };
        bool have_finisher = false;
        for (const Cand& k : fin) {
            if (rc) break;
            ++tried;
            int e = 0;
            double fmin = INFINITY;
            const bool finished = race(k, best.est_s, &e, &fmin);
            if (rc) break;
            if (finished) {
                const double est_s = (double)e * k.ms * 1e-3;
                if (est_s < best.est_s) best = Cand{est_s, (double)e, k.ms, k.gamma, k.S};
                have_finisher = true;
            }
            if (fmin < lowest_f) {
                lowest_f = fmin;
                lowest = Cand{(double)e * k.ms * 1e-3, (double)e, k.ms, k.gamma, k.S};
            }
        }
        if (!rc && !std::isfinite(best.est_s) && std::isfinite(lowest_f)) best = lowest;
        // The winner once more in workgroups half as large (unless the caller
        // fixed the size): the same wavefronts over twice the compute units
        // shorten a sample's latency where few wavefronts share a unit, while
        // each hot set combines half as many samples' pending sums (more flush
        // requests per update) and refreshes its views at another pace, which
        // moves the stable step as well.  Measured on the URL-shaped instance
        // at 512 wavefronts and 0.075 of the rule: 256-thread workgroups 52 M
        // updates/s and 1e-9 after 81 epochs, 512-thread 49.5 M and 86,
        // 1024-thread 39 M and no convergence.  It is timed for one epoch and
        // kept if it finishes in less kernel time.
        if (!rc && have_finisher && c->o.threads_per_block == 0 && best.S.block >= 512) {
            Cand h = best;
            h.S.block = best.S.block / 2;
            c->shape = h.S;
            I.gamma = h.gamma;
            float ms = 0.0f;
            hipError_t he = hipSuccess;
            if ((rc = reset_state(c)) == ASAGA_OK) {
                he = hipEventRecord(e0, c->st);
                if (he == hipSuccess) rc = asaga_updates(c, I.m);
                if (!rc && he == hipSuccess) he = hipEventRecord(e1, c->st);
                if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
                if (!rc && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                if (!rc && he != hipSuccess)
                    rc = fail(c, ASAGA_E_HIP, std::string("autotune timing: ") + hipGetErrorString(he));
            }
            if (!rc && ms > 0.0f) {
                ++tried;
                h.ms = ms;
                int e = 0;
                double fmin = INFINITY;
                if (race(h, best.est_s, &e, &fmin) && (double)e * h.ms * 1e-3 < best.est_s)
                    best = Cand{(double)e * h.ms * 1e-3, (double)e, h.ms, h.gamma, h.S};
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        c->shape = base;
        return rc;
    }
    if (!std::isfinite(best.est_s)) {
        c->shape = base;
        I.gamma = c->o.step > 0.0 ? c->o.step : I.rule * std::min(1.0, kStepGroups / groups_in_flight(base));
        reset_state(c);
        return fail(c, ASAGA_E_DIVERGED, "no probed launch shape and step reduced the gradient norm steadily");
    }
    c->shape = best.S;
    I.gamma = best.gamma;
    // With FP32 state the run ends with an FP64 polish after asaga_widen.
    // The FP64 kernel serves its atomics faster, so at the same launch more
    // updates are in flight and, by Theorem 2, its largest stable step is
    // smaller: the Covtype-shaped instance at 1024 wavefronts overlaps 2587
    // updates in FP64 against 1615 with FP32 x and FP64 abar, and diverges in
    // FP64 at the largest step stable there.  When the choice is the largest
    // stable step probed at its count, the polish takes the next smaller one.
    c->widen_gamma = 0.0;
    if (c->mixed)
        for (const Cand& q : stable_cands)
            if (q.S.waves == best.S.waves) {  // recorded from the largest step down
                if (q.gamma == best.gamma) c->widen_gamma = best.gamma * std::exp2(-1.0 / 3.0);
                break;
            }
    if ((rc = reset_state(c))) return rc;
    if (rep) {
        rep->candidates = tried;
        rep->waves = best.S.waves;
        rep->hot_columns = best.S.hot;
        rep->hot_tier_columns = best.S.tier;
        rep->gamma = best.gamma;
        rep->ms_per_epoch = best.ms;
        rep->est_epochs = best.est_e;
        rep->est_seconds = best.est_s;
        rep->step_groups = 0.0;
        rep->step_cap = 0.0;
        rep->widen_gamma = c->widen_gamma > 0.0 ? c->widen_gamma : best.gamma;
        rep->threads_per_block = best.S.block;
    }
    return ASAGA_OK;
}

int asaga_overlap_estimate(const int64_t* log, int64_t n_logged, int64_t every, double clock_hz,
                           double updates_per_s, asaga_overlap_report* out) {
    if (!out || (n_logged > 0 && !log) || n_logged < 0 || every < 1 || !(clock_hz > 0.0))
        return fail(nullptr, ASAGA_E_ARG, "bad overlap estimate arguments");
    std::vector<int64_t> st, en;
    for (int64_t i = 0; i < n_logged; ++i) {
        const int64_t a = log[2 * i], b = log[2 * i + 1];
        if (a == 0) continue;
        if (b < a) return fail(nullptr, ASAGA_E_ARG, "overlap log pair ends before it starts");
        st.push_back(a);
        en.push_back(b);
    }
    *out = asaga_overlap_report{};
    out->logged = (int64_t)st.size();
    out->every = every;
    out->updates_per_s = updates_per_s;
    if (st.empty()) return ASAGA_OK;
    std::vector<int64_t> ss = st, es = en;
    std::sort(ss.begin(), ss.end());
    std::sort(es.begin(), es.end());
    std::vector<double> tau(st.size()), lat(st.size());
    double tsum = 0.0, lsum = 0.0;
    for (size_t i = 0; i < st.size(); ++i) {
        // started strictly before st[i], minus those already ended by then:
        // an interval that ended by st[i] also started before it
        const int64_t started = std::lower_bound(ss.begin(), ss.end(), st[i]) - ss.begin();
        const int64_t ended = std::upper_bound(es.begin(), es.end(), st[i]) - es.begin();
        tau[i] = (double)std::max<int64_t>(0, started - ended) * (double)every;
        lat[i] = (double)(en[i] - st[i]) / clock_hz * 1e6;
        tsum += tau[i];
        lsum += lat[i];
    }
    auto pct = [](std::vector<double> v, double q) {
        std::sort(v.begin(), v.end());
        return v[(size_t)std::min<double>((double)v.size() - 1, std::floor(q * (double)(v.size() - 1) + 0.5))];
    };
    out->tau_mean = tsum / (double)st.size();
    out->tau_p50 = pct(tau, 0.5);
    out->tau_p99 = pct(tau, 0.99);
    out->tau_max = *std::max_element(tau.begin(), tau.end());
    out->latency_mean_us = lsum / (double)st.size();
    out->latency_p99_us = pct(lat, 0.99);
    out->little = updates_per_s * out->latency_mean_us * 1e-6;
    return ASAGA_OK;
}

int asaga_overlap(asaga_ctx* c, int64_t n_epochs, asaga_overlap_report* out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!out || n_epochs < 1) return fail(c, ASAGA_E_ARG, "need a report and n_epochs >= 1");
    if (c->d_insts || c->shape.serial || !c->d_tau)
        return fail(c, ASAGA_E_STATE, "overlap logging needs a single-instance async context");
    const Inst& I = c->inst[0];
    int dev = 0, khz = 0;
    HIPCHK(c, hipGetDevice(&dev));
    HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(c, ASAGA_E_HIP, "the device reports no wall-clock rate");
    std::vector<int64_t> all;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    double secs = 0.0;
    int rc = ASAGA_OK;
    for (int64_t e = 0; e < n_epochs && !rc; ++e) {
        hipError_t he = launch_fill_i64(c->d_tau, 0, 2 * c->tau_cap, c->st);
        if (he == hipSuccess)
            he = launch_fill_i64(reinterpret_cast<long long*>(c->d_tau_count), 0, 1, c->st);
        if (he == hipSuccess) he = hipEventRecord(e0, c->st);
        if (he != hipSuccess) {
            rc = fail(c, ASAGA_E_HIP, std::string("overlap: ") + hipGetErrorString(he));
            break;
        }
        c->tau_on = true;
        rc = asaga_updates(c, I.m);
        c->tau_on = false;
        if (rc) break;
        he = hipEventRecord(e1, c->st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        unsigned long long used = 0;
        if (he == hipSuccess) he = hipMemcpy(&used, c->d_tau_count, 8, hipMemcpyDeviceToHost);
        const int64_t pairs = std::min<int64_t>((int64_t)used, c->tau_cap);
        const size_t at = all.size();
        all.resize(at + 2 * (size_t)pairs);
        if (he == hipSuccess && pairs > 0)
            he = hipMemcpy(all.data() + at, c->d_tau, (size_t)pairs * 16, hipMemcpyDeviceToHost);
        if (he != hipSuccess) rc = fail(c, ASAGA_E_HIP, std::string("overlap: ") + hipGetErrorString(he));
        secs += ms * 1e-3;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    rc = asaga_overlap_estimate(all.data(), (int64_t)all.size() / 2, (int64_t)kTauEvery, (double)khz * 1e3,
                                secs > 0.0 ? (double)(n_epochs * I.m) / secs : 0.0, out);
    if (rc) return fail(c, rc, asaga_last_error(nullptr));
    return check_flag(c);
}

int asaga_instance_get(asaga_ctx* c, int32_t inst, asaga_instance* out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!out) return fail(c, ASAGA_E_ARG, "NULL instance output");
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst];
    out->m = I.m;
    out->t = I.t;
    out->lambda = I.lambda;
    out->gamma = I.gamma;
    out->L = I.L;
    out->fold = I.fold;
    out->active = I.active ? 1 : 0;
    return ASAGA_OK;
}

int asaga_info_get(asaga_ctx* c, asaga_info* out) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    if (!out) return fail(c, ASAGA_E_ARG, "NULL info");
    const Inst& I = c->inst[0];
    out->n = c->n;
    out->d = c->d;
    out->nnz = c->nnz;
    out->delta_r = I.delta_r;
    out->t = I.t;
    out->L = I.L;
    out->gamma = I.gamma;
    out->lambda = I.lambda;
    out->waves = c->shape.waves;
    if (c->d_insts && c->o.waves == 0) {
        int n_act = 0;
        for (const Inst& J : c->inst) n_act += J.active ? 1 : 0;
        out->waves = (int32_t)batched_share(c, c->shape, n_act) * (c->shape.block / 64);
    }
    out->lanes_per_sample = c->shape.lanes;
    out->n_inst = (int32_t)c->inst.size();
    out->hot_columns = c->shape.hot;
    out->flush_every = c->shape.flush;
    out->threads_per_block = c->shape.block;
    out->hot_tier_columns = c->shape.tier;
    out->hot_tier_every = c->shape.serial ? c->shape.tier_every : tier_every_for(c, c->shape);
    out->hot_reload_from = out->hot_columns;
    if (c->shape.serial && !c->d_insts) {
        const int rf = view_reload_from(c, I, c->shape.hot, 1.0);
        if (rf < c->shape.hot) out->hot_reload_from = rf;
    } else if (!c->d_insts) {
        const double w = (double)((c->shape.waves * 64 + c->shape.block - 1) / c->shape.block);
        const int hot = stable_hot(c, I, c->shape.hot, w);
        const int rf = view_reload_from(c, I, hot, w);
        if (rf < hot) out->hot_reload_from = rf;
    } else if (c->d_insts && !c->plan_h.empty() && c->plan_h[0].reload_from < out->hot_columns) {
        out->hot_reload_from = c->plan_h[0].reload_from;
    }
    return ASAGA_OK;
}

int asaga_sync(asaga_ctx* c) {
    if (!c) return fail(nullptr, ASAGA_E_ARG, "NULL context");
    HIPCHK(c, hipStreamSynchronize(c->st));
    return check_flag(c);
}

int asaga_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out_host) {
    if (count < 0 || n < 1 || (!out_host && count > 0)) return fail(nullptr, ASAGA_E_ARG, "bad sample stream arguments");
    if (count == 0) return ASAGA_OK;
    int64_t* d = nullptr;
    hipError_t e = hipMalloc(&d, (size_t)count * 8);
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = launch_sample_stream(seed, t0, count, n, d, nullptr);
    if (e == hipSuccess) e = hipMemcpy(out_host, d, (size_t)count * 8, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_HIP, std::string("sample stream: ") + hipGetErrorString(e));
    return ASAGA_OK;
}

int asaga_request_ceiling(int64_t columns, double* atomic_per_s, double* mixed_per_s) {
    if (columns < 1 || columns > kMaxD || !atomic_per_s || !mixed_per_s)
        return fail(nullptr, ASAGA_E_ARG, "bad request ceiling arguments");
    double* xa = nullptr;
    hipError_t e = hipMalloc(&xa, (size_t)(2 * columns + 1) * sizeof(double));
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = launch_fill_f64(xa, 0.0, 2 * columns + 1, 1, st);
    // 4096 workgroups of 256 threads (2^19 lane pairs), 256 operations each
    const int blocks = 4096, iters = 256;
    double rate[2] = {0.0, 0.0};
    for (int mode = 0; mode < 2 && e == hipSuccess; ++mode) {
        e = launch_request_probe(xa, columns, blocks, 8, mode, xa + 2 * columns, st);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess) e = launch_request_probe(xa, columns, blocks, iters, mode, xa + 2 * columns, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        const double pairs = (double)blocks * 256.0 / 2.0;
        if (e == hipSuccess) rate[mode] = pairs * iters * (mode == 0 ? 1.0 : 2.0) / ((double)ms * 1e-3);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamSynchronize(st);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(xa);
    if (e != hipSuccess) return fail(nullptr, ASAGA_E_HIP, std::string("request ceiling: ") + hipGetErrorString(e));
    *atomic_per_s = rate[0];
    *mixed_per_s = rate[1];
    return ASAGA_OK;
}

const char* asaga_last_error(const asaga_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void asaga_free(asaga_ctx* c) {
    if (!c) return;
    free_all(c);
    delete c;
}

}  // extern "C"
