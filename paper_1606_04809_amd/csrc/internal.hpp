// Internal interface between the C-ABI host code (asaga.hip) and the device
// code (kernels.hip).  Not installed; not part of the public ABI.
//
// Device layout of one instance's state (columns relabelled by descending
// count, so the most-used columns are 0, 1, 2, ...), in an allocation of 2d
// doubles:
//   FP64 layout:   xa[2c] = x_c, xa[2c + 1] = abar_c (FP64)
//   mixed layout:  x_c FP32 in the low 4 bytes of xa[2c], abar_c FP64 in xa[2c + 1]
//   FP32 layout:   xf[2c] = x_c, xf[2c + 1] = abar_c (FP32, xf = (float*)xa; the
//                  first 8d bytes)
// so that one pair holds everything a sample reads and writes for a column,
// and two adjacent lanes reach both halves with one memory request (in the
// mixed layout the halves have different types: two requests).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asaga {

constexpr int kLayF64 = 0;
constexpr int kLayMixed = 1;
constexpr int kLayF32 = 2;

// Per-instance arguments of the update kernels.  A single solve is one
// instance whose row list is the identity (rows == nullptr).
struct InstArgs {
    const int32_t* rows;  // [m] training rows of the instance, or nullptr (= 0..n-1)
    double* xa;           // [2d] interleaved x / abar (layout above)
    void* alpha;          // [m]  FP64 or FP32 scalar memory, one per training row
    const double* D;      // [d]  m / cnt_c (0 for columns the instance never touches)
    int64_t m;            // number of training rows
    double gamma;
    double lambda;
    double inv_m;
    uint64_t seed;
    uint64_t t0;          // sample counter of the first update of this launch
    uint64_t count;       // updates this launch applies to the instance (0: skip it)
    int32_t blocks;       // batched: workgroups serving the instance
    int32_t frozen;       // 1: the memory (alpha, abar) is held fixed, only x is written
                          //    (the inner steps of sparse SVRG)
    int32_t reload_from;  // hot columns [reload_from, hot) that a workgroup did not write
                          //    are read again from global memory at each full flush
                          //    (>= hot: none)
    // overlap log (nullptr: off): a sample whose counter hashes to 0 modulo
    // kTauEvery (an independent thinning, unrelated to which lane group or
    // round runs it) takes the next entry e = (*tau_count)++ below tau_cap and
    // writes its read-start and writes-visible clock ticks to tau_log[2e],
    // tau_log[2e + 1]
    long long* tau_log;
    unsigned long long* tau_count;
    uint64_t tau_cap;
};
constexpr uint64_t kTauEvery = 1024;
constexpr int32_t kNoReload = 1 << 20;  // above any hot-set size

// Batched launches: workgroup b serves instance inst, as its rank-th
// workgroup (inst < 0: idle).
struct BlockMap {
    int32_t inst;
    int32_t rank;
};

struct MatArgs {
    const int64_t* rowptr;
    const int32_t* colidx;  // relabelled column indices
    const void* val;
    const double* b;
    int64_t n;
    int64_t d;
    int32_t val_dtype;   // ASAGA_VAL_*
    int32_t loss;        // ASAGA_LOSS_*
};

// Hot-set parameters the update kernels receive.
struct HotArgs {
    int hot, flush, tier, tier_every;
};

// launch shape and variant of the Sparse SAGA update kernel
struct UpdateShape {
    int lanes;        // lanes per sample: 64, 32, 16 or 8
    int waves;        // wavefronts in flight (1 for serial)
    int block;        // threads per workgroup
    int hot;          // columns [0, hot) combined in LDS per workgroup (0: none)
    int flush;        // samples per lane group between flushes of the LDS buffer
    int tier;         // columns [0, tier) flush every round, [tier, hot) every tier_every rounds
    int tier_every;
    bool serial;      // one wave, ordered: agent-scope fence between updates
    bool racy;        // plain read-modify-write (negative control)
    int layout;       // kLay*: state layout (FP32 x and alpha unless kLayF64)
};

// A read-only view of a vector: element v at p[v * stride], FP64 or FP32.
struct XView {
    const void* p;
    int64_t stride;
    int32_t f32;
};

hipError_t launch_updates(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag, hipStream_t st);
// One persistent grid of n_blocks workgroups over all instances, workgroup b
// serving instance dev_map[b].inst; instance k applies samples
// t0_k + epoch*count_k .. t0_k + (epoch+1)*count_k - 1.
hipError_t launch_updates_batched(const MatArgs& A, const InstArgs* dev_insts, const BlockMap* dev_map,
                                  int n_blocks, uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st);
// workgroups of the batched update kernel that fit on the device at once
int batched_resident_blocks(const UpdateShape& S, int32_t val_dtype);
size_t update_lds_bytes(const UpdateShape& S);

// initialisation
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st);
// stop test of a batch after epoch `epoch` of a call: proxy[k] = ||abar_k +
// lambda_k x_k||^2 for each instance k < n_inst still running; at or below
// thr[k] the instance is switched off (insts[k].count = 0, ran[k] = epoch + 1)
hipError_t launch_batch_proxy(InstArgs* insts, int n_inst, int64_t d, int layout, const double* thr, double* proxy,
                              int32_t* ran, int32_t epoch, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t count, int64_t stride, hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t st);
hipError_t launch_fill_i64(long long* p, long long v, int64_t count, hipStream_t st);
// cnt_c += #{j < m : c in S_rows[j]}; hot_first: the most-used columns are the
// lowest indices (after relabelling)
hipError_t launch_colcount(const MatArgs& A, const int32_t* rows, int64_t m, int32_t* cnt, bool hot_first,
                           hipStream_t st);
// out[k] = rank[in[k]]
hipError_t launch_relabel(const int32_t* in, int64_t nnz, const int32_t* rank, int32_t* out, hipStream_t st);
// D_c = m / cnt_c (0 if cnt_c = 0); stats[0] = max cnt, stats[1] = min positive cnt
hipError_t launch_reweight(const int32_t* cnt, int64_t d, int64_t m, double* D, int32_t* stats, hipStream_t st);
// bits of max_i ||a_i||^2 over the rows into *maxbits (uint64 ordering of non-negative doubles)
hipError_t launch_rownorm_max(const MatArgs& A, const int32_t* rows, int64_t m, unsigned long long* maxbits,
                              hipStream_t st);
// device-side CSR validation for borrowed device arrays: bits of *bad
hipError_t launch_validate(const MatArgs& A, int64_t nnz, int32_t* bad, hipStream_t st);

// evaluation: z_j = a_rows[j] . x
hipError_t launch_rowdot(const MatArgs& A, const int32_t* rows, int64_t m, XView x, double* z, hipStream_t st);
// tmp_j = phi(z_j; b_rows[j])
hipError_t launch_phi_terms(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double* tmp,
                            hipStream_t st);
// coef_j = phi'(z_j; b_rows[j]) * scale
hipError_t launch_dphi_coef(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double scale,
                            double* coef, hipStream_t st);
// coef_j = alpha_j * scale
hipError_t launch_alpha_coef(const void* alpha, bool f32, int64_t m, double scale, double* coef, hipStream_t st);
// out[c * stride] += sum_j coef_j a_rows[j],c   (atomic FP64)
hipError_t launch_scatter(const MatArgs& A, const int32_t* rows, int64_t m, const double* coef, double* out,
                          int64_t stride, hipStream_t st);
// g_c += lambda x_c
hipError_t launch_axpy_x(XView x, int64_t d, double lambda, double* g, hipStream_t st);
// sum of in[0..count) (two stages, pairwise over blocks) into *out; part needs kSumParts doubles
constexpr int kSumParts = 1024;
hipError_t launch_sum(const double* in, int64_t count, double* part, double* out, hipStream_t st);
hipError_t launch_sum_x2(XView x, int64_t d, double* part, double* out, hipStream_t st);
// *f = sums[0] / m + (lambda / 2) sums[1]: the objective from its two sums (one thread)
hipError_t launch_objective_finish(const double* sums, double m, double lambda, double* f, hipStream_t st);
// out[v] = x[rank[v]]  (back to the caller's column order)
hipError_t launch_gather_view(XView x, const int32_t* rank, int64_t d, double* out, hipStream_t st);
// slot[rank[v] * stride] = in[v]  (into the relabelled order; f32 stores a float in the slot)
hipError_t launch_scatter_slots(const double* in, const int32_t* rank, int64_t d, void* slot, int64_t stride, bool f32,
                                hipStream_t st);
hipError_t launch_widen_f32(const float* in, int64_t count, double* out, hipStream_t st);
// the FP32 x of the mixed-precision layout (low half of xa[2c]) widened in place to FP64
hipError_t launch_widen_x_slots(double* xa, int64_t d, hipStream_t st);
hipError_t launch_narrow_f64(const double* in, int64_t count, float* out, hipStream_t st);
// out[c * out_stride] = x[c], c < d  (a view copied to FP64)
hipError_t launch_copy_view(XView x, int64_t d, double* out, int64_t out_stride, hipStream_t st);
// slot[c * stride] = in[c], c < d, as FP32 (f32) or FP64
hipError_t launch_store_slots(const double* in, int64_t d, void* slot, int64_t stride, bool f32, hipStream_t st);

hipError_t launch_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out, hipStream_t st);
// memory-side request probe: blocks x 256 threads, iters operations per lane
// pair into xa[2 * cols]; mode 0 atomics only, mode 1 one coherent read and
// one atomic per iteration
hipError_t launch_request_probe(double* xa, int64_t cols, int blocks, int iters, int mode, double* sink,
                                hipStream_t st);

int device_cu_count();

}  // namespace asaga
