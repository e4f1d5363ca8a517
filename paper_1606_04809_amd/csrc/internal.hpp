// Internal interface between the C-ABI host code (asaga.hip) and the device
// code (kernels.hip).  Not installed; not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace asaga {

// Per-instance arguments of the update kernels.  A single solve is one
// instance whose row list is the identity (rows == nullptr).
struct InstArgs {
    const int32_t* rows;  // [m] training rows of the instance, or nullptr (= 0..n-1)
    void* x;              // [d]  FP64 or FP32 iterate
    void* alpha;          // [m]  FP64 or FP32 scalar memory, one per training row
    double* abar;         // [d]  running average (1/m) sum_j alpha_j a_rows[j]
    const double* D;      // [d]  m / cnt_v (0 for columns the instance never touches)
    int64_t m;            // number of training rows
    double gamma;
    double lambda;
    double inv_m;
    uint64_t seed;
    uint64_t t0;          // sample counter of the first update of this launch
    uint64_t count;       // updates this launch applies to the instance
};

struct MatArgs {
    const int64_t* rowptr;
    const int32_t* colidx;
    const void* val;
    const double* b;
    int64_t n;
    int64_t d;
    int32_t val_dtype;   // ASAGA_VAL_*
    int32_t loss;        // ASAGA_LOSS_*
};

// launch shape and variant of the Sparse SAGA update kernel
struct UpdateShape {
    int lanes;        // lanes per sample: 64, 32, 16 or 8
    int waves;        // wavefronts in flight (1 for serial)
    bool serial;      // one wave, ordered: agent-scope fence between updates
    bool racy;        // plain read-modify-write (negative control)
    bool mixed;       // FP32 x and alpha
};

hipError_t launch_updates(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag, hipStream_t st);
// Instance k applies samples t0_k + epoch*count_k .. t0_k + (epoch+1)*count_k - 1.
hipError_t launch_updates_batched(const MatArgs& A, const InstArgs* dev_insts, int n_inst, int waves_per_inst,
                                  uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st);

// initialisation
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st);
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t st);
hipError_t launch_colcount(const MatArgs& A, const int32_t* rows, int64_t m, int32_t* cnt, hipStream_t st);
// D_v = m / cnt_v (0 if cnt_v = 0); stats[0] = max cnt, stats[1] = min positive cnt
hipError_t launch_reweight(const int32_t* cnt, int64_t d, int64_t m, double* D, int32_t* stats, hipStream_t st);
// bits of max_i ||a_i||^2 over the rows into *maxbits (uint64 ordering of non-negative doubles)
hipError_t launch_rownorm_max(const MatArgs& A, const int32_t* rows, int64_t m, unsigned long long* maxbits,
                              hipStream_t st);
// device-side CSR validation for borrowed device arrays: bits of *bad
hipError_t launch_validate(const MatArgs& A, int64_t nnz, int32_t* bad, hipStream_t st);

// evaluation: z_j = a_rows[j] . x
hipError_t launch_rowdot(const MatArgs& A, const int32_t* rows, int64_t m, const void* x, bool x_f32, double* z,
                         hipStream_t st);
// tmp_j = phi(z_j; b_rows[j])
hipError_t launch_phi_terms(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double* tmp,
                            hipStream_t st);
// coef_j = phi'(z_j; b_rows[j]) * scale
hipError_t launch_dphi_coef(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double scale,
                            double* coef, hipStream_t st);
// coef_j = alpha_j * scale
hipError_t launch_alpha_coef(const void* alpha, bool f32, int64_t m, double scale, double* coef, hipStream_t st);
// out_v += sum_j coef_j a_rows[j],v   (atomic FP64)
hipError_t launch_scatter(const MatArgs& A, const int32_t* rows, int64_t m, const double* coef, double* out,
                          hipStream_t st);
// g_v += lambda x_v
hipError_t launch_axpy_x(const void* x, bool x_f32, int64_t d, double lambda, double* g, hipStream_t st);
// sum of in[0..count) (two stages, pairwise over blocks) into *out; part needs kSumParts doubles
constexpr int kSumParts = 1024;
hipError_t launch_sum(const double* in, int64_t count, bool square, double* part, double* out, hipStream_t st);
hipError_t launch_sum_x2(const void* x, bool x_f32, int64_t d, double* part, double* out, hipStream_t st);
// conversions between the FP64 host-facing form and the state's storage type
hipError_t launch_widen_f32(const float* in, int64_t count, double* out, hipStream_t st);
hipError_t launch_narrow_f64(const double* in, int64_t count, float* out, hipStream_t st);

hipError_t launch_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out, hipStream_t st);

int device_cu_count();

}  // namespace asaga
