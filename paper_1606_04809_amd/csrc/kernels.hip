// Device code of the gfx950 Sparse SAGA / ASAGA library.
//
// The hot kernel is k_update: the Sparse SAGA update of Section 2 (Eq.
// SparseSAGA, with the projected L2 term of Section 4.2) applied lock-free by
// many wavefronts at once, as Algorithm 2 describes: each sample reads x and
// abar on its support without any lock (inconsistent reads), forms the dot
// product, the scalar gradient change delta = phi'(z) - alpha_i, and adds its
// update to x, abar and alpha_i with hardware atomic additions (Property 3).
//
// Mapping to CDNA (64-wide wavefronts):
//   * a group of G lanes (G = 64, 32, 16 or 8) owns one sample at a time, so a
//     wavefront carries 64/G samples; the sample index comes from a
//     counter-based stream, so no queue or global counter is needed;
//   * the row's column indices and values stream in coalesced, G entries per
//     load instruction; up to 128 entries per row stay in registers between
//     the read phase and the write phase;
//   * x, abar and D are gathered per entry; x and abar with relaxed
//     agent-scope atomic loads (coherent across the XCDs' L2 caches), D with
//     plain loads (read-only, cacheable);
//   * the dot product is reduced inside the group with cross-lane shuffles;
//   * the scatter uses global FP64/FP32 atomic add (no return value).
// There is no matrix-core work: the update is a sparse gather/scatter.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asaga.h"
#include "internal.hpp"

namespace asaga {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// SplitMix64 (Steele, Lea & Flood 2014): output number t+1 of the generator
// started from state `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// uniform index in [0, m): high word of the 128-bit product (Lemire)
__device__ __forceinline__ int64_t sample_index(uint64_t seed, uint64_t t, int64_t m) {
    return (int64_t)__umul64hi(splitmix64(seed, t), (uint64_t)m);
}

__device__ __forceinline__ double widen(double v) { return v; }
__device__ __forceinline__ double widen(float v) { return (double)v; }
__device__ __forceinline__ double widen(uint16_t bits) { return (double)__uint_as_float((uint32_t)bits << 16); }

// phi(z; b) of the logistic (log(1+exp(-bz))) or squared ((z-b)^2/2) loss
__device__ __forceinline__ double phi(double z, double b, int loss) {
    if (loss == ASAGA_LOSS_SQUARED) return 0.5 * (z - b) * (z - b);
    const double m = b * z;
    return m > 0.0 ? log1p(exp(-m)) : -m + log1p(exp(m));
}

// phi'(z; b): logistic -b / (1 + exp(b z)) evaluated without overflow
__device__ __forceinline__ double dphi(double z, double b, int loss) {
    if (loss == ASAGA_LOSS_SQUARED) return z - b;
    const double m = b * z;
    if (m > 0.0) {
        const double e = exp(-m);
        return -b * e / (1.0 + e);
    }
    return -b / (1.0 + exp(m));
}

// Shared-state access.  Relaxed atomics at agent scope: no ordering, but the
// value read is the one in the device-coherent level, not a stale line of
// another XCD's L2.
template <typename T>
__device__ __forceinline__ T load_state(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool RACY, typename T>
__device__ __forceinline__ void add_state(T* p, T v) {
    if constexpr (RACY) {
        // non-thread-safe read-modify-write (negative control)
        const T o = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p, o + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// sum over the G lanes of a group (G a power of two dividing 64)
template <int G>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) v += __shfl_xor(v, m, G);
    return v;
}

// ---------------------------------------------------------------------------
// the Sparse SAGA update of one sample, applied by a group of G lanes
// ---------------------------------------------------------------------------

template <int G, bool SERIAL, bool RACY, typename VT, typename XT>
__device__ __forceinline__ void apply_update(const MatArgs& A, const InstArgs& I, uint64_t t, int gl, int* flag) {
    constexpr int R = 128 / G;  // entries per lane kept in registers (rows up to 128 entries)
    const VT* __restrict__ val = static_cast<const VT*>(A.val);
    XT* x = static_cast<XT*>(I.x);
    XT* alpha = static_cast<XT*>(I.alpha);

    // sample (Algorithm 2: sample first, then read only the support)
    const int64_t j = sample_index(I.seed, t, I.m);
    const int64_t i = I.rows ? (int64_t)I.rows[j] : j;
    const int64_t rs = A.rowptr[i];
    const int64_t re = A.rowptr[i + 1];

    // read phase: x_hat, abar and D on S_i; partial dot product
    int32_t cc[R];
    double vv[R], xx[R], aa[R], dd[R];
    double zp = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t k = rs + gl + (int64_t)r * G;
        if (k < re) {
            const int32_t c = A.colidx[k];
            cc[r] = c;
            vv[r] = widen(val[k]);
            xx[r] = (double)load_state(x + c);
            aa[r] = load_state(I.abar + c);
            dd[r] = I.D[c];
            zp += vv[r] * xx[r];
        }
    }
    for (int64_t k = rs + gl + (int64_t)R * G; k < re; k += G) zp += widen(val[k]) * (double)load_state(x + A.colidx[k]);
    const double z = group_sum<G>(zp);

    // scalar gradient change against the memory
    double g = dphi(z, A.b[i], A.loss);
    if constexpr (sizeof(XT) == 4) g = (double)(float)g;  // stored memory is FP32: delta exact in FP64
    const double delta = g - (double)load_state(alpha + j);
    if (gl == 0 && !isfinite(delta)) *flag = 1;

    // write phase: x_v -= gamma (delta a_v + D_v (abar_v + lambda x_hat_v)); abar_v += delta a_v / m
    const double gam = I.gamma, lam = I.lambda, dm = delta * I.inv_m;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t k = rs + gl + (int64_t)r * G;
        if (k < re) {
            const double step = -gam * (delta * vv[r] + dd[r] * (aa[r] + lam * xx[r]));
            add_state<RACY>(x + cc[r], (XT)step);
            add_state<RACY>(I.abar + cc[r], dm * vv[r]);
        }
    }
    for (int64_t k = rs + gl + (int64_t)R * G; k < re; k += G) {
        const int32_t c = A.colidx[k];
        const double v = widen(val[k]);
        const double xo = (double)load_state(x + c);
        const double ab = load_state(I.abar + c);
        const double step = -gam * (delta * v + I.D[c] * (ab + lam * xo));
        add_state<RACY>(x + c, (XT)step);
        add_state<RACY>(I.abar + c, dm * v);
    }
    if (gl == 0) add_state<RACY>(alpha + j, (XT)delta);
    if constexpr (SERIAL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
}

// One instance: updates t0 .. t0+count-1, sample slot s = wave*(64/G) + group,
// strided by the number of slots in the grid.
template <int G, bool SERIAL, bool RACY, typename VT, typename XT>
__global__ void __launch_bounds__(256) k_update(MatArgs A, InstArgs I, int* flag) {
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t slots = (((uint64_t)gridDim.x * blockDim.x) >> 6) * SPW;
    for (uint64_t s = wave * SPW + (uint64_t)(lane / G); s < I.count; s += slots)
        apply_update<G, SERIAL, RACY, VT, XT>(A, I, I.t0 + s, lane & (G - 1), flag);
}

// Many instances in one persistent grid: waves_per_inst consecutive
// wavefronts serve one instance.
template <int G, typename VT, typename XT>
__global__ void __launch_bounds__(256) k_update_batched(MatArgs A, const InstArgs* insts, int n_inst, int wpi,
                                                        uint64_t epoch, int* flag) {
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int inst = (int)(wave / (uint64_t)wpi);
    if (inst >= n_inst) return;
    const InstArgs I = insts[inst];
    const uint64_t lw = wave % (uint64_t)wpi;
    const uint64_t slots = (uint64_t)wpi * SPW;
    const uint64_t t0 = I.t0 + epoch * I.count;
    for (uint64_t s = lw * SPW + (uint64_t)(lane / G); s < I.count; s += slots)
        apply_update<G, false, false, VT, XT>(A, I, t0 + s, lane & (G - 1), flag);
}

// ---------------------------------------------------------------------------
// launchers for the update kernels
// ---------------------------------------------------------------------------

template <typename VT, typename XT>
static hipError_t launch_updates_t(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag,
                                   hipStream_t st) {
    if (I.count == 0) return hipSuccess;
    if (S.serial) {
        k_update<64, true, false, VT, XT><<<1, 64, 0, st>>>(A, I, flag);
        return hipGetLastError();
    }
    const int threads = 256;
    const int blocks = (S.waves * 64 + threads - 1) / threads;
#define ASAGA_LAUNCH(GG)                                                                   \
    case GG:                                                                               \
        if (S.racy)                                                                        \
            k_update<GG, false, true, VT, XT><<<blocks, threads, 0, st>>>(A, I, flag);     \
        else                                                                               \
            k_update<GG, false, false, VT, XT><<<blocks, threads, 0, st>>>(A, I, flag);    \
        break;
    switch (S.lanes) {
        ASAGA_LAUNCH(64)
        ASAGA_LAUNCH(32)
        ASAGA_LAUNCH(16)
        ASAGA_LAUNCH(8)
        default: return hipErrorInvalidValue;
    }
#undef ASAGA_LAUNCH
    return hipGetLastError();
}

hipError_t launch_updates(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag, hipStream_t st) {
    switch (A.val_dtype) {
        case ASAGA_VAL_F64:
            return S.mixed ? launch_updates_t<double, float>(A, I, S, flag, st)
                           : launch_updates_t<double, double>(A, I, S, flag, st);
        case ASAGA_VAL_F32:
            return S.mixed ? launch_updates_t<float, float>(A, I, S, flag, st)
                           : launch_updates_t<float, double>(A, I, S, flag, st);
        case ASAGA_VAL_BF16:
            return S.mixed ? launch_updates_t<uint16_t, float>(A, I, S, flag, st)
                           : launch_updates_t<uint16_t, double>(A, I, S, flag, st);
    }
    return hipErrorInvalidValue;
}

template <typename VT, typename XT>
static hipError_t launch_batched_t(const MatArgs& A, const InstArgs* insts, int n_inst, int wpi, uint64_t epoch,
                                   const UpdateShape& S, int* flag, hipStream_t st) {
    const int threads = 256;
    const int64_t waves = (int64_t)n_inst * wpi;
    const int blocks = (int)((waves * 64 + threads - 1) / threads);
    switch (S.lanes) {
        case 64: k_update_batched<64, VT, XT><<<blocks, threads, 0, st>>>(A, insts, n_inst, wpi, epoch, flag); break;
        case 32: k_update_batched<32, VT, XT><<<blocks, threads, 0, st>>>(A, insts, n_inst, wpi, epoch, flag); break;
        case 16: k_update_batched<16, VT, XT><<<blocks, threads, 0, st>>>(A, insts, n_inst, wpi, epoch, flag); break;
        case 8: k_update_batched<8, VT, XT><<<blocks, threads, 0, st>>>(A, insts, n_inst, wpi, epoch, flag); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_updates_batched(const MatArgs& A, const InstArgs* dev_insts, int n_inst, int waves_per_inst,
                                  uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    switch (A.val_dtype) {
        case ASAGA_VAL_F64:
            return S.mixed ? launch_batched_t<double, float>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st)
                           : launch_batched_t<double, double>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st);
        case ASAGA_VAL_F32:
            return S.mixed ? launch_batched_t<float, float>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st)
                           : launch_batched_t<float, double>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st);
        case ASAGA_VAL_BF16:
            return S.mixed ? launch_batched_t<uint16_t, float>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st)
                           : launch_batched_t<uint16_t, double>(A, dev_insts, n_inst, waves_per_inst, epoch, S, flag, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// initialisation kernels
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t items, int threads, int cap = 65536) {
    int64_t b = (items + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

template <typename T>
__global__ void k_fill(T* p, T v, int64_t count) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<int32_t><<<grid_for(count, 256), 256, 0, st>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<double><<<grid_for(count, 256), 256, 0, st>>>(p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<float><<<grid_for(count, 256), 256, 0, st>>>(p, v, count);
    return hipGetLastError();
}

// 16 lanes per row for the evaluation and set-up passes (not on the hot path)
constexpr int kRowLanes = 16;

__device__ __forceinline__ int64_t row_of(const int32_t* rows, int64_t j) { return rows ? (int64_t)rows[j] : j; }

__global__ void k_colcount(MatArgs A, const int32_t* rows, int64_t m, int32_t* cnt) {
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes) atomicAdd(cnt + A.colidx[k], 1);
    }
}

hipError_t launch_colcount(const MatArgs& A, const int32_t* rows, int64_t m, int32_t* cnt, hipStream_t st) {
    k_colcount<<<grid_for(m * kRowLanes, 256), 256, 0, st>>>(A, rows, m, cnt);
    return hipGetLastError();
}

__global__ void k_reweight(const int32_t* cnt, int64_t d, int64_t m, double* D, int32_t* stats) {
    int32_t mx = 0, mn = 0x7fffffff;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = cnt[v];
        D[v] = c > 0 ? (double)m / (double)c : 0.0;
        if (c > mx) mx = c;
        if (c > 0 && c < mn) mn = c;
    }
    atomicMax(stats + 0, mx);
    atomicMin(stats + 1, mn);
}

hipError_t launch_reweight(const int32_t* cnt, int64_t d, int64_t m, double* D, int32_t* stats, hipStream_t st) {
    k_reweight<<<grid_for(d, 256, 1024), 256, 0, st>>>(cnt, d, m, D, stats);
    return hipGetLastError();
}

template <typename VT>
__global__ void k_rownorm_max(MatArgs A, const int32_t* rows, int64_t m, unsigned long long* maxbits) {
    const VT* val = static_cast<const VT*>(A.val);
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    double best = 0.0;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        double s = 0.0;
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes) {
            const double v = widen(val[k]);
            s += v * v;
        }
        s = group_sum<kRowLanes>(s);
        if (s > best) best = s;
    }
    if (gl == 0) atomicMax(maxbits, (unsigned long long)__double_as_longlong(best));
}

hipError_t launch_rownorm_max(const MatArgs& A, const int32_t* rows, int64_t m, unsigned long long* maxbits,
                              hipStream_t st) {
    const int blocks = grid_for(m * kRowLanes, 256);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_rownorm_max<double><<<blocks, 256, 0, st>>>(A, rows, m, maxbits); break;
        case ASAGA_VAL_F32: k_rownorm_max<float><<<blocks, 256, 0, st>>>(A, rows, m, maxbits); break;
        case ASAGA_VAL_BF16: k_rownorm_max<uint16_t><<<blocks, 256, 0, st>>>(A, rows, m, maxbits); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// bad bits: 1 rowptr, 2 empty row, 4 column out of range, 8 columns not
// strictly increasing, 16 non-finite value, 32 bad label
template <typename VT>
__global__ void k_validate(MatArgs A, int64_t nnz, int32_t* bad) {
    const VT* val = static_cast<const VT*>(A.val);
    int32_t flags = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = A.rowptr[i], e = A.rowptr[i + 1];
        if (s < 0 || e > nnz || e < s) {
            flags |= 1;
            continue;
        }
        if (e == s) flags |= 2;
        int64_t prev = -1;
        for (int64_t k = s; k < e; ++k) {
            const int64_t c = A.colidx[k];
            if (c < 0 || c >= A.d) flags |= 4;
            if (c <= prev) flags |= 8;
            prev = c;
            if (!isfinite(widen(val[k]))) flags |= 16;
        }
        const double b = A.b[i];
        if (!isfinite(b) || (A.loss == ASAGA_LOSS_LOGISTIC && b != 1.0 && b != -1.0)) flags |= 32;
    }
    if (flags) atomicOr(bad, flags);
}

hipError_t launch_validate(const MatArgs& A, int64_t nnz, int32_t* bad, hipStream_t st) {
    const int blocks = grid_for(A.n, 256);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_validate<double><<<blocks, 256, 0, st>>>(A, nnz, bad); break;
        case ASAGA_VAL_F32: k_validate<float><<<blocks, 256, 0, st>>>(A, nnz, bad); break;
        case ASAGA_VAL_BF16: k_validate<uint16_t><<<blocks, 256, 0, st>>>(A, nnz, bad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// evaluation kernels (objective, gradient, re-anchoring of abar)
// ---------------------------------------------------------------------------

template <typename VT, typename XT>
__global__ void k_rowdot(MatArgs A, const int32_t* rows, int64_t m, const XT* x, double* z) {
    const VT* val = static_cast<const VT*>(A.val);
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        double s = 0.0;
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes)
            s += widen(val[k]) * (double)x[A.colidx[k]];
        s = group_sum<kRowLanes>(s);
        if (gl == 0) z[j] = s;
    }
}

template <typename XT>
static hipError_t launch_rowdot_x(const MatArgs& A, const int32_t* rows, int64_t m, const XT* x, double* z,
                                  hipStream_t st) {
    const int blocks = grid_for(m * kRowLanes, 256);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_rowdot<double, XT><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        case ASAGA_VAL_F32: k_rowdot<float, XT><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        case ASAGA_VAL_BF16: k_rowdot<uint16_t, XT><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rowdot(const MatArgs& A, const int32_t* rows, int64_t m, const void* x, bool x_f32, double* z,
                         hipStream_t st) {
    return x_f32 ? launch_rowdot_x<float>(A, rows, m, static_cast<const float*>(x), z, st)
                 : launch_rowdot_x<double>(A, rows, m, static_cast<const double*>(x), z, st);
}

__global__ void k_phi_terms(MatArgs A, const int32_t* rows, int64_t m, const double* z, double* tmp) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        tmp[j] = phi(z[j], A.b[row_of(rows, j)], A.loss);
}

hipError_t launch_phi_terms(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double* tmp,
                            hipStream_t st) {
    k_phi_terms<<<grid_for(m, 256), 256, 0, st>>>(A, rows, m, z, tmp);
    return hipGetLastError();
}

__global__ void k_dphi_coef(MatArgs A, const int32_t* rows, int64_t m, const double* z, double scale, double* coef) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        coef[j] = dphi(z[j], A.b[row_of(rows, j)], A.loss) * scale;
}

hipError_t launch_dphi_coef(const MatArgs& A, const int32_t* rows, int64_t m, const double* z, double scale,
                            double* coef, hipStream_t st) {
    k_dphi_coef<<<grid_for(m, 256), 256, 0, st>>>(A, rows, m, z, scale, coef);
    return hipGetLastError();
}

template <typename XT>
__global__ void k_alpha_coef(const XT* alpha, int64_t m, double scale, double* coef) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x)
        coef[j] = (double)alpha[j] * scale;
}

hipError_t launch_alpha_coef(const void* alpha, bool f32, int64_t m, double scale, double* coef, hipStream_t st) {
    if (f32)
        k_alpha_coef<float><<<grid_for(m, 256), 256, 0, st>>>(static_cast<const float*>(alpha), m, scale, coef);
    else
        k_alpha_coef<double><<<grid_for(m, 256), 256, 0, st>>>(static_cast<const double*>(alpha), m, scale, coef);
    return hipGetLastError();
}

template <typename VT>
__global__ void k_scatter(MatArgs A, const int32_t* rows, int64_t m, const double* coef, double* out) {
    const VT* val = static_cast<const VT*>(A.val);
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        const double cj = coef[j];
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes)
            __hip_atomic_fetch_add(out + A.colidx[k], cj * widen(val[k]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_scatter(const MatArgs& A, const int32_t* rows, int64_t m, const double* coef, double* out,
                          hipStream_t st) {
    const int blocks = grid_for(m * kRowLanes, 256);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_scatter<double><<<blocks, 256, 0, st>>>(A, rows, m, coef, out); break;
        case ASAGA_VAL_F32: k_scatter<float><<<blocks, 256, 0, st>>>(A, rows, m, coef, out); break;
        case ASAGA_VAL_BF16: k_scatter<uint16_t><<<blocks, 256, 0, st>>>(A, rows, m, coef, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename XT>
__global__ void k_axpy_x(const XT* x, int64_t d, double lambda, double* g) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d; v += (int64_t)gridDim.x * blockDim.x)
        g[v] += lambda * (double)x[v];
}

hipError_t launch_axpy_x(const void* x, bool x_f32, int64_t d, double lambda, double* g, hipStream_t st) {
    if (x_f32)
        k_axpy_x<float><<<grid_for(d, 256), 256, 0, st>>>(static_cast<const float*>(x), d, lambda, g);
    else
        k_axpy_x<double><<<grid_for(d, 256), 256, 0, st>>>(static_cast<const double*>(x), d, lambda, g);
    return hipGetLastError();
}

// two-stage sum: each thread keeps a compensated (Neumaier) running sum over
// a strided slice, blocks reduce pairwise in LDS, one block reduces the
// kSumParts block results.
__device__ __forceinline__ void neumaier(double& s, double& c, double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

template <int THREADS>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = THREADS / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

template <typename T, bool SQUARE>
__global__ void __launch_bounds__(256) k_sum_stage1(const T* in, int64_t count, double* part) {
    double s = 0.0, c = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        double v = (double)in[k];
        if (SQUARE) v *= v;
        neumaier(s, c, v);
    }
    const double r = block_sum<256>(s + c);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kSumParts) k_sum_stage2(const double* part, double* out) {
    const double r = block_sum<kSumParts>(part[threadIdx.x]);
    if (threadIdx.x == 0) *out = r;
}

template <typename T, bool SQUARE>
static hipError_t launch_sum_t(const T* in, int64_t count, double* part, double* out, hipStream_t st) {
    k_sum_stage1<T, SQUARE><<<kSumParts, 256, 0, st>>>(in, count, part);
    k_sum_stage2<<<1, kSumParts, 0, st>>>(part, out);
    return hipGetLastError();
}

hipError_t launch_sum(const double* in, int64_t count, bool square, double* part, double* out, hipStream_t st) {
    return square ? launch_sum_t<double, true>(in, count, part, out, st)
                  : launch_sum_t<double, false>(in, count, part, out, st);
}

hipError_t launch_sum_x2(const void* x, bool x_f32, int64_t d, double* part, double* out, hipStream_t st) {
    return x_f32 ? launch_sum_t<float, true>(static_cast<const float*>(x), d, part, out, st)
                 : launch_sum_t<double, true>(static_cast<const double*>(x), d, part, out, st);
}

__global__ void k_widen(const float* in, int64_t count, double* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (double)in[k];
}
__global__ void k_narrow(const double* in, int64_t count, float* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (float)in[k];
}

hipError_t launch_widen_f32(const float* in, int64_t count, double* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_widen<<<grid_for(count, 256), 256, 0, st>>>(in, count, out);
    return hipGetLastError();
}
hipError_t launch_narrow_f64(const double* in, int64_t count, float* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_narrow<<<grid_for(count, 256), 256, 0, st>>>(in, count, out);
    return hipGetLastError();
}

__global__ void k_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = sample_index(seed, t0 + (uint64_t)k, n);
}

hipError_t launch_sample_stream(uint64_t seed, uint64_t t0, int64_t count, int64_t n, int64_t* out, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_sample_stream<<<grid_for(count, 256), 256, 0, st>>>(seed, t0, count, n, out);
    return hipGetLastError();
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace asaga
