// Device code of the gfx950 Sparse SAGA / ASAGA library.
//
// The hot kernel is k_update: the Sparse SAGA update of Section 2 (Eq.
// SparseSAGA, with the projected L2 term of Section 4.2) applied lock-free by
// many wavefronts at once, as Algorithm 2 describes: each sample reads x and
// abar on its support without any lock (inconsistent reads), forms the dot
// product and the scalar gradient change delta = phi'(z) - alpha_i, and adds
// its update to x, abar and alpha_i with atomic additions (Property 3).
//
// Mapping to CDNA4 (64-wide wavefronts).  Measured on MI355X: FP64 global
// atomics execute at the memory side, which serves about 2.3e10 requests/s,
// where one request is one wave instruction's lanes that fall in one 64-byte
// line (up to 8 FP64 adds), and a single address takes at most 8.3e7
// atomics/s.  Hence:
//   * a group of G lanes (64, 32, 16 or 8) owns one sample; the sample index
//     comes from a counter-based stream, so no queue or global counter, and
//     the next sample's row bounds are fetched while the current one runs;
//   * the read phase gathers x_c with one lane per row entry; the dot product
//     is reduced inside the group with cross-lane shuffles;
//   * the write phase works in lane pairs, one row entry per pair: the even
//     lane carries x_c, the odd lane abar_c.  x and abar are interleaved per
//     column (16 bytes in FP64, 8 in the FP32 layout), so the pair's load and
//     the pair's atomic add are each one memory request (in the mixed layout,
//     FP32 x beside FP64 abar, the add takes two);
//   * rows of up to 2G entries keep their column indices, values and state
//     in registers between the read and the write phase; longer rows are
//     processed in chunks and read again;
//   * columns are relabelled by descending count, so the most-used columns
//     are [0, H).  Each workgroup keeps them in LDS: a view of the global
//     values and its own pending additions (LDS atomics run at ~1e12/s).
//     Every F samples per group the workgroup adds its pending sums to the
//     global state with line-coalesced atomics and refreshes the touched
//     part of the view from the values those atomics return; the first tier
//     of hot columns (those nearly every row touches) is flushed every
//     round, the rest of the hot set every few rounds, when the untouched
//     views of the rarest hot columns are reloaded too if the host finds
//     their lag too long for the step.  Reads of hot columns touch only
//     LDS; this removes the per-line serialisation of the columns every row
//     touches, and the tag stalls of reading lines with atomics in flight.
// The same kernels run the inner steps of sparse SVRG (Appendix C) with the
// memory frozen (InstArgs::frozen: no abar or alpha writes), and can log a
// sample of updates' read and completion clocks (InstArgs::tau_log).
// There is no matrix-core work: the update is a sparse gather/scatter.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "asaga.h"
#include "internal.hpp"

namespace asaga {

// LDS of a workgroup with a hot set of H columns, both halves interleaved
// like the state:  [0, 2H)   view: the global (x, abar) values at the last flush
//                  [2H, 4H)  pend: the workgroup's own additions since then
// in FP64 (FP64 and mixed layouts) or FP32 (FP32 layout: 16 bytes per column,
// so twice the columns fit).
extern __shared__ double lds[];

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

// State layouts (kLay* in internal.hpp): x and alpha are FP32 in the mixed
// and FP32 layouts; abar is FP32 too in the FP32 layout, where a column's
// (x, abar) pair takes 8 bytes instead of 16.
template <int LAY>
constexpr bool kX32 = LAY != kLayF64;
template <int LAY>
constexpr bool kS32 = LAY == kLayF32;

// hot-set LDS entry i (view or pending half) in the layout's precision
template <int LAY>
__device__ __forceinline__ double lds_get(int i) {
    if constexpr (kS32<LAY>) return (double)reinterpret_cast<const float*>(lds)[i];
    else return lds[i];
}

template <int LAY>
__device__ __forceinline__ void lds_add(int i, double w) {
    if constexpr (kS32<LAY>) atomicAdd(reinterpret_cast<float*>(lds) + i, (float)w);
    else atomicAdd(&lds[i], w);
}

// Shared-state reads: relaxed atomics at agent scope (no ordering; the value
// comes from the device-coherent level).
template <int LAY>
__device__ __forceinline__ double load_alpha(const void* alpha, int64_t j) {
    if constexpr (kX32<LAY>)
        return (double)__hip_atomic_load(const_cast<float*>(static_cast<const float*>(alpha)) + j, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    else
        return __hip_atomic_load(const_cast<double*>(static_cast<const double*>(alpha)) + j, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
}

template <bool RACY, typename T>
__device__ __forceinline__ void add_global(T* p, T v) {
    if constexpr (RACY) {
        // non-thread-safe read-modify-write (negative control)
        const T o = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p, o + v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// add w to slot (c, comp) of the state: LDS pending sum for hot columns,
// global atomic otherwise.  In the FP32 layout both lanes of a pair add to
// the same 8 bytes with the same instruction: one memory request.
template <bool RACY, int LAY>
__device__ __forceinline__ void add_slot(double* xa, int32_t c, int comp, int hot, double w) {
    if (c < hot) {
        lds_add<LAY>(2 * hot + 2 * c + comp, w);
    } else if constexpr (kS32<LAY>) {
        add_global<RACY, float>(reinterpret_cast<float*>(xa) + 2 * (int64_t)c + comp, (float)w);
    } else if (LAY == kLayMixed && comp == 0) {
        add_global<RACY, float>(reinterpret_cast<float*>(xa + 2 * (int64_t)c), (float)w);
    } else {
        add_global<RACY, double>(xa + 2 * (int64_t)c + comp, w);
    }
}

template <bool RACY, int LAY>
__device__ __forceinline__ void add_alpha(void* alpha, int64_t j, double delta) {
    if constexpr (kX32<LAY>)
        add_global<RACY, float>(static_cast<float*>(alpha) + j, (float)delta);
    else
        add_global<RACY, double>(static_cast<double*>(alpha) + j, delta);
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

// The (x_c, abar_c) pair of column c: one 16-byte load (FP32 layout: 8
// bytes) with the sc1 cache policy (served from the device-coherent level,
// like an agent-scope atomic load; lines that atomics modify are served from
// there whatever the policy), through a buffer descriptor whose range check
// returns zeros for an offset past the state (the CDNA descriptor word 3 is
// 0x00020000).
struct Pair {
    double x, a;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const double* xa, int64_t d) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(xa), (short)0, (int)(d * 16), 0x00020000);
}

// Columns below `hot` are served from LDS: their load gets an offset past
// the descriptor's range, which the hardware drops (it returns zeros and
// sends no request), so the read needs no branch.  The FP32 layout's pair
// is one 8-byte load.
template <int LAY>
__device__ __forceinline__ Pair load_pair(__amdgpu_buffer_rsrc_t r, int32_t c, int hot) {
    constexpr int kSC1 = 16;
    Pair p;
    if constexpr (kS32<LAY>) {
        const int off = c >= hot ? c * 8 : (int)0x7ffffff0;
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kSC1);
        p.x = (double)__uint_as_float(v[0]);
        p.a = (double)__uint_as_float(v[1]);
    } else {
        const int off = c >= hot ? c * 16 : (int)0x7ffffff0;
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kSC1);
        if (LAY == kLayMixed) p.x = (double)__uint_as_float(v[0]);
        else p.x = __longlong_as_double((long long)(((uint64_t)v[1] << 32) | v[0]));
        p.a = __longlong_as_double((long long)(((uint64_t)v[3] << 32) | v[2]));
    }
    return p;
}

// Row of one sample: j (index into the instance's rows), i (matrix row),
// bounds, label, and (asynchronous mode) an early read of alpha_j.
struct RowRef {
    int64_t j, i, rs, re;
    double b, alpha;
};

template <bool SERIAL, int LAY>
__device__ __forceinline__ RowRef row_ref(const MatArgs& A, const InstArgs& I, uint64_t t) {
    RowRef r;
    r.j = sample_index(I.seed, t, I.m);
    r.i = I.rows ? (int64_t)I.rows[r.j] : r.j;
    r.rs = A.rowptr[r.i];
    r.re = A.rowptr[r.i + 1];
    r.b = A.b[r.i];
    r.alpha = SERIAL ? 0.0 : load_alpha<LAY>(I.alpha, r.j);
    return r;
}

// Sample j is processed by one group of G lanes working in pairs: the pair
// (2e, 2e+1) takes the row entries e, e + G/2, e + G, ...  Both lanes of a
// pair load the entry's column, value and (x_c, abar_c) pair (one request
// each for the pair); the even lane adds a_c x_hat_c to the dot product and
// later adds the x step, the odd lane adds the abar step.  Rows of up to
// P * G / 2 entries are held in registers between the two phases, with all
// their loads issued together; longer rows are processed in chunks and read
// again for the write phase.
template <int G, int P, bool SERIAL, bool RACY, int LAY, typename VT>
__device__ __forceinline__ void apply_update(const MatArgs& A, const InstArgs& I, const RowRef& rr, int gl, int hot,
                                             int* flag) {
    constexpr int E = G / 2;
    constexpr int CAP = P * E;
    const int comp = gl & 1;
    const int e = gl >> 1;
    const VT* __restrict__ val = static_cast<const VT*>(A.val);
    const __amdgpu_buffer_rsrc_t rsrc = state_rsrc(I.xa, A.d);
    const int64_t len = rr.re - rr.rs;

    // read phase
    int32_t cc[P];
    double vv[P], xs[P], as[P], dd[P];
    double zp = 0.0;
    if (len <= CAP) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int64_t q = (int64_t)p * E + e;
            const int64_t k = rr.rs + (q < len ? q : 0);  // idle lanes re-read entry 0
            cc[p] = A.colidx[k];
            vv[p] = widen(val[k]);
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const Pair pr = load_pair<LAY>(rsrc, cc[p], hot);
            xs[p] = pr.x;
            as[p] = pr.a;
            dd[p] = I.D[cc[p]];
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int64_t q = (int64_t)p * E + e;
            if (q < len) {
                if (cc[p] < hot) {
                    const int h = 2 * cc[p];
                    xs[p] = lds_get<LAY>(h) + lds_get<LAY>(2 * hot + h);
                    as[p] = lds_get<LAY>(h + 1) + lds_get<LAY>(2 * hot + h + 1);
                }
                if (comp == 0) zp += vv[p] * xs[p];
            }
        }
    } else {
        for (int64_t k = rr.rs + gl; k < rr.re; k += G) {
            const int32_t c = A.colidx[k];
            double x = load_pair<LAY>(rsrc, c, hot).x;
            if (c < hot) x = lds_get<LAY>(2 * c) + lds_get<LAY>(2 * hot + 2 * c);
            zp += widen(val[k]) * x;
        }
    }
    const double z = group_sum<G>(zp);

    // scalar gradient change against the memory
    double g = dphi(z, rr.b, A.loss);
    if constexpr (kX32<LAY>) g = (double)(float)g;  // stored memory is FP32
    const double al = SERIAL ? load_alpha<LAY>(I.alpha, rr.j) : rr.alpha;
    const double delta = g - al;
    if (gl == 0 && !isfinite(delta)) *flag = 1;
    // What the memory entry gains: with FP32 memory the atomic addition
    // stores fl32(alpha_j + fl32(delta)), which differs from g when |delta|
    // is far below alpha_j's precision; abar receives that change, not delta,
    // so that it stays the average of the stored memory (exactly when no
    // other sample changed alpha_j between this read and the addition).
    double dmem = delta;
    if constexpr (kX32<LAY>) dmem = (double)((float)al + (float)delta) - al;

    // write phase: x_c += -gamma (delta a_c + D_c (abar_c + lambda x_hat_c)) on even lanes,
    //              abar_c += dmem a_c / m on odd lanes
    const double gam = I.gamma, lam = I.lambda, dm = dmem * I.inv_m;
    // frozen memory: the odd lanes (abar) write nothing
    const bool writes = !(I.frozen && comp == 1);
    if (len <= CAP) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int64_t q = (int64_t)p * E + e;
            if (q < len && writes) {
                const double w = comp == 0 ? -gam * (delta * vv[p] + dd[p] * (as[p] + lam * xs[p])) : dm * vv[p];
                add_slot<RACY, LAY>(I.xa, cc[p], comp, hot, w);
            }
        }
    } else {
        for (int64_t k = rr.rs + e; k < rr.re; k += E) {
            const int32_t c = A.colidx[k];
            const double v = widen(val[k]);
            Pair pr = load_pair<LAY>(rsrc, c, hot);
            if (c < hot) {
                pr.x = lds_get<LAY>(2 * c) + lds_get<LAY>(2 * hot + 2 * c);
                pr.a = lds_get<LAY>(2 * c + 1) + lds_get<LAY>(2 * hot + 2 * c + 1);
            }
            const double w = comp == 0 ? -gam * (delta * v + I.D[c] * (pr.a + lam * pr.x)) : dm * v;
            if (writes) add_slot<RACY, LAY>(I.xa, c, comp, hot, w);
        }
    }
    if (gl == 0 && !I.frozen) add_alpha<RACY, LAY>(I.alpha, rr.j, delta);
    if constexpr (SERIAL) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
}

// The global value of slot q of the interleaved state (x in FP32 for the
// mixed layout, both halves for the FP32 layout), read at the
// device-coherent level.
template <int LAY>
__device__ __forceinline__ double load_slot(const double* xa, int q) {
    if constexpr (kS32<LAY>)
        return (double)__hip_atomic_load(reinterpret_cast<float*>(const_cast<double*>(xa)) + q, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    if (LAY == kLayMixed && (q & 1) == 0)
        return (double)__hip_atomic_load(reinterpret_cast<float*>(const_cast<double*>(xa) + q), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return __hip_atomic_load(const_cast<double*>(xa) + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Add the workgroup's pending sums of hot columns [0, upto) to the global
// state and clear them.  A slot with a pending sum takes, as its new view, the
// value its returning atomic add reports plus the sum (the global value
// including every flush so far).  Every other slot of a column at or above
// `reload_from` reads its global value again; the rest keep their view until
// the workgroup next writes them.  (A workgroup writes a hot column of
// probability p_v about once in 1/(p_v * samples per round) rounds, while the
// other workgroups apply about W of its updates, each a step of about
// gamma D_v: without a reload, the view of the rarer hot columns lags by
// about W D_v samples.)  Consecutive threads take consecutive slots, so each
// wave instruction covers 512 contiguous bytes (8 lines; FP32 layout: 256
// bytes, 4 lines).
//
// FP32 layout: a slot is flushed when its pending sum exceeds half a unit
// in the last place of the view.  The returning atomic gives the old value,
// so the rounding error of the addition (TwoSum of old and the pending sum)
// is known exactly; it stays pending and rides along with the workgroup's
// next contribution to the slot, so the hot columns' FP32 sums are
// compensated.  What is still pending at the end of a launch (at most half
// a unit in the last place per slot and workgroup) is dropped.
template <int LAY>
__device__ __forceinline__ void flush_and_refresh(double* xa, int hot, int upto, int reload_from) {
    if constexpr (kS32<LAY>) {
        float* lf = reinterpret_cast<float*>(lds);
        float* gs = reinterpret_cast<float*>(xa);
        for (int q = threadIdx.x; q < 2 * upto; q += blockDim.x) {
            const float w = lf[2 * hot + q];
            if (fabsf(w) > fabsf(lf[q]) * 0x1p-24f) {
                const float old = __hip_atomic_fetch_add(gs + q, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const float s = old + w;
                const float bv = s - old;
                lf[q] = s;
                lf[2 * hot + q] = (old - (s - bv)) + (w - bv);
            } else if (q >= 2 * reload_from) {
                lf[q] = __hip_atomic_load(gs + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        return;
    }
    for (int q = threadIdx.x; q < 2 * upto; q += blockDim.x) {
        const double w = lds[2 * hot + q];
        if (w != 0.0) {
            double now;
            if (LAY == kLayMixed && (q & 1) == 0)
                now = (double)(__hip_atomic_fetch_add(reinterpret_cast<float*>(xa + q), (float)w, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) + (float)w);
            else
                now = __hip_atomic_fetch_add(xa + q, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + w;
            lds[q] = now;
            lds[2 * hot + q] = 0.0;
        } else if (q >= 2 * reload_from) {
            lds[q] = load_slot<LAY>(xa, q);
        }
    }
}

template <int LAY>
__device__ __forceinline__ void load_view(const double* xa, int hot) {
    for (int q = threadIdx.x; q < 2 * hot; q += blockDim.x) {
        if constexpr (kS32<LAY>) {
            reinterpret_cast<float*>(lds)[q] = (float)load_slot<LAY>(xa, q);
            reinterpret_cast<float*>(lds)[2 * hot + q] = 0.0f;
        } else {
            lds[q] = load_slot<LAY>(xa, q);
            lds[2 * hot + q] = 0.0;
        }
    }
}

// The samples of one launch for one instance, spread over `slots` lane
// groups: group `slot` applies samples s = slot + k * slots, k = 0, 1, ...
// The row bounds of the next sample are fetched while the current one is
// processed.  With a hot set, all groups of the workgroup advance in rounds
// of `flush` samples; after each round the workgroup flushes the first
// `tier` hot columns, and all hot columns every `tier_every` rounds (then
// reloading the view of the slots from `reload_from` on that it did not
// write) and at the end of the launch.
template <int G, int P, bool SERIAL, bool RACY, int LAY, typename VT>
__device__ __forceinline__ void run_slots(const MatArgs& A, const InstArgs& I, uint64_t t0, uint64_t slot,
                                          uint64_t slots, HotArgs H, int* flag) {
    const int gl = threadIdx.x & (G - 1);
    const int hot = H.hot;
    const uint64_t kmax = (I.count + slots - 1) / slots;
    // a group with no sample and no workgroup flush to take part in
    if (hot == 0 && slot >= I.count) return;
    if (hot > 0) {
        load_view<LAY>(I.xa, hot);
        __syncthreads();
    }
    const uint64_t round = hot > 0 ? (uint64_t)H.flush : kmax;
    RowRef cur{0, 0, 0, 0, 0.0, 0.0};
    if (slot < I.count) cur = row_ref<SERIAL, LAY>(A, I, t0 + slot);
    uint64_t r = 0;
    for (uint64_t k0 = 0; k0 < kmax; k0 += round, ++r) {
        const uint64_t k1 = k0 + round < kmax ? k0 + round : kmax;
        for (uint64_t k = k0; k < k1; ++k) {
            const uint64_t s = slot + k * slots;
            const uint64_t s2 = s + slots;
            RowRef nxt{0, 0, 0, 0, 0.0, 0.0};
            if (s2 < I.count) nxt = row_ref<SERIAL, LAY>(A, I, t0 + s2);
            // sampled overlap log: clock at the read, and once the sample's
            // global writes are visible device-wide
            const bool logged = I.tau_log != nullptr && s < I.count &&
                                splitmix64(0x7A05EEDull, t0 + s) % kTauEvery == 0;
            long long t_read = 0;
            if (logged) t_read = wall_clock64();
            if (s < I.count) apply_update<G, P, SERIAL, RACY, LAY, VT>(A, I, cur, gl, hot, flag);
            if (logged) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                const long long t_done = wall_clock64();
                if (gl == 0) {
                    const unsigned long long e = __hip_atomic_fetch_add(I.tau_count, 1ull, __ATOMIC_RELAXED,
                                                                        __HIP_MEMORY_SCOPE_AGENT);
                    if (e < I.tau_cap) {
                        I.tau_log[2 * e] = t_read;
                        I.tau_log[2 * e + 1] = t_done;
                    }
                }
            }
            cur = nxt;
        }
        if (hot > 0) {
            const bool last = k1 == kmax;
            const bool all = last || (r + 1) % (uint64_t)H.tier_every == 0;
            __syncthreads();
            const int upto = all ? hot : H.tier;
            flush_and_refresh<LAY>(I.xa, hot, upto, all && !last && I.reload_from < upto ? I.reload_from : upto);
            __syncthreads();
        }
    }
}

// P = 4 passes in registers: rows of up to 2G entries take the fast path.
constexpr int kPasses = 4;

// Ordered execution (SERIAL): the first lane group of the first workgroup
// applies every sample of the launch in stream order, reading the memory
// value alpha_j only after the previous sample's writes and waiting for its
// own writes before the next sample (an agent-scope fence), which makes the
// run the sequential Sparse SAGA of Section 2.  The other lane groups apply
// nothing but take part in the workgroup's flushes of the LDS hot set, so
// the hot-set combining, the tiered flush, the view refresh and reload, the
// long-row chunks and every lane-group width run the same code as in the
// asynchronous launch.
template <int G, bool SERIAL>
__device__ __forceinline__ void slot_range(uint64_t rank, uint64_t n_blocks, uint64_t count, uint64_t* slot,
                                           uint64_t* slots) {
    if constexpr (SERIAL) {
        *slots = 1;
        *slot = rank == 0 && threadIdx.x < G ? 0 : count;  // count: no sample
    } else {
        const uint64_t groups = blockDim.x / G;
        *slot = rank * groups + threadIdx.x / G;
        *slots = n_blocks * groups;
    }
}

template <int G, bool SERIAL, bool RACY, int LAY, typename VT>
__global__ void __launch_bounds__(1024) k_update(MatArgs A, InstArgs I, HotArgs H, int* flag) {
    uint64_t slot, slots;
    slot_range<G, SERIAL>(blockIdx.x, gridDim.x, I.count, &slot, &slots);
    run_slots<G, kPasses, SERIAL, RACY, LAY, VT>(A, I, I.t0, slot, slots, H, flag);
}

// Many instances in one persistent grid: the block map says which instance
// each workgroup serves and as which of that instance's workgroups.
template <int G, bool SERIAL, int LAY, typename VT>
__global__ void __launch_bounds__(1024) k_update_batched(MatArgs A, const InstArgs* insts, const BlockMap* map,
                                                        uint64_t epoch, HotArgs H, int* flag) {
    const BlockMap bm = map[blockIdx.x];
    if (bm.inst < 0) return;
    const InstArgs I = insts[bm.inst];
    if (I.count == 0 || bm.rank >= I.blocks) return;  // instance switched off: its state stays as it is
    uint64_t slot, slots;
    slot_range<G, SERIAL>(bm.rank, I.blocks, I.count, &slot, &slots);
    run_slots<G, kPasses, SERIAL, false, LAY, VT>(A, I, I.t0 + epoch * I.count, slot, slots, H, flag);
}

// ---------------------------------------------------------------------------
// launchers for the update kernels
// ---------------------------------------------------------------------------

size_t update_lds_bytes(const UpdateShape& S) {
    return (size_t)S.hot * 4 * (S.layout == kLayF32 ? sizeof(float) : sizeof(double));
}

static HotArgs hot_args(const UpdateShape& S) {
    HotArgs H;
    H.hot = S.hot;
    H.flush = S.flush > 0 ? S.flush : 1;
    H.tier = S.tier > 0 && S.tier < S.hot ? S.tier : S.hot;
    H.tier_every = S.tier_every > 0 ? S.tier_every : 1;
    return H;
}

template <int G, bool SERIAL, int LAY, typename VT>
static hipError_t launch_update_g(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int blocks, int* flag,
                                  hipStream_t st) {
    const size_t lds = update_lds_bytes(S);
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_update<G, SERIAL, false, LAY, VT>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_update<G, SERIAL, false, LAY, VT><<<blocks, S.block, lds, st>>>(A, I, hot_args(S), flag);
    return hipGetLastError();
}

template <bool SERIAL, int LAY, typename VT>
static hipError_t launch_update_s(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int blocks, int* flag,
                                  hipStream_t st) {
    switch (S.lanes) {
        case 64: return launch_update_g<64, SERIAL, LAY, VT>(A, I, S, blocks, flag, st);
        case 32: return launch_update_g<32, SERIAL, LAY, VT>(A, I, S, blocks, flag, st);
        case 16: return launch_update_g<16, SERIAL, LAY, VT>(A, I, S, blocks, flag, st);
        case 8: return launch_update_g<8, SERIAL, LAY, VT>(A, I, S, blocks, flag, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LAY, typename VT>
static hipError_t launch_updates_t(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag,
                                   hipStream_t st) {
    if (I.count == 0) return hipSuccess;
    // ordered: one workgroup, whose first lane group applies the samples
    if (S.serial) return launch_update_s<true, LAY, VT>(A, I, S, 1, flag, st);
    const int threads = S.block;
    const int blocks = (S.waves * 64 + threads - 1) / threads;
    if (S.racy) {
        const HotArgs none{0, 1, 0, 1};
        switch (S.lanes) {
            case 64: k_update<64, false, true, LAY, VT><<<blocks, threads, 0, st>>>(A, I, none, flag); break;
            case 32: k_update<32, false, true, LAY, VT><<<blocks, threads, 0, st>>>(A, I, none, flag); break;
            case 16: k_update<16, false, true, LAY, VT><<<blocks, threads, 0, st>>>(A, I, none, flag); break;
            case 8: k_update<8, false, true, LAY, VT><<<blocks, threads, 0, st>>>(A, I, none, flag); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    return launch_update_s<false, LAY, VT>(A, I, S, blocks, flag, st);
}

template <typename VT>
static hipError_t launch_updates_v(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag,
                                   hipStream_t st) {
    switch (S.layout) {
        case kLayF64: return launch_updates_t<kLayF64, VT>(A, I, S, flag, st);
        case kLayMixed: return launch_updates_t<kLayMixed, VT>(A, I, S, flag, st);
        case kLayF32: return launch_updates_t<kLayF32, VT>(A, I, S, flag, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_updates(const MatArgs& A, const InstArgs& I, const UpdateShape& S, int* flag, hipStream_t st) {
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: return launch_updates_v<double>(A, I, S, flag, st);
        case ASAGA_VAL_F32: return launch_updates_v<float>(A, I, S, flag, st);
        case ASAGA_VAL_BF16: return launch_updates_v<uint16_t>(A, I, S, flag, st);
    }
    return hipErrorInvalidValue;
}

template <int G, bool SERIAL, int LAY, typename VT>
static hipError_t launch_batched_gs(const MatArgs& A, const InstArgs* insts, const BlockMap* map, int n_blocks,
                                    uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    const size_t lds = update_lds_bytes(S);
    if (lds > 65536) {
        const hipError_t e =
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_update_batched<G, SERIAL, LAY, VT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_update_batched<G, SERIAL, LAY, VT><<<n_blocks, S.block, lds, st>>>(A, insts, map, epoch, hot_args(S), flag);
    return hipGetLastError();
}

template <int G, int LAY, typename VT>
static hipError_t launch_batched_g(const MatArgs& A, const InstArgs* insts, const BlockMap* map, int n_blocks,
                                   uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    return S.serial ? launch_batched_gs<G, true, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st)
                    : launch_batched_gs<G, false, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
}

template <int G, int LAY, typename VT>
static int resident_g(const UpdateShape& S) {
    const size_t lds = update_lds_bytes(S);
    const void* fn = reinterpret_cast<const void*>(&k_update_batched<G, false, LAY, VT>);
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, S.block, lds) != hipSuccess) return 0;
    return per_cu * device_cu_count();
}

template <int LAY, typename VT>
static hipError_t launch_batched_t(const MatArgs& A, const InstArgs* insts, const BlockMap* map, int n_blocks,
                                   uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    switch (S.lanes) {
        case 64: return launch_batched_g<64, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        case 32: return launch_batched_g<32, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        case 16: return launch_batched_g<16, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        case 8: return launch_batched_g<8, LAY, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        default: return hipErrorInvalidValue;
    }
}

template <int LAY, typename VT>
static int resident_t(const UpdateShape& S) {
    switch (S.lanes) {
        case 64: return resident_g<64, LAY, VT>(S);
        case 32: return resident_g<32, LAY, VT>(S);
        case 16: return resident_g<16, LAY, VT>(S);
        case 8: return resident_g<8, LAY, VT>(S);
        default: return 0;
    }
}

template <typename VT>
static hipError_t launch_batched_v(const MatArgs& A, const InstArgs* insts, const BlockMap* map, int n_blocks,
                                   uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    switch (S.layout) {
        case kLayF64: return launch_batched_t<kLayF64, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        case kLayMixed: return launch_batched_t<kLayMixed, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
        case kLayF32: return launch_batched_t<kLayF32, VT>(A, insts, map, n_blocks, epoch, S, flag, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_updates_batched(const MatArgs& A, const InstArgs* dev_insts, const BlockMap* dev_map,
                                  int n_blocks, uint64_t epoch, const UpdateShape& S, int* flag, hipStream_t st) {
    if (n_blocks <= 0) return hipSuccess;
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: return launch_batched_v<double>(A, dev_insts, dev_map, n_blocks, epoch, S, flag, st);
        case ASAGA_VAL_F32: return launch_batched_v<float>(A, dev_insts, dev_map, n_blocks, epoch, S, flag, st);
        case ASAGA_VAL_BF16: return launch_batched_v<uint16_t>(A, dev_insts, dev_map, n_blocks, epoch, S, flag, st);
    }
    return hipErrorInvalidValue;
}

template <typename VT>
static int resident_v(const UpdateShape& S) {
    switch (S.layout) {
        case kLayF64: return resident_t<kLayF64, VT>(S);
        case kLayMixed: return resident_t<kLayMixed, VT>(S);
        case kLayF32: return resident_t<kLayF32, VT>(S);
    }
    return 0;
}

int batched_resident_blocks(const UpdateShape& S, int32_t val_dtype) {
    switch (val_dtype) {
        case ASAGA_VAL_F64: return resident_v<double>(S);
        case ASAGA_VAL_F32: return resident_v<float>(S);
        case ASAGA_VAL_BF16: return resident_v<uint16_t>(S);
    }
    return 0;
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
__global__ void k_fill(T* p, T v, int64_t count, int64_t stride) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        p[k * stride] = v;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<int32_t><<<grid_for(count, 256), 256, 0, st>>>(p, v, count, 1);
    return hipGetLastError();
}
hipError_t launch_fill_i64(long long* p, long long v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<long long><<<grid_for(count, 256), 256, 0, st>>>(p, v, count, 1);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t count, int64_t stride, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<double><<<grid_for(count, 256), 256, 0, st>>>(p, v, count, stride);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, float v, int64_t count, hipStream_t st) {
    if (count <= 0) return hipSuccess;
    k_fill<float><<<grid_for(count, 256), 256, 0, st>>>(p, v, count, 1);
    return hipGetLastError();
}

// 16 lanes per row for the evaluation and set-up passes (not on the hot path)
constexpr int kRowLanes = 16;

__device__ __forceinline__ int64_t row_of(const int32_t* rows, int64_t j) { return rows ? (int64_t)rows[j] : j; }

// Column counts.  Columns in [c0, c0 + C) are counted in an LDS histogram
// per workgroup (C <= kCountTile) and added to the global counts once per
// workgroup, so the columns nearly every row touches do not serialise on
// one address; with `rest` set, columns outside the tile are counted with
// global atomics in the same pass.
constexpr int kCountTile = 16384;

__global__ void __launch_bounds__(1024) k_colcount(MatArgs A, const int32_t* rows, int64_t m, int32_t* cnt, int32_t c0,
                                                   int32_t C, int rest) {
    __shared__ int32_t h[kCountTile];
    for (int q = threadIdx.x; q < C; q += blockDim.x) h[q] = 0;
    __syncthreads();
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes) {
            const int32_t c = A.colidx[k];
            const int32_t q = c - c0;
            if (q >= 0 && q < C) atomicAdd(&h[q], 1);
            else if (rest) atomicAdd(cnt + c, 1);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < C; q += blockDim.x)
        if (h[q]) atomicAdd(cnt + c0 + q, h[q]);
}

hipError_t launch_colcount(const MatArgs& A, const int32_t* rows, int64_t m, int32_t* cnt, bool hot_first,
                           hipStream_t st) {
    const int threads = 1024;
    const int blocks = grid_for(m * kRowLanes, threads, 1024);
    if (hot_first || A.d <= kCountTile) {
        // one pass: [0, tile) in LDS, the rest by global atomics
        const int32_t C = (int32_t)(A.d < kCountTile ? A.d : kCountTile);
        k_colcount<<<blocks, threads, 0, st>>>(A, rows, m, cnt, 0, C, 1);
        return hipGetLastError();
    }
    if (A.d <= 16 * (int64_t)kCountTile) {
        // column order unknown (before relabelling): one LDS pass per tile
        for (int64_t c0 = 0; c0 < A.d; c0 += kCountTile) {
            const int32_t C = (int32_t)(A.d - c0 < kCountTile ? A.d - c0 : kCountTile);
            k_colcount<<<blocks, threads, 0, st>>>(A, rows, m, cnt, (int32_t)c0, C, 0);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    k_colcount<<<blocks, threads, 0, st>>>(A, rows, m, cnt, 0, 0, 1);
    return hipGetLastError();
}

__global__ void k_relabel(const int32_t* in, int64_t nnz, const int32_t* rank, int32_t* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = rank[in[k]];
}

hipError_t launch_relabel(const int32_t* in, int64_t nnz, const int32_t* rank, int32_t* out, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    k_relabel<<<grid_for(nnz, 256), 256, 0, st>>>(in, nnz, rank, out);
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

// sum over the kRowLanes lanes of a row group
__device__ __forceinline__ double row_sum(double v) { return group_sum<kRowLanes>(v); }

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
        s = row_sum(s);
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

__device__ __forceinline__ double xget(const XView& X, int64_t v) {
    return X.f32 ? (double)static_cast<const float*>(X.p)[v * X.stride] : static_cast<const double*>(X.p)[v * X.stride];
}

template <typename VT>
__global__ void k_rowdot(MatArgs A, const int32_t* rows, int64_t m, XView x, double* z) {
    const VT* val = static_cast<const VT*>(A.val);
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        double s = 0.0;
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes) s += widen(val[k]) * xget(x, A.colidx[k]);
        s = row_sum(s);
        if (gl == 0) z[j] = s;
    }
}

hipError_t launch_rowdot(const MatArgs& A, const int32_t* rows, int64_t m, XView x, double* z, hipStream_t st) {
    const int blocks = grid_for(m * kRowLanes, 256);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_rowdot<double><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        case ASAGA_VAL_F32: k_rowdot<float><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        case ASAGA_VAL_BF16: k_rowdot<uint16_t><<<blocks, 256, 0, st>>>(A, rows, m, x, z); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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

// out[c * stride] += sum_j coef_j a_rows[j],c.  The most-used columns
// [0, hot) (the lowest labels after relabelling) are summed per workgroup in
// LDS and added to global memory once per workgroup; the others take one
// global atomic per entry.  Without this, every row's atomic on the handful
// of columns nearly all rows touch serialises on a few cache lines.
constexpr int kScatterHot = 4096;
constexpr int kScatterBlocks = 1024;

template <typename VT>
__global__ void __launch_bounds__(256) k_scatter(MatArgs A, const int32_t* rows, int64_t m, const double* coef,
                                                 double* out, int64_t stride, int hot) {
    __shared__ double acc[kScatterHot];
    for (int q = threadIdx.x; q < hot; q += blockDim.x) acc[q] = 0.0;
    __syncthreads();
    const VT* val = static_cast<const VT*>(A.val);
    const int gl = threadIdx.x & (kRowLanes - 1);
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) / kRowLanes;
    for (int64_t j = grp; j < m; j += ngrp) {
        const int64_t i = row_of(rows, j);
        const double cj = coef[j];
        for (int64_t k = A.rowptr[i] + gl; k < A.rowptr[i + 1]; k += kRowLanes) {
            const int32_t c = A.colidx[k];
            const double w = cj * widen(val[k]);
            if (c < hot)
                atomicAdd(&acc[c], w);
            else
                __hip_atomic_fetch_add(out + (int64_t)c * stride, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < hot; q += blockDim.x) {
        const double w = acc[q];
        if (w != 0.0) __hip_atomic_fetch_add(out + (int64_t)q * stride, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_scatter(const MatArgs& A, const int32_t* rows, int64_t m, const double* coef, double* out,
                          int64_t stride, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const int blocks = grid_for(m * kRowLanes, 256, kScatterBlocks);
    const int hot = (int)(A.d < kScatterHot ? A.d : kScatterHot);
    switch (A.val_dtype) {
        case ASAGA_VAL_F64: k_scatter<double><<<blocks, 256, 0, st>>>(A, rows, m, coef, out, stride, hot); break;
        case ASAGA_VAL_F32: k_scatter<float><<<blocks, 256, 0, st>>>(A, rows, m, coef, out, stride, hot); break;
        case ASAGA_VAL_BF16: k_scatter<uint16_t><<<blocks, 256, 0, st>>>(A, rows, m, coef, out, stride, hot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_axpy_x(XView x, int64_t d, double lambda, double* g) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d; v += (int64_t)gridDim.x * blockDim.x)
        g[v] += lambda * xget(x, v);
}

hipError_t launch_axpy_x(XView x, int64_t d, double lambda, double* g, hipStream_t st) {
    k_axpy_x<<<grid_for(d, 256), 256, 0, st>>>(x, d, lambda, g);
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

template <bool SQUARE>
__global__ void __launch_bounds__(256) k_sum_stage1(XView x, int64_t count, double* part) {
    double s = 0.0, c = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        double v = xget(x, k);
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

hipError_t launch_sum(const double* in, int64_t count, double* part, double* out, hipStream_t st) {
    k_sum_stage1<false><<<kSumParts, 256, 0, st>>>(XView{in, 1, 0}, count, part);
    k_sum_stage2<<<1, kSumParts, 0, st>>>(part, out);
    return hipGetLastError();
}

hipError_t launch_sum_x2(XView x, int64_t d, double* part, double* out, hipStream_t st) {
    k_sum_stage1<true><<<kSumParts, 256, 0, st>>>(x, d, part);
    k_sum_stage2<<<1, kSumParts, 0, st>>>(part, out);
    return hipGetLastError();
}

// In-graph stop test of a batch, after epoch `epoch` of a call (0-based):
// for every instance still running, r_k = ||abar_k + lambda_k x_k||^2, the
// gradient of instance k's objective with each row's scalar derivative
// taken from the memory (alpha_j, from when row j was last sampled) instead
// of at x: O(d) instead of a pass over the instance's rows.  An instance
// with r_k <= thr[k] is switched off for the rest of the call (count = 0 in
// its descriptor, which the call's later launches read) and ran[k] = epoch
// + 1 records the epochs it applied.  One workgroup per instance; the
// threads read x and abar by column in the state layout LAY.
template <int LAY>
__global__ void __launch_bounds__(1024) k_batch_proxy(InstArgs* insts, int64_t d, const double* thr, double* proxy,
                                                      int32_t* ran, int32_t epoch) {
    const int k = blockIdx.x;
    if (insts[k].count == 0) return;  // off before this epoch (the whole workgroup returns)
    const double* xd = insts[k].xa;
    const float* xf = reinterpret_cast<const float*>(xd);
    const double lam = insts[k].lambda;
    double s = 0.0, c = 0.0;
#pragma unroll 4
    for (int64_t v = threadIdx.x; v < d; v += 1024) {
        double x, ab;
        if (LAY == kLayF64) {
            x = xd[2 * v];
            ab = xd[2 * v + 1];
        } else if (LAY == kLayMixed) {
            x = (double)xf[4 * v];
            ab = xd[2 * v + 1];
        } else {
            x = (double)xf[2 * v];
            ab = (double)xf[2 * v + 1];
        }
        const double g = ab + lam * x;
        neumaier(s, c, g * g);
    }
    const double r = block_sum<1024>(s + c);
    if (threadIdx.x == 0) {
        proxy[k] = r;
        if (r <= thr[k]) {
            insts[k].count = 0;
            ran[k] = epoch + 1;
        }
    }
}

hipError_t launch_batch_proxy(InstArgs* insts, int n_inst, int64_t d, int layout, const double* thr, double* proxy,
                              int32_t* ran, int32_t epoch, hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    switch (layout) {
        case kLayF64: k_batch_proxy<kLayF64><<<n_inst, 1024, 0, st>>>(insts, d, thr, proxy, ran, epoch); break;
        case kLayMixed: k_batch_proxy<kLayMixed><<<n_inst, 1024, 0, st>>>(insts, d, thr, proxy, ran, epoch); break;
        case kLayF32: k_batch_proxy<kLayF32><<<n_inst, 1024, 0, st>>>(insts, d, thr, proxy, ran, epoch); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_objective_finish(const double* sums, double m, double lambda, double* f) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *f = sums[0] / m + 0.5 * lambda * sums[1];
}

hipError_t launch_objective_finish(const double* sums, double m, double lambda, double* f, hipStream_t st) {
    k_objective_finish<<<1, 64, 0, st>>>(sums, m, lambda, f);
    return hipGetLastError();
}

__global__ void k_gather_view(XView x, const int32_t* rank, int64_t d, double* out) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d; v += (int64_t)gridDim.x * blockDim.x)
        out[v] = xget(x, rank[v]);
}

hipError_t launch_gather_view(XView x, const int32_t* rank, int64_t d, double* out, hipStream_t st) {
    k_gather_view<<<grid_for(d, 256), 256, 0, st>>>(x, rank, d, out);
    return hipGetLastError();
}

__global__ void k_scatter_slots(const double* in, const int32_t* rank, int64_t d, void* slot, int64_t stride, int f32) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d; v += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = (int64_t)rank[v] * stride;
        if (f32) static_cast<float*>(slot)[q] = (float)in[v];
        else static_cast<double*>(slot)[q] = in[v];
    }
}

hipError_t launch_scatter_slots(const double* in, const int32_t* rank, int64_t d, void* slot, int64_t stride, bool f32,
                                hipStream_t st) {
    k_scatter_slots<<<grid_for(d, 256), 256, 0, st>>>(in, rank, d, slot, stride, f32 ? 1 : 0);
    return hipGetLastError();
}

__global__ void k_widen(const float* in, int64_t count, double* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (double)in[k];
}
__global__ void k_narrow(const double* in, int64_t count, float* out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        out[k] = (float)in[k];
}

__global__ void k_copy_view(XView x, int64_t d, double* out, int64_t out_stride) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d; c += (int64_t)gridDim.x * blockDim.x)
        out[c * out_stride] = xget(x, c);
}

hipError_t launch_copy_view(XView x, int64_t d, double* out, int64_t out_stride, hipStream_t st) {
    k_copy_view<<<grid_for(d, 256), 256, 0, st>>>(x, d, out, out_stride);
    return hipGetLastError();
}

__global__ void k_store_slots(const double* in, int64_t d, void* slot, int64_t stride, int f32) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d; c += (int64_t)gridDim.x * blockDim.x) {
        if (f32) static_cast<float*>(slot)[c * stride] = (float)in[c];
        else static_cast<double*>(slot)[c * stride] = in[c];
    }
}

hipError_t launch_store_slots(const double* in, int64_t d, void* slot, int64_t stride, bool f32, hipStream_t st) {
    k_store_slots<<<grid_for(d, 256), 256, 0, st>>>(in, d, slot, stride, f32 ? 1 : 0);
    return hipGetLastError();
}

// x_c stored as FP32 in the low half of slot xa[2c] -> FP64 in the whole slot
__global__ void k_widen_x_slots(double* xa, int64_t d) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < d; c += (int64_t)gridDim.x * blockDim.x) {
        const float v = reinterpret_cast<const float*>(xa + 2 * c)[0];
        xa[2 * c] = (double)v;
    }
}

hipError_t launch_widen_x_slots(double* xa, int64_t d, hipStream_t st) {
    if (d <= 0) return hipSuccess;
    k_widen_x_slots<<<grid_for(d, 256), 256, 0, st>>>(xa, d);
    return hipGetLastError();
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

// Memory-side request ceiling (a diagnostic of the atomic-rate bound): every
// lane pair touches a pseudo-random 16-byte (x, abar) slot of a state of
// `cols` columns per operation, one memory request per pair, as the update
// kernel's cold columns do.  mode 0: one FP64 atomic addition per iteration;
// mode 1: one device-coherent read and one atomic addition (to another
// slot).  The reads feed a value that is stored only if it takes an
// impossible value, so that they are kept.
__global__ void k_request_probe(double* xa, int64_t cols, int iters, int mode, double* sink) {
    const uint64_t pair = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 1;
    const int comp = threadIdx.x & 1;
    double acc = 0.0;
    for (int it = 0; it < iters; ++it) {
        const uint64_t h = splitmix64(0x5EEDull, pair * (uint64_t)iters + (uint64_t)it);
        const int64_t c1 = (int64_t)(h % (uint64_t)cols);
        const int64_t c2 = (int64_t)((h >> 32) % (uint64_t)cols);
        if (mode == 1) acc += __hip_atomic_load(xa + 2 * c1 + comp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(xa + 2 * c2 + comp, 1e-300, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (acc == -1.0) sink[0] = acc;
}

hipError_t launch_request_probe(double* xa, int64_t cols, int blocks, int iters, int mode, double* sink,
                                hipStream_t st) {
    k_request_probe<<<blocks, 256, 0, st>>>(xa, cols, iters, mode, sink);
    return hipGetLastError();
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace asaga
