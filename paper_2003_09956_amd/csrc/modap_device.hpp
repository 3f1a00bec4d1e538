// Device-side types shared by the kernels and the host half of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace modap {

// Iteration state codes held on the device (mirrored in modap_stats.state).
enum : int32_t {
    ST_RUNNING = 0,
    ST_CONVERGED = 1,
    ST_NO_DIRECTION = 2,
    ST_NUMERIC = 3,
    ST_LIMIT = 4,
    ST_BAD_ROW = 5,
    ST_UNCERTIFIED = 6,   // the FP64 certificate cannot confirm eps: eps_abs lies below its rounding bound
};

// The iteration state after one feasibility check and its decision.
struct alignas(16) State {
    int64_t sweeps;       // checks done
    int64_t steps;        // steps taken
    int64_t sched_pos;    // next drift-schedule row
    int64_t v_idx;        // drift-schedule row applied by the next sweep (-1: none)
    double s;             // step scale of the last step (x <- x - s*y)
    double dmax;          // last check: max_i max(r_i,0)/||a_i||
    double binf;          // last check: max_i |b_i|
    double ynorm;         // last check: ||y||
    double eps_abs;       // last check: threshold applied
    int64_t h;            // last check: violated rows
    int32_t status;       // ST_*
    int32_t feasible;     // last check found x eps-feasible
    int32_t vpend_valid;  // a one-shot translation waits for the next sweep
    int32_t certified;    // the stop was confirmed by the FP64 certificate
    double bdrift;        // last certificate: max_i |b_i - exact b_i| it corrected
    double pad;
};

// Device-resident control block of one context.  The state after the check
// of sweep j (and the decision taken on it) lives in slot j & 1.  It is
// written once, from slot (j-1)&1, by the first kernel of sweep j+1, or by the
// stage kernel that ends a call; kernel boundaries order every write before
// its readers, so no device-wide fence is needed anywhere.
struct alignas(128) Ctrl {
    State st[2];
    int64_t step_limit;   // no step is taken once steps reaches this (set per call)
    int64_t sched_len;    // rows in the drift schedule
    uint32_t barrier;     // arrivals at the grid barriers of a resident launch (zero before each)
    uint32_t fault;       // a resident launch gave up waiting at a grid barrier
    uint32_t exits;       // workgroups of a resident launch that have left it (zero before each)
    uint32_t pad32;
    int64_t pad[12];
};

// Totals of the sweep's per-workgroup scalars, formed by the reduction.
struct alignas(32) Totals {
    int64_t h;
    double dmax;
    double binf;
    double bdrift;      // certificate only: max_i |b_i - exact b_i| before the rebase
};

// Parameters of the decision taken after every check.
struct Decide {
    double lambda;
    double eps;
    int32_t eps_relative;
    int32_t rule;         // 0 fixed length (eq. 12), 1 relaxed average (Alg. 1)
    int32_t track;        // an eps-feasible check does not stop the iteration
    int32_t pad;
};

// Storage traits: 16-byte vector loads of VEC elements; Acc = dot-product
// accumulator and the type of the working vectors x and v of a sweep.
template <int DT> struct Store;
template <> struct Store<0> {  // IEEE binary64
    using T = double;
    using Acc = double;
    static constexpr int VEC = 2;
};
template <> struct Store<1> {  // IEEE binary32
    using T = float;
    using Acc = float;
    static constexpr int VEC = 4;
};
template <> struct Store<2> {  // bfloat16 bit patterns
    using T = uint16_t;
    using Acc = float;
    static constexpr int VEC = 8;
};

// What a sweep needs to settle the previous check before it runs: sweep j of
// a call (all but the first) takes the decision of check j-1 itself, from the
// state in slot (j-2)&1 and the totals and norm parts of reduction j-1, and
// commits it to slot (j-1)&1.  Every workgroup takes the same decision from the
// same data in the same order; one of them writes it.
struct Pending {
    Ctrl *ctl;
    int64_t j;
    const Totals *tot;
    const double *ynp;
    int32_t R;              // norm parts
    int32_t decide;         // 0: slot (j-1)&1 already holds the state this sweep runs under
    Decide dp;
};

struct SweepArgs {
    const void *A;          // [m x ldA] storage type, rows padded with zeros to ldA
    int64_t ldA;            // multiple of the 16-byte vector width
    int64_t m, n;
    const double *b_in;     // [m]
    double *b_out;          // [m] or null; written (may alias b_in) only when a translation applies
    const double *nu;       // [m] ||a_i||^2
    const void *work;       // [3 x ldA] Acc: the point x, the translation v, the direction y
    Pending pd;             // the state this sweep runs under (whether to run, step, translation)
    int32_t check_status;   // 1: do nothing unless the state is ST_RUNNING
    int32_t pad;
    double *r_out;          // [m] or null
    void *part;             // [grid x ldPart] Acc partial sums of y
    int64_t ldPart;
    int64_t *h_part;        // [grid]
    double *dmax_part;      // [grid]
    double *binf_part;      // [grid]
    // rows of workgroup b: from b*block_stride, one step of rows every
    // step_stride rows, below min(m, b*block_stride + rows_per_block)
    int64_t rows_per_block;
    int64_t block_stride;
    int64_t step_stride;
};

struct ReduceArgs {
    const void *part;       // [G x ldPart] Acc (float or double per acc_f64)
    int64_t ldPart;
    int32_t G;              // partial-y rows
    int32_t acc_f64;
    int32_t Gs;             // per-workgroup scalar partials (h, dmax, binf)
    int32_t apply_step;     // iteration mode: make the step of state (j-1)&1 permanent in x first
    int64_t n, ldA;
    double *y;              // [n] in: previous direction (apply_step), out: this sweep's
    const Ctrl *ctl;        // iteration mode: state slot (j-1)&1 (skip when stopped)
    int64_t j;
    int32_t iterate;
    int32_t pad;
    const int64_t *h_part;
    const double *dmax_part;
    const double *binf_part;
    Totals *tot;            // out (workgroup 0)
    double *ynp;            // out [gridDim.x]
    double *x;              // iteration mode: [n] FP64 approximation
    void *work;             // iteration mode: out [3 x ldA] Acc x, drift row due next, y
    const double *V;        // drift schedule [T x ldV] or null
    int64_t ldV;
    double *wsum;           // iteration mode: [ldA] FP64 sum of the translations applied since the
                            // last rebase of b (the exact data are bref + A wsum)
    const double *vpend;    // [ldA] one-shot translation
    int32_t has_v;          // the sweep was compiled with the translation (it applied the state's)
    int32_t pad2;
};

struct StageArgs {
    Ctrl *ctl;
    int64_t j;              // iteration whose check is settled (stage) / next iteration (prime)
    const Totals *tot;
    const double *ynp;
    int32_t R;
    int32_t pad;
    Decide dp;
    double *x;              // [ldA] FP64 approximation (stage: x <- x - s*y)
    const double *y;        // [ldA]
    const double *vpend;    // [ldA] one-shot translation
    const double *V;        // drift schedule [T x ldV] or null
    int64_t ldV;
    int64_t n, ldA;
    void *work;             // out [2 x ldA] Acc
};

// One system as the FP64 certificate of a stop sees it (certify.hpp).
struct CertArgs {
    const void *A;          // [m x ldA] storage type
    int64_t ldA, m, n;
    double *b;              // [m] working right-hand side (rebased)
    double *bref;           // [m] right-hand side at zero translation (rebased)
    const double *nu;       // [m] ||a_i||^2
    double *x;              // [ldA] FP64 approximation
    double *wsum;           // [ldA] translations applied since the last rebase (cleared)
    const double *V;        // drift schedule [T x ldV] or null (working vectors after a step)
    int64_t ldV;
    void *work;             // [3 x ldA] working vectors of the next sweep
    Ctrl *ctl;
    int32_t sl;             // the committed state slot, read and rewritten in place
    int32_t R;              // ceil(n / 64): parts of ||y||^2
    double *wt;             // [m] r_i/||a_i||^2 for violated rows, else 0
    int64_t *h_part;        // [dot workgroups]
    double *dmax_part;      // [dot workgroups]
    double *binf_part;      // [dot workgroups]
    double *drift_part;     // [dot workgroups]
    int32_t Gs;             // dot workgroups: ceil(m / 4)
    int32_t bands;          // row bands of cert_axpy
    int64_t rows_per_band;
    double *part;           // [bands x ldA] FP64 partial y
    double *y;              // [ldA] FP64 y of the certificate
    double *ynp;            // [R]
    Totals *tot;
    Decide dp;
};

__host__ __device__ __forceinline__ int slot_of(int64_t j) { return (int)(j & 1); }

// Accesses through a pointer known to address global memory.  A pointer read
// from memory is otherwise taken as generic: its accesses become flat ones,
// which the compiler must count as LDS accesses too when it places waits.
// (A structure is moved as 16-byte words: an aggregate copy would drop the
// address space.)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T load_global(const T *p) {
    if constexpr (sizeof(T) % 16 == 0 && alignof(T) >= 16) {
        const __attribute__((address_space(1))) u32x4 *q = (const __attribute__((address_space(1))) u32x4 *)p;
        u32x4 w[sizeof(T) / 16];
#pragma unroll
        for (int i = 0; i < (int)(sizeof(T) / 16); ++i) w[i] = q[i];
        T v;
        __builtin_memcpy(&v, w, sizeof(T));
        return v;
    } else {
        return *(const __attribute__((address_space(1))) T *)p;
    }
}
template <typename T>
__device__ __forceinline__ void store_global(T *p, const T &v) {
    if constexpr (sizeof(T) % 16 == 0 && alignof(T) >= 16) {
        __attribute__((address_space(1))) u32x4 *q = (__attribute__((address_space(1))) u32x4 *)p;
        u32x4 w[sizeof(T) / 16];
        __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
        for (int i = 0; i < (int)(sizeof(T) / 16); ++i) q[i] = w[i];
    } else {
        *(__attribute__((address_space(1))) T *)p = v;
    }
}

// x - s*y with one rounding.
__device__ __forceinline__ double step_point(double x, double s, double y) {
    return __fma_rn(-s, y, x);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// A DPP lane move inside each row of 16 lanes (CTRL is the gfx9 DPP control:
// 0x00-0xFF quad permutations, 0x140 row mirror, 0x141 half-row mirror).
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float lane_value(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over each row of 16 lanes of a wavefront whose lanes are all active,
// without the LDS permute unit: DPP adds with partners xor 1, xor 2, then the
// half-row and row mirrors.  The two operands of every add are the same pair
// in both lanes, so all 16 lanes of a row hold identical sums.
template <typename T>
__device__ __forceinline__ T row_total(T v) {
    v += dpp_move<0xB1>(v);   // quad permutation [1,0,3,2]
    v += dpp_move<0x4E>(v);   // quad permutation [2,3,0,1]
    v += dpp_move<0x141>(v);  // half-row mirror
    v += dpp_move<0x140>(v);  // row mirror
    return v;
}
// Sum over the 64 lanes of a wavefront whose lanes are all active, the same
// bits in every lane: the row sums, read as scalars and added as
// (row0 + row1) + (row2 + row3).  Used on the per-row paths, where the
// permute round trips of wave_sum sit on the critical path.
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
    v = row_total(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// The gfx950 lane swaps.  With halves, lanes 32-63 of a trade places with
// lanes 0-31 of b; without, in each half of the wavefront the upper 16 lanes
// of a trade places with the lower 16 of b.  Returns the sum of the two
// results: lanes 0-31 hold a(l) + a(l+32) and lanes 32-63 b(l-32) + b(l)
// (halves), or lanes 16q .. 16q+15 the same pattern of quarters.  With a == b
// every lane gets v(l) + v(l ^ 32) (or ^ 16): the bits of a shuffle and an
// add, without the permute unit.
template <typename T>
__device__ __forceinline__ T lane_swap_add(T a, T b, bool halves) {
    if constexpr (sizeof(T) == 4) {
        const auto r = halves ? __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, a),
                                                                 __builtin_bit_cast(uint32_t, b), false, false)
                              : __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, a),
                                                                 __builtin_bit_cast(uint32_t, b), false, false);
        return __builtin_bit_cast(T, (uint32_t)r[0]) + __builtin_bit_cast(T, (uint32_t)r[1]);
    } else {
        const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
        const uint32_t al = (uint32_t)ua, ah = (uint32_t)(ua >> 32), bl = (uint32_t)ub, bh = (uint32_t)(ub >> 32);
        const auto lo = halves ? __builtin_amdgcn_permlane32_swap(al, bl, false, false)
                               : __builtin_amdgcn_permlane16_swap(al, bl, false, false);
        const auto hi = halves ? __builtin_amdgcn_permlane32_swap(ah, bh, false, false)
                               : __builtin_amdgcn_permlane16_swap(ah, bh, false, false);
        const T a2 = __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
        const T b2 = __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
        return a2 + b2;
    }
}
// v(l) + v(l ^ O) in every lane, O = 16 or 32 (all lanes active).
template <int O, typename T>
__device__ __forceinline__ T xor_add(T v) {
    static_assert(O == 16 || O == 32, "swaps of quarters or halves");
    return lane_swap_add(v, v, O == 32);
}

// NaN-propagating maximum (fmax would drop a NaN).
__device__ __forceinline__ double max_nan(double a, double b) {
    return (b > a || b != b) ? b : a;
}

// NaN-propagating maximum over the 64 lanes of a wavefront whose lanes are
// all active (the moves of wave_total, with max_nan for the adds); every lane
// returns the same value.
__device__ __forceinline__ double wave_max_nan(double v) {
    v = max_nan(v, dpp_move<0xB1>(v));
    v = max_nan(v, dpp_move<0x4E>(v));
    v = max_nan(v, dpp_move<0x141>(v));
    v = max_nan(v, dpp_move<0x140>(v));
    return max_nan(max_nan(lane_value(v, 0), lane_value(v, 16)), max_nan(lane_value(v, 32), lane_value(v, 48)));
}

// ||y|| from its per-workgroup parts, in a fixed order.  Called by a whole
// wavefront; every lane returns the same value, in every workgroup.
__device__ __forceinline__ double ynorm_of(const double *ynp, int R, int lane) {
    double s = 0.0;
    for (int r = lane; r < R; r += 64) s += load_global(ynp + r);
    s = wave_total(s);   // DPP moves: no permute round trips before the decision
    return sqrt(s);
}

// The decision after a check (eq. 10 test, then eq. 12 or Algorithm 1 step).
__device__ __forceinline__ State decide(const State &p, const Totals &t, double ynorm, const Decide &d,
                                        int64_t step_limit, int64_t sched_len) {
    State s = p;
    if (p.status != ST_RUNNING) return s;
    s.sweeps = p.sweeps + 1;
    s.vpend_valid = 0;
    s.certified = 0;
    s.dmax = t.dmax;
    s.binf = t.binf;
    s.h = t.h;
    s.ynorm = ynorm;
    s.eps_abs = d.eps_relative ? d.eps * t.binf : d.eps;
    s.s = 0.0;
    s.v_idx = -1;
    s.feasible = t.dmax <= s.eps_abs;
    if (s.feasible) {
        if (d.track) {
            if (p.sched_pos < sched_len) {
                s.v_idx = p.sched_pos;
                s.sched_pos = p.sched_pos + 1;
            }
        } else {
            s.status = ST_CONVERGED;
        }
    } else if (!isfinite(t.dmax) || !isfinite(ynorm) || !isfinite(t.binf)) {
        s.status = ST_NUMERIC;
    } else if (p.steps >= step_limit) {
        s.status = ST_LIMIT;
    } else if (!(ynorm > 0.0) || t.h == 0) {
        s.status = ST_NO_DIRECTION;
    } else {
        s.s = d.rule == 0 ? d.lambda / ynorm : d.lambda / (double)t.h;
        s.steps = p.steps + 1;
        if (p.sched_pos < sched_len) {
            s.v_idx = p.sched_pos;
            s.sched_pos = p.sched_pos + 1;
        }
    }
    return s;
}

// The state that sweep pd.j runs under (see Pending).  Called by whole
// wavefronts (the norm of y is summed across the wavefront); `writer` commits
// a fresh decision.
__device__ __forceinline__ State sweep_state(const Pending &pd, int lane, bool writer) {
    if (!pd.decide) return load_global(&pd.ctl->st[slot_of(pd.j - 1)]);
    // every load first (none depends on another), then the decision
    const State p = load_global(&pd.ctl->st[slot_of(pd.j - 2)]);
    const Totals t = load_global(pd.tot);
    const int64_t limit = load_global(&pd.ctl->step_limit);
    const int64_t len = load_global(&pd.ctl->sched_len);
    const double yn = ynorm_of(pd.ynp, pd.R, lane);
    const State s = decide(p, t, yn, pd.dp, limit, len);
    if (writer) store_global(&pd.ctl->st[slot_of(pd.j - 1)], s);
    return s;
}

}  // namespace modap
