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
};

// Device-resident control block of one context.  Every kernel of an
// iteration reads it; only the last workgroup of the reduction writes it, so
// the host never has to synchronise between iterations.
struct alignas(128) Ctrl {
    int32_t status;       // ST_*
    int32_t vpend_valid;  // a one-shot translation waits in vpend
    int64_t steps;        // steps taken
    int64_t sweeps;       // checks done
    int64_t step_limit;   // no step is taken once steps reaches this
    int64_t v_idx;        // drift schedule row applied by the next sweep (-1: none)
    int64_t sched_pos;    // next drift schedule row
    int64_t sched_len;    // rows in the drift schedule
    double s;             // pending step: the next sweep works at x - s*y
    double dmax;          // last check
    double binf;
    double ynorm;
    double eps_abs;
    int64_t h;
    uint32_t ticket;      // last-workgroup election in the reduction
    int32_t feasible;     // the last check found x eps-feasible
    int64_t pad1[2];
};

// Per-sweep outputs of a stateless evaluation.
struct alignas(64) EvalOut {
    int64_t h;
    double dmax;
    double binf;
    double ynorm;
    uint32_t ticket;
    uint32_t pad;
};

// Storage traits: 16-byte vector loads of VEC elements; Acc = dot-product
// accumulator; X = register copy of x and v.
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

struct SweepArgs {
    const void *A;          // [m x ldA] storage type, rows padded with zeros to ldA
    int64_t ldA;            // multiple of the 16-byte vector width
    int64_t m, n;
    const double *b_in;     // [m]
    double *b_out;          // [m] or null; written (may alias b_in) only when a translation applies
    const double *nu;       // [m] ||a_i||^2
    const double *x;        // [n]
    const double *ystep;    // [n] or null: the sweep works at x - ctl->s * ystep
    const double *vpend;    // [n] one-shot translation, used when ctl->vpend_valid
    const double *V;        // drift schedule [T x ldV] or null; row ctl->v_idx when >= 0
    int64_t ldV;
    const Ctrl *ctl;
    int32_t check_status;   // 1: do nothing unless ctl->status == ST_RUNNING
    int32_t pad;
    double *r_out;          // [m] or null
    void *part;             // [grid x ldPart] Acc partial sums of y
    int64_t ldPart;
    int64_t *h_part;        // [grid]
    double *dmax_part;      // [grid]
    double *binf_part;      // [grid]
    int64_t rows_per_block;
};

struct ReduceArgs {
    const void *part;       // [G x ldPart] Acc (float or double per acc_f64)
    int64_t ldPart;
    int32_t G;
    int32_t acc_f64;
    int64_t n;
    double *y;              // [n] out (iteration mode: also the previous y, read first)
    double *x;              // [n] iteration mode: x <- x - s*y_prev (materialise the pending step)
    Ctrl *ctl;              // iteration mode when non-null
    EvalOut *eval;          // evaluation mode when ctl is null
    const int64_t *h_part;
    const double *dmax_part;
    const double *binf_part;
    double *ynorm_part;     // [gridDim.x]
    double lambda, eps;
    int32_t eps_relative;
    int32_t rule;           // 0 fixed length (eq. 12), 1 relaxed average (Alg. 1)
    int32_t track;          // an eps-feasible check does not stop the iteration
    int32_t pad;
};

// x - s*y with one rounding, so every kernel forms the same value.
__device__ __forceinline__ double step_point(double x, double s, double y) {
    return __fma_rn(-s, y, x);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// NaN-propagating maximum (fmax would drop a NaN).
__device__ __forceinline__ double max_nan(double a, double b) {
    return (b > a || b != b) ? b : a;
}

}  // namespace modap
