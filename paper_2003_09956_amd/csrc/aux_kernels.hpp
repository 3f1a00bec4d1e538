// Kernels around the sweep: row norms, the reduction of the partial y with
// the stop test and the step, control-block updates, in-place row
// replacement and the flush of a pending translation.
#pragma once

#include "modap_device.hpp"

namespace modap {

template <int DT>
__device__ __forceinline__ double load_elem(const void *A, int64_t idx) {
    if constexpr (DT == 0) {
        return reinterpret_cast<const double *>(A)[idx];
    } else if constexpr (DT == 1) {
        return (double)reinterpret_cast<const float *>(A)[idx];
    } else {
        const uint32_t u = ((uint32_t)reinterpret_cast<const uint16_t *>(A)[idx]) << 16;
        return (double)__uint_as_float(u);
    }
}

// nu_i = ||a_i||^2 in FP64 (section 2: the denominator of the reflection
// vector).  One wavefront per row, a fixed summation order.  Reports the
// first zero or non-finite row through *bad (atomic minimum of the index).
template <int DT>
__global__ __launch_bounds__(256) void row_norms(const void *A, int64_t ldA, int64_t m, int64_t n,
                                                 double *nu, unsigned long long *bad) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
        const double v = load_elem<DT>(A, row * ldA + j);
        s = __fma_rn(v, v, s);
    }
    s = wave_sum(s);
    if (lane == 0) {
        nu[row] = s;
        if (!(s > 0.0) || !isfinite(s)) atomicMin(bad, (unsigned long long)row);
    }
}

// Raises *flag when any of p[0..count) is NaN or infinite.
__global__ void check_finite(const double *p, int64_t count, int *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!isfinite(p[i])) atomicOr(flag, 1);
    }
}

// Sum of the workgroup partials of y in a fixed order (FP64), with the
// iteration's decision taken by the last workgroup to finish:
//   eps-feasible (eq. 10)      -> converged, no step
//   otherwise                  -> s = lambda/||y|| (eq. 12) or lambda/h (Alg. 1)
// In iteration mode the pending step of the previous iteration is first made
// permanent: x <- x - s_prev * y_prev, column by column, before y is replaced.
template <typename Acc>
__global__ __launch_bounds__(1024) void reduce_y(const ReduceArgs a) {
    constexpr int COLS = 64;
    constexpr int RG = 16;
    Ctrl *ctl = a.ctl;
    if (ctl && ctl->status != ST_RUNNING) return;
    const double s_prev = ctl ? ctl->s : 0.0;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int rg = tid >> 6;
    const int64_t col = (int64_t)blockIdx.x * COLS + lane;
    const Acc *part = reinterpret_cast<const Acc *>(a.part);

    double acc = 0.0;
    if (col < a.n) {
        for (int g = rg; g < a.G; g += RG) acc += (double)part[(int64_t)g * a.ldPart + col];
    }
    __shared__ double sh[RG][COLS];
    sh[rg][lane] = acc;
    __syncthreads();
    if (rg == 0) {
        double yv = 0.0;
#pragma unroll
        for (int r = 0; r < RG; ++r) yv += sh[r][lane];
        double sq = 0.0;
        if (col < a.n) {
            if (ctl && a.x && s_prev != 0.0) a.x[col] = step_point(a.x[col], s_prev, a.y[col]);
            a.y[col] = yv;
            sq = yv * yv;
        }
        sq = wave_sum(sq);
        if (lane == 0) a.ynorm_part[blockIdx.x] = sq;
    }

    // Elect the last workgroup (release our writes, then count).
    __shared__ int is_last;
    unsigned *ticket = ctl ? &ctl->ticket : &a.eval->ticket;
    if (tid == 0) {
        __threadfence();
        const unsigned t = atomicAdd(ticket, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();

    int64_t h = 0;
    double dm = 0.0, bm = 0.0, ys = 0.0;
    for (int g = tid; g < a.G; g += 1024) {
        h += a.h_part[g];
        dm = max_nan(dm, a.dmax_part[g]);
        bm = max_nan(bm, a.binf_part[g]);
    }
    for (int b = tid; b < (int)gridDim.x; b += 1024) ys += a.ynorm_part[b];
    // fixed-order reduction: butterfly within each wavefront, then wavefronts in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        h += __shfl_xor(h, o, 64);
        dm = max_nan(dm, __shfl_xor(dm, o, 64));
        bm = max_nan(bm, __shfl_xor(bm, o, 64));
        ys += __shfl_xor(ys, o, 64);
    }
    __shared__ int64_t hw[16];
    __shared__ double dw[16], bw[16], yw[16];
    if (lane == 0) {
        hw[rg] = h;
        dw[rg] = dm;
        bw[rg] = bm;
        yw[rg] = ys;
    }
    __syncthreads();
    if (tid != 0) return;
    h = 0;
    dm = 0.0;
    bm = 0.0;
    ys = 0.0;
    for (int w = 0; w < 16; ++w) {
        h += hw[w];
        dm = max_nan(dm, dw[w]);
        bm = max_nan(bm, bw[w]);
        ys += yw[w];
    }
    const double ynorm = sqrt(ys);
    if (!ctl) {
        a.eval->h = h;
        a.eval->dmax = dm;
        a.eval->binf = bm;
        a.eval->ynorm = ynorm;
        a.eval->ticket = 0u;
        return;
    }
    const double eps_abs = a.eps_relative ? a.eps * bm : a.eps;
    ctl->sweeps += 1;
    ctl->dmax = dm;
    ctl->binf = bm;
    ctl->ynorm = ynorm;
    ctl->h = h;
    ctl->eps_abs = eps_abs;
    ctl->vpend_valid = 0;
    ctl->s = 0.0;
    ctl->v_idx = -1;
    ctl->feasible = dm <= eps_abs;
    if (dm <= eps_abs) {
        if (a.track) {
            // no step; the data keep changing and the next sweep checks again
            if (ctl->sched_pos < ctl->sched_len) ctl->v_idx = ctl->sched_pos++;
        } else {
            ctl->status = ST_CONVERGED;
        }
    } else if (!isfinite(dm) || !isfinite(ynorm) || !isfinite(bm)) {
        ctl->status = ST_NUMERIC;
    } else if (ctl->steps >= ctl->step_limit) {
        ctl->status = ST_LIMIT;
    } else if (!(ynorm > 0.0) || h == 0) {
        ctl->status = ST_NO_DIRECTION;
    } else {
        ctl->s = a.rule == 0 ? a.lambda / ynorm : a.lambda / (double)h;
        ctl->steps += 1;
        if (ctl->sched_pos < ctl->sched_len) ctl->v_idx = ctl->sched_pos++;
    }
    ctl->ticket = 0u;
}

// Start of an iterate/solve call: a stop that came from a previous call's
// tolerance, step limit or missing direction is re-examined by the next sweep.
__global__ void ctl_begin(Ctrl *c, int64_t max_steps) {
    if (threadIdx.x != 0) return;
    const int32_t st = c->status;
    if (st == ST_CONVERGED || st == ST_LIMIT || st == ST_NO_DIRECTION) c->status = ST_RUNNING;
    c->step_limit = max_steps < 0 ? INT64_MAX : c->steps + max_steps;
}

// A new approximation: counters restart, no step is pending.
__global__ void ctl_restart(Ctrl *c) {
    if (threadIdx.x != 0) return;
    if (c->status != ST_BAD_ROW) c->status = ST_RUNNING;
    c->s = 0.0;
    c->steps = 0;
    c->sweeps = 0;
    c->dmax = c->binf = c->ynorm = c->eps_abs = 0.0;
    c->h = 0;
    c->feasible = 0;
}

// One-shot translation: vpend <- (pending ? vpend : 0) + v.  A single
// workgroup, so the pending flag is read before it is set.
__global__ __launch_bounds__(1024) void vpend_add(Ctrl *c, double *vpend, const double *v, int64_t n) {
    const int valid = c->vpend_valid;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) vpend[j] = valid ? vpend[j] + v[j] : v[j];
    __syncthreads();
    if (threadIdx.x == 0) c->vpend_valid = 1;
}

// Move a drift-schedule translation that is due at the next sweep into the
// one-shot slot (used before the schedule buffer is replaced).
__global__ __launch_bounds__(1024) void sched_to_vpend(Ctrl *c, double *vpend, const double *V,
                                                       int64_t ldV, int64_t n) {
    const int64_t idx = c->v_idx;
    const int valid = c->vpend_valid;
    if (idx >= 0 && V) {
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
            vpend[j] = (valid ? vpend[j] : 0.0) + V[idx * ldV + j];
    }
    __syncthreads();
    if (threadIdx.x == 0 && idx >= 0) {
        c->vpend_valid = V ? 1 : valid;
        c->v_idx = -1;
    }
}

__global__ void ctl_set_drift(Ctrl *c, int64_t T) {
    if (threadIdx.x != 0) return;
    c->sched_len = T;
    c->sched_pos = 0;
    c->v_idx = -1;
}

// Row replacement in place (one workgroup per replaced row): copy the new
// coefficients, refresh ||a_i||^2, and store b_i so that a translation still
// pending for the next sweep leaves the new row's right-hand side as given.
template <int DT>
__global__ __launch_bounds__(256) void scatter_rows(void *A, int64_t ldA, int64_t m, int64_t n,
                                                    const int64_t *rows, const void *new_rows,
                                                    const double *new_b, double *b, double *nu,
                                                    Ctrl *ctl, const double *vpend) {
    using T = typename Store<DT>::T;
    const int64_t q = blockIdx.x;
    const int64_t i = rows[q];
    if (i < 0 || i >= m) {
        if (threadIdx.x == 0) ctl->status = ST_BAD_ROW;
        return;
    }
    const int valid = ctl->vpend_valid;
    T *dst = reinterpret_cast<T *>(A) + i * ldA;
    const T *src = reinterpret_cast<const T *>(new_rows) + q * n;
    double s2 = 0.0, sv = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const T raw = src[j];
        dst[j] = raw;
        const double v = load_elem<DT>(src, j);
        s2 = __fma_rn(v, v, s2);
        if (valid) sv = __fma_rn(v, vpend[j], sv);
    }
    s2 = wave_sum(s2);
    sv = wave_sum(sv);
    __shared__ double p2[4], pv[4];
    if ((threadIdx.x & 63) == 0) {
        p2[threadIdx.x >> 6] = s2;
        pv[threadIdx.x >> 6] = sv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t2 = ((p2[0] + p2[1]) + p2[2]) + p2[3];
        const double tv = ((pv[0] + pv[1]) + pv[2]) + pv[3];
        nu[i] = t2;
        b[i] = valid ? new_b[q] - tv : new_b[q];
        if (!(t2 > 0.0) || !isfinite(t2) || !isfinite(new_b[q])) ctl->status = ST_BAD_ROW;
    }
}

// Apply a pending one-shot translation to b with a pass of its own (used when
// b is read back): b_i += <a_i, vpend>, FP64, one wavefront per row.
template <int DT>
__global__ __launch_bounds__(256) void flush_translation(const void *A, int64_t ldA, int64_t m,
                                                         int64_t n, const Ctrl *ctl,
                                                         const double *vpend, double *b) {
    if (!ctl->vpend_valid) return;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) s = __fma_rn(load_elem<DT>(A, row * ldA + j), vpend[j], s);
    s = wave_sum(s);
    if (lane == 0) b[row] += s;
}

__global__ void ctl_clear_vpend(Ctrl *c) {
    if (threadIdx.x == 0) c->vpend_valid = 0;
}

// Make a pending step permanent (used when x is read back): x <- x - s*y.
__global__ void materialize_x(const Ctrl *c, double *x, const double *y, int64_t n) {
    const double s = c->s;
    if (s == 0.0) return;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        x[j] = step_point(x[j], s, y[j]);
}

__global__ void ctl_clear_step(Ctrl *c) {
    if (threadIdx.x == 0) c->s = 0.0;
}

}  // namespace modap
