// Kernels around the sweep: row norms, the fixed-order reduction of the
// partial y, the stage kernel that settles each iteration, control-block
// updates made between calls, in-place row replacement and the exact
// right-hand side read back by a query.
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

// Threads of a reduction workgroup.  Measured on the FP32 n = 8192 system
// with 256 partials: 256 threads took 5.2 us, 1024 threads 6.9 us (with
// permute-unit sums and 8 loads in flight; 4.3 us now at 256).
constexpr int kReduceThreads = 256;

// Column sums of the workgroup partials of y, in a fixed order, in FP64.
// Workgroup b writes its share of ||y||^2 to ynp[b]; workgroup 0 also forms
// the totals of h, dmax and binf.  The stop test and the step are taken from
// these by the next sweep (or by the stage kernel at the end of a call).  In
// iteration mode it first makes the previous step permanent in x and then
// writes the working vectors of the next sweep.
template <typename Acc>
__global__ __launch_bounds__(kReduceThreads) void reduce_y(const ReduceArgs a) {
    constexpr int COLS = 64;                    // columns per workgroup
    constexpr int VW = 16 / (int)sizeof(Acc);   // columns per 16-byte load
    constexpr int LPRR = COLS / VW;             // lanes per partial row
    constexpr int RPW = 64 / LPRR;              // partial rows per wavefront load
    constexpr int NWR = kReduceThreads / 64;    // wavefronts per workgroup
    constexpr int RG = NWR * RPW;               // row groups per workgroup
    constexpr int U = 16;                       // loads in flight per lane
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int rg = (tid >> 6) * RPW + lane / LPRR;
    const int cl = lane % LPRR;
    const int64_t col = (int64_t)blockIdx.x * COLS + tid;   // column of threads 0..63
    // ldPart is a multiple of 64 and covers every workgroup's columns
    const Acc *pc = reinterpret_cast<const Acc *>(a.part) + (int64_t)blockIdx.x * COLS + cl * VW;

    // Every load that does not depend on the state is issued before the state
    // is examined: the first batch of partial rows, the column's x and
    // previous y, and (workgroup 0) the first scalar partials.
    uint4 v[U];
    auto issue = [&](int g0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = min(g0 + u * RG, a.G - 1);
            v[u] = *reinterpret_cast<const uint4 *>(pc + (int64_t)g * a.ldPart);
        }
    };
    issue(rg);
    const bool colw = a.work && tid < COLS && col < a.n;
    double xo = 0.0, yo = 0.0, wso = 0.0;
    int64_t slen = 0;
    if (colw) {
        xo = load_global(a.x + col);
        yo = load_global(a.y + col);
        if (a.wsum) wso = load_global(a.wsum + col);
        if (a.V) slen = load_global(&a.ctl->sched_len);
    }
    int64_t h = 0;
    double dm = 0.0, bm = 0.0;
    if (blockIdx.x == 0 && tid < a.Gs) {
        h = load_global(a.h_part + tid);
        dm = load_global(a.dmax_part + tid);
        bm = load_global(a.binf_part + tid);
    }
    State S{};
    if (a.iterate) {
        S = load_global(&a.ctl->st[slot_of(a.j - 1)]);
        if (S.status != ST_RUNNING) return;
    }
    // The drift row due next depends on the state only: requested now, so
    // that it arrives while the partial rows are summed.  So is the
    // translation this sweep applied (one-shot part and drift row), which is
    // added to the running sum of translations in FP64.
    const bool due = colw && a.V && S.sched_pos < slen;
    const double vdue = due ? load_global(a.V + S.sched_pos * a.ldV + col) : 0.0;
    const bool ap = colw && a.wsum && a.has_v && S.vpend_valid;
    const bool ar = colw && a.wsum && a.has_v && a.V && S.v_idx >= 0;
    const double vap = (ap ? load_global(a.vpend + col) : 0.0) + (ar ? load_global(a.V + S.v_idx * a.ldV + col) : 0.0);

    // Batches of U independent 16-byte loads (partial rows rg, rg+RG, ...),
    // each batch summed in order, batches in order: a fixed order for a given G.
    double acc[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) acc[k] = 0.0;
    for (int g0 = rg; g0 < a.G; g0 += U * RG) {
        if (g0 != rg) issue(g0);
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            double bsum = 0.0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                Acc e[VW];
                __builtin_memcpy(e, &v[u], 16);
                if (g0 + u * RG < a.G) bsum += (double)e[k];
            }
            acc[k] += bsum;
        }
    }
    __shared__ double sh[RG][COLS];
#pragma unroll
    for (int k = 0; k < VW; ++k) sh[rg][cl * VW + k] = acc[k];
    __syncthreads();
    if (tid < 64) {
        double yv = 0.0;
#pragma unroll 8
        for (int r = 0; r < RG; ++r) yv += sh[r][tid];
        double sq = 0.0;
        if (col < a.n) {
            if (colw) {
                // the step decided on the previous check becomes permanent in
                // FP64, then the working vectors of the next sweep: x, the
                // drift row due next (applied if the next decision moves on),
                // and this sweep's y
                if (a.apply_step && S.s != 0.0) {
                    xo = step_point(xo, S.s, yo);
                    a.x[col] = xo;
                }
                Acc *w = reinterpret_cast<Acc *>(a.work);
                w[col] = (Acc)xo;
                w[a.ldA + col] = (Acc)vdue;
                w[2 * a.ldA + col] = (Acc)yv;
                if (ap || ar) a.wsum[col] = wso + vap;
            }
            a.y[col] = yv;
            sq = yv * yv;
        }
        sq = wave_total(sq);
        if (tid == 0) a.ynp[blockIdx.x] = sq;
    }
    if (blockIdx.x != 0) return;

    for (int g = tid + kReduceThreads; g < a.Gs; g += kReduceThreads) {
        h += a.h_part[g];
        dm = max_nan(dm, a.dmax_part[g]);
        bm = max_nan(bm, a.binf_part[g]);
    }
    // across each wavefront with DPP moves (no permute round trips): h as an
    // FP64 sum of integers below 2^53 (exact), the maxima in any order
    h = (int64_t)wave_total((double)h);
    dm = wave_max_nan(dm);
    bm = wave_max_nan(bm);
    __shared__ int64_t hw[NWR];
    __shared__ double dw[NWR], bw[NWR];
    if (lane == 0) {
        hw[wv] = h;
        dw[wv] = dm;
        bw[wv] = bm;
    }
    __syncthreads();
    if (tid != 0) return;
    Totals t{};
    for (int w = 0; w < NWR; ++w) {
        t.h += hw[w];
        t.dmax = max_nan(t.dmax, dw[w]);
        t.binf = max_nan(t.binf, bw[w]);
    }
    *a.tot = t;
}

// End of a call: settle the last check j (no sweep follows to do it).  Every
// workgroup takes the decision from the check's totals (the same arithmetic in
// every workgroup), workgroup 0 records it in slot j & 1, and each workgroup,
// for its columns, makes the step permanent in FP64 (x <- x - s*y, eq. 12 or
// Algorithm 1) and writes x and the translation due next into the working
// vectors.
template <typename Acc>
__global__ __launch_bounds__(256) void stage_iter(const StageArgs a) {
    const State p = a.ctl->st[slot_of(a.j - 1)];
    if (p.status != ST_RUNNING) {
        if (blockIdx.x == 0 && threadIdx.x == 0) a.ctl->st[slot_of(a.j)] = p;
        return;
    }
    __shared__ State sst;
    if (threadIdx.x < 64) {
        const double yn = ynorm_of(a.ynp, a.R, threadIdx.x);
        const State cur = decide(p, *a.tot, yn, a.dp, a.ctl->step_limit, a.ctl->sched_len);
        if (threadIdx.x == 0) {
            sst = cur;
            if (blockIdx.x == 0) a.ctl->st[slot_of(a.j)] = cur;
        }
    }
    __syncthreads();
    const double s = sst.s;
    const double *vrow = (a.V && sst.v_idx >= 0) ? a.V + sst.v_idx * a.ldV : nullptr;
    Acc *wx = reinterpret_cast<Acc *>(a.work);
    Acc *wv = wx + a.ldA;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        double xv = a.x[j];
        if (s != 0.0) {
            xv = step_point(xv, s, a.y[j]);
            a.x[j] = xv;
        }
        wx[j] = (Acc)xv;
        wv[j] = vrow ? (Acc)vrow[j] : (Acc)0;
    }
}

// Working vectors for the first sweep of a call (or an evaluation) from the
// committed state in slot (j-1)&1: x as it is, and the pending translation
// (one-shot part plus the drift row due).
template <typename Acc>
__global__ __launch_bounds__(256) void prime_work(const StageArgs a) {
    const State &p = a.ctl->st[slot_of(a.j - 1)];
    const bool use_p = p.vpend_valid != 0;
    const double *vrow = (a.V && p.v_idx >= 0) ? a.V + p.v_idx * a.ldV : nullptr;
    Acc *wx = reinterpret_cast<Acc *>(a.work);
    Acc *wv = wx + a.ldA;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double v = (use_p ? a.vpend[j] : 0.0) + (vrow ? vrow[j] : 0.0);
        wx[j] = (Acc)a.x[j];
        wv[j] = (Acc)v;
    }
}

// Working vectors of a stateless sweep at x: x in the accumulation type, no
// translation, no previous direction (zero-padded to ldA).
template <typename Acc>
__global__ __launch_bounds__(256) void stage_point(const double *x, int64_t n, int64_t ldA, void *work) {
    Acc *w = reinterpret_cast<Acc *>(work);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < ldA; j += (int64_t)gridDim.x * blockDim.x) {
        w[j] = j < n ? (Acc)x[j] : (Acc)0;
        w[ldA + j] = (Acc)0;
        w[2 * ldA + j] = (Acc)0;
    }
}

// The totals of a reduction to caller memory (either pointer may be null).
__global__ void copy_totals(const Totals *t, int64_t *h, double *dmax) {
    if (threadIdx.x != 0) return;
    const Totals v = *t;
    if (h) *h = v.h;
    if (dmax) *dmax = v.dmax;
}

// The control kernels below run between calls as a single thread (or a
// single workgroup) on the committed state in slot `sl`.

// Start of an iterate/solve call: a stop that came from a previous call's
// tolerance, step limit or missing direction is re-examined by the next sweep.
__global__ void ctl_begin(Ctrl *c, int sl, int64_t max_steps) {
    if (threadIdx.x != 0) return;
    State &s = c->st[sl];
    if (s.status == ST_CONVERGED || s.status == ST_LIMIT || s.status == ST_NO_DIRECTION) s.status = ST_RUNNING;
    c->step_limit = max_steps < 0 ? INT64_MAX : s.steps + max_steps;
}

// A fresh state (set_system): both slots.
__global__ void ctl_init(Ctrl *c) {
    if (threadIdx.x != 0) return;
    State s{};
    s.v_idx = -1;
    s.status = ST_RUNNING;
    c->st[0] = s;
    c->st[1] = s;
    c->step_limit = INT64_MAX;
    c->sched_len = 0;
    c->barrier = 0;
    c->fault = 0;
    c->exits = 0;
}

// A new approximation: counters restart, no step is pending.
__global__ void ctl_restart(Ctrl *c, int sl) {
    if (threadIdx.x != 0) return;
    State &s = c->st[sl];
    if (s.status != ST_BAD_ROW) s.status = ST_RUNNING;
    s.s = 0.0;
    s.steps = 0;
    s.sweeps = 0;
    s.dmax = s.binf = s.ynorm = s.eps_abs = 0.0;
    s.h = 0;
    s.feasible = 0;
}

// One-shot translation: vpend <- (pending ? vpend : 0) + v.  A single
// workgroup, so the pending flag is read before it is set.
__global__ __launch_bounds__(1024) void vpend_add(Ctrl *c, int sl, double *vpend, const double *v, int64_t n) {
    const int valid = c->st[sl].vpend_valid;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) vpend[j] = valid ? vpend[j] + v[j] : v[j];
    __syncthreads();
    if (threadIdx.x == 0) c->st[sl].vpend_valid = 1;
}

// Move a drift-schedule translation that is due at the next sweep into the
// one-shot slot (used before the schedule buffer is replaced or b is read).
__global__ __launch_bounds__(1024) void sched_to_vpend(Ctrl *c, int sl, double *vpend, const double *V,
                                                       int64_t ldV, int64_t n) {
    const int64_t idx = c->st[sl].v_idx;
    const int valid = c->st[sl].vpend_valid;
    if (idx >= 0 && V) {
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
            vpend[j] = (valid ? vpend[j] : 0.0) + V[idx * ldV + j];
    }
    __syncthreads();
    if (threadIdx.x == 0 && idx >= 0) {
        c->st[sl].vpend_valid = V ? 1 : valid;
        c->st[sl].v_idx = -1;
    }
}

__global__ void ctl_set_drift(Ctrl *c, int sl, int64_t T) {
    if (threadIdx.x != 0) return;
    c->sched_len = T;
    c->st[sl].sched_pos = 0;
    c->st[sl].v_idx = -1;
}

// Row replacement in place (one workgroup per replaced row): copy the new
// coefficients, refresh ||a_i||^2, and store the right-hand sides.  A
// translation still pending for the next sweep (the one-shot part and the
// drift row due) has already happened to the data the caller sees, so it must
// not move the new row: b_i is stored as new_b - <a_new, pending>, which the
// next sweep's translation brings back to new_b.  The exact data are
// bref + A wsum, so bref_i = new_b - <a_new, wsum + pending>.  Nothing is
// written once the state holds ST_BAD_ROW (for instance after a duplicate
// device-side row index).
template <int DT>
__global__ __launch_bounds__(256) void scatter_rows(void *A, int64_t ldA, int64_t m, int64_t n,
                                                    const int64_t *rows, const void *new_rows,
                                                    const double *new_b, double *b, double *bref, double *nu,
                                                    Ctrl *ctl, int sl, const double *vpend, const double *V,
                                                    int64_t ldV, const double *wsum) {
    using T = typename Store<DT>::T;
    const int64_t q = blockIdx.x;
    const State st = load_global(&ctl->st[sl]);
    if (st.status == ST_BAD_ROW) return;
    const int64_t i = rows[q];
    if (i < 0 || i >= m) {
        if (threadIdx.x == 0) ctl->st[sl].status = ST_BAD_ROW;
        return;
    }
    const bool valid = st.vpend_valid != 0;
    const double *vrow = (V && st.v_idx >= 0) ? V + st.v_idx * ldV : nullptr;
    T *dst = reinterpret_cast<T *>(A) + i * ldA;
    const T *src = reinterpret_cast<const T *>(new_rows) + q * n;
    double s2 = 0.0, sv = 0.0, sw = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += 256) {
        const T raw = src[j];
        dst[j] = raw;
        const double v = load_elem<DT>(src, j);
        s2 = __fma_rn(v, v, s2);
        const double pj = (valid ? vpend[j] : 0.0) + (vrow ? vrow[j] : 0.0);
        sv = __fma_rn(v, pj, sv);
        sw = __fma_rn(v, wsum[j], sw);
    }
    s2 = wave_sum(s2);
    sv = wave_sum(sv);
    sw = wave_sum(sw);
    __shared__ double p2[4], pv[4], pw[4];
    if ((threadIdx.x & 63) == 0) {
        p2[threadIdx.x >> 6] = s2;
        pv[threadIdx.x >> 6] = sv;
        pw[threadIdx.x >> 6] = sw;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t2 = ((p2[0] + p2[1]) + p2[2]) + p2[3];
        const double tv = ((pv[0] + pv[1]) + pv[2]) + pv[3];
        const double tw = ((pw[0] + pw[1]) + pw[2]) + pw[3];
        nu[i] = t2;
        b[i] = new_b[q] - tv;
        bref[i] = new_b[q] - (tw + tv);
        if (!(t2 > 0.0) || !isfinite(t2) || !isfinite(new_b[q])) ctl->st[sl].status = ST_BAD_ROW;
    }
}

// Device-side row indices of a replacement: one thread per index claims its
// row in `claim` (zero outside this pair of kernels); an index out of range or
// claimed twice puts the state in ST_BAD_ROW before any row is written.
__global__ void claim_rows(const int64_t *rows, int64_t k, int64_t m, int *claim, Ctrl *ctl, int sl) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < k; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = rows[q];
        if (i < 0 || i >= m || atomicAdd(claim + i, 1) != 0) ctl->st[sl].status = ST_BAD_ROW;
    }
}

// Releases the claims of claim_rows (after the replacement).
__global__ void release_rows(const int64_t *rows, int64_t k, int64_t m, int *claim) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < k; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = rows[q];
        if (i >= 0 && i < m) claim[i] = 0;
    }
}

// The right-hand side of the data as the caller sees them, in FP64 and
// without changing any state: out_i = bref_i + <a_i, wsum + pending>, with
// the pending translation (one-shot part and due drift row) of slot sl.  One
// wavefront per row, a fixed summation order.
template <int DT>
__global__ __launch_bounds__(256) void rhs_exact(const void *A, int64_t ldA, int64_t m, int64_t n, const Ctrl *ctl,
                                                 int sl, const double *bref, const double *wsum,
                                                 const double *vpend, const double *V, int64_t ldV, double *out) {
    const State st = load_global(&ctl->st[sl]);
    const bool valid = st.vpend_valid != 0;
    const double *vrow = (V && st.v_idx >= 0) ? V + st.v_idx * ldV : nullptr;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
        const double t = wsum[j] + ((valid ? vpend[j] : 0.0) + (vrow ? vrow[j] : 0.0));
        s = __fma_rn(load_elem<DT>(A, row * ldA + j), t, s);
    }
    s = wave_sum(s);
    if (lane == 0) out[row] = bref[row] + s;
}

}  // namespace modap
