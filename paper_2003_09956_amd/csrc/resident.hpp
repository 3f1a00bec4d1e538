// Resident iteration for small systems: many iterations in one launch.
//
// For a system of a few MiB the two-kernel iteration (sweep, then reduction)
// is bound by latency, not bandwidth: each kernel costs a few microseconds
// whatever its size.  Here one cooperative launch of G workgroups runs K
// iterations of the method (section 3: Map of the positive slices, eq. 7,
// Reduce(+), the eq. 10 test, the step of eq. 12 or Algorithm 1, the
// translation of the data) with one grid barrier per iteration and no other
// synchronisation:
//
//   * each workgroup copies its band of rows (and their b, ||a_i||^2) into
//     LDS once, and reads them from there in every iteration;
//   * per iteration it sweeps its band (eight wavefronts, four rows at a time
//     each, lanes over the columns) and writes one partial y and its h, dmax,
//     ||b||inf to one of two buffers (alternating by iteration);
//   * after the barrier every workgroup sums all G partials in the same order,
//     takes the same decision and step in FP64 on its own copy of x, y and the
//     running sum of translations (identical arithmetic on identical data
//     gives identical results in every workgroup), and goes on.
// A workgroup can be at most one barrier ahead of another, so it never
// overwrites partials that another is still reading.
//
// Every wait at the barrier is bounded by the device's constant clock: a
// workgroup that waits longer than timeout_ticks raises ctl->fault and
// leaves, and so do the others once they see it, so the grid always drains.
// A launch with a fault writes nothing back (its results are void).
//
// At the end workgroup 0 writes x, y, the translation sum, the working
// vectors of the two-kernel path and the final state (into both slots); each
// workgroup writes the translated b of its band.  Semantics per iteration are
// those of the two-kernel path (check, step, data update); only the order of
// the sum over row bands differs.
#pragma once

#include <type_traits>

#include "modap_device.hpp"

namespace modap {

struct ResidentArgs {
    const void *A;          // [m x ldA] storage type
    int64_t ldA, m, n;
    int32_t ldR;            // LDS row length: n rounded up to 64 (at most 512)
    int32_t rows;           // rows per workgroup
    double *b;              // [m]
    const double *nu;       // [m]
    double *x, *y, *wsum;   // [ldA]
    const double *vpend;    // [ldA]
    const double *V;        // [T x ldV] or null
    int64_t ldV;
    void *work;             // [3 x ldA] working vectors of the two-kernel path (written at the end)
    Ctrl *ctl;
    int64_t j0;             // the launch runs under the committed state of slot (j0-1)&1
    int64_t K;              // iterations
    Decide dp;
    void *part;             // [2 x kResidentMaxGrid x ldR] accumulation type
    int64_t *h_part;        // [2 x G]
    double *dmax_part;      // [2 x G]
    double *binf_part;      // [2 x G]
    int64_t timeout_ticks;  // constant-clock (100 MHz) ticks a workgroup waits at the barrier
};

// Arrival k (k = 0, 1, ...) at the grid barrier of a resident launch: every
// workgroup's writes before it are visible to every workgroup after it.
// false if the wait timed out or another workgroup gave up.  A workgroup that
// gives up sets the top bit of the arrival counter (so that one read tells a
// waiting workgroup both) and raises ctl->fault for the host.
constexpr uint32_t kBarrierFault = 0x80000000u;

__device__ __forceinline__ bool resident_barrier(Ctrl *ctl, uint32_t target, int64_t timeout_ticks) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    __shared__ int ok;
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(&ctl->barrier, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long t0 = wall_clock64();
        uint32_t seen;
        for (;;) {
            seen = __hip_atomic_load(&ctl->barrier, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (seen >= target) break;
            if (wall_clock64() - t0 > timeout_ticks) {
                seen = kBarrierFault;
                __hip_atomic_fetch_or(&ctl->barrier, kBarrierFault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->fault, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok = (seen & kBarrierFault) == 0;
    }
    __syncthreads();
    return ok != 0;
}

template <int DT>
__device__ __forceinline__ typename Store<DT>::Acc widen(typename Store<DT>::T v) {
    if constexpr (DT == 2)
        return __uint_as_float((uint32_t)v << 16);
    else
        return v;
}

// Totals of four per-lane values over the 64 lanes of a wavefront whose lanes
// are all active: the total of d_j in lanes 16j .. 16j+15.  The lane swaps
// pair the halves and then the quarters of the wavefront (value j and j+2
// share a swap across the halves, j and j+1 across the quarters), each pair
// added lower lane first, and a DPP sum inside each row of 16 lanes finishes:
// three exchanges for the four values instead of one full sum each.
template <typename T>
__device__ __forceinline__ T quad_total(T d0, T d1, T d2, T d3) {
    const T e02 = lane_swap_add(d0, d2, true);   // lanes 0-31: d0, lanes 32-63: d2
    const T e13 = lane_swap_add(d1, d3, true);   // lanes 0-31: d1, lanes 32-63: d3
    return row_total(lane_swap_add(e02, e13, false));
}

constexpr int kResidentMaxCols = 512;   // LDS row length limit (8 columns per lane)
constexpr int kResidentMaxGrid = 32;    // workgroups of a resident launch at most
constexpr int kResidentThreads = 512;   // threads of a resident workgroup (8 wavefronts)
constexpr int kResidentWaves = kResidentThreads / 64;
constexpr int kResidentRowsAtOnce = 4;  // rows a wavefront sweeps at once
constexpr int kResidentStaticLds = 1024; // bytes of static LDS a resident workgroup uses at most

// CPL = columns per lane (the LDS row length is 64 CPL); a template
// parameter, so that a row's loads are issued together and its values stay in
// registers between the dot products and the sum of positive slices.
template <int DT, int CPL>
__global__ __launch_bounds__(kResidentThreads) void resident_iterate(const ResidentArgs a) {
    using S = Store<DT>;
    using T = typename S::T;
    using Acc = typename S::Acc;
    constexpr int ldR = 64 * CPL;
    constexpr int NT = kResidentThreads, NW = kResidentWaves, RA = kResidentRowsAtOnce;
    constexpr int CPT = (ldR + NT - 1) / NT;   // columns per thread in the column-wise phases
    static_assert(NW * RA <= 64, "one wavefront reduces the rows' shares");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int G = (int)gridDim.x, g = (int)blockIdx.x;
    const int64_t r0 = (int64_t)g * a.rows;
    const int nr = (int)max((int64_t)0, min(a.m, r0 + a.rows) - r0);

    // LDS: the band of rows, its b, ||a_i||^2 and ||a_i||, the FP64 x, y
    // and translation sum, x and v in the accumulation type, the
    // wavefronts' partial y
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    auto up16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    size_t off = 0;
    T *As = reinterpret_cast<T *>(lds);
    off += up16((size_t)a.rows * ldR * sizeof(T));
    double *bs = reinterpret_cast<double *>(lds + off);
    off += up16((size_t)a.rows * sizeof(double));
    double *nus = reinterpret_cast<double *>(lds + off);
    off += up16((size_t)a.rows * sizeof(double));
    double *snus = reinterpret_cast<double *>(lds + off);
    off += up16((size_t)a.rows * sizeof(double));
    double *x64 = reinterpret_cast<double *>(lds + off);
    off += (size_t)ldR * sizeof(double);
    double *y64 = reinterpret_cast<double *>(lds + off);
    off += (size_t)ldR * sizeof(double);
    double *ws = reinterpret_cast<double *>(lds + off);
    off += (size_t)ldR * sizeof(double);
    Acc *xa = reinterpret_cast<Acc *>(lds + off);
    off += up16((size_t)ldR * sizeof(Acc));
    Acc *va = reinterpret_cast<Acc *>(lds + off);
    off += up16((size_t)ldR * sizeof(Acc));
    Acc *yw = reinterpret_cast<Acc *>(lds + off);   // [NW][ldR]
    __shared__ double hw[NW * RA], dw[NW * RA], bw[NW * RA], qw[NW];
    __shared__ State st_shared;   // the decision, taken by the last wavefront
    static_assert((3 * NW * RA + NW) * sizeof(double) + sizeof(State) <= kResidentStaticLds,
                  "static LDS within what the host plans for");

    // the band, the committed state and the vectors
    const T *Ag = reinterpret_cast<const T *>(a.A);
    for (int i = tid; i < nr * ldR; i += NT) {
        const int r = i / ldR, c = i - r * ldR;
        As[i] = c < a.n ? Ag[(r0 + r) * a.ldA + c] : (T)0;
    }
    for (int i = tid; i < nr; i += NT) {
        bs[i] = a.b[r0 + i];
        nus[i] = a.nu[r0 + i];
        snus[i] = sqrt(nus[i]);
    }
    // every thread holds the state and takes every decision itself (the same
    // arithmetic on the same values in every thread of every workgroup);
    // the step limit and the schedule length do not change during a launch
    State st = load_global(&a.ctl->st[slot_of(a.j0 - 1)]);
    const int64_t step_limit = load_global(&a.ctl->step_limit);
    const int64_t sched_len = load_global(&a.ctl->sched_len);
    {
        const bool pv = st.vpend_valid != 0;
        const int64_t vi = st.v_idx;
        for (int c = tid; c < ldR; c += NT) {
            const bool in = c < a.n;
            const double xv = in ? a.x[c] : 0.0;
            const double vv = in ? (pv ? a.vpend[c] : 0.0) + ((a.V && vi >= 0) ? a.V[vi * a.ldV + c] : 0.0) : 0.0;
            x64[c] = xv;
            xa[c] = (Acc)xv;
            va[c] = (Acc)vv;
            ws[c] = in ? a.wsum[c] : 0.0;
            y64[c] = in ? a.y[c] : 0.0;
        }
    }
    __syncthreads();

    // [2][kResidentMaxGrid][ldR]: workgroup g's partial y is row g of its
    // half (a wavefront's loads and stores of it cover 64 consecutive
    // columns); rows G.. are never read into a sum
    Acc *part = reinterpret_cast<Acc *>(a.part);
    bool failed = false;
    for (int64_t it = 0; it < a.K; ++it) {
        // the state this sweep runs under
        if (st.status != ST_RUNNING) break;
        const bool pv = st.vpend_valid != 0;
        const int64_t vi = st.v_idx, sp = st.sched_pos;
        const bool apply = pv || vi >= 0;
        const int par = (int)(it & 1);
        Acc xr[CPL], vr[CPL], yacc[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            xr[k] = xa[lane + 64 * k];
            vr[k] = apply ? va[lane + 64 * k] : (Acc)0;
            yacc[k] = (Acc)0;
        }
        // lane 16j of a wavefront settles row j of each of its batches and
        // keeps that row's share of h, dmax and ||b||inf
        static_assert(RA == 4, "the four rows of a batch are reduced together");
        const int jl = lane >> 4;
        const bool settler = (lane & 15) == 0;
        double h = 0.0, dmax = 0.0, binf = 0.0;
        // (compiled with and without the translation of the data)
        auto sweep_band = [&](auto with_translation) {
            constexpr bool AP = decltype(with_translation)::value;
            // wavefront w takes rows w, w + NW, w + 2 NW, ..., RA of them at a
            // time and without branches, so that their loads, dot products,
            // wavefront sums and divisions overlap (rows past the band count as
            // satisfied and are not written)
            for (int base = 0; base < nr; base += NW * RA) {
                Acc av[RA][CPL], dot[RA], tdot[RA];
                bool ok[RA];
#pragma unroll
                for (int j = 0; j < RA; ++j) {
                    const int r = base + wave + NW * j;
                    ok[j] = r < nr;
                    const T *row = As + (ok[j] ? r : 0) * ldR;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) av[j][k] = widen<DT>(row[lane + 64 * k]);
                    dot[j] = (Acc)0;
                    tdot[j] = (Acc)0;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) {
                        dot[j] = fma(xr[k], av[j][k], dot[j]);
                        if constexpr (AP) tdot[j] = fma(vr[k], av[j][k], tdot[j]);
                    }
                }
                const double dj = quad_total(dot[0], dot[1], dot[2], dot[3]);
                double tj = 0.0;
                if constexpr (AP) tj = quad_total(tdot[0], tdot[1], tdot[2], tdot[3]);
                const int rj = base + wave + NW * jl;
                const bool okj = settler && rj < nr;
                const int rc = okj ? rj : 0;
                double bb = bs[rc];
                if constexpr (AP) bb += tj;
                const double rr = okj ? dj - bb : -1.0;
                if (okj) {
                    bs[rj] = bb;
                    binf = max_nan(binf, fabs(bb));
                }
                const bool pos = rr > 0.0;
                h += pos ? 1.0 : 0.0;
                const double d = rr / snus[rc];
                dmax = pos ? max_nan(dmax, d) : (rr != rr ? rr : dmax);
                const Acc w = pos ? (Acc)(rr / nus[rc]) : (Acc)0;
#pragma unroll
                for (int j = 0; j < RA; ++j) {
                    const Acc wj = lane_value(w, 16 * j);
#pragma unroll
                    for (int k = 0; k < CPL; ++k) yacc[k] = fma(wj, av[j][k], yacc[k]);
                }
            }
        };
        if (apply)
            sweep_band(std::integral_constant<bool, true>{});
        else
            sweep_band(std::integral_constant<bool, false>{});
        // the wavefronts' partials, summed in wavefront order
#pragma unroll
        for (int k = 0; k < CPL; ++k) yw[wave * ldR + lane + 64 * k] = yacc[k];
        if (settler) {
            hw[wave * RA + jl] = h;
            dw[wave * RA + jl] = dmax;
            bw[wave * RA + jl] = binf;
        }
        __syncthreads();
        // the workgroup's partial y and totals, stored as agent-scope atomics:
        // they are written through to where every workgroup reads them as
        // they are stored, so the release at the barrier finds nothing left
        // to write back
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + NT * k;
            if (c < ldR) {
                Acc sum = yw[c];
#pragma unroll
                for (int w = 1; w < NW; ++w) sum += yw[w * ldR + c];
                __hip_atomic_store(&part[((int64_t)par * kResidentMaxGrid + g) * ldR + c], sum, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (wave == NW - 1) {   // the workgroup's shares of h, dmax, ||b||inf
            const bool in = lane < NW * RA;
            const double hh = wave_total(in ? hw[lane] : 0.0);   // integers below 2^53: exact
            const double dd = wave_max_nan(in ? dw[lane] : 0.0);
            const double bm = wave_max_nan(in ? bw[lane] : 0.0);
            if (lane == 0) {
                __hip_atomic_store(&a.h_part[par * G + g], (int64_t)hh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.dmax_part[par * G + g], dd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&a.binf_part[par * G + g], bm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // Before the barrier (they depend on the state this sweep ran under
        // only): the translation this sweep applied joins the FP64 sum, and the
        // drift row due after a step (row sched_pos: the decision either takes
        // it or none) is requested, so that it arrives during the wait.
        const bool next_due = a.V && sp < sched_len;
        double vcand[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + NT * k;
            vcand[k] = (c < a.n && next_due) ? a.V[sp * a.ldV + c] : 0.0;
            if (c < a.n && apply) ws[c] += (pv ? a.vpend[c] : 0.0) + ((a.V && vi >= 0) ? a.V[vi * a.ldV + c] : 0.0);
        }
        if (!resident_barrier(a.ctl, (uint32_t)(it + 1) * (uint32_t)G, a.timeout_ticks)) {
            failed = true;
            break;
        }
        // every workgroup: y as the sum of the G partials in workgroup order,
        // FP64, and ||y||^2 in a fixed order, by the threads that hold a
        // column; the totals (an integer sum and two maxima, exact in any
        // order) and the decision by the last wavefront, once, shared through
        // LDS.  Every load is issued before the first use (slots past G are
        // not read; lanes past G read slot G-1 and are masked out).
        const bool decider = wave == NW - 1;
        const int gl = min(lane, G - 1);
        int64_t hr = 0;
        double dr = 0.0, br = 0.0;
        if (decider) {
            hr = a.h_part[par * G + gl];
            dr = a.dmax_part[par * G + gl];
            br = a.binf_part[par * G + gl];
        }
        double q = 0.0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + NT * k;
            if (c >= ldR) continue;
            const Acc *pc = part + (int64_t)par * kResidentMaxGrid * ldR + c;
            Acc t[kResidentMaxGrid];
#pragma unroll
            for (int gg = 0; gg < kResidentMaxGrid; ++gg) t[gg] = gg < G ? pc[(int64_t)gg * ldR] : (Acc)0;
            double s = 0.0;
#pragma unroll
            for (int gg = 0; gg < kResidentMaxGrid; ++gg) s += gg < G ? (double)t[gg] : 0.0;
            y64[c] = s;
            q += s * s;
        }
        if (wave * 64 < ldR) q = wave_total(q);   // (the other wavefronts hold no column)
        if (lane == 0) qw[wave] = q;
        Totals t{};
        if (decider) {   // (while the other wavefronts wait for their loads)
            t.h = (int64_t)wave_total(lane < G ? (double)hr : 0.0);   // integers below 2^53: exact
            t.dmax = wave_max_nan(lane < G ? dr : 0.0);
            t.binf = wave_max_nan(lane < G ? br : 0.0);
        }
        __syncthreads();
        if (decider) {
            double qq = qw[0];
#pragma unroll
            for (int w = 1; w < NW; ++w) qq += qw[w];
            const State s = decide(st, t, sqrt(qq), a.dp, step_limit, sched_len);
            if (lane == 0) st_shared = s;
        }
        __syncthreads();
        st = st_shared;
        // the step (x <- x - s y, one rounding) and the translation due at the
        // next sweep (the row requested before the barrier, when one is due)
        const double step = st.s;
        const bool take = st.v_idx >= 0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int c = tid + NT * k;
            if (c >= a.n) continue;
            if (step != 0.0) x64[c] = step_point(x64[c], step, y64[c]);
            xa[c] = (Acc)x64[c];
            va[c] = take ? (Acc)vcand[k] : (Acc)0;
        }
        __syncthreads();
    }
    // The last workgroup to leave clears the arrival counters for the next
    // launch on this stream (a kernel, not a memory set, so that the stream's
    // work stays kernels only).  Every workgroup has then left its loop, so
    // none is still reading them; a fault stays raised in ctl->fault.
    __syncthreads();
    if (tid == 0) {
        const uint32_t out = __hip_atomic_fetch_add(&a.ctl->exits, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (out == (uint32_t)G - 1) {
            __hip_atomic_store(&a.ctl->barrier, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&a.ctl->exits, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (failed) return;

    // write back: the band's b; workgroup 0 the vectors and the state
    for (int i = tid; i < nr; i += NT) a.b[r0 + i] = bs[i];
    if (g != 0) return;
    const State p = st;
    const double *vrow_next = (a.V && p.v_idx >= 0) ? a.V + p.v_idx * a.ldV : nullptr;
    Acc *wx = reinterpret_cast<Acc *>(a.work);
    for (int c = tid; c < a.n; c += NT) {
        a.x[c] = x64[c];
        a.y[c] = y64[c];
        a.wsum[c] = ws[c];
        wx[c] = (Acc)x64[c];
        wx[a.ldA + c] = vrow_next ? (Acc)vrow_next[c] : (Acc)0;
        wx[2 * a.ldA + c] = (Acc)y64[c];
    }
    if (tid == 0) {
        store_global(&a.ctl->st[0], p);
        store_global(&a.ctl->st[1], p);
    }
}

}  // namespace modap
