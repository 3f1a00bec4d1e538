// Batched sweep: many independent systems advanced together.
//
// Every system of a batch is the problem of the single-system library (the
// sweep of section 3, the eps test of eq. 10, the step of eq. 12 or
// Algorithm 1, the translation of the data), and every system keeps its own
// state.  Two kernels advance all of them by one iteration:
//
//   sweep_batch   a persistent grid takes work items -- bands of rows of one
//                 system -- from a device queue until it is empty.  One
//                 wavefront streams one row at a time (its dot products need
//                 no barrier); the four wavefronts of a workgroup take every
//                 fourth row of the band; the item's x and v are staged in
//                 LDS and each lane keeps C 16-byte chunks of its partial y in
//                 registers, C = 1, 2, 4 or 8 chosen per system from its row
//                 length.  Each item writes
//                 its own partial y and scalars, so a system's result does not
//                 depend on which workgroup took which item, nor on the other
//                 systems in the batch.
//   reduce_batch  one workgroup per 64 columns of a system: the system's item
//                 partials summed in item order, the previous step made
//                 permanent in x, and the next sweep's working vectors.
//
// The decision on a check is taken, as in the single-system library, by the
// first kernel of the next sweep: every item of system s settles check j-1 of
// s from the state in slot (j-2)&1 and the totals of the last reduction; the
// system's first item commits it to slot (j-1)&1.
#pragma once

#include "modap_device.hpp"
#include "sweep_wide.hpp"

namespace modap {

// One system of a batch, as the batch kernels see it.
struct BatchSys {
    const void *A;          // [m x ldA] storage type, rows padded with zeros
    int64_t ldA, m, n;
    double *b;              // [m]
    const double *nu;       // [m] ||a_i||^2
    double *x, *y;          // [ldA] FP64, zero-padded
    const double *vpend;    // [ldA] one-shot translation
    double *wsum;           // [ldA] FP64 sum of the translations applied since the last rebase
    const double *V;        // drift schedule [T x ldA] or null
    void *work;             // [3 x ldA] Acc: x, v and y of the next sweep
    Ctrl *ctl;
    Totals *tot;
    double *ynp;            // [R] norm parts of y
    int32_t R;              // 64-column blocks: ceil(n/64)
    int32_t C;              // 16-byte chunks per lane: (64/RPW)*VEC*C >= ldA
    int32_t RPW;            // rows a wavefront sweeps at once: 1, or 4 (16 lanes per row)
    int32_t pad;
    int64_t item0, nitems;  // the system's work items
    int64_t part0;          // Acc offset of the first item's partial y (stride ldA)
    int64_t rows_per_item;
};

// A 64-column block of one system (one workgroup of the reduction).
struct BatchCol {
    int32_t sys;
    int32_t blk;
};

struct BatchArgs {
    const BatchSys *sys;
    int32_t nsys;
    int32_t nitems;
    const int32_t *item_sys;  // [nitems] the system of each item; a system's items are consecutive
    const int32_t *item_order;  // [nitems] the item handed out at each queue position
    void *part;               // per-item partial y
    int64_t *h_part;          // [nitems]
    double *dmax_part;        // [nitems]
    double *binf_part;        // [nitems]
    int32_t *queue;           // next item to take; zero before every sweep
    int64_t j;                // index of this iteration (all systems advance together)
    int32_t decide;           // the sweep settles the previous check (all but a call's first)
    int32_t apply_step;       // the reduction makes the previous step permanent first
    Decide dp;
    int32_t check_status;     // skip systems whose state is not ST_RUNNING
    int32_t write_b;          // store the translated b (0: a stateless sweep, e.g. for timing)
};

constexpr int kBatchWaves = 4;  // wavefronts per workgroup of sweep_batch
constexpr int kBatchCmax = 8;   // largest C compiled

// Stage the item's x_j = x_{j-1} - s*y_{j-1} (one rounding) and v in LDS,
// zero from ldA to COLS (all threads of the workgroup; the caller syncs).
template <int DT>
__device__ __forceinline__ void batch_stage(const BatchSys &S, bool apply_v, double s, typename Store<DT>::Acc *xs,
                                            typename Store<DT>::Acc *vs, int COLS) {
    using Acc = typename Store<DT>::Acc;
    constexpr int AV = 16 / (int)sizeof(Acc);
    const int tid = threadIdx.x;
    const int64_t ldA = S.ldA;
    const Acc *wx = reinterpret_cast<const Acc *>(S.work);
    const Acc *wv = wx + ldA;
    const Acc *wy = wx + 2 * ldA;
    for (int col = tid * AV; col < COLS; col += 256 * AV) {
        Acc xv[AV], vv[AV];
        if (col < ldA) {
            const uint4 ux = load_global(reinterpret_cast<const uint4 *>(wx + col));
            __builtin_memcpy(xv, &ux, 16);
            if (s != 0.0) {
                Acc yv[AV];
                const uint4 uy = load_global(reinterpret_cast<const uint4 *>(wy + col));
                __builtin_memcpy(yv, &uy, 16);
#pragma unroll
                for (int q = 0; q < AV; ++q) xv[q] = (Acc)step_point((double)xv[q], s, (double)yv[q]);
            }
            if (apply_v) {
                const uint4 uv = load_global(reinterpret_cast<const uint4 *>(wv + col));
                __builtin_memcpy(vv, &uv, 16);
            } else {
#pragma unroll
                for (int q = 0; q < AV; ++q) vv[q] = (Acc)0;
            }
        } else {
#pragma unroll
            for (int q = 0; q < AV; ++q) xv[q] = vv[q] = (Acc)0;
        }
        uint4 ux, uv;
        __builtin_memcpy(&ux, xv, 16);
        __builtin_memcpy(&uv, vv, 16);
        *reinterpret_cast<uint4 *>(xs + col) = ux;
        *reinterpret_cast<uint4 *>(vs + col) = uv;
    }
}

// End of a work item: the wavefronts' partials of y summed in LDS and
// written as the item's partial (lanes with `owner` set hold the partial of
// their columns col_of(c)), and the item's h, dmax and ||b||inf.
template <int DT, int C, typename ColOf>
__device__ __forceinline__ void batch_item_end(const BatchArgs &a, const BatchSys &S, int64_t k, int64_t band,
                                               typename Store<DT>::Acc (&yacc)[C][Store<DT>::VEC], int64_t h,
                                               double dmax, double binf,
                                               typename Store<DT>::Acc (*lds)[kBatchCmax * 64 * Store<DT>::VEC],
                                               int64_t *hsh, double *dsh, double *bsh, ColOf col_of, bool owner) {
    using Acc = typename Store<DT>::Acc;
    constexpr int VEC = Store<DT>::VEC;
    constexpr int AV = 16 / (int)sizeof(Acc);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t ldA = S.ldA;
    // The wavefronts' partials are summed pairwise in LDS (the staging space
    // is free once every wavefront has left the row loop):
    // (w0 + w2) + (w1 + w3); wavefront 0 writes the item's partial.
    auto put = [&](Acc *dst) {
        if (!owner) return;
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                uint4 w;
                __builtin_memcpy(&w, &yacc[c][e], 16);
                *reinterpret_cast<uint4 *>(dst + col_of(c) + e) = w;
            }
    };
    auto add = [&](const Acc *src) {
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                Acc t4[AV];
                const uint4 u = *reinterpret_cast<const uint4 *>(src + col_of(c) + e);
                __builtin_memcpy(t4, &u, 16);
#pragma unroll
                for (int q = 0; q < AV; ++q) yacc[c][e + q] += t4[q];
            }
    };
    if (lane == 0) {
        hsh[wave] = h;
        dsh[wave] = dmax;
        bsh[wave] = binf;
    }
    __syncthreads();
    if (wave >= 2) put(lds[wave - 2]);
    __syncthreads();
    if (wave < 2) add(lds[wave]);
    __syncthreads();
    if (wave == 1) put(lds[0]);
    __syncthreads();
    if (wave == 0 && owner) {
        add(lds[0]);
        Acc *part = reinterpret_cast<Acc *>(a.part) + S.part0 + band * ldA;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (col_of(c) >= ldA) continue;
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                uint4 w;
                __builtin_memcpy(&w, &yacc[c][e], 16);
                *reinterpret_cast<uint4 *>(part + col_of(c) + e) = w;
            }
        }
    }
    if (tid == 0) {
        int64_t hh = 0;
        double dd = 0.0, bm = 0.0;
        for (int g = 0; g < kBatchWaves; ++g) {
            hh += hsh[g];
            dd = max_nan(dd, dsh[g]);
            bm = max_nan(bm, bsh[g]);
        }
        a.h_part[k] = hh;
        a.dmax_part[k] = dd;
        a.binf_part[k] = bm;
    }
}

// One work item: rows [r0, r1) of system S, wavefront w taking rows r0+w,
// r0+w+4, ...  The item's x (with the previous step applied) and v are staged
// once in LDS, and every lane reads its columns from there for each row; the
// lane's partial y and two rows in flight stay in registers.  Every branch
// that guards a barrier is uniform over the workgroup.
template <int DT, int C>
__device__ void batch_item(const BatchArgs &a, const BatchSys &Sref, int64_t k,
                           typename Store<DT>::Acc (*lds)[kBatchCmax * 64 * Store<DT>::VEC],
                           int64_t *hsh, double *dsh, double *bsh) {
    using St = Store<DT>;
    using Acc = typename St::Acc;
    using T = typename St::T;
    constexpr int VEC = St::VEC;
    constexpr int CW = 64 * VEC;                   // columns per chunk
    constexpr int AV = 16 / (int)sizeof(Acc);      // Acc per 16-byte vector
    constexpr int COLS = C * CW;                   // staged columns (>= ldA)
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform per wavefront
    // The system's fields are read once per item: held in memory, they would
    // be read again after every store the compiler cannot tell apart from them.
    const BatchSys S = Sref;
    const int64_t band = k - S.item0;
    const int64_t r0 = band * S.rows_per_item;
    const int64_t r1 = min(S.m, r0 + S.rows_per_item);
    const int64_t ldA = S.ldA;
    auto col_of = [&](int c) -> int { return c * CW + lane * VEC; };
    const char *Ab = reinterpret_cast<const char *>(S.A);
    const int64_t row_bytes = ldA * (int64_t)sizeof(T);

    // this wavefront's rows; the first two are requested before the state is settled
    const int64_t nrows = r1 - r0;
    const int64_t nmine = nrows > wave ? (nrows - wave + kBatchWaves - 1) / kBatchWaves : 0;
    auto row_of = [&](int64_t t) -> int64_t { return r0 + wave + t * kBatchWaves; };
    // Rows are read through a buffer resource per row (range = the padded
    // row, so columns past it read as zeros), b and nu ahead of the row.  A
    // step past the wavefront's last row reads the item's first row again
    // (from L2): every pass of the row loop issues the same loads, so the
    // compiler can count exactly which of them a row still waits for.
    const uint32_t row_range = (uint32_t)row_bytes;
    auto load_row = [&](uint4 (&buf)[C], double &bi, double &ni, int64_t t) {
        const int64_t row = t < nmine ? row_of(t) : r0;
        bi = load_global(S.b + row);
        ni = load_global(S.nu + row);
        const __amdgpu_buffer_rsrc_t rr = row_resource(Ab + row * row_bytes, row_range);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[c] = load_row_vec(rr, (uint32_t)(col_of(c) * (int)sizeof(T)));
    };
    uint4 bufA[C], bufB[C];
    double bA, nA, bB, nB;
    load_row(bufA, bA, nA, 0);
    load_row(bufB, bB, nB, 1);

    Pending pd{S.ctl, a.j, S.tot, S.ynp, S.R, a.decide, a.dp};
    const State st = sweep_state(pd, lane, band == 0 && tid == 0);
    if (a.check_status && st.status != ST_RUNNING) return;
    const bool apply_v = st.vpend_valid || st.v_idx >= 0;
    const double s = a.decide ? st.s : 0.0;

    // stage x_j = x_{j-1} - s*y_{j-1} (one rounding) and v, zero past ldA
    batch_stage<DT>(S, apply_v, s, lds[0], lds[1], COLS);
    const Acc *xs = lds[0];
    const Acc *vs = lds[1];
    __syncthreads();

    Acc yacc[C][VEC];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) yacc[c][e] = (Acc)0;
    int64_t h = 0;
    double dmax = 0.0, binf = 0.0;
    // The translated b of the wavefront's rows is collected in a register,
    // lane i holding that of the wavefront's row 64 q + i, and written for
    // 64 rows at a time: a global store inside the row loop would leave
    // loads and stores outstanding together, and the compiler would then wait
    // for every outstanding load before each use of a row.
    const bool keep_b = apply_v && a.write_b;
    double bkeep = 0.0;
    auto write_b = [&](int64_t t_last) {
        const int64_t t0 = t_last & ~(int64_t)63;
        if (t0 + lane <= t_last) store_global(S.b + row_of(t0 + lane), bkeep);
        __builtin_amdgcn_s_waitcnt(0);  // the stores are done before rows are counted again
    };
    auto process = [&](uint4 (&buf)[C], double bi, double ni, int64_t t) {
        Acc dot = (Acc)0, tdot = (Acc)0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC], xv[VEC], vv[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                const uint4 ux = *reinterpret_cast<const uint4 *>(xs + col_of(c) + e);
                __builtin_memcpy(&xv[e], &ux, 16);
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) dot = fma(xv[e], av[e], dot);
            if (apply_v) {
#pragma unroll
                for (int e = 0; e < VEC; e += AV) {
                    const uint4 uv = *reinterpret_cast<const uint4 *>(vs + col_of(c) + e);
                    __builtin_memcpy(&vv[e], &uv, 16);
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e) tdot = fma(vv[e], av[e], tdot);
            }
        }
        dot = wave_total(dot);
        double bb = bi;
        if (apply_v) bb += (double)wave_total(tdot);
        if (keep_b && lane == (int)(t & 63)) bkeep = bb;
        const double r = (double)dot - bb;
        binf = max_nan(binf, fabs(bb));
        if (r > 0.0) {
            ++h;
            dmax = max_nan(dmax, r / sqrt(ni));
            const Acc w = (Acc)(r / ni);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                Acc av[VEC];
                unpack<DT>(buf[c], av);
#pragma unroll
                for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(w, av[e], yacc[c][e]);
            }
        } else if (r != r) {
            dmax = r;
        }
    };
    int64_t t = 0;
    for (; t + 2 <= nmine; t += 2) {
        process(bufA, bA, nA, t);   // t is even: never the 64th row of a group
        load_row(bufA, bA, nA, t + 2);
        process(bufB, bB, nB, t + 1);
        if (keep_b && (((t + 2) & 63) == 0 || t + 2 == nmine)) write_b(t + 1);
        load_row(bufB, bB, nB, t + 3);
    }
    if (t < nmine) {
        process(bufA, bA, nA, t);
        if (keep_b) write_b(t);
    }

    batch_item_end<DT, C>(a, S, k, band, yacc, h, dmax, binf, lds, hsh, dsh, bsh, col_of, true);
}

// One work item of a system with short rows (ldA <= 16 VEC C elements): a row
// takes 16 lanes, so a wavefront sweeps RPW = 4 consecutive rows at once.
// Their dot products are reduced over 16 lanes (DPP only), and their
// residuals, weights and counts are formed by their own lanes; the row
// groups' partials of y are added once per item.  At step t wavefront w takes
// rows r0 + 4 (4 t + w) + g, g = lane / 16.  The item's rows are read through
// one buffer resource, padding columns and rows past the item as zeros.  (A
// form with eight rows of 8 lanes measured no faster, and its registers cost
// the whole persistent kernel an occupancy level.)
template <int DT, int C>
__device__ void batch_item_short(const BatchArgs &a, const BatchSys &Sref, int64_t k,
                                 typename Store<DT>::Acc (*lds)[kBatchCmax * 64 * Store<DT>::VEC],
                                 int64_t *hsh, double *dsh, double *bsh) {
    using St = Store<DT>;
    using Acc = typename St::Acc;
    using T = typename St::T;
    constexpr int VEC = St::VEC;
    constexpr int RPW = 4, LPR = 16;               // rows per wavefront, lanes per row
    constexpr int CW = LPR * VEC;                  // columns per chunk
    constexpr int AV = 16 / (int)sizeof(Acc);
    constexpr int COLS = C * CW;
    constexpr int64_t PER = kBatchWaves * RPW;     // rows per step of the workgroup
    constexpr uint32_t kOutside = 0x80000000u;     // a byte offset past every item
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane / LPR, gl = lane % LPR;
    const BatchSys S = Sref;
    const int64_t band = k - S.item0;
    const int64_t r0 = band * S.rows_per_item;
    const int64_t r1 = min(S.m, r0 + S.rows_per_item);
    const int64_t ldA = S.ldA;
    auto col_of = [&](int c) -> int { return c * CW + gl * VEC; };
    const int64_t row_bytes = ldA * (int64_t)sizeof(T);
    const int64_t nrows = r1 - r0;
    const int64_t nmine = nrows > wave * RPW ? (nrows - wave * RPW + PER - 1) / PER : 0;
    auto row_of = [&](int64_t t) -> int64_t { return r0 + (t * kBatchWaves + wave) * RPW + g; };
    const __amdgpu_buffer_rsrc_t rr =
        row_resource(reinterpret_cast<const char *>(S.A) + r0 * row_bytes, (uint32_t)(nrows * row_bytes));
    // as in batch_item, a step past the wavefront's last one issues the same
    // loads (here all outside the item: zeros, no memory traffic)
    auto load_rows = [&](uint4 (&buf)[C], double &bi, double &ni, int64_t t) {
        const int64_t row = row_of(t);
        const bool ok = t < nmine && row < r1;
        const int64_t rc = ok ? row : r0;
        bi = load_global(S.b + rc);
        ni = load_global(S.nu + rc);
        const uint32_t base = (uint32_t)((rc - r0) * row_bytes);
#pragma unroll
        for (int c = 0; c < C; ++c)
            buf[c] = load_row_vec(rr, ok && col_of(c) < ldA ? base + (uint32_t)(col_of(c) * (int)sizeof(T)) : kOutside);
    };
    uint4 bufA[C], bufB[C];
    double bA, nA, bB, nB;
    load_rows(bufA, bA, nA, 0);
    load_rows(bufB, bB, nB, 1);

    Pending pd{S.ctl, a.j, S.tot, S.ynp, S.R, a.decide, a.dp};
    const State st = sweep_state(pd, lane, band == 0 && tid == 0);
    if (a.check_status && st.status != ST_RUNNING) return;
    const bool apply_v = st.vpend_valid || st.v_idx >= 0;
    batch_stage<DT>(S, apply_v, a.decide ? st.s : 0.0, lds[0], lds[1], COLS);
    const Acc *xs = lds[0];
    const Acc *vs = lds[1];
    __syncthreads();

    Acc yacc[C][VEC];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) yacc[c][e] = (Acc)0;
    int64_t h = 0;
    double dmax = 0.0, binf = 0.0;
    // the translated b of the wavefront's rows, collected as in batch_item:
    // lane i holds that of the wavefront's row 64 q + i (its rows numbered
    // 4 t + g), written for 64 rows at a time
    const bool keep_b = apply_v && a.write_b;
    double bkeep = 0.0;
    auto write_b = [&](int64_t t_last) {
        const int64_t q_last = t_last * RPW + RPW - 1;
        const int64_t q = (q_last & ~(int64_t)63) + lane;
        if (q <= q_last) {
            const int64_t row = r0 + ((q / RPW) * kBatchWaves + wave) * RPW + q % RPW;
            if (row < r1) store_global(S.b + row, bkeep);
        }
        __builtin_amdgcn_s_waitcnt(0);  // the stores are done before rows are counted again
    };
    auto process = [&](uint4 (&buf)[C], double bi, double ni, int64_t t) {
        const bool ok = row_of(t) < r1;
        Acc dot = (Acc)0, tdot = (Acc)0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC], xv[VEC], vv[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                const uint4 ux = *reinterpret_cast<const uint4 *>(xs + col_of(c) + e);
                __builtin_memcpy(&xv[e], &ux, 16);
            }
#pragma unroll
            for (int e = 0; e < VEC; ++e) dot = fma(xv[e], av[e], dot);
            if (apply_v) {
#pragma unroll
                for (int e = 0; e < VEC; e += AV) {
                    const uint4 uv = *reinterpret_cast<const uint4 *>(vs + col_of(c) + e);
                    __builtin_memcpy(&vv[e], &uv, 16);
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e) tdot = fma(vv[e], av[e], tdot);
            }
        }
        dot = row_total(dot);
        double bb = bi;
        if (apply_v) bb += (double)row_total(tdot);
        if (keep_b) {
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const double bq = lane_value(bb, q * LPR);
                if (lane == (int)((t * RPW + q) & 63)) bkeep = bq;
            }
        }
        const double r = ok ? (double)dot - bb : -1.0;
        if (ok) binf = max_nan(binf, fabs(bb));
        const bool pos = r > 0.0;
        h += (pos && gl == 0) ? 1 : 0;
        const double d = r / sqrt(ni);
        dmax = pos ? max_nan(dmax, d) : (r != r ? r : dmax);
        const Acc w = pos ? (Acc)(r / ni) : (Acc)0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(w, av[e], yacc[c][e]);
        }
    };
    int64_t t = 0;
    for (; t + 2 <= nmine; t += 2) {
        process(bufA, bA, nA, t);   // t is even: its rows never end a group of 64
        load_rows(bufA, bA, nA, t + 2);
        process(bufB, bB, nB, t + 1);
        if (keep_b && ((((t + 2) * RPW) & 63) == 0 || t + 2 == nmine)) write_b(t + 1);
        load_rows(bufB, bB, nB, t + 3);
    }
    if (t < nmine) {
        process(bufA, bA, nA, t);
        if (keep_b) write_b(t);
    }
    // the row groups' partials (lanes gl, gl + 16, gl + 32, gl + 48 hold the
    // same columns), added pairwise: (g0 + g1) + (g2 + g3), the same bits in
    // every group
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            Acc v = yacc[c][e];
#pragma unroll
            for (int o = LPR; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
            if constexpr (LPR <= 16) v = xor_add<16>(v);
            if constexpr (LPR <= 32) v = xor_add<32>(v);
            yacc[c][e] = v;
        }
    h = (decltype(h))wave_total((double)h);   // an integer below 2^53: exact
    dmax = wave_max_nan(dmax);
    binf = wave_max_nan(binf);
    batch_item_end<DT, C>(a, S, k, band, yacc, h, dmax, binf, lds, hsh, dsh, bsh, col_of, g == 0);
}

// Persistent sweep over every item of the batch.  Each workgroup takes queue
// positions until they are exhausted (every workgroup reaches the end); a
// position names an item through item_order, largest items first, so that the
// last items to start are small ones and the workgroups finish together.
template <int DT>
__global__ __launch_bounds__(256) void sweep_batch(const BatchArgs a) {
    using Acc = typename Store<DT>::Acc;
    constexpr int VEC = Store<DT>::VEC;
    __shared__ __attribute__((aligned(16))) Acc lds[2][kBatchCmax * 64 * VEC];
    __shared__ int64_t hsh[kBatchWaves];
    __shared__ double dsh[kBatchWaves], bsh[kBatchWaves];
    __shared__ int s_pos;
    if (threadIdx.x == 0) s_pos = atomicAdd(a.queue, 1);
    __syncthreads();
    int pos = s_pos;
    while (pos < a.nitems) {
        // the next position is requested while this item runs; it reaches
        // the other threads through LDS after the item's last barrier
        int next = 0;
        __syncthreads();  // every thread has read s_pos
        if (threadIdx.x == 0) next = atomicAdd(a.queue, 1);
        const int k = load_global(a.item_order + pos);
        const BatchSys &S = a.sys[a.item_sys[k]];
        if (S.RPW == 4) {
            switch (S.C) {
                case 1: batch_item_short<DT, 1>(a, S, k, lds, hsh, dsh, bsh); break;
                case 2: batch_item_short<DT, 2>(a, S, k, lds, hsh, dsh, bsh); break;
                default: batch_item_short<DT, 4>(a, S, k, lds, hsh, dsh, bsh); break;
            }
        } else {
            switch (S.C) {
                case 1: batch_item<DT, 1>(a, S, k, lds, hsh, dsh, bsh); break;
                case 2: batch_item<DT, 2>(a, S, k, lds, hsh, dsh, bsh); break;
                case 4: batch_item<DT, 4>(a, S, k, lds, hsh, dsh, bsh); break;
                default: batch_item<DT, 8>(a, S, k, lds, hsh, dsh, bsh); break;
            }
        }
        if (threadIdx.x == 0) s_pos = next;
        __syncthreads();  // the item's use of LDS is over, and s_pos is set
        pos = s_pos;
    }
}

// Column sums of a system's item partials (item order, FP64), the previous
// step made permanent in x, and the next sweep's working vectors.  One
// workgroup per 64-column block; block 0 of a system also forms its totals.
// Workgroup 0 empties the item queue for the next sweep.  The work of a block
// is small, so its time is the chain of dependent loads: the system's fields
// come in one request, and then the state, the partials and every vector of
// the block's columns that does not depend on the state are requested
// together; the state only decides whether they are used.  Only the drift
// rows, whose index is in the state, wait for it.
template <typename Acc>
__global__ __launch_bounds__(256) void reduce_batch(const BatchArgs a, const BatchCol *cols) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0;
    const BatchCol cb = cols[blockIdx.x];
    const BatchSys S = a.sys[cb.sys];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t col = (int64_t)cb.blk * 64 + lane;
    const bool in = col < S.n;
    const State P = S.ctl->st[slot_of(a.j - 1)];
    const int64_t sched_len = S.ctl->sched_len;
    const Acc *part = reinterpret_cast<const Acc *>(a.part) + S.part0;
    double acc = 0.0;
    if (in)
        for (int64_t q = wave; q < S.nitems; q += kBatchWaves) acc += (double)part[q * S.ldA + col];
    double xo = 0.0, yprev = 0.0, ws = 0.0, vp = 0.0;
    if (wave == 0 && in) {
        xo = S.x[col];
        yprev = S.y[col];
        ws = S.wsum[col];
        vp = S.vpend[col];
    }
    int64_t h = 0;
    double dm = 0.0, bm = 0.0;
    if (cb.blk == 0)
        for (int64_t q = tid; q < S.nitems; q += 256) {
            h += a.h_part[S.item0 + q];
            dm = max_nan(dm, a.dmax_part[S.item0 + q]);
            bm = max_nan(bm, a.binf_part[S.item0 + q]);
        }
    if (P.status != ST_RUNNING) return;
    __shared__ double sh[kBatchWaves][64];
    sh[wave][lane] = acc;
    __shared__ int64_t hw[kBatchWaves];
    __shared__ double dw[kBatchWaves], bw[kBatchWaves];
    if (cb.blk == 0) {
        // DPP moves, no permute round trips: h an FP64 sum of integers below
        // 2^53 (exact), the maxima in any order
        h = (int64_t)wave_total((double)h);
        dm = wave_max_nan(dm);
        bm = wave_max_nan(bm);
        if (lane == 0) {
            hw[wave] = h;
            dw[wave] = dm;
            bw[wave] = bm;
        }
    }
    __syncthreads();
    if (wave != 0) return;
    double yv = 0.0;
#pragma unroll
    for (int g = 0; g < kBatchWaves; ++g) yv += sh[g][lane];
    double sq = 0.0;
    if (in) {
        if (a.apply_step && P.s != 0.0) {
            xo = step_point(xo, P.s, yprev);
            S.x[col] = xo;
        }
        // the translation the sweep applied joins the FP64 sum of translations
        const bool ap = P.vpend_valid != 0, ar = S.V && P.v_idx >= 0;
        if (ap || ar) S.wsum[col] = ws + ((ap ? vp : 0.0) + (ar ? S.V[P.v_idx * S.ldA + col] : 0.0));
        const bool due = S.V && P.sched_pos < sched_len;
        Acc *w = reinterpret_cast<Acc *>(S.work);
        w[col] = (Acc)xo;
        w[S.ldA + col] = due ? (Acc)S.V[P.sched_pos * S.ldA + col] : (Acc)0;
        w[2 * S.ldA + col] = (Acc)yv;
        S.y[col] = yv;
        sq = yv * yv;
    }
    sq = wave_sum(sq);
    if (lane == 0) S.ynp[cb.blk] = sq;
    if (cb.blk == 0 && lane == 0) {
        Totals t{};
        for (int g = 0; g < kBatchWaves; ++g) {
            t.h += hw[g];
            t.dmax = max_nan(t.dmax, dw[g]);
            t.binf = max_nan(t.binf, bw[g]);
        }
        *S.tot = t;
    }
}

// Start of a call, one thread per system: a stop that came from a previous
// call's tolerance, step limit or missing direction is re-examined, and the
// step limit of this call is set (-1: none).
__global__ void begin_batch(const BatchArgs a, int64_t max_steps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nsys) return;
    Ctrl *c = a.sys[i].ctl;
    State &s = c->st[slot_of(a.j - 1)];
    if (s.status == ST_CONVERGED || s.status == ST_LIMIT || s.status == ST_NO_DIRECTION) s.status = ST_RUNNING;
    c->step_limit = max_steps < 0 ? INT64_MAX : s.steps + max_steps;
}

// Working vectors of a call's first sweep from each system's committed state
// (one workgroup per system); workgroup 0 empties the item queue.
template <typename Acc>
__global__ __launch_bounds__(256) void prime_batch(const BatchArgs a) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *a.queue = 0;
    const BatchSys &S = a.sys[blockIdx.x];
    const State &p = S.ctl->st[slot_of(a.j - 1)];
    const bool use_p = p.vpend_valid != 0;
    const double *vrow = (S.V && p.v_idx >= 0) ? S.V + p.v_idx * S.ldA : nullptr;
    Acc *w = reinterpret_cast<Acc *>(S.work);
    for (int64_t col = threadIdx.x; col < S.n; col += blockDim.x) {
        const double v = (use_p ? S.vpend[col] : 0.0) + (vrow ? vrow[col] : 0.0);
        w[col] = (Acc)S.x[col];
        w[S.ldA + col] = (Acc)v;
    }
}

// End of a call: settle each system's last check (one workgroup per system).
__global__ __launch_bounds__(256) void settle_batch(const BatchArgs a) {
    const BatchSys &S = a.sys[blockIdx.x];
    const State p = S.ctl->st[slot_of(a.j - 1)];
    if (p.status != ST_RUNNING) {
        if (threadIdx.x == 0) S.ctl->st[slot_of(a.j)] = p;
        return;
    }
    __shared__ State sst;
    if (threadIdx.x < 64) {
        const double yn = ynorm_of(S.ynp, S.R, threadIdx.x);
        const State cur = decide(p, *S.tot, yn, a.dp, S.ctl->step_limit, S.ctl->sched_len);
        if (threadIdx.x == 0) {
            sst = cur;
            S.ctl->st[slot_of(a.j)] = cur;
        }
    }
    __syncthreads();
    const double s = sst.s;
    if (s == 0.0) return;
    for (int64_t col = threadIdx.x; col < S.n; col += blockDim.x) S.x[col] = step_point(S.x[col], s, S.y[col]);
}

// Status and certificate flag of every system in slot sl (one thread each).
__global__ void gather_states(const BatchArgs a, int sl, int2 *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.nsys) return;
    const State &s = a.sys[i].ctl->st[sl];
    out[i] = make_int2(s.status, s.certified);
}

// Number of systems whose state in slot sl is ST_RUNNING (one workgroup).
__global__ __launch_bounds__(256) void count_running(const BatchArgs a, int sl, int *out) {
    int cnt = 0;
    for (int i = threadIdx.x; i < a.nsys; i += 256) cnt += a.sys[i].ctl->st[sl].status == ST_RUNNING;
    cnt = wave_sum(cnt);
    __shared__ int w[4];
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) *out = w[0] + w[1] + w[2] + w[3];
}

}  // namespace modap
