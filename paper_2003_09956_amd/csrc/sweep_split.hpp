// Split-row two-phase sweep for rows too long to keep on chip.
//
// The same sweep as sweep_wide.hpp (section 3's Map of positive slices and
// Reduce(+), the eq. 10 measures and the translation update), for rows whose
// length exceeds what one workgroup can hold in registers.  The row is cut
// into column tiles of TW = BLOCK*VEC*C columns:
//
//   phase 1 (split_dot):    for each (row band, column tile): partial dots
//                           <a_i[tile], x[tile]> and <a_i[tile], v[tile]>
//   split_finish:           per row, the partial dots summed over the tiles in
//                           a fixed order (FP64): b'_i, r_i, w_i = r_i/||a_i||^2
//                           when r_i > 0 (else 0), and h, dmax, binf
//   phase 2 (split_axpy):   for each (row band, column tile): the violated rows
//                           of the band are listed first, then only those rows
//                           are read again, y[tile] += w_i a_i[tile]
//
// Phase 1 reads all of A and phase 2 only the violated rows, so the sweep
// moves (1 + h/m) times the bytes of A.  The partial y of each row band is
// summed over the bands by the reduction kernel, as for the one-pass sweep.
#pragma once

#include "modap_device.hpp"
#include "sweep_wide.hpp"

namespace modap {

struct SplitArgs {
    const void *A;
    int64_t ldA, m, n;
    const double *b_in;
    double *b_out;
    const double *nu;
    const void *work;        // [3 x ldA] Acc working vectors x, v, y
    Pending pd;              // settled by split_dot; the later kernels read slot (j-1)&1
    int32_t check_status;
    int32_t ntiles;          // column tiles
    int64_t rows_per_band;
    void *pdot;              // [ntiles x m] Acc partial dots (x), then (v) at + ntiles*m
    double *w;               // [m] step weights r_i/||a_i||^2 of violated rows, else 0
    double *r_out;           // [m] or null
    void *part;              // [bands x ldPart] Acc partial y
    int64_t ldPart;
    int64_t *h_part;         // [finish blocks]
    double *dmax_part;
    double *binf_part;
};

template <int DT, int BLOCK, int C, bool HAS_V>
__global__ __launch_bounds__(BLOCK) void split_dot(const SplitArgs a) {
    using S = Store<DT>;
    using Acc = typename S::Acc;
    using T = typename S::T;
    constexpr int VEC = S::VEC;
    constexpr int NW = BLOCK / 64;
    constexpr int CW = BLOCK * VEC;
    constexpr int TW = CW * C;
    constexpr int AV = 16 / (int)sizeof(Acc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const State st = sweep_state(a.pd, lane, blockIdx.x == 0 && blockIdx.y == 0 && tid == 0);
    if (a.check_status && st.status != ST_RUNNING) return;
    const double s = a.pd.decide ? st.s : 0.0;   // step decided on the previous check

    const int64_t tile0 = (int64_t)blockIdx.y * TW;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_band;
    const int64_t r1 = min(a.m, r0 + a.rows_per_band);
    if (r1 <= r0) return;
    auto col_of = [&](int c) -> int64_t { return tile0 + (int64_t)c * CW + tid * VEC; };

    Acc xr[C][VEC], vr[C][VEC];
    const Acc *wx = reinterpret_cast<const Acc *>(a.work);
    const Acc *wv = wx + a.ldA;
    const Acc *wy = wx + 2 * a.ldA;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t col = min(col_of(c), a.ldA - VEC);
        const bool in = col_of(c) < a.ldA;
#pragma unroll
        for (int e = 0; e < VEC; e += AV) {
            const uint4 ux = *reinterpret_cast<const uint4 *>(wx + col + e);
            __builtin_memcpy(&xr[c][e], &ux, 16);
            if (HAS_V) {
                const uint4 uv = *reinterpret_cast<const uint4 *>(wv + col + e);
                __builtin_memcpy(&vr[c][e], &uv, 16);
            }
            if (s != 0.0) {
                Acc yv[AV];
                const uint4 uy = *reinterpret_cast<const uint4 *>(wy + col + e);
                __builtin_memcpy(yv, &uy, 16);
#pragma unroll
                for (int k = 0; k < AV; ++k) xr[c][e + k] = (Acc)step_point((double)xr[c][e + k], s, (double)yv[k]);
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (!in || !HAS_V) vr[c][e] = (Acc)0;
            if (!in) xr[c][e] = (Acc)0;
        }
    }
    const char *Ab = reinterpret_cast<const char *>(a.A);
    const int64_t row_bytes = a.ldA * (int64_t)sizeof(T);
    // Rows through a buffer resource each (columns past the padded row read
    // as zeros).  Loads past the band re-read its last row, so every pass of
    // the row loop issues the same loads and the compiler can count which of
    // them a row still waits for.
    const uint32_t row_range = (uint32_t)row_bytes;
    auto load_row = [&](uint4 (&buf)[C], int64_t row) {
        const __amdgpu_buffer_rsrc_t rr = row_resource(Ab + min(row, r1 - 1) * row_bytes, row_range);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[c] = load_row_vec(rr, (uint32_t)(col_of(c) * (int64_t)sizeof(T)));
    };
    Acc *pd = reinterpret_cast<Acc *>(a.pdot);
    Acc *pt = pd + (int64_t)a.ntiles * a.m;
    __shared__ Acc red[2][NW][2];
    uint4 bufA[C], bufB[C];
    Acc kd = (Acc)0, kt = (Acc)0;
    auto process = [&](const uint4 (&buf)[C], int64_t row, int64_t t) {
        Acc d = (Acc)0, td = (Acc)0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                d = fma(xr[c][e], av[e], d);
                if (HAS_V) td = fma(vr[c][e], av[e], td);
            }
        }
        d = wave_total(d);
        if (HAS_V) td = wave_total(td);
        const int pp = (int)(t & 1);
        if (lane == 0) {
            red[pp][wave][0] = d;
            red[pp][wave][1] = td;
        }
        __syncthreads();
        // thread t mod BLOCK keeps the tile dots of the band's row t; they
        // are written BLOCK rows at a time (no global store in the row loop,
        // so that only loads are outstanding there)
        if (tid == (int)(t & (BLOCK - 1))) {
            Acc s = (Acc)0, ts = (Acc)0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                s += red[pp][w][0];
                ts += red[pp][w][1];
            }
            kd = s;
            kt = ts;
        }
    };
    auto write_out = [&](int64_t t_last) {
        const int64_t t0 = t_last & ~(int64_t)(BLOCK - 1);
        if (t0 + tid <= t_last) {
            pd[(int64_t)blockIdx.y * a.m + r0 + t0 + tid] = kd;
            pt[(int64_t)blockIdx.y * a.m + r0 + t0 + tid] = kt;
        }
        __builtin_amdgcn_s_waitcnt(0);  // the stores are done before rows are counted again
    };
    const int64_t nrows = r1 - r0;
    load_row(bufA, r0);
    load_row(bufB, r0 + 1);
    int64_t t = 0;
    for (; t + 2 <= nrows; t += 2) {
        process(bufA, r0 + t, t);
        if (((t + 1) & (BLOCK - 1)) == 0) write_out(t);
        load_row(bufA, r0 + t + 2);
        process(bufB, r0 + t + 1, t + 1);
        if (((t + 2) & (BLOCK - 1)) == 0 || t + 2 == nrows) write_out(t + 1);
        load_row(bufB, r0 + t + 3);
    }
    if (t < nrows) {
        process(bufA, r0 + t, t);
        write_out(t);
    }
}

// Per row: sum the tile dots in order, apply the translation, form r_i and
// the step weight; per workgroup: h, dmax, binf.
template <typename Acc>
__global__ __launch_bounds__(256) void split_finish(const SplitArgs a, int has_v) {
    const State &st = a.pd.ctl->st[slot_of(a.pd.j - 1)];
    if (a.check_status && st.status != ST_RUNNING) return;
    const bool apply_v = has_v && (st.vpend_valid || st.v_idx >= 0);
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const Acc *pd = reinterpret_cast<const Acc *>(a.pdot);
    const Acc *pt = pd + (int64_t)a.ntiles * a.m;
    int64_t h = 0;
    double dmax = 0.0, binf = 0.0;
    if (row < a.m) {
        double d = 0.0, td = 0.0;
        for (int t = 0; t < a.ntiles; ++t) {
            d += (double)pd[(int64_t)t * a.m + row];
            if (apply_v) td += (double)pt[(int64_t)t * a.m + row];
        }
        double bb = a.b_in[row];
        if (apply_v) {
            bb += td;
            if (a.b_out) a.b_out[row] = bb;
        }
        const double r = d - bb;
        if (a.r_out) a.r_out[row] = r;
        binf = fabs(bb);
        double w = 0.0;
        if (r > 0.0) {
            h = 1;
            dmax = r / sqrt(a.nu[row]);
            w = r / a.nu[row];
        } else if (r != r) {
            dmax = r;
        }
        a.w[row] = w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        h += __shfl_xor(h, o, 64);
        dmax = max_nan(dmax, __shfl_xor(dmax, o, 64));
        binf = max_nan(binf, __shfl_xor(binf, o, 64));
    }
    __shared__ int64_t hs[4];
    __shared__ double ds[4], bs[4];
    if ((threadIdx.x & 63) == 0) {
        hs[threadIdx.x >> 6] = h;
        ds[threadIdx.x >> 6] = dmax;
        bs[threadIdx.x >> 6] = binf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t hh = 0;
        double dd = 0.0, bm = 0.0;
        for (int k = 0; k < 4; ++k) {
            hh += hs[k];
            dd = max_nan(dd, ds[k]);
            bm = max_nan(bm, bs[k]);
        }
        a.h_part[blockIdx.x] = hh;
        a.dmax_part[blockIdx.x] = dd;
        a.binf_part[blockIdx.x] = bm;
    }
}

// Phase 2: y[tile] partial of one row band over its violated rows only.
template <int DT, int BLOCK, int C>
__global__ __launch_bounds__(BLOCK) void split_axpy(const SplitArgs a) {
    using S = Store<DT>;
    using Acc = typename S::Acc;
    using T = typename S::T;
    constexpr int VEC = S::VEC;
    constexpr int CW = BLOCK * VEC;
    constexpr int TW = CW * C;
    constexpr int AV = 16 / (int)sizeof(Acc);
    constexpr int LIST = 4096;   // rows per band at most (checked by the host)
    const State &st = a.pd.ctl->st[slot_of(a.pd.j - 1)];
    if (a.check_status && st.status != ST_RUNNING) return;
    const int tid = threadIdx.x;
    const int64_t tile0 = (int64_t)blockIdx.y * TW;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_band;
    const int64_t r1 = min(a.m, r0 + a.rows_per_band);
    auto col_of = [&](int c) -> int64_t { return tile0 + (int64_t)c * CW + tid * VEC; };

    // list the violated rows of the band, in row order: BLOCK rows at a time,
    // each wavefront's flags compacted with a ballot, wavefronts in order
    constexpr int NWV = BLOCK / 64;
    __shared__ int list[LIST];
    __shared__ int wcount[NWV];
    const int lane = tid & 63, wave = tid >> 6;
    int nv = 0;
    for (int64_t base = r0; base < r1; base += BLOCK) {
        const int64_t r = base + tid;
        const bool f = r < r1 && a.w[r] != 0.0;
        const unsigned long long bal = __ballot(f);
        const int before = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int off = nv;
        for (int w = 0; w < wave; ++w) off += wcount[w];
        if (f) list[off + before] = (int)(r - r0);
        int total = 0;
        for (int w = 0; w < NWV; ++w) total += wcount[w];
        __syncthreads();
        nv += total;
    }

    Acc yacc[C][VEC];
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int e = 0; e < VEC; ++e) yacc[c][e] = (Acc)0;
    const char *Ab = reinterpret_cast<const char *>(a.A);
    const int64_t row_bytes = a.ldA * (int64_t)sizeof(T);
    // as in split_dot: a buffer resource per row, and loads past the list
    // re-read its last row so that every pass of the loop issues the same loads
    const uint32_t row_range = (uint32_t)row_bytes;
    auto load_row = [&](uint4 (&buf)[C], double &wk, int k) {
        const int64_t row = r0 + list[min(k, nv - 1)];
        wk = a.w[row];   // ahead of the row (loads return in order)
        const __amdgpu_buffer_rsrc_t rr = row_resource(Ab + row * row_bytes, row_range);
#pragma unroll
        for (int c = 0; c < C; ++c) buf[c] = load_row_vec(rr, (uint32_t)(col_of(c) * (int64_t)sizeof(T)));
    };
    auto accumulate = [&](const uint4 (&buf)[C], double w) {
        const Acc wk = (Acc)w;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(wk, av[e], yacc[c][e]);
        }
    };
    uint4 bufA[C], bufB[C];
    double wA, wB;
    if (nv > 0) {
        load_row(bufA, wA, 0);
        load_row(bufB, wB, 1);
        int k = 0;
        for (; k + 2 <= nv; k += 2) {
            // the scheduling barriers keep each refill right after the use of
            // its buffer, so that one row is always in flight
            accumulate(bufA, wA);
            load_row(bufA, wA, k + 2);
            __builtin_amdgcn_sched_barrier(0);
            accumulate(bufB, wB);
            load_row(bufB, wB, k + 3);
            __builtin_amdgcn_sched_barrier(0);
        }
        if (k < nv) accumulate(bufA, wA);
    }
    Acc *part = reinterpret_cast<Acc *>(a.part) + (int64_t)blockIdx.x * a.ldPart;
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int e = 0; e < VEC; e += AV) {
            uint4 w;
            __builtin_memcpy(&w, &yacc[c][e], 16);
            *reinterpret_cast<uint4 *>(part + col_of(c) + e) = w;
        }
    }
}

}  // namespace modap
