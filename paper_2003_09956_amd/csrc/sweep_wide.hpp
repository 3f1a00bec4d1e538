// Fused one-pass sweep over A for rows that fit on chip.
//
// One sweep of the pseudo-projection method (section 3: Map of the positive
// slices, eq. 7, then Reduce(+)) together with the eps-feasibility measures of
// eq. 10 and the data update by translation, in a single read of A:
//
//   b'_i = b_i + <a_i, v>                     (translation by +v, when one applies)
//   r_i  = <a_i, x> - b'_i
//   y   += (r_i/||a_i||^2) a_i   if r_i > 0   (while the row is still in registers)
//   h   += [r_i > 0],  dmax = max r_i/||a_i||,  binf = max |b'_i|
//
// x, v and y come from the working vectors written once per iteration by the
// reduction kernel, in the accumulation type; the step decided on the previous
// check (x_j = x_{j-1} - s*y_{j-1}) is applied while they are staged.
//
// Thread shape: LPR lanes (a multiple of the 64-wide wavefront, or 16 or 32
// for short rows, several rows to a wavefront) share a row;
// a workgroup of BLOCK lanes holds BLOCK/LPR row groups, and each row group
// takes RS consecutive rows per step, with the rows of the next PD-1 steps in
// flight (PD at the start).  The row is cut into C chunks of LPR*VEC
// columns; lane l owns VEC consecutive columns of every chunk, so each
// wavefront load of a chunk is 64 contiguous 16-byte vectors (1 KiB).  The
// chunks are visited in an order rotated by the workgroup index, so that the
// workgroups do not all read the same part of the working vectors at once.
// The lane's slices of x, v and of the partial y stay in registers for the
// whole sweep; the next PD-1 steps' rows are loaded (non-temporally: A is read
// once per sweep) while the current ones are reduced.  Dot products are
// reduced across the wavefront by DPP moves and lane reads (the same value in
// every lane) and across the wavefronts of a row group through LDS, in a fixed
// order, so results do not depend on timing.
// Each workgroup owns a fixed set of rows (a contiguous band, or row blocks
// taken in turn with the other workgroups) and writes one partial y; the
// reduction kernel sums the partials in a fixed order.
#pragma once

#include "modap_device.hpp"

namespace modap {

// A buffer resource for one row: wave-uniform base (scalar registers), range
// = the padded row in bytes, raw addressing (word 3 is the gfx9 value for
// untyped dword access).  A load addressed past the range returns zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_resource(const char *row, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char *>(row), (short)0, (int)bytes, 0x00020000);
}

// One 16-byte vector of a row through its resource, at a 32-bit per-lane byte
// offset.  Rows of A are read exactly once per sweep: the load is non-temporal
// (aux bit 1) so that the working vectors, b and the partials keep the caches;
// measured, a cached load makes the sweep 11-19% slower.
__device__ __forceinline__ uint4 load_row_vec(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    const u32x4 t = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 2);
    return make_uint4(t.x, t.y, t.z, t.w);
}

// Sum over each group of LPR = 16 or 32 consecutive lanes (every lane of a
// group holds the same bits): the DPP stages of a 16-lane row, then for 32
// lanes one lane swap with the partner row.
template <int LPR, typename T>
__device__ __forceinline__ T group_total(T v) {
    static_assert(LPR == 16 || LPR == 32, "groups of 16 or 32 lanes");
    v = row_total(v);
    if constexpr (LPR == 32) v = xor_add<16>(v);
    return v;
}

template <int DT>
__device__ __forceinline__ void unpack(const uint4 &u, typename Store<DT>::Acc (&o)[Store<DT>::VEC]);

template <>
__device__ __forceinline__ void unpack<0>(const uint4 &u, double (&o)[2]) {
    o[0] = __hiloint2double((int)u.y, (int)u.x);
    o[1] = __hiloint2double((int)u.w, (int)u.z);
}
template <>
__device__ __forceinline__ void unpack<1>(const uint4 &u, float (&o)[4]) {
    o[0] = __uint_as_float(u.x);
    o[1] = __uint_as_float(u.y);
    o[2] = __uint_as_float(u.z);
    o[3] = __uint_as_float(u.w);
}
// bfloat16 -> float is exact: the 16 stored bits are the upper half of the float.
template <>
__device__ __forceinline__ void unpack<2>(const uint4 &u, float (&o)[8]) {
    o[0] = __uint_as_float(u.x << 16);
    o[1] = __uint_as_float(u.x & 0xffff0000u);
    o[2] = __uint_as_float(u.y << 16);
    o[3] = __uint_as_float(u.y & 0xffff0000u);
    o[4] = __uint_as_float(u.z << 16);
    o[5] = __uint_as_float(u.z & 0xffff0000u);
    o[6] = __uint_as_float(u.w << 16);
    o[7] = __uint_as_float(u.w & 0xffff0000u);
}

template <int DT, int BLOCK, int LPR, int C, int RS, int PD, bool HAS_V>
__global__ __launch_bounds__(BLOCK) void sweep_wide(const SweepArgs a) {
    using S = Store<DT>;
    using Acc = typename S::Acc;
    using T = typename S::T;
    constexpr int VEC = S::VEC;
    constexpr int NG = BLOCK / LPR;   // row groups per workgroup
    constexpr int WPG = LPR / 64;     // wavefronts per row group
    constexpr int NW = BLOCK / 64;
    constexpr int CW = LPR * VEC;     // columns per chunk
    constexpr int AV = 16 / (int)sizeof(Acc);  // working-vector elements per 16-byte load
    // SUB: rows of 16 or 32 lanes, 64/LPR of them to a wavefront
    constexpr bool SUB = LPR < 64;
    constexpr int GPW = SUB ? 64 / LPR : 1;   // row groups per wavefront
    static_assert((LPR % 64 == 0 || LPR == 16 || LPR == 32) && BLOCK % LPR == 0 && BLOCK % 64 == 0,
                  "row groups are whole wavefronts, or 16 or 32 lanes");
    static_assert(VEC % AV == 0, "a lane's columns are whole 16-byte vectors of the working vectors");
    static_assert(PD >= 2, "at least one step is in flight while another is reduced");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    // the row group is the same for every lane of a wavefront when LPR is a
    // multiple of 64: say so, so that row addresses stay in scalar registers
    const int grp = SUB ? tid / LPR : __builtin_amdgcn_readfirstlane(tid / LPR);
    const int gl = tid % LPR;
    const int rot = (int)(blockIdx.x % C);

    // first column of register chunk c (chunks visited in rotated order)
    auto col_of = [&](int c) -> int64_t {
        const int cc = c + rot < C ? c + rot : c + rot - C;
        return (int64_t)cc * CW + gl * VEC;
    };

    // A step takes NG*RS consecutive rows; the workgroup's steps are either
    // consecutive (a band of rows) or step_stride rows apart (the workgroups
    // take consecutive row blocks in turn, so that at any time they all read
    // one contiguous region of A).
    const int64_t r0 = (int64_t)blockIdx.x * a.block_stride;
    const int64_t r1 = min(a.m, r0 + a.rows_per_block);
    const int64_t nsteps = r1 > r0 ? (r1 - r0 + a.step_stride - 1) / a.step_stride : 0;
    const char *Ab = reinterpret_cast<const char *>(a.A);
    const int64_t row_bytes = a.ldA * (int64_t)sizeof(T);

    auto row_of = [&](int64_t t, int q) -> int64_t { return r0 + t * a.step_stride + grp * RS + q; };
    // Loads are issued unconditionally so that no branch separates them: a row
    // index past the band is clamped to the band's last row, and the results
    // of rows past the band are never used.  A step past the last one (the
    // ring's look-ahead at the end of the band) reads row 0, which every
    // workgroup shares from L2, instead of a row of its own: every pass of the
    // row loop then issues the same loads, which lets the compiler count
    // exactly which of them a row still waits for.
    //
    // Each row is read through a buffer resource whose range is the padded
    // row: the chunks of a lane that lie past it read as zeros, which is what
    // the products need there, and the per-lane address is a 32-bit offset.
    const uint32_t row_range = (uint32_t)row_bytes;
    uint32_t coff[C];
#pragma unroll
    for (int c = 0; c < C; ++c) coff[c] = (uint32_t)(col_of(c) * (int64_t)sizeof(T));
    // Short rows (SUB): the wavefront's GPW*RS consecutive rows of a step
    // through one resource based at its first row; a lane's chunk past its
    // padded row, and a row past the band, are given an offset outside the
    // range (zeros, no memory traffic).
    constexpr uint32_t kOutside = 0x80000000u;
    bool cin[C];
#pragma unroll
    for (int c = 0; c < C; ++c) cin[c] = col_of(c) < a.ldA;
    auto load_rows = [&](uint4 (&buf)[RS][C], double (&bi)[RS], double (&nui)[RS], int64_t t) {
        const bool live = t < nsteps;
        if constexpr (SUB) {
            const int64_t rw = r0 + t * a.step_stride + (int64_t)(wave * GPW) * RS;   // uniform
            const int64_t rb = live ? min(rw, r1 - 1) : 0;
            const __amdgpu_buffer_rsrc_t rr = row_resource(Ab + rb * row_bytes, (uint32_t)(GPW * RS) * row_range);
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int64_t row = row_of(t, q);
                const bool ok = live && row < r1;
                const int64_t rc = ok ? row : rb;
                bi[q] = a.b_in[rc];
                nui[q] = a.nu[rc];
                const uint32_t base = (uint32_t)((rc - rb) * row_bytes);
#pragma unroll
                for (int c = 0; c < C; ++c) buf[q][c] = load_row_vec(rr, ok && cin[c] ? base + coff[c] : kOutside);
            }
        } else {
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const int64_t row = live ? min(row_of(t, q), r1 - 1) : 0;
                // b and nu first: loads return in order, so once the row has
                // arrived they have too, and no register of a reduced row is
                // still waiting for data when the buffer is refilled
                bi[q] = a.b_in[row];
                nui[q] = a.nu[row];
                const __amdgpu_buffer_rsrc_t rr = row_resource(Ab + row * row_bytes, row_range);
#pragma unroll
                for (int c = 0; c < C; ++c) buf[q][c] = load_row_vec(rr, coff[c]);
            }
        }
    };

    // The rows of the first PD steps (from HBM), then this lane's slices of
    // the working vectors x, v and (when the previous step is still to be
    // applied) y, padded with zeros to ldA (from L2): none of these loads
    // depends on the state, so they are all in flight while the state is
    // settled.  yacc holds the slice of y until the step is applied.
    uint4 buf[PD][RS][C];
    double bq[PD][RS], nq[PD][RS];
#pragma unroll
    for (int k = 0; k < PD; ++k) load_rows(buf[k], bq[k], nq[k], k);

    Acc xr[C][VEC];
    Acc vr[C][VEC];
    Acc yacc[C][VEC];
    const Acc *wx = reinterpret_cast<const Acc *>(a.work);
    const Acc *wv = wx + a.ldA;
    const Acc *wy = wx + 2 * a.ldA;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t col = min(col_of(c), a.ldA - VEC);
#pragma unroll
        for (int e = 0; e < VEC; e += AV) {
            const uint4 ux = *reinterpret_cast<const uint4 *>(wx + col + e);
            __builtin_memcpy(&xr[c][e], &ux, 16);
            if (HAS_V) {
                const uint4 uv = *reinterpret_cast<const uint4 *>(wv + col + e);
                __builtin_memcpy(&vr[c][e], &uv, 16);
            } else {
#pragma unroll
                for (int k = 0; k < AV; ++k) vr[c][e + k] = (Acc)0;
            }
            if (a.pd.decide) {
                const uint4 uy = *reinterpret_cast<const uint4 *>(wy + col + e);
                __builtin_memcpy(&yacc[c][e], &uy, 16);
            }
        }
    }
    const State st = sweep_state(a.pd, lane, blockIdx.x == 0 && tid == 0);
    if (a.check_status && st.status != ST_RUNNING) return;
    const bool apply_v = HAS_V && (st.vpend_valid || st.v_idx >= 0);
    // the step decided on the previous check: x_j = x_{j-1} - s*y_{j-1}, one rounding
    const double s = a.pd.decide ? st.s : 0.0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const bool in = col_of(c) < a.ldA;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (s != 0.0) xr[c][e] = (Acc)step_point((double)xr[c][e], s, (double)yacc[c][e]);
            if (!in) {
                xr[c][e] = (Acc)0;
                vr[c][e] = (Acc)0;
            }
            yacc[c][e] = (Acc)0;
        }
    }

    int64_t h = 0;
    double dmax = 0.0, binf = 0.0;
    __shared__ Acc red[2][NW][RS][2];

    // Per-row results bound for global memory (the translated b, and r when
    // asked for) are staged in LDS and written together every KS steps and
    // after the last one.  A global store inside the row loop would leave
    // loads and stores outstanding together; the compiler can then no longer
    // count which loads have returned and waits for all of them, the
    // prefetched rows included, before each use of a row.
    constexpr int SR = NG * RS;                   // rows per step
    constexpr int KS = SR >= 256 ? 1 : 256 / SR;  // steps per write-out
    __shared__ double bst[KS * SR], rst[KS * SR];
    const bool stage_b = apply_v && a.b_out != nullptr;
    const bool stage_r = a.r_out != nullptr;
    auto write_out = [&](int64_t t_last) {
        const int64_t t0 = t_last - t_last % KS;
        const int cnt = (int)(t_last - t0 + 1) * SR;
        __syncthreads();
        for (int i = tid; i < cnt; i += BLOCK) {
            const int64_t row = r0 + (t0 + i / SR) * a.step_stride + i % SR;
            if (row < r1) {
                if (stage_b) a.b_out[row] = bst[i];
                if (stage_r) a.r_out[row] = rst[i];
            }
        }
        // every store has completed before the loop's loads are counted again
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    auto process = [&](const uint4 (&buf)[RS][C], const double (&bi)[RS], const double (&nui)[RS], int64_t t) {
        Acc dot[RS], tdot[RS];
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            dot[q] = (Acc)0;
            tdot[q] = (Acc)0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                Acc av[VEC];
                unpack<DT>(buf[q][c], av);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    dot[q] = fma(xr[c][e], av[e], dot[q]);
                    if (HAS_V) tdot[q] = fma(vr[c][e], av[e], tdot[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            if constexpr (SUB) {
                dot[q] = group_total<LPR>(dot[q]);
                if (HAS_V) tdot[q] = group_total<LPR>(tdot[q]);
            } else {
                dot[q] = wave_total(dot[q]);
                if (HAS_V) tdot[q] = wave_total(tdot[q]);
            }
        }
        if (WPG > 1) {
            const int pp = (int)(t & 1);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < RS; ++q) {
                    red[pp][wave][q][0] = dot[q];
                    red[pp][wave][q][1] = tdot[q];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                Acc d = (Acc)0, td = (Acc)0;
#pragma unroll
                for (int w = 0; w < WPG; ++w) {
                    d += red[pp][grp * WPG + w][q][0];
                    if (HAS_V) td += red[pp][grp * WPG + w][q][1];
                }
                dot[q] = d;
                tdot[q] = td;
            }
        }
        if constexpr (SUB) {
            // the groups of a wavefront settle their rows side by side, without
            // branches (a row past the band counts as satisfied)
#pragma unroll
            for (int q = 0; q < RS; ++q) {
                const bool ok = row_of(t, q) < r1;
                double bb = bi[q];
                if (apply_v) bb += (double)tdot[q];
                const double r = ok ? (double)dot[q] - bb : -1.0;
                const int si = (int)(t % KS) * SR + grp * RS + q;
                if (ok && stage_b && gl == 0) bst[si] = bb;
                if (ok && stage_r && gl == 0) rst[si] = r;
                if (ok) binf = max_nan(binf, fabs(bb));
                const bool pos = r > 0.0;
                h += pos ? 1 : 0;
                const double d = r / sqrt(nui[q]);
                dmax = pos ? max_nan(dmax, d) : (r != r ? r : dmax);
                const Acc w = pos ? (Acc)(r / nui[q]) : (Acc)0;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Acc av[VEC];
                    unpack<DT>(buf[q][c], av);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(w, av[e], yacc[c][e]);
                }
            }
            return;
        }
#pragma unroll
        for (int q = 0; q < RS; ++q) {
            const int64_t row = row_of(t, q);
            if (row >= r1) continue;
            double bb = bi[q];
            if (apply_v) bb += (double)tdot[q];
            const double r = (double)dot[q] - bb;
            const int si = (int)(t % KS) * SR + grp * RS + q;
            if (stage_b && gl == 0) bst[si] = bb;
            if (stage_r && gl == 0) rst[si] = r;
            binf = max_nan(binf, fabs(bb));
            if (r > 0.0) {
                ++h;
                dmax = max_nan(dmax, r / sqrt(nui[q]));
                const Acc w = (Acc)(r / nui[q]);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Acc av[VEC];
                    unpack<DT>(buf[q][c], av);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(w, av[e], yacc[c][e]);
                }
            } else if (r != r) {
                dmax = r;  // NaN: reported as a numeric failure
            }
        }
    };

    // A ring of PD steps' rows: while one is reduced the next PD-1 are in
    // flight, and a buffer is refilled (PD steps ahead) as soon as it has been
    // reduced.  nsteps is the same for the whole workgroup, so every branch
    // below is uniform and the barriers inside process() are reached by all
    // lanes.
    int64_t t = 0;
    for (; t + PD <= nsteps; t += PD) {
#pragma unroll
        for (int k = 0; k < PD; ++k) {
            const int64_t tk = t + k;
            process(buf[k], bq[k], nq[k], tk);
            if ((stage_b || stage_r) && ((tk + 1) % KS == 0 || tk + 1 == nsteps)) write_out(tk);
            load_rows(buf[k], bq[k], nq[k], tk + PD);
        }
    }
    // the last nsteps % PD steps, already in the ring
#pragma unroll
    for (int k = 0; k < PD - 1; ++k) {
        const int64_t tk = t + k;
        if (tk < nsteps) {
            process(buf[k], bq[k], nq[k], tk);
            if ((stage_b || stage_r) && ((tk + 1) % KS == 0 || tk + 1 == nsteps)) write_out(tk);
        }
    }

    // Partial y of this workgroup (the chunk columns past ldA are zero in
    // yacc and lie inside the covered width ldPart).
    Acc *part = reinterpret_cast<Acc *>(a.part) + (int64_t)blockIdx.x * a.ldPart;
    if (NG == 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                uint4 w;
                __builtin_memcpy(&w, &yacc[c][e], 16);
                *reinterpret_cast<uint4 *>(part + col_of(c) + e) = w;
            }
        }
    } else {
        // The row groups' partials meet in LDS and are summed in group order;
        // chunk c of the result is written by row group c % NG, each lane its
        // own columns, in whole 16-byte vectors.
        __shared__ __attribute__((aligned(16))) Acc ysh[NG][C * CW];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                uint4 w;
                __builtin_memcpy(&w, &yacc[c][e], 16);
                *reinterpret_cast<uint4 *>(&ysh[grp][col_of(c) + e]) = w;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c % NG != grp) continue;
#pragma unroll
            for (int e = 0; e < VEC; e += AV) {
                Acc sum[AV];
#pragma unroll
                for (int k = 0; k < AV; ++k) sum[k] = (Acc)0;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    Acc t[AV];
                    const uint4 u = *reinterpret_cast<const uint4 *>(&ysh[g][col_of(c) + e]);
                    __builtin_memcpy(t, &u, 16);
#pragma unroll
                    for (int k = 0; k < AV; ++k) sum[k] += t[k];
                }
                uint4 w;
                __builtin_memcpy(&w, sum, 16);
                *reinterpret_cast<uint4 *>(part + col_of(c) + e) = w;
            }
        }
    }

    __shared__ int64_t hs[NG];
    __shared__ double ds[NG], bs[NG];
    if (gl == 0) {
        hs[grp] = h;
        ds[grp] = dmax;
        bs[grp] = binf;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t hh = 0;
        double dd = 0.0, bbm = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            hh += hs[g];
            dd = max_nan(dd, ds[g]);
            bbm = max_nan(bbm, bs[g]);
        }
        a.h_part[blockIdx.x] = hh;
        a.dmax_part[blockIdx.x] = dd;
        a.binf_part[blockIdx.x] = bbm;
    }
}

}  // namespace modap
