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
// Thread shape: LPR lanes (a multiple of the 64-wide wavefront) share a row;
// a workgroup of BLOCK lanes works on BLOCK/LPR rows at a time.  Lane l of a
// row group owns the columns c*LPR*VEC + l*VEC + [0, VEC) for chunk c < C, so
// each wavefront load of a chunk is 64 contiguous 16-byte vectors (1 KiB).  The
// lane's slices of x, v and of the partial y stay in registers for the whole
// sweep; the next row's vectors are loaded while the current row is reduced.
// Dot products are reduced across the wavefront with a butterfly (identical in
// every lane) and across the wavefronts of a row group through LDS, in a fixed
// order, so the result does not depend on timing.  Each workgroup owns a
// contiguous band of rows and writes one partial y; a second kernel sums the
// partials in a fixed order.
#pragma once

#include "modap_device.hpp"

namespace modap {

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

template <int DT, int BLOCK, int LPR, int C, bool HAS_V>
__global__ __launch_bounds__(BLOCK) void sweep_wide(const SweepArgs a) {
    using S = Store<DT>;
    using Acc = typename S::Acc;
    using T = typename S::T;
    constexpr int VEC = S::VEC;
    constexpr int NG = BLOCK / LPR;   // row groups per workgroup
    constexpr int WPG = LPR / 64;     // wavefronts per row group
    constexpr int NW = BLOCK / 64;
    constexpr int CW = LPR * VEC;     // columns per chunk
    static_assert(LPR % 64 == 0 && BLOCK % LPR == 0, "row groups are whole wavefronts");

    const Ctrl *ctl = a.ctl;
    if (a.check_status && ctl->status != ST_RUNNING) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int grp = tid / LPR;
    const int gl = tid % LPR;

    const double s = a.ystep ? ctl->s : 0.0;
    const double *vp = nullptr;
    const double *vs = nullptr;
    if (HAS_V) {
        if (a.vpend && ctl->vpend_valid) vp = a.vpend;
        if (a.V && ctl->v_idx >= 0) vs = a.V + ctl->v_idx * a.ldV;
    }
    const bool apply_v = HAS_V && (vp != nullptr || vs != nullptr);

    // Stage this lane's slices of the working point x - s*y and of v.
    Acc xr[C][VEC];
    Acc vr[C][VEC];
    Acc yacc[C][VEC];
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int64_t col = (int64_t)c * CW + gl * VEC + e;
            double xv = 0.0, vv = 0.0;
            if (col < a.n) {
                xv = a.x[col];
                if (s != 0.0) xv = step_point(xv, s, a.ystep[col]);
                if (HAS_V) {
                    if (vp) vv += vp[col];
                    if (vs) vv += vs[col];
                }
            }
            xr[c][e] = (Acc)xv;
            vr[c][e] = (Acc)vv;
            yacc[c][e] = (Acc)0;
        }
    }

    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_block;
    const int64_t r1 = min(a.m, r0 + a.rows_per_block);
    const int64_t nsteps = r1 > r0 ? (r1 - r0 + NG - 1) / NG : 0;
    const char *Ab = reinterpret_cast<const char *>(a.A);
    const int64_t row_bytes = a.ldA * (int64_t)sizeof(T);

    int64_t h = 0;
    double dmax = 0.0, binf = 0.0;

    __shared__ Acc red[2][NW][2];

    auto load_row = [&](uint4 (&buf)[C], double &bi, double &nui, int64_t row) {
        if (row < r1) {
            const char *rp = Ab + row * row_bytes;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const int64_t col = (int64_t)c * CW + gl * VEC;
                if (col < a.ldA)
                    buf[c] = *reinterpret_cast<const uint4 *>(rp + col * (int64_t)sizeof(T));
                else
                    buf[c] = make_uint4(0u, 0u, 0u, 0u);
            }
            bi = a.b_in[row];
            nui = a.nu[row];
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) buf[c] = make_uint4(0u, 0u, 0u, 0u);
            bi = 0.0;
            nui = 1.0;
        }
    };

    auto process = [&](const uint4 (&buf)[C], double bi, double nui, int64_t row, int64_t t) {
        Acc dot = (Acc)0, tdot = (Acc)0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Acc av[VEC];
            unpack<DT>(buf[c], av);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                dot = fma(xr[c][e], av[e], dot);
                if (HAS_V) tdot = fma(vr[c][e], av[e], tdot);
            }
        }
        dot = wave_sum(dot);
        if (HAS_V) tdot = wave_sum(tdot);
        if (WPG > 1) {
            const int pp = (int)(t & 1);
            if (lane == 0) {
                red[pp][wave][0] = dot;
                red[pp][wave][1] = tdot;
            }
            __syncthreads();
            Acc d = (Acc)0, td = (Acc)0;
#pragma unroll
            for (int w = 0; w < WPG; ++w) {
                d += red[pp][grp * WPG + w][0];
                if (HAS_V) td += red[pp][grp * WPG + w][1];
            }
            dot = d;
            tdot = td;
        }
        if (row < r1) {
            double bb = bi;
            if (apply_v) {
                bb += (double)tdot;
                if (a.b_out && gl == 0) a.b_out[row] = bb;
            }
            const double r = (double)dot - bb;
            if (a.r_out && gl == 0) a.r_out[row] = r;
            binf = max_nan(binf, fabs(bb));
            if (r > 0.0) {
                ++h;
                dmax = max_nan(dmax, r / sqrt(nui));
                const Acc w = (Acc)(r / nui);
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    Acc av[VEC];
                    unpack<DT>(buf[c], av);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) yacc[c][e] = fma(w, av[e], yacc[c][e]);
                }
            } else if (r != r) {
                dmax = r;  // NaN: reported as a numeric failure
            }
        }
    };

    uint4 bufA[C], bufB[C];
    double bA = 0.0, nA = 1.0, bB = 0.0, nB = 1.0;
    if (nsteps > 0) load_row(bufA, bA, nA, r0 + grp);
    for (int64_t t = 0; t < nsteps; t += 2) {
        const int64_t rowA = r0 + grp + t * NG;
        if (t + 1 < nsteps) load_row(bufB, bB, nB, rowA + NG);
        process(bufA, bA, nA, rowA, t);
        if (t + 1 < nsteps) {
            if (t + 2 < nsteps) load_row(bufA, bA, nA, rowA + 2 * NG);
            process(bufB, bB, nB, rowA + NG, t + 1);
        }
    }

    // Partial y of this workgroup.
    Acc *part = reinterpret_cast<Acc *>(a.part) + (int64_t)blockIdx.x * a.ldPart;
    if (NG == 1) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) part[(int64_t)c * CW + gl * VEC + e] = yacc[c][e];
        }
    } else {
        __shared__ Acc ysh[NG][C * CW];
#pragma unroll
        for (int c = 0; c < C; ++c) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) ysh[grp][c * CW + gl * VEC + e] = yacc[c][e];
        }
        __syncthreads();
        for (int col = tid; col < C * CW; col += BLOCK) {
            Acc acc = (Acc)0;
#pragma unroll
            for (int g = 0; g < NG; ++g) acc += ysh[g][col];
            part[col] = acc;
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
