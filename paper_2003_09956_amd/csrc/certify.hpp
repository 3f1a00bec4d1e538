// FP64 certificate of an eps-feasible stop.
//
// With FP32 or BF16 storage the sweep decides the stop from FP32 dot products,
// and the right-hand side it carries has been translated by FP32 dot products
// of v rounded to FP32, so the point it calls eps-feasible (eq. 10) is
// eps-feasible only up to those roundings.  The certificate re-decides such a
// stop on the same stored rows, with x and the translations in FP64 and FP64
// accumulation:
//
//   b_i  = bref_i + <a_i, wsum>          the exact data: bref is the right-hand
//                                         side at zero translation and wsum the
//                                         FP64 sum of every translation applied
//   r_i  = <a_i, x> - b_i                (section 2)
//   d_i  = max(r_i + g_i, 0)/||a_i||      an upper bound of the distance of eq. 10,
//                                         g_i bounding the rounding of r_i
//   y    = sum over r_i > 0 of (r_i/||a_i||^2) a_i,  h = #{r_i > 0}   (eq. 7, section 3)
//
// The rounding bound is the standard one for a dot product of n terms
// accumulated in any order (Higham, Accuracy and Stability of Numerical
// Algorithms, sect. 3.1): |fl(sum) - sum| <= gamma_n sum |terms| with
// gamma_n = n u/(1 - n u), u = 2^-53.  Both dot products, the sum bref + <a,w>
// and the difference stay within 4 gamma_{n+4} (sum_j |a_ij|(|x_j| + |w_j|) +
// |bref_i|); the norm, its square root and the division add at most a factor
// (1 + 2 gamma_{n+4}).  So max_i d_i bounds the true largest distance from
// above, and a stop it confirms is eps-feasible on the exact data.
//
// If the bound exceeds eps_abs, the certificate's own y and h decide a step
// (eq. 12 or Algorithm 1) in place of the stop, and the iteration goes on.
// Either way b and bref are rebased to the exact right-hand side and wsum is
// cleared, which removes whatever the working-precision translations had
// accumulated.
//
// Four kernels, each a no-op unless the committed state is an uncertified
// stop (so they may be queued without knowing whether one is due):
//   cert_dot     one wavefront per row: r_i, d_i, the step weight, the rebase
//   cert_axpy    (row band, column tile): y partial over the band's violated rows
//   cert_reduce  64 columns per workgroup: y and ||y||^2 parts; totals
//   cert_decide  one workgroup: the decision, the step, the working vectors
#pragma once

#include "aux_kernels.hpp"
#include "modap_device.hpp"

namespace modap {


// The certificate runs only on a stop that it has not confirmed yet.
__device__ __forceinline__ bool cert_due(const Ctrl *c, int sl) {
    const State s = load_global(&c->st[sl]);
    return s.status == ST_CONVERGED && s.certified == 0;
}

// gamma_k = k u / (1 - k u), u = 2^-53.
__device__ __forceinline__ double gamma_of(int64_t k) {
    const double ku = (double)k * 0x1p-53;
    return ku / (1.0 - ku);
}

template <int DT>
__global__ __launch_bounds__(256) void cert_dot(const CertArgs a) {
    if (!cert_due(a.ctl, a.sl)) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t row = (int64_t)blockIdx.x * 4 + wave;
    int64_t h = 0;
    double dup = 0.0, binf = 0.0, drift = 0.0;
    if (row < a.m) {
        double dx = 0.0, dw = 0.0, sc = 0.0;
        for (int64_t j = lane; j < a.n; j += 64) {
            const double e = load_elem<DT>(a.A, row * a.ldA + j);
            const double xj = a.x[j], wj = a.wsum[j];
            dx = __fma_rn(e, xj, dx);
            dw = __fma_rn(e, wj, dw);
            sc = __fma_rn(fabs(e), fabs(xj) + fabs(wj), sc);
        }
        dx = wave_sum(dx);
        dw = wave_sum(dw);
        sc = wave_sum(sc);
        const double br = a.bref[row];
        const double bi = br + dw;
        const double r = dx - bi;
        const double nu = a.nu[row];
        const double gm = gamma_of(a.n + 4);
        const double g = 4.0 * gm * (sc + fabs(br));
        const double d = ((r + g) / sqrt(nu)) * (1.0 + 2.0 * gm);
        drift = fabs(a.b[row] - bi);
        if (lane == 0) {
            a.b[row] = bi;
            a.bref[row] = bi;
            a.wt[row] = r > 0.0 ? r / nu : 0.0;
        }
        h = r > 0.0 ? 1 : 0;
        dup = d > 0.0 ? d : (d != d ? d : 0.0);
        binf = fabs(bi);
    }
    __shared__ int64_t hs[4];
    __shared__ double ds[4], bs[4], fs[4];
    if (lane == 0) {
        hs[wave] = h;
        ds[wave] = dup;
        bs[wave] = binf;
        fs[wave] = drift;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.h_part[blockIdx.x] = ((hs[0] + hs[1]) + hs[2]) + hs[3];
        a.dmax_part[blockIdx.x] = max_nan(max_nan(ds[0], ds[1]), max_nan(ds[2], ds[3]));
        a.binf_part[blockIdx.x] = max_nan(max_nan(bs[0], bs[1]), max_nan(bs[2], bs[3]));
        a.drift_part[blockIdx.x] = max_nan(max_nan(fs[0], fs[1]), max_nan(fs[2], fs[3]));
    }
}

// Partial y of one row band over one column tile of 256 VEC-element vectors
// (VEC = 16 bytes of the storage type): the band's violated rows are listed
// in row order, 256 at a time (a ballot per wavefront, wavefronts in order),
// and each is added in FP64, four rows in flight, in row order.
template <int DT>
__global__ __launch_bounds__(256) void cert_axpy(const CertArgs a) {
    if (!cert_due(a.ctl, a.sl)) return;
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::VEC;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t col = (int64_t)blockIdx.y * (256 * VEC) + (int64_t)tid * VEC;
    const bool in = col < a.ldA;
    const int64_t r0 = (int64_t)blockIdx.x * a.rows_per_band;
    const int64_t r1 = min(a.m, r0 + a.rows_per_band);
    double acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.0;
    __shared__ int64_t list[256];
    __shared__ double wl[256];
    __shared__ int wcount[4];
    const T *A = reinterpret_cast<const T *>(a.A);
    auto fetch = [&](int64_t row) -> uint4 {
        return in ? *reinterpret_cast<const uint4 *>(A + row * a.ldA + col) : make_uint4(0, 0, 0, 0);
    };
    auto add_row = [&](const uint4 &u, double w) {
        double av[VEC];
        if constexpr (DT == 0) {
            av[0] = __hiloint2double((int)u.y, (int)u.x);
            av[1] = __hiloint2double((int)u.w, (int)u.z);
        } else if constexpr (DT == 1) {
            av[0] = (double)__uint_as_float(u.x);
            av[1] = (double)__uint_as_float(u.y);
            av[2] = (double)__uint_as_float(u.z);
            av[3] = (double)__uint_as_float(u.w);
        } else {
            const uint32_t wds[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                av[2 * k] = (double)__uint_as_float(wds[k] << 16);
                av[2 * k + 1] = (double)__uint_as_float(wds[k] & 0xffff0000u);
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = __fma_rn(w, av[e], acc[e]);
    };
    for (int64_t base = r0; base < r1; base += 256) {
        const int64_t r = base + tid;
        const double w = r < r1 ? a.wt[r] : 0.0;
        const bool f = w != 0.0;
        const unsigned long long bal = __ballot(f);
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int off = 0, total = 0;
        for (int q = 0; q < 4; ++q) {
            if (q < wave) off += wcount[q];
            total += wcount[q];
        }
        if (f) {
            const int at = off + __popcll(bal & ((1ull << lane) - 1ull));
            list[at] = r;
            wl[at] = w;
        }
        __syncthreads();
        int k = 0;
        for (; k + 4 <= total; k += 4) {
            const uint4 u0 = fetch(list[k]), u1 = fetch(list[k + 1]), u2 = fetch(list[k + 2]), u3 = fetch(list[k + 3]);
            add_row(u0, wl[k]);
            add_row(u1, wl[k + 1]);
            add_row(u2, wl[k + 2]);
            add_row(u3, wl[k + 3]);
        }
        for (; k < total; ++k) add_row(fetch(list[k]), wl[k]);
        __syncthreads();   // the list is rewritten by the next chunk
    }
    if (in) {
        double *p = a.part + (int64_t)blockIdx.x * a.ldA + col;
#pragma unroll
        for (int e = 0; e < VEC; ++e) p[e] = acc[e];
    }
}

// y as the sum of the band partials in band order, the parts of ||y||^2, and
// (workgroup 0) the totals of the dot workgroups' scalars.
__global__ __launch_bounds__(256) void cert_reduce(const CertArgs a) {
    if (!cert_due(a.ctl, a.sl)) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (col < a.n)
        for (int q = wave; q < a.bands; q += 4) s += a.part[(int64_t)q * a.ldA + col];
    __shared__ double sh[4][64];
    sh[wave][lane] = s;
    int64_t h = 0;
    double dm = 0.0, bm = 0.0, fm = 0.0;
    if (blockIdx.x == 0) {
        for (int g = tid; g < a.Gs; g += 256) {
            h += a.h_part[g];
            dm = max_nan(dm, a.dmax_part[g]);
            bm = max_nan(bm, a.binf_part[g]);
            fm = max_nan(fm, a.drift_part[g]);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            h += __shfl_xor(h, o, 64);
            dm = max_nan(dm, __shfl_xor(dm, o, 64));
            bm = max_nan(bm, __shfl_xor(bm, o, 64));
            fm = max_nan(fm, __shfl_xor(fm, o, 64));
        }
    }
    __shared__ int64_t hw[4];
    __shared__ double dw[4], bw[4], fw[4];
    if (lane == 0) {
        hw[wave] = h;
        dw[wave] = dm;
        bw[wave] = bm;
        fw[wave] = fm;
    }
    __syncthreads();
    if (wave != 0) return;
    const double yv = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
    double sq = 0.0;
    if (col < a.n) {
        a.y[col] = yv;
        sq = yv * yv;
    }
    sq = wave_sum(sq);
    if (lane == 0) a.ynp[blockIdx.x] = sq;
    if (blockIdx.x == 0 && lane == 0) {
        Totals t{};
        for (int q = 0; q < 4; ++q) {
            t.h += hw[q];
            t.dmax = max_nan(t.dmax, dw[q]);
            t.binf = max_nan(t.binf, bw[q]);
            t.bdrift = max_nan(t.bdrift, fw[q]);
        }
        *a.tot = t;
    }
}

// The decision on the certificate (one workgroup, so the state is read by
// every thread before thread 0 rewrites it).  The stop being certified is
// undone -- the same state, running, one check fewer -- and decided again from
// the certificate's totals: a confirmed stop is marked certified; otherwise
// the step is taken in FP64 from the certificate's y and the next sweep's
// working vectors are written (x, and the drift row due after the step).  A
// failure with no row violated in FP64 means eps_abs lies below the rounding
// bound: ST_UNCERTIFIED.  wsum is cleared (b and bref hold the exact data).
template <typename Acc>
__global__ __launch_bounds__(1024) void cert_decide(const CertArgs a) {
    const State p = load_global(&a.ctl->st[a.sl]);
    if (!(p.status == ST_CONVERGED && p.certified == 0)) return;
    __shared__ State sst;
    if (threadIdx.x < 64) {
        const double yn = ynorm_of(a.ynp, a.R, threadIdx.x);
        const Totals t = load_global(a.tot);
        State q = p;
        q.status = ST_RUNNING;
        q.sweeps = p.sweeps - 1;
        q.feasible = 0;
        State s = decide(q, t, yn, a.dp, load_global(&a.ctl->step_limit), load_global(&a.ctl->sched_len));
        if (s.status == ST_CONVERGED) s.certified = 1;
        if (s.status == ST_NO_DIRECTION && t.h == 0) s.status = ST_UNCERTIFIED;
        s.bdrift = t.bdrift;
        if (threadIdx.x == 0) sst = s;
    }
    __syncthreads();
    const State s = sst;
    const double *vrow = (a.V && s.v_idx >= 0) ? a.V + s.v_idx * a.ldV : nullptr;
    Acc *wx = reinterpret_cast<Acc *>(a.work);
    Acc *wv = wx + a.ldA;
    for (int64_t j = threadIdx.x; j < a.n; j += blockDim.x) {
        a.wsum[j] = 0.0;
        if (s.status != ST_RUNNING) continue;
        double xv = a.x[j];
        if (s.s != 0.0) {
            xv = step_point(xv, s.s, a.y[j]);
            a.x[j] = xv;
        }
        wx[j] = (Acc)xv;
        wv[j] = vrow ? (Acc)vrow[j] : (Acc)0;
    }
    __syncthreads();
    if (threadIdx.x == 0) store_global(&a.ctl->st[a.sl], s);
}

}  // namespace modap
