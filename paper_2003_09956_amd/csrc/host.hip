// Host half of the library: the C ABI declared in include/modap.h.
//
// A context owns a device copy of the system (rows padded with zeros to a
// 16-byte multiple), its FP64 row norms, the approximation x, the last y, a
// one-shot translation slot, an optional drift schedule, the per-workgroup
// partials, the working vectors of the next sweep and a device control block.
// One iteration is two kernels on the context's stream: the fused sweep
// (which first settles the previous check: stop decision and step length)
// and the fixed-order reduction of y (which makes the previous step permanent
// in x and writes the next sweep's working vectors); a stage kernel settles
// the last check of a call.  The host never waits between iterations; solve()
// reads the control block once per batch of queued iterations.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "aux_kernels.hpp"
#include "aux_launch.hpp"
#include "certify.hpp"
#include "host_common.hpp"
#include "trace.hpp"
#include "internal.hpp"
#include "modap.h"
#include "resident.hpp"
#include "sweep_split.hpp"
#include "modap_device.hpp"
#include "sweep_table.hpp"

using namespace modap;

struct modap_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    std::string err;

    // system
    bool loaded = false;
    int64_t m = 0, n = 0, ldA = 0;
    int dt = 0;
    size_t es = 0;
    void *A = nullptr;
    double *b = nullptr, *nu = nullptr, *x = nullptr, *y = nullptr, *vpend = nullptr;
    double *bref = nullptr;      // [m] right-hand side at zero translation: the data are bref + A wsum
    double *wsum = nullptr;      // [ldA] FP64 sum of the translations applied since the last rebase
    int *claim = nullptr;        // [m] row claims of a device-side replacement (zero between calls)
    double *V = nullptr;
    int64_t T = 0;
    bool vpend_maybe = false;   // a translation may be pending on the device
    int64_t jn = 0;             // index of the next iteration; state of jn-1 is committed

    // kernel shape and scratch
    modap_tile tile{};
    bool tile_forced = false;
    const SweepKernel *kern_nov = nullptr, *kern_v = nullptr;
    // split-row two-phase form (tile kind 1)
    const SplitKernels *skern = nullptr;
    int ntiles = 0;
    int64_t rows_per_band = 0;
    int finish_blocks = 0;
    void *pdot = nullptr;
    size_t pdot_bytes = 0;
    double *wrow = nullptr;
    int64_t rows_per_block = 0;  // one-pass sweep: row mapping (see SweepArgs)
    int64_t block_stride = 0;
    int64_t step_stride = 0;
    int64_t ldPart = 0;
    void *part = nullptr;
    size_t part_bytes = 0;
    int64_t *h_part = nullptr;
    double *dmax_part = nullptr, *binf_part = nullptr;
    int part_grid = 0;
    double *ynp = nullptr;
    Totals *tot = nullptr;
    void *work = nullptr;        // [3 x ldA] accumulation type: x, v and y of the next sweep
    void *work_eval = nullptr;

    Ctrl *ctl = nullptr;
    State *hst = nullptr;        // pinned [2]
    double *x_eval = nullptr, *y_eval = nullptr, *r_eval = nullptr;
    unsigned long long *bad = nullptr;
    int *flag = nullptr;

    // staging for host-side update inputs
    void *stage = nullptr;
    size_t stage_bytes = 0;

    // resident iteration of small systems (resident.hpp): one launch of many
    // iterations on a few workgroups holding their rows in LDS
    bool res_ok = false;
    int res_grid = 0, res_rows = 0, res_ldR = 0;
    size_t res_lds = 0;
    void *res_part = nullptr;
    int64_t *res_h = nullptr;
    double *res_dmax = nullptr, *res_binf = nullptr;

    // FP64 certificate scratch (allocated at the first certificate of a system)
    double *cert_wt = nullptr, *cert_part = nullptr, *cert_y = nullptr, *cert_ynp = nullptr;
    int64_t *cert_h = nullptr;
    double *cert_dmax = nullptr, *cert_binf = nullptr, *cert_drift = nullptr;
    Totals *cert_tot = nullptr;
    int cert_bands = 0;
    int64_t cert_rows_per_band = 0;

    std::vector<hipEvent_t> events;
    hipEvent_t sync_ev[2] = {nullptr, nullptr};
};

namespace {

using namespace modap_host;

const SweepKernel *kernels_for(int dt, int *count) {
    switch (dt) {
        case 0: return sweep_kernels_0(count);
        case 1: return sweep_kernels_1(count);
        default: return sweep_kernels_2(count);
    }
}

// The compiled kernel of a shape; depth 0 takes the shallowest one compiled.
const SweepKernel *find_kernel(int dt, int block, int lpr, int chunks, int rs, int depth, bool has_v) {
    int cnt = 0;
    const SweepKernel *t = kernels_for(dt, &cnt);
    const SweepKernel *hit = nullptr;
    for (int i = 0; i < cnt; ++i)
        if (t[i].block == block && t[i].lpr == lpr && t[i].chunks == chunks && t[i].rs == rs &&
            t[i].has_v == has_v && (depth == 0 ? (!hit || t[i].pd < hit->pd) : t[i].pd == depth))
            hit = &t[i];
    return hit;
}

int64_t coverage(int dt, int lpr, int chunks) { return (int64_t)lpr * vec_elems(dt) * chunks; }

const SplitKernels *split_for(int dt) {
    switch (dt) {
        case 0: return split_kernels_0();
        case 1: return split_kernels_1();
        default: return split_kernels_2();
    }
}

constexpr int64_t kMaxBandRows = 4096;  // rows per band of the split-row form (its row list)

// Built-in choice of the fused sweep's shape (what measured fastest on the
// headline systems): the smallest row coverage that holds a padded row; among
// equal coverage, about 32 elements (128 bytes of FP32) per lane per row, then
// the smaller workgroup, one row per step and the shallowest prefetch.
bool choose_shape(int dt, int64_t ldA, modap_tile *out) {
    int cnt = 0;
    const SweepKernel *t = kernels_for(dt, &cnt);
    const SweepKernel *best = nullptr;
    int64_t best_cov = 0;
    int best_score = INT_MAX;
    for (int i = 0; i < cnt; ++i) {
        if (!t[i].has_v) continue;
        const int64_t cov = coverage(dt, t[i].lpr, t[i].chunks);
        if (cov < ldA) continue;
        const int epl = t[i].chunks * vec_elems(dt);
        const int score = std::abs(epl - 32) * 16 + (t[i].block == 256 ? 0 : t[i].block == 512 ? 4 : 8) +
                          (t[i].rs == 1 ? 0 : 2) + 4 * (t[i].pd - 2) + (t[i].lpr == t[i].block ? 0 : 1);
        if (!best || cov < best_cov || (cov == best_cov && score < best_score)) {
            best = &t[i];
            best_cov = cov;
            best_score = score;
        }
    }
    if (!best) {
        const SplitKernels *sk = split_for(dt);
        out->kind = 1;
        out->block = sk->block;
        out->lanes_per_row = sk->block;
        out->chunks = sk->chunks;
        out->grid = 0;
        out->rows_per_step = 1;
        out->depth = 0;
        out->interleave = 0;
        return true;
    }
    out->kind = 0;
    out->block = best->block;
    out->lanes_per_row = best->lpr;
    out->chunks = best->chunks;
    out->grid = 0;
    out->rows_per_step = best->rs;
    out->depth = best->pd;
    out->interleave = 0;
    return true;
}

modap_status ensure_scalar_parts(modap_ctx *c, int count) {
    if (count <= c->part_grid) return MODAP_OK;
    free_dev(c->h_part);
    free_dev(c->dmax_part);
    free_dev(c->binf_part);
    HIP_TRY(c, hipMalloc(&c->h_part, sizeof(int64_t) * count));
    HIP_TRY(c, hipMalloc(&c->dmax_part, sizeof(double) * count));
    HIP_TRY(c, hipMalloc(&c->binf_part, sizeof(double) * count));
    c->part_grid = count;
    return MODAP_OK;
}

modap_status ensure_part(modap_ctx *c, size_t need) {
    if (need <= c->part_bytes) return MODAP_OK;
    free_dev(c->part);
    HIP_TRY(c, hipMalloc(&c->part, need));
    c->part_bytes = need;
    return MODAP_OK;
}

// Split-row form: column tiles of 256*VEC*C columns, row bands of at most
// kMaxBandRows rows; grid = number of row bands (0: about two workgroups per
// compute unit over bands x tiles).
modap_status configure_split(modap_ctx *c, modap_tile t) {
    const SplitKernels *sk = split_for(c->dt);
    if (t.block != sk->block || t.lanes_per_row != sk->block || t.chunks != sk->chunks)
        return fail(c, MODAP_E_INVAL, "no compiled split-row kernel of that shape for this storage type");
    const int64_t tw = (int64_t)sk->block * vec_elems(c->dt) * sk->chunks;
    const int ntiles = (int)((c->ldA + tw - 1) / tw);
    int64_t bands = t.grid > 0 ? t.grid : std::max<int64_t>(1, (2 * c->cu_count + ntiles - 1) / ntiles);
    int64_t rpb = (c->m + bands - 1) / bands;
    rpb = std::min(rpb, kMaxBandRows);
    bands = (c->m + rpb - 1) / rpb;
    const size_t acc = acc_size(c->dt);
    modap_status st;
    if ((st = ensure_part(c, (size_t)bands * (size_t)ntiles * (size_t)tw * acc))) return st;
    const size_t pd = 2 * (size_t)ntiles * (size_t)c->m * acc;
    if (pd > c->pdot_bytes) {
        free_dev(c->pdot);
        HIP_TRY(c, hipMalloc(&c->pdot, pd));
        c->pdot_bytes = pd;
    }
    if (!c->wrow) HIP_TRY(c, hipMalloc(&c->wrow, sizeof(double) * (size_t)c->m));
    c->finish_blocks = (int)((c->m + 255) / 256);
    if ((st = ensure_scalar_parts(c, c->finish_blocks))) return st;
    c->skern = sk;
    c->ntiles = ntiles;
    c->rows_per_band = rpb;
    c->ldPart = (int64_t)ntiles * tw;
    t.grid = (int)bands;
    t.rows_per_step = 1;
    t.depth = 0;
    t.interleave = 0;
    c->tile = t;
    c->kern_v = c->kern_nov = nullptr;
    return MODAP_OK;
}

// Resolve the tile into kernels, grid and scratch.
modap_status configure(modap_ctx *c, const modap_tile &want) {
    modap_tile t = want;
    if (t.kind == 1) return configure_split(c, t);
    if (t.kind != 0) return fail(c, MODAP_E_INVAL, "tile kind must be 0 (one pass) or 1 (split rows)");
    if (t.rows_per_step <= 0) t.rows_per_step = 1;
    if (t.depth < 0) return fail(c, MODAP_E_INVAL, "tile depth must be >= 0");
    const SweepKernel *kv = find_kernel(c->dt, t.block, t.lanes_per_row, t.chunks, t.rows_per_step, t.depth, true);
    if (!kv) return fail(c, MODAP_E_INVAL, "no compiled sweep kernel of that shape for this storage type");
    t.depth = kv->pd;
    const SweepKernel *kn = find_kernel(c->dt, t.block, t.lanes_per_row, t.chunks, t.rows_per_step, t.depth, false);
    if (!kn) return fail(c, MODAP_E_INVAL, "no compiled sweep kernel of that shape for this storage type");
    const int64_t cov = coverage(c->dt, t.lanes_per_row, t.chunks);
    if (cov < c->ldA) return fail(c, MODAP_E_INVAL, "sweep shape does not cover a row");
    const int per_step = (t.block / t.lanes_per_row) * t.rows_per_step;
    // By default one workgroup per CU: with every row group keeping depth-1
    // steps of rows in flight, a second workgroup per CU adds no bandwidth
    // but doubles the partial y written at the end of the sweep.
    int grid = t.grid > 0 ? t.grid : c->cu_count;
    if (t.interleave != 0 && t.interleave != 1) return fail(c, MODAP_E_INVAL, "tile interleave must be 0 or 1");
    int64_t rpb, block_stride, step_stride;
    if (t.interleave) {
        // workgroup b takes row blocks b, b + grid, b + 2*grid, ... of per_step rows
        grid = (int)std::min<int64_t>(grid, (c->m + per_step - 1) / per_step);
        rpb = c->m;
        block_stride = per_step;
        step_stride = (int64_t)grid * per_step;
    } else {
        rpb = (c->m + grid - 1) / grid;
        rpb = ((rpb + per_step - 1) / per_step) * per_step;
        grid = (int)((c->m + rpb - 1) / rpb);
        block_stride = rpb;
        step_stride = per_step;
    }
    const size_t acc = acc_size(c->dt);
    modap_status st;
    if ((st = ensure_part(c, (size_t)grid * (size_t)cov * acc))) return st;
    if ((st = ensure_scalar_parts(c, grid))) return st;
    c->skern = nullptr;
    c->kern_v = kv;
    c->kern_nov = kn;
    c->rows_per_block = rpb;
    c->block_stride = block_stride;
    c->step_stride = step_stride;
    c->ldPart = cov;
    t.grid = grid;
    c->tile = t;
    return MODAP_OK;
}

modap_status check_ctx(modap_ctx *c, bool need_system) {
    if (!c) return MODAP_E_INVAL;
    if (need_system && !c->loaded) return fail(c, MODAP_E_STATE, "no system loaded (call modap_set_system first)");
    return MODAP_OK;
}

modap_status check_params(modap_ctx *c, const modap_params *p) {
    const char *msg = nullptr;
    const modap_status st = modap_host::check_params(p, &msg);
    return st ? fail(c, st, msg) : MODAP_OK;
}


modap_status ensure_stage(modap_ctx *c, size_t bytes) {
    if (bytes <= c->stage_bytes) return MODAP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_dev(c->stage);
    HIP_TRY(c, hipMalloc(&c->stage, bytes));
    c->stage_bytes = bytes;
    return MODAP_OK;
}

// Copy caller data (host or device) to a device pointer, stream-ordered.
modap_status to_device(modap_ctx *c, void *dst, const void *src, size_t bytes, int on_dev) {
    if (bytes == 0) return MODAP_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    return MODAP_OK;
}

modap_status from_device(modap_ctx *c, void *dst, const void *src, size_t bytes, int on_dev) {
    if (bytes == 0) return MODAP_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    return MODAP_OK;
}

double sweep_bytes(const modap_ctx *c, bool with_v) {
    return (double)c->m * (double)c->n * (double)c->es + 16.0 * (double)c->m + (with_v ? 8.0 * (double)c->m : 0.0);
}

bool translation_possible(const modap_ctx *c) { return c->vpend_maybe || (c->V && c->T > 0); }

int reduce_grid(const modap_ctx *c) { return (int)((c->n + 63) / 64); }

int last_slot(const modap_ctx *c) { return (int)((c->jn - 1) & 1); }

Decide decide_params(const modap_params *p, int track) {
    Decide d{};
    d.lambda = p->lambda;
    d.eps = p->eps;
    d.eps_relative = p->eps_relative;
    d.rule = p->step;
    d.track = track;
    return d;
}

SweepArgs sweep_args(modap_ctx *c) {
    SweepArgs a{};
    a.A = c->A;
    a.ldA = c->ldA;
    a.m = c->m;
    a.n = c->n;
    a.b_in = c->b;
    a.nu = c->nu;
    a.work = c->work;
    a.pd.ctl = c->ctl;
    a.pd.j = c->jn;
    a.pd.tot = c->tot;
    a.pd.ynp = c->ynp;
    a.pd.R = reduce_grid(c);
    a.pd.decide = 0;
    a.part = c->part;
    a.ldPart = c->ldPart;
    a.h_part = c->h_part;
    a.dmax_part = c->dmax_part;
    a.binf_part = c->binf_part;
    a.rows_per_block = c->rows_per_block;
    a.block_stride = c->block_stride;
    a.step_stride = c->step_stride;
    return a;
}

// Launch the sweep of the configured form (events: start/end of its kernels).
modap_status launch_sweep(modap_ctx *c, const SweepArgs &a, bool hv, hipEvent_t e0, hipEvent_t e1) {
    if (!c->skern) {
        HIP_TRY(c, (hv ? c->kern_v : c->kern_nov)->launch(a, c->tile.grid, c->stream, e0, e1));
        return MODAP_OK;
    }
    SplitArgs s{};
    s.A = a.A;
    s.ldA = a.ldA;
    s.m = a.m;
    s.n = a.n;
    s.b_in = a.b_in;
    s.b_out = a.b_out;
    s.nu = a.nu;
    s.work = a.work;
    s.pd = a.pd;
    s.check_status = a.check_status;
    s.ntiles = c->ntiles;
    s.rows_per_band = c->rows_per_band;
    s.pdot = c->pdot;
    s.w = c->wrow;
    s.r_out = a.r_out;
    s.part = c->part;
    s.ldPart = c->ldPart;
    s.h_part = c->h_part;
    s.dmax_part = c->dmax_part;
    s.binf_part = c->binf_part;
    if (e0) HIP_TRY(c, hipEventRecord(e0, c->stream));
    HIP_TRY(c, c->skern->dot(s, c->tile.grid, c->ntiles, hv, c->stream));
    HIP_TRY(c, c->skern->finish(s, c->finish_blocks, hv, c->stream));
    HIP_TRY(c, c->skern->axpy(s, c->tile.grid, c->ntiles, c->stream));
    if (e1) HIP_TRY(c, hipEventRecord(e1, c->stream));
    return MODAP_OK;
}

ReduceArgs reduce_args(modap_ctx *c) {
    ReduceArgs r{};
    r.part = c->part;
    r.ldPart = c->ldPart;
    r.G = c->tile.grid;
    r.Gs = c->skern ? c->finish_blocks : c->tile.grid;
    r.acc_f64 = c->dt == 0;
    r.n = c->n;
    r.ldA = c->ldA;
    r.x = c->x;
    r.V = c->V;
    r.ldV = c->ldA;
    r.h_part = c->h_part;
    r.dmax_part = c->dmax_part;
    r.binf_part = c->binf_part;
    r.tot = c->tot;
    r.ynp = c->ynp;
    r.vpend = c->vpend;
    return r;
}

modap_status launch_reduce(modap_ctx *c, const ReduceArgs &r, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    if (e0 || e1) {
        ReduceArgs copy = r;
        void *args[] = {&copy};
        const void *f = r.acc_f64 ? reinterpret_cast<const void *>(&reduce_y<double>)
                                  : reinterpret_cast<const void *>(&reduce_y<float>);
        HIP_TRY(c, hipExtLaunchKernel(f, dim3(reduce_grid(c)), dim3(kReduceThreads), args, 0, c->stream, e0, e1, 0));
        return MODAP_OK;
    }
    if (r.acc_f64)
        hipLaunchKernelGGL(reduce_y<double>, dim3(reduce_grid(c)), dim3(kReduceThreads), 0, c->stream, r);
    else
        hipLaunchKernelGGL(reduce_y<float>, dim3(reduce_grid(c)), dim3(kReduceThreads), 0, c->stream, r);
    LAUNCH_TRY(c, "reduce_y launch");
    return MODAP_OK;
}

hipEvent_t event_at(modap_ctx *c, size_t i) {
    while (c->events.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    return c->events[i];
}

// Create the events of `iters` queued iterations of which every `every`-th is
// profiled, before any is queued: creating one while the device runs ahead
// of the host would leave the device idle.
modap_status reserve_events(modap_ctx *c, int64_t iters, int64_t every) {
    if (every <= 0 || iters <= 0) return MODAP_OK;
    const int64_t need = 4 * ((iters + every - 1) / every);
    if (!event_at(c, (size_t)need - 1)) return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
    return MODAP_OK;
}

// Profiling: events 4i..4i+3 of iteration i mark the sweep's start and end
// and the reduction's start and end, recorded by the kernel dispatches
// themselves.
bool profile_events(modap_ctx *c, size_t first, hipEvent_t (&e)[4]) {
    for (int k = 0; k < 4; ++k) {
        e[k] = event_at(c, first + k);
        if (!e[k]) return false;
    }
    return true;
}

StageArgs stage_args(modap_ctx *c, const modap_params *p, int track, int64_t j) {
    StageArgs g{};
    g.ctl = c->ctl;
    g.j = j;
    g.tot = c->tot;
    g.ynp = c->ynp;
    g.R = reduce_grid(c);
    if (p) g.dp = decide_params(p, track);
    g.x = c->x;
    g.y = c->y;
    g.vpend = c->vpend;
    g.V = c->V;
    g.ldV = c->ldA;
    g.n = c->n;
    g.ldA = c->ldA;
    g.work = c->work;
    return g;
}

int stage_grid(const modap_ctx *c) { return (int)std::min<int64_t>(1024, (c->n + 255) / 256); }

// Working vectors of the next sweep from the committed state (call start).
modap_status enqueue_prime(modap_ctx *c, void *work, const double *x) {
    StageArgs g = stage_args(c, nullptr, 0, c->jn);
    g.x = const_cast<double *>(x);
    g.work = work;
    if (c->dt == 0)
        hipLaunchKernelGGL(prime_work<double>, dim3(stage_grid(c)), dim3(256), 0, c->stream, g);
    else
        hipLaunchKernelGGL(prime_work<float>, dim3(stage_grid(c)), dim3(256), 0, c->stream, g);
    LAUNCH_TRY(c, "prime_work launch");
    return MODAP_OK;
}

// Queue iteration i of a call: the sweep (which first settles the previous
// check, except in the first iteration of a call) at the current x on the
// current data, then the reduction of y (which makes the previous step
// permanent in x and writes the next sweep's working vectors).
modap_status enqueue_iteration(modap_ctx *c, const modap_params *p, int track, int64_t i, size_t *ev_used,
                               double *bytes) {
    const bool hv = translation_possible(c);
    const int64_t j = c->jn;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (p->profile > 0 && i % p->profile == 0) {
        if (!profile_events(c, *ev_used, ev)) return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
        *ev_used += 4;
    }
    SweepArgs a = sweep_args(c);
    a.b_out = c->b;
    a.pd.j = j;
    a.pd.decide = i > 0;   // the first sweep of a call runs under the committed state
    a.pd.dp = decide_params(p, track);
    a.check_status = 1;
    modap_status st;
    if ((st = launch_sweep(c, a, hv, ev[0], ev[1]))) return st;
    ReduceArgs r = reduce_args(c);
    r.y = c->y;
    r.ctl = c->ctl;
    r.j = j;
    r.iterate = 1;
    r.apply_step = i > 0;
    r.work = c->work;
    r.wsum = hv ? c->wsum : nullptr;   // no translation: nothing to add to the sum
    r.has_v = hv;
    if ((st = launch_reduce(c, r, ev[2], ev[3]))) return st;
    c->jn = j + 1;
    *bytes += sweep_bytes(c, hv);
    return MODAP_OK;
}

// End of a call that queued iterations: settle the last check (decision,
// step) with the stage kernel, so the committed state is in slot (jn-1)&1.
modap_status enqueue_settle(modap_ctx *c, const modap_params *p, int track) {
    StageArgs g = stage_args(c, p, track, c->jn - 1);
    if (c->dt == 0)
        hipLaunchKernelGGL(stage_iter<double>, dim3(stage_grid(c)), dim3(256), 0, c->stream, (const StageArgs)g);
    else
        hipLaunchKernelGGL(stage_iter<float>, dim3(stage_grid(c)), dim3(256), 0, c->stream, (const StageArgs)g);
    LAUNCH_TRY(c, "stage_iter launch");
    return MODAP_OK;
}

modap_status read_state(modap_ctx *c, State *out) {
    uint32_t bf[2] = {0, 0};
    HIP_TRY(c, hipMemcpyAsync(out, &c->ctl->st[last_slot(c)], sizeof(State), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(bf, &c->ctl->barrier, sizeof bf, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (bf[1])
        return fail(c, MODAP_E_DEVICE,
                    "a resident launch gave up waiting at a grid barrier; the context's data are void until set_system");
    return MODAP_OK;
}

void fill_stats(modap_stats *o, const State &k) {
    o->iters = k.steps;
    o->sweeps = k.sweeps;
    o->converged = k.feasible;
    o->state = k.status;
    o->max_viol = k.dmax;
    o->h = k.h;
    o->y_norm = k.ynorm;
    o->b_inf = k.binf;
    o->eps_abs = k.eps_abs;
    o->certified = k.certified;
    o->b_drift = k.bdrift;
}

modap_status profile_totals(modap_ctx *c, size_t ev_used, modap_stats *o) {
    double sw = 0.0, rd = 0.0;
    int64_t cnt = 0;
    for (size_t i = 0; i + 3 < ev_used; i += 4) {
        float a = 0.f, b = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&a, c->events[i], c->events[i + 1]));
        HIP_TRY(c, hipEventElapsedTime(&b, c->events[i + 2], c->events[i + 3]));
        sw += a;
        rd += b;
        ++cnt;
    }
    o->sweep_ms = sw;
    o->reduce_ms = rd;
    o->profiled = cnt;
    return MODAP_OK;
}

modap_status status_of(modap_ctx *c, const State &k, bool solve) {
    switch (k.status) {
        case ST_RUNNING:
        case ST_CONVERGED: return MODAP_OK;
        case ST_LIMIT: return solve ? fail(c, MODAP_E_NOT_CONVERGED, "step limit reached before eps-feasibility") : MODAP_OK;
        case ST_NO_DIRECTION: return fail(c, MODAP_E_INFEASIBLE, "a row is violated but y = 0: no step direction");
        case ST_NUMERIC: return fail(c, MODAP_E_NUMERIC, "NaN or infinity in the iteration");
        case ST_BAD_ROW: return fail(c, MODAP_E_ZERO_ROW, "a replaced row is zero, not finite, out of range or repeated");
        case ST_UNCERTIFIED:
            return fail(c, MODAP_E_NOT_CONVERGED, "the FP64 certificate cannot confirm the stop: eps_abs lies below "
                                                  "its rounding bound");
        default: return fail(c, MODAP_E_DEVICE, "unknown device state");
    }
}

void release_cert(modap_ctx *c) {
    free_dev(c->cert_wt);
    free_dev(c->cert_part);
    free_dev(c->cert_y);
    free_dev(c->cert_ynp);
    free_dev(c->cert_h);
    free_dev(c->cert_dmax);
    free_dev(c->cert_binf);
    free_dev(c->cert_drift);
    free_dev(c->cert_tot);
    c->cert_bands = 0;
}

void release_resident(modap_ctx *c) {
    free_dev(c->res_part);
    free_dev(c->res_h);
    free_dev(c->res_dmax);
    free_dev(c->res_binf);
    c->res_ok = false;
}

void release_system(modap_ctx *c) {
    release_cert(c);
    release_resident(c);
    free_dev(c->bref);
    free_dev(c->wsum);
    free_dev(c->claim);
    free_dev(c->A);
    free_dev(c->wrow);
    free_dev(c->b);
    free_dev(c->nu);
    free_dev(c->x);
    free_dev(c->y);
    free_dev(c->vpend);
    free_dev(c->V);
    free_dev(c->ynp);
    free_dev(c->work);
    free_dev(c->work_eval);
    free_dev(c->x_eval);
    free_dev(c->y_eval);
    free_dev(c->r_eval);
    c->T = 0;
    c->loaded = false;
}

modap_status launch_scatter(modap_ctx *c, int64_t k, const int64_t *rows, const void *new_rows, const double *nb) {
    HIP_TRY(c, aux_scatter_rows(c->dt, c->A, c->ldA, c->m, c->n, k, rows, new_rows, nb, c->b, c->bref, c->nu,
                                c->ctl, last_slot(c), c->vpend, c->V, c->ldA, c->wsum, c->stream));
    return MODAP_OK;
}

// Resident iteration (resident.hpp): systems whose rows hold at most 512
// elements and whose A, with rows padded to a multiple of 64 elements, fits
// in the LDS of at most kResidentMaxGrid workgroups at kResidentBand bytes
// each.  The grid is the larger of that minimum and one workgroup per
// kResidentRows rows (fewer rows per workgroup shorten the sweep; more
// workgroups lengthen the barrier).
constexpr int64_t kResidentBand = 96 * 1024;
constexpr int64_t kResidentRows = 32;
constexpr int64_t kResidentTimeoutTicks = 100000000;   // one second of the 100 MHz constant clock

modap_status plan_resident(modap_ctx *c) {
    release_resident(c);
    const int64_t ldR = (c->n + 63) / 64 * 64;
    if (ldR > kResidentMaxCols) return MODAP_OK;
    const int64_t row_bytes = ldR * (int64_t)c->es;
    const int64_t gmin = (c->m * row_bytes + kResidentBand - 1) / kResidentBand;
    if (gmin > kResidentMaxGrid) return MODAP_OK;
    int64_t rows_target = kResidentRows;
    if (const char *e = std::getenv("MODAP_RESIDENT_ROWS")) rows_target = std::max<int64_t>(4, std::atoll(e));
    int64_t grid = std::min<int64_t>(kResidentMaxGrid, std::max(gmin, (c->m + rows_target - 1) / rows_target));
    const int64_t rows = (c->m + grid - 1) / grid;
    grid = (c->m + rows - 1) / rows;
    const size_t lds = resident_lds_bytes(c->dt, (int)rows, (int)ldR);
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess ||
        lds + kResidentStaticLds > (size_t)max_lds)
        return MODAP_OK;
    const size_t acc = acc_size(c->dt);
    HIP_TRY(c, hipMalloc(&c->res_part, 2 * (size_t)kResidentMaxGrid * (size_t)ldR * acc));
    HIP_TRY(c, hipMalloc(&c->res_h, 2 * sizeof(int64_t) * (size_t)grid));
    HIP_TRY(c, hipMalloc(&c->res_dmax, 2 * sizeof(double) * (size_t)grid));
    HIP_TRY(c, hipMalloc(&c->res_binf, 2 * sizeof(double) * (size_t)grid));
    c->res_grid = (int)grid;
    c->res_rows = (int)rows;
    c->res_ldR = (int)ldR;
    c->res_lds = lds;
    c->res_ok = true;
    return MODAP_OK;
}

// The resident path runs unless the caller forced a tile of the two-kernel
// sweep, asked for per-iteration kernel timings, or set MODAP_RESIDENT=0.
bool use_resident(const modap_ctx *c, const modap_params *p) {
    if (!c->res_ok || c->tile_forced || p->profile > 0) return false;
    const char *e = std::getenv("MODAP_RESIDENT");
    return !(e && e[0] == '0');
}

// Queue K resident iterations from the committed state (the launch settles
// every check it makes, so no stage kernel follows).
modap_status launch_resident(modap_ctx *c, const modap_params *p, int track, int64_t K, double *bytes) {
    const bool hv = translation_possible(c);
    // (the arrival counters were cleared by the last workgroup of the previous
    // launch, or by set_system; the fault flag stays raised)
    ResidentArgs r{};
    r.A = c->A;
    r.ldA = c->ldA;
    r.m = c->m;
    r.n = c->n;
    r.ldR = c->res_ldR;
    r.rows = c->res_rows;
    r.b = c->b;
    r.nu = c->nu;
    r.x = c->x;
    r.y = c->y;
    r.wsum = c->wsum;
    r.vpend = c->vpend;
    r.V = c->V;
    r.ldV = c->ldA;
    r.work = c->work;
    r.ctl = c->ctl;
    r.j0 = c->jn;
    r.K = K;
    r.dp = decide_params(p, track);
    r.part = c->res_part;
    r.h_part = c->res_h;
    r.dmax_part = c->res_dmax;
    r.binf_part = c->res_binf;
    r.timeout_ticks = kResidentTimeoutTicks;
    if (const char *e = std::getenv("MODAP_RESIDENT_TIMEOUT_TICKS")) r.timeout_ticks = std::atoll(e);   // tests
    HIP_TRY(c, aux_resident_launch(c->dt, r, c->res_grid, c->res_lds, c->stream));
    c->jn += K;
    *bytes += (double)K * sweep_bytes(c, hv);
    return MODAP_OK;
}

// Scratch of the FP64 certificate: row bands of at least 256 rows, at most
// 128 bands (the band partials of y are FP64 rows of ldA).
modap_status ensure_cert(modap_ctx *c) {
    if (c->cert_bands > 0) return MODAP_OK;
    const int64_t rpb = std::max<int64_t>(256, (c->m + 127) / 128);
    const int bands = (int)((c->m + rpb - 1) / rpb);
    const int64_t gs = (c->m + 3) / 4;
    HIP_TRY(c, hipMalloc(&c->cert_wt, sizeof(double) * (size_t)c->m));
    HIP_TRY(c, hipMalloc(&c->cert_part, sizeof(double) * (size_t)bands * (size_t)c->ldA));
    HIP_TRY(c, hipMalloc(&c->cert_y, sizeof(double) * (size_t)c->ldA));
    HIP_TRY(c, hipMalloc(&c->cert_ynp, sizeof(double) * (size_t)reduce_grid(c)));
    HIP_TRY(c, hipMalloc(&c->cert_h, sizeof(int64_t) * (size_t)gs));
    HIP_TRY(c, hipMalloc(&c->cert_dmax, sizeof(double) * (size_t)gs));
    HIP_TRY(c, hipMalloc(&c->cert_binf, sizeof(double) * (size_t)gs));
    HIP_TRY(c, hipMalloc(&c->cert_drift, sizeof(double) * (size_t)gs));
    HIP_TRY(c, hipMalloc(&c->cert_tot, sizeof(Totals)));
    c->cert_rows_per_band = rpb;
    c->cert_bands = bands;
    return MODAP_OK;
}

// Queue the FP64 certificate of the committed state (a no-op on the device
// unless that state is an uncertified stop).
modap_status enqueue_certify(modap_ctx *c, const modap_params *p) {
    modap_status st;
    if ((st = ensure_cert(c))) return st;
    CertArgs v{};
    v.A = c->A;
    v.ldA = c->ldA;
    v.m = c->m;
    v.n = c->n;
    v.b = c->b;
    v.bref = c->bref;
    v.nu = c->nu;
    v.x = c->x;
    v.wsum = c->wsum;
    v.V = c->V;
    v.ldV = c->ldA;
    v.work = c->work;
    v.ctl = c->ctl;
    v.sl = last_slot(c);
    v.wt = c->cert_wt;
    v.h_part = c->cert_h;
    v.dmax_part = c->cert_dmax;
    v.binf_part = c->cert_binf;
    v.drift_part = c->cert_drift;
    v.bands = c->cert_bands;
    v.rows_per_band = c->cert_rows_per_band;
    v.part = c->cert_part;
    v.y = c->cert_y;
    v.ynp = c->cert_ynp;
    v.tot = c->cert_tot;
    v.dp = decide_params(p, 0);
    HIP_TRY(c, aux_certify(c->dt, v, c->stream));
    return MODAP_OK;
}

// Tuning cache: lines "dt ldA m block lanes_per_row chunks rows_per_step depth interleave grid".
const char *tune_cache_path() {
    const char *p = std::getenv("MODAP_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

bool cache_lookup(const modap_ctx *c, modap_tile *t) {
    const char *path = tune_cache_path();
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    long long dt, lda, m;
    int blk, lpr, ch, rs, depth, il, grid;
    bool found = false;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "%lld %lld %lld %d %d %d %d %d %d %d", &dt, &lda, &m, &blk, &lpr, &ch, &rs, &depth,
                        &il, &grid) != 10)
            continue;  // not a line of this format
        if (dt == c->dt && lda == c->ldA && m == c->m) {  // the last matching line wins
            t->kind = 0;
            t->block = blk;
            t->lanes_per_row = lpr;
            t->chunks = ch;
            t->rows_per_step = rs;
            t->depth = depth;
            t->interleave = il;
            t->grid = grid;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const modap_ctx *c, const modap_tile &t) {
    const char *path = tune_cache_path();
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%d %lld %lld %d %d %d %d %d %d %d\n", c->dt, (long long)c->ldA, (long long)c->m, t.block,
                 t.lanes_per_row, t.chunks, t.rows_per_step, t.depth, t.interleave, t.grid);
    std::fclose(f);
}

}  // namespace

extern "C" {

const char *modap_strerror(modap_status s) {
    switch (s) {
        case MODAP_OK: return "ok";
        case MODAP_E_INVAL: return "invalid argument";
        case MODAP_E_ZERO_ROW: return "zero or non-finite row";
        case MODAP_E_NOMEM: return "out of memory";
        case MODAP_E_DEVICE: return "device error";
        case MODAP_E_STATE: return "invalid state";
        case MODAP_E_NOT_CONVERGED: return "not converged within max_iters";
        case MODAP_E_INFEASIBLE: return "no step direction (infeasible system)";
        case MODAP_E_NUMERIC: return "non-finite value in the iteration";
        default: return "unknown status";
    }
}

const char *modap_last_error(modap_ctx *c) { return c ? c->err.c_str() : "null context"; }

modap_status modap_create(int device, void *hip_stream, modap_ctx **out) {
    if (!out) return MODAP_E_INVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return MODAP_E_DEVICE;
    if (device < 0 || device >= ndev) return MODAP_E_INVAL;
    modap_ctx *c = new (std::nothrow) modap_ctx();
    if (!c) return MODAP_E_NOMEM;
    c->device = device;
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MODAP_E_DEVICE;
    }
    c->cu_count = prop.multiProcessorCount;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);  // NULL: the device's default stream
    bool ok = hipMalloc(&c->ctl, sizeof(Ctrl)) == hipSuccess && hipMalloc(&c->tot, sizeof(Totals)) == hipSuccess &&
              hipMalloc(&c->bad, sizeof(unsigned long long)) == hipSuccess &&
              hipMalloc(&c->flag, sizeof(int)) == hipSuccess &&
              hipHostMalloc(&c->hst, 2 * sizeof(State), hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&c->sync_ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->sync_ev[1], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        modap_destroy(c);
        return MODAP_E_NOMEM;
    }
    hipLaunchKernelGGL(ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl);
    if (hipPeekAtLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        (void)hipGetLastError();
        modap_destroy(c);
        return MODAP_E_DEVICE;
    }
    *out = c;
    return MODAP_OK;
}

void modap_destroy(modap_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    release_system(c);
    free_dev(c->part);
    free_dev(c->pdot);
    free_dev(c->wrow);
    free_dev(c->h_part);
    free_dev(c->dmax_part);
    free_dev(c->binf_part);
    free_dev(c->ctl);
    free_dev(c->tot);
    free_dev(c->bad);
    free_dev(c->flag);
    free_dev(c->stage);
    if (c->hst) (void)hipHostFree(c->hst);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->sync_ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

modap_status modap_set_system(modap_ctx *c, int64_t m, int64_t n, modap_dtype storage, const void *A, int64_t lda,
                              const double *b, const double *x0, int on_dev) {
    TraceRange trace_("modap_set_system");
    modap_status st = check_ctx(c, false);
    if (st) return st;
    const char *msg = nullptr;
    if ((st = check_system(m, n, lda, A, b, (int)storage, &msg))) return fail(c, st, msg);
    if (!on_dev) {
        if (!all_finite(b, m)) return fail(c, MODAP_E_INVAL, "b has a non-finite entry");
        if (x0 && !all_finite(x0, n)) return fail(c, MODAP_E_INVAL, "x0 has a non-finite entry");
    }
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    release_system(c);
    c->dt = (int)storage;
    c->es = elem_size(c->dt);
    c->m = m;
    c->n = n;
    const int64_t v = vec_elems(c->dt);
    c->ldA = (n + v - 1) / v * v;
    c->vpend_maybe = false;
    c->jn = 0;
    const size_t abytes = (size_t)m * (size_t)c->ldA * c->es;
    HIP_TRY(c, hipMalloc(&c->A, abytes));
    HIP_TRY(c, hipMalloc(&c->b, sizeof(double) * m));
    HIP_TRY(c, hipMalloc(&c->bref, sizeof(double) * m));
    HIP_TRY(c, hipMalloc(&c->claim, sizeof(int) * m));
    HIP_TRY(c, hipMalloc(&c->nu, sizeof(double) * m));
    // x, y, the one-shot translation and the evaluation point are padded with
    // zeros to ldA so that the sweep reads whole 16-byte vectors of them.
    const size_t vbytes = sizeof(double) * (size_t)c->ldA;
    HIP_TRY(c, hipMalloc(&c->x, vbytes));
    HIP_TRY(c, hipMalloc(&c->y, vbytes));
    HIP_TRY(c, hipMalloc(&c->vpend, vbytes));
    HIP_TRY(c, hipMalloc(&c->wsum, vbytes));
    HIP_TRY(c, hipMalloc(&c->x_eval, vbytes));
    HIP_TRY(c, hipMalloc(&c->y_eval, vbytes));
    const size_t wbytes = 3 * acc_size(c->dt) * (size_t)c->ldA;
    HIP_TRY(c, hipMalloc(&c->work, wbytes));
    HIP_TRY(c, hipMalloc(&c->work_eval, wbytes));
    HIP_TRY(c, hipMemsetAsync(c->work, 0, wbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->work_eval, 0, wbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->x, 0, vbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->x_eval, 0, vbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->y_eval, 0, vbytes, c->stream));
    HIP_TRY(c, hipMalloc(&c->r_eval, sizeof(double) * m));
    HIP_TRY(c, hipMalloc(&c->ynp, sizeof(double) * (size_t)reduce_grid(c)));
    if (c->ldA != n) HIP_TRY(c, hipMemsetAsync(c->A, 0, abytes, c->stream));
    HIP_TRY(c, hipMemcpy2DAsync(c->A, (size_t)c->ldA * c->es, A, (size_t)lda * c->es, (size_t)n * c->es, (size_t)m,
                                on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    if ((st = to_device(c, c->b, b, sizeof(double) * m, on_dev))) return st;
    if (x0 && (st = to_device(c, c->x, x0, sizeof(double) * n, on_dev))) return st;
    HIP_TRY(c, hipMemsetAsync(c->y, 0, vbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->vpend, 0, vbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->wsum, 0, vbytes, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->claim, 0, sizeof(int) * m, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->bref, c->b, sizeof(double) * m, hipMemcpyDeviceToDevice, c->stream));
    const unsigned long long none = ULLONG_MAX;
    HIP_TRY(c, hipMemcpyAsync(c->bad, &none, sizeof none, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
    const int nb = (int)((m + 3) / 4);
    switch (c->dt) {
        case 0: hipLaunchKernelGGL(row_norms<0>, dim3(nb), dim3(256), 0, c->stream, (const void *)c->A, c->ldA, m, n, c->nu, c->bad); break;
        case 1: hipLaunchKernelGGL(row_norms<1>, dim3(nb), dim3(256), 0, c->stream, (const void *)c->A, c->ldA, m, n, c->nu, c->bad); break;
        default: hipLaunchKernelGGL(row_norms<2>, dim3(nb), dim3(256), 0, c->stream, (const void *)c->A, c->ldA, m, n, c->nu, c->bad); break;
    }
    LAUNCH_TRY(c, "row_norms launch");
    if (on_dev) {
        hipLaunchKernelGGL(check_finite, dim3(64), dim3(256), 0, c->stream, (const double *)c->b, m, c->flag);
        hipLaunchKernelGGL(check_finite, dim3(64), dim3(256), 0, c->stream, (const double *)c->x, n, c->flag);
        LAUNCH_TRY(c, "check_finite launch");
    }
    hipLaunchKernelGGL(ctl_init, dim3(1), dim3(64), 0, c->stream, c->ctl);
    LAUNCH_TRY(c, "ctl_init launch");
    unsigned long long bad = 0;
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, c->bad, sizeof bad, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (flag) {
        release_system(c);
        return fail(c, MODAP_E_INVAL, "b or x0 has a non-finite entry");
    }
    if (bad != ULLONG_MAX) {
        release_system(c);
        return fail(c, MODAP_E_ZERO_ROW, "row " + std::to_string(bad) + " is zero or not finite");
    }
    modap_tile t{};
    bool ok = false;
    if (c->tile_forced) {
        t = c->tile;
        t.grid = 0;
        ok = configure(c, t) == MODAP_OK;
    }
    if (!ok && cache_lookup(c, &t)) ok = configure(c, t) == MODAP_OK;
    if (!ok) {
        if (!choose_shape(c->dt, c->ldA, &t)) {
            release_system(c);
            return fail(c, MODAP_E_INVAL, "rows too long for the one-pass sweep shapes");
        }
        c->tile_forced = false;
        if ((st = configure(c, t))) {
            release_system(c);
            return st;
        }
    }
    if ((st = plan_resident(c))) {
        release_system(c);
        return st;
    }
    c->loaded = true;
    c->err.clear();
    return MODAP_OK;
}

modap_status modap_set_x(modap_ctx *c, const double *x, int on_dev) {
    TraceRange trace_("modap_set_x");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if (x && !on_dev && !all_finite(x, c->n)) return fail(c, MODAP_E_INVAL, "x has a non-finite entry");
    DeviceGuard g(c->device);
    if (x) {
        if ((st = to_device(c, c->x, x, sizeof(double) * c->n, on_dev))) return st;
    } else {
        HIP_TRY(c, hipMemsetAsync(c->x, 0, sizeof(double) * c->ldA, c->stream));
    }
    hipLaunchKernelGGL(ctl_restart, dim3(1), dim3(64), 0, c->stream, c->ctl, last_slot(c));
    LAUNCH_TRY(c, "ctl_restart launch");
    return MODAP_OK;
}

modap_status modap_update_coeffs(modap_ctx *c, int64_t k, const int64_t *rows, const void *new_rows,
                                 const double *new_b, const double *v, int on_dev) {
    TraceRange trace_("modap_update_coeffs");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    const char *msg = nullptr;
    if (k < 0 || k > c->m) return fail(c, MODAP_E_INVAL, "k out of range");
    if (k > 0 && (!rows || !new_rows || !new_b)) return fail(c, MODAP_E_INVAL, "rows, new_rows and new_b are required");
    DeviceGuard g(c->device);
    const size_t rbytes = (size_t)k * (size_t)c->n * c->es;
    if (k > 0 && !on_dev) {
        if ((st = check_rows(k, rows, new_rows, new_b, c->m, &msg))) return fail(c, st, msg);
        if ((st = check_new_rows(c->dt, new_rows, k, c->n, &msg))) return fail(c, st, msg);
    }
    if (v && !on_dev && !all_finite(v, c->n)) return fail(c, MODAP_E_INVAL, "translation has a non-finite entry");
    const int64_t *d_rows = rows;
    const void *d_new = new_rows;
    const double *d_b = new_b;
    const double *d_v = v;
    if (!on_dev) {
        const size_t o1 = 0, o2 = o1 + (size_t)k * 8, o3 = (o2 + rbytes + 15) / 16 * 16, o4 = o3 + (size_t)k * 8;
        const size_t total = o4 + (v ? (size_t)c->n * 8 : 0);
        if ((st = ensure_stage(c, total + 16))) return st;
        char *s = reinterpret_cast<char *>(c->stage);
        if (k > 0) {
            if ((st = to_device(c, s + o1, rows, (size_t)k * 8, 0))) return st;
            if ((st = to_device(c, s + o2, new_rows, rbytes, 0))) return st;
            if ((st = to_device(c, s + o3, new_b, (size_t)k * 8, 0))) return st;
        }
        if (v && (st = to_device(c, s + o4, v, (size_t)c->n * 8, 0))) return st;
        d_rows = reinterpret_cast<const int64_t *>(s + o1);
        d_new = s + o2;
        d_b = reinterpret_cast<const double *>(s + o3);
        d_v = v ? reinterpret_cast<const double *>(s + o4) : nullptr;
    }
    if (k > 0 && on_dev) HIP_TRY(c, aux_claim_rows(d_rows, k, c->m, c->claim, c->ctl, last_slot(c), c->stream));
    if (k > 0 && (st = launch_scatter(c, k, d_rows, d_new, d_b))) return st;
    if (k > 0 && on_dev) HIP_TRY(c, aux_release_rows(d_rows, k, c->m, c->claim, c->stream));
    if (d_v) {
        hipLaunchKernelGGL(vpend_add, dim3(1), dim3(1024), 0, c->stream, c->ctl, last_slot(c), c->vpend, d_v, c->n);
        LAUNCH_TRY(c, "vpend_add launch");
        c->vpend_maybe = true;
    }
    return MODAP_OK;
}

modap_status modap_set_drift(modap_ctx *c, int64_t T, const double *V, int64_t ldv, int on_dev) {
    TraceRange trace_("modap_set_drift");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    const char *msg = nullptr;
    if ((st = check_drift(T, V, ldv, c->n, !on_dev, &msg))) return fail(c, st, msg);
    DeviceGuard g(c->device);
    const int sl = last_slot(c);
    if (c->V) {
        hipLaunchKernelGGL(sched_to_vpend, dim3(1), dim3(1024), 0, c->stream, c->ctl, sl, c->vpend,
                           (const double *)c->V, c->ldA, c->n);
        LAUNCH_TRY(c, "sched_to_vpend launch");
        c->vpend_maybe = true;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_dev(c->V);
    c->T = 0;
    if (T > 0 && V) {
        // rows padded with zeros to ldA, like x
        const size_t vb = sizeof(double) * (size_t)T * (size_t)c->ldA;
        HIP_TRY(c, hipMalloc(&c->V, vb));
        HIP_TRY(c, hipMemsetAsync(c->V, 0, vb, c->stream));
        HIP_TRY(c, hipMemcpy2DAsync(c->V, sizeof(double) * c->ldA, V, sizeof(double) * ldv, sizeof(double) * c->n,
                                    (size_t)T, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
        c->T = T;
    }
    if (on_dev && c->T > 0) {
        HIP_TRY(c, hipMemsetAsync(c->flag, 0, sizeof(int), c->stream));
        hipLaunchKernelGGL(check_finite, dim3(64), dim3(256), 0, c->stream, (const double *)c->V, c->T * c->ldA, c->flag);
        int flag = 0;
        HIP_TRY(c, hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (flag) {
            free_dev(c->V);
            c->T = 0;
            hipLaunchKernelGGL(ctl_set_drift, dim3(1), dim3(64), 0, c->stream, c->ctl, sl, (int64_t)0);
            return fail(c, MODAP_E_INVAL, "drift has a non-finite entry");
        }
    }
    hipLaunchKernelGGL(ctl_set_drift, dim3(1), dim3(64), 0, c->stream, c->ctl, sl, c->T);
    LAUNCH_TRY(c, "ctl_set_drift launch");
    return MODAP_OK;
}

modap_status modap_iterate(modap_ctx *c, const modap_params *p, int64_t k, modap_stats *out) {
    TraceRange trace_("modap_iterate");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if ((st = check_params(c, p))) return st;
    if (k < 0) return fail(c, MODAP_E_INVAL, "k < 0");
    DeviceGuard g(c->device);
    const auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(ctl_begin, dim3(1), dim3(64), 0, c->stream, c->ctl, last_slot(c), (int64_t)-1);
    LAUNCH_TRY(c, "ctl_begin launch");
    size_t ev = 0;
    double bytes = 0.0;
    const int track = p->track != 0;
    if (use_resident(c, p)) {
        // one launch of many iterations (each launch settles its own checks)
        for (int64_t done = 0; done < k;) {
            const int64_t K = std::min<int64_t>(k - done, int64_t(1) << 20);
            if ((st = launch_resident(c, p, track, K, &bytes))) return st;
            done += K;
        }
    } else {
        if ((st = enqueue_prime(c, c->work, c->x))) return st;
        if ((st = reserve_events(c, k, p->profile))) return st;
        for (int64_t i = 0; i < k; ++i)
            if ((st = enqueue_iteration(c, p, track, i, &ev, &bytes))) return st;
        if (k > 0 && (st = enqueue_settle(c, p, track))) return st;
    }
    if (k > 0 && p->certify && (st = enqueue_certify(c, p))) return st;
    if (!out) return MODAP_OK;
    State kc;
    if ((st = read_state(c, &kc))) return st;
    *out = modap_stats{};
    fill_stats(out, kc);
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out->hbm_bytes = bytes;
    out->resident = use_resident(c, p) ? 1 : 0;
    if (p->profile && (st = profile_totals(c, ev, out))) return st;
    if (!kc.vpend_valid && kc.v_idx < 0) c->vpend_maybe = false;
    return status_of(c, kc, false);
}

modap_status modap_solve(modap_ctx *c, const modap_params *p, modap_stats *out) {
    TraceRange trace_("modap_solve");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if ((st = check_params(c, p))) return st;
    DeviceGuard g(c->device);
    const auto t0 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(ctl_begin, dim3(1), dim3(64), 0, c->stream, c->ctl, last_slot(c), (int64_t)p->max_iters);
    LAUNCH_TRY(c, "ctl_begin launch");
    const bool resident = use_resident(c, p);
    if (!resident && (st = enqueue_prime(c, c->work, c->x))) return st;
    const int64_t total = p->max_iters + 1;  // the last sweep checks the last step
    if (!resident && (st = reserve_events(c, std::min<int64_t>(total, 4096), p->profile))) return st;
    size_t ev = 0;
    double bytes = 0.0;
    auto observed = t0;
    State kc;
    // Passes of queued iterations until the device stops; a stop at
    // eps-feasibility that the FP64 certificate does not confirm has taken a
    // step instead, and the next pass goes on from there.  The step limit is
    // the device's, so a pass may queue more iterations than remain.  The host
    // reads the state of the chunk before the newest one, so the device never
    // waits for it.
    for (;;) {
        int64_t queued = 0, chunk = resident ? 16 : 1;
        int slot = 0, pending = -1;
        bool done = false;
        while (queued < total && !done) {
            TraceRange trace_chunk("modap_solve chunk");
            const int64_t cnt = std::min(chunk, total - queued);
            if (resident) {
                if ((st = launch_resident(c, p, 0, cnt, &bytes))) return st;
            } else {
                for (int64_t i = 0; i < cnt; ++i)
                    if ((st = enqueue_iteration(c, p, 0, queued + i, &ev, &bytes))) return st;
            }
            queued += cnt;
            // the newest settled state: the check before the last queued sweep
            // (two-kernel path), or the last check of the launch (resident path)
            HIP_TRY(c, hipMemcpyAsync(&c->hst[slot], &c->ctl->st[slot_of(c->jn - (resident ? 1 : 2))], sizeof(State),
                                      hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(c, hipEventRecord(c->sync_ev[slot], c->stream));
            if (pending >= 0) {
                HIP_TRY(c, hipEventSynchronize(c->sync_ev[pending]));
                if (c->hst[pending].status != ST_RUNNING) done = true;
            }
            pending = slot;
            slot ^= 1;
            chunk = std::min<int64_t>(chunk * 2, resident ? 1024 : 64);
        }
        if (!resident && (st = enqueue_settle(c, p, 0))) return st;
        if ((st = read_state(c, &kc))) return st;
        observed = std::chrono::steady_clock::now();
        if (!(p->certify && kc.status == ST_CONVERGED && !kc.certified)) break;
        if ((st = enqueue_certify(c, p))) return st;
        if ((st = read_state(c, &kc))) return st;
        bytes += sweep_bytes(c, false);
        observed = std::chrono::steady_clock::now();
        if (kc.status != ST_RUNNING) break;
    }
    if (out) {
        *out = modap_stats{};
        fill_stats(out, kc);
        out->seconds = std::chrono::duration<double>(observed - t0).count();
        out->hbm_bytes = bytes;
        out->resident = resident ? 1 : 0;
        if (p->profile && (st = profile_totals(c, ev, out))) return st;
    }
    if (!kc.vpend_valid && kc.v_idx < 0) c->vpend_maybe = false;
    if (kc.status == ST_RUNNING) return fail(c, MODAP_E_NOT_CONVERGED, "step limit reached before eps-feasibility");
    return status_of(c, kc, true);
}

modap_status modap_eval_sweep(modap_ctx *c, const double *x, double *r, double *y, int64_t *h, double *max_viol,
                              int on_dev) {
    TraceRange trace_("modap_eval_sweep");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if (!x || !y) return fail(c, MODAP_E_INVAL, "x and y are required");
    DeviceGuard g(c->device);
    if ((st = to_device(c, c->x_eval, x, sizeof(double) * c->n, on_dev))) return st;
    if ((st = enqueue_prime(c, c->work_eval, c->x_eval))) return st;
    const bool hv = translation_possible(c);
    SweepArgs a = sweep_args(c);
    a.b_out = nullptr;
    a.work = c->work_eval;
    a.check_status = 0;
    a.r_out = r ? c->r_eval : nullptr;
    if ((st = launch_sweep(c, a, hv, nullptr, nullptr))) return st;
    ReduceArgs ra = reduce_args(c);
    ra.y = c->y_eval;
    ra.ctl = nullptr;
    ra.iterate = 0;
    if ((st = launch_reduce(c, ra))) return st;
    Totals to;
    HIP_TRY(c, hipMemcpyAsync(&to, c->tot, sizeof to, hipMemcpyDeviceToHost, c->stream));
    if ((st = from_device(c, y, c->y_eval, sizeof(double) * c->n, on_dev))) return st;
    if (r && (st = from_device(c, r, c->r_eval, sizeof(double) * c->m, on_dev))) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (h) *h = to.h;
    if (max_viol) *max_viol = to.dmax;
    return MODAP_OK;
}

modap_status modap_query(modap_ctx *c, double *x, double *b, modap_stats *out, int on_dev) {
    TraceRange trace_("modap_query");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    DeviceGuard g(c->device);
    if (x && (st = from_device(c, x, c->x, sizeof(double) * c->n, on_dev))) return st;
    if (b) {
        // the data as the caller sees them, every translation applied, in FP64;
        // nothing is committed, so reading b does not change the iteration
        HIP_TRY(c, aux_rhs_exact(c->dt, c->A, c->ldA, c->m, c->n, c->ctl, last_slot(c), c->bref, c->wsum, c->vpend,
                                 c->V, c->ldA, c->r_eval, c->stream));
        if ((st = from_device(c, b, c->r_eval, sizeof(double) * c->m, on_dev))) return st;
    }
    State kc;
    if ((st = read_state(c, &kc))) return st;
    if (out) {
        *out = modap_stats{};
        fill_stats(out, kc);
    }
    return MODAP_OK;
}

modap_status modap_set_tile(modap_ctx *c, const modap_tile *t) {
    if (!c) return MODAP_E_INVAL;
    DeviceGuard g(c->device);
    if (!t) {
        c->tile_forced = false;
        if (!c->loaded) return MODAP_OK;
        modap_tile d{};
        if (!choose_shape(c->dt, c->ldA, &d)) return fail(c, MODAP_E_INVAL, "no built-in shape");
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return configure(c, d);
    }
    if (!c->loaded) {
        c->tile = *t;
        c->tile_forced = true;
        return MODAP_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const modap_tile keep = c->tile;
    modap_status st = configure(c, *t);
    if (st) {
        const std::string msg = c->err;
        (void)configure(c, keep);
        return fail(c, st, msg);
    }
    c->tile_forced = true;
    return MODAP_OK;
}

modap_status modap_autotune(modap_ctx *c, int reps, modap_tile *best) {
    TraceRange trace_("modap_autotune");
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if (reps < 1) return fail(c, MODAP_E_INVAL, "reps < 1");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const modap_tile keep = c->tile;
    const bool hv = translation_possible(c);
    if (!event_at(c, 2 * (size_t)reps - 1)) return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
    if ((st = enqueue_prime(c, c->work_eval, c->x))) return st;
    int cnt = 0;
    const SweepKernel *tab = kernels_for(c->dt, &cnt);
    modap_tile win = keep;
    float win_ms = 1e30f;
    std::vector<float> times;
    // The built-in shape is timed first, and a challenger must beat the
    // incumbent by kMargin: near-equal shapes do not flip with timing noise.
    constexpr float kMargin = 0.98f;
    std::vector<modap_tile> order;
    modap_tile def{};
    if (choose_shape(c->dt, c->ldA, &def) && def.kind == 0) order.push_back(def);
    for (int i = 0; i < cnt; ++i) {
        if (tab[i].has_v != hv) continue;
        if (coverage(c->dt, tab[i].lpr, tab[i].chunks) < c->ldA) continue;
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tab[i].func, tab[i].block, 0) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        for (int trial = 0; trial < 2 * std::max(2, per_cu); ++trial) {
            const int mult = trial / 2 + 1, il = trial % 2;
            modap_tile t{0, tab[i].block, tab[i].lpr, tab[i].chunks, c->cu_count * mult, tab[i].rs, tab[i].pd, il};
            if (mult > 1 && mult != per_cu && mult != 2) continue;
            order.push_back(t);
        }
    }
    for (const modap_tile &t : order) {
        if (configure(c, t) != MODAP_OK) continue;
        SweepArgs a = sweep_args(c);
        a.b_out = nullptr;
        a.work = c->work_eval;
        a.check_status = 0;
        const SweepKernel *k = hv ? c->kern_v : c->kern_nov;
        // an untimed sweep, then `reps` timed ones back to back (as the
        // iterations run; a host wait after each would leave the device idle
        // between them); the shortest counts, the work being the same each time
        HIP_TRY(c, k->launch(a, c->tile.grid, c->stream, nullptr, nullptr));
        for (int r = 0; r < reps; ++r)
            HIP_TRY(c, k->launch(a, c->tile.grid, c->stream, event_at(c, 2 * (size_t)r), event_at(c, 2 * (size_t)r + 1)));
        HIP_TRY(c, hipEventSynchronize(event_at(c, 2 * (size_t)reps - 1)));
        times.clear();
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&ms, event_at(c, 2 * (size_t)r), event_at(c, 2 * (size_t)r + 1)));
            times.push_back(ms);
        }
        const float best_ms = *std::min_element(times.begin(), times.end());
        if (best_ms < win_ms * kMargin || win_ms == 1e30f) {
            win_ms = best_ms;
            win = c->tile;
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
    }
    if ((st = configure(c, win))) {
        (void)configure(c, keep);
        return st;
    }
    c->tile_forced = true;
    cache_store(c, c->tile);
    if (best) *best = c->tile;
    return MODAP_OK;
}

modap_status modap_get_tile(modap_ctx *c, modap_tile *t) {
    modap_status st = check_ctx(c, true);
    if (st) return st;
    if (!t) return fail(c, MODAP_E_INVAL, "tile is NULL");
    *t = c->tile;
    return MODAP_OK;
}

}  // extern "C"

// Launchers of the auxiliary kernels for the other translation units.
namespace modap {

hipError_t aux_row_norms(int dt, const void *A, int64_t ldA, int64_t m, int64_t n, double *nu,
                         unsigned long long *bad, hipStream_t s) {
    const int nb = (int)((m + 3) / 4);
    switch (dt) {
        case 0: hipLaunchKernelGGL(row_norms<0>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, nu, bad); break;
        case 1: hipLaunchKernelGGL(row_norms<1>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, nu, bad); break;
        default: hipLaunchKernelGGL(row_norms<2>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, nu, bad); break;
    }
    return hipPeekAtLastError();
}

hipError_t aux_check_finite(const double *p, int64_t count, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(check_finite, dim3(64), dim3(256), 0, s, p, count, flag);
    return hipPeekAtLastError();
}

hipError_t aux_ctl_init(Ctrl *c, hipStream_t s) {
    hipLaunchKernelGGL(ctl_init, dim3(1), dim3(64), 0, s, c);
    return hipPeekAtLastError();
}

hipError_t aux_scatter_rows(int dt, void *A, int64_t ldA, int64_t m, int64_t n, int64_t k, const int64_t *rows,
                            const void *new_rows, const double *new_b, double *b, double *bref, double *nu, Ctrl *ctl,
                            int sl, const double *vpend, const double *V, int64_t ldV, const double *wsum,
                            hipStream_t s) {
    switch (dt) {
        case 0: hipLaunchKernelGGL(scatter_rows<0>, dim3(k), dim3(256), 0, s, A, ldA, m, n, rows, new_rows, new_b, b, bref, nu, ctl, sl, vpend, V, ldV, wsum); break;
        case 1: hipLaunchKernelGGL(scatter_rows<1>, dim3(k), dim3(256), 0, s, A, ldA, m, n, rows, new_rows, new_b, b, bref, nu, ctl, sl, vpend, V, ldV, wsum); break;
        default: hipLaunchKernelGGL(scatter_rows<2>, dim3(k), dim3(256), 0, s, A, ldA, m, n, rows, new_rows, new_b, b, bref, nu, ctl, sl, vpend, V, ldV, wsum); break;
    }
    return hipPeekAtLastError();
}

hipError_t aux_claim_rows(const int64_t *rows, int64_t k, int64_t m, int *claim, Ctrl *ctl, int sl, hipStream_t s) {
    const int grid = (int)std::min<int64_t>(1024, (k + 255) / 256);
    hipLaunchKernelGGL(claim_rows, dim3(grid), dim3(256), 0, s, rows, k, m, claim, ctl, sl);
    return hipPeekAtLastError();
}

hipError_t aux_release_rows(const int64_t *rows, int64_t k, int64_t m, int *claim, hipStream_t s) {
    const int grid = (int)std::min<int64_t>(1024, (k + 255) / 256);
    hipLaunchKernelGGL(release_rows, dim3(grid), dim3(256), 0, s, rows, k, m, claim);
    return hipPeekAtLastError();
}

hipError_t aux_vpend_add(Ctrl *c, int sl, double *vpend, const double *v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(vpend_add, dim3(1), dim3(1024), 0, s, c, sl, vpend, v, n);
    return hipPeekAtLastError();
}

hipError_t aux_sched_to_vpend(Ctrl *c, int sl, double *vpend, const double *V, int64_t ldV, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(sched_to_vpend, dim3(1), dim3(1024), 0, s, c, sl, vpend, V, ldV, n);
    return hipPeekAtLastError();
}

hipError_t aux_ctl_set_drift(Ctrl *c, int sl, int64_t T, hipStream_t s) {
    hipLaunchKernelGGL(ctl_set_drift, dim3(1), dim3(64), 0, s, c, sl, T);
    return hipPeekAtLastError();
}

hipError_t aux_rhs_exact(int dt, const void *A, int64_t ldA, int64_t m, int64_t n, const Ctrl *ctl, int sl,
                         const double *bref, const double *wsum, const double *vpend, const double *V, int64_t ldV,
                         double *out, hipStream_t s) {
    const int nb = (int)((m + 3) / 4);
    switch (dt) {
        case 0: hipLaunchKernelGGL(rhs_exact<0>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, ctl, sl, bref, wsum, vpend, V, ldV, out); break;
        case 1: hipLaunchKernelGGL(rhs_exact<1>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, ctl, sl, bref, wsum, vpend, V, ldV, out); break;
        default: hipLaunchKernelGGL(rhs_exact<2>, dim3(nb), dim3(256), 0, s, A, ldA, m, n, ctl, sl, bref, wsum, vpend, V, ldV, out); break;
    }
    return hipPeekAtLastError();
}

bool static_sweep_plan(int dt, int64_t ldA, int64_t m, int64_t n, int cu_count, StaticPlan *out) {
    modap_tile t{};
    if (!choose_shape(dt, ldA, &t) || t.kind != 0) return false;
    const SweepKernel *k = find_kernel(dt, t.block, t.lanes_per_row, t.chunks, t.rows_per_step, t.depth, false);
    if (!k) return false;
    // the row mapping of configure() for a band of rows per workgroup
    const int per_step = (t.block / t.lanes_per_row) * t.rows_per_step;
    int grid = std::max(1, cu_count);
    int64_t rpb = (m + grid - 1) / grid;
    rpb = ((rpb + per_step - 1) / per_step) * per_step;
    grid = (int)((m + rpb - 1) / rpb);
    out->k = k;
    out->grid = grid;
    out->R = (int)((n + 63) / 64);
    out->cov = coverage(dt, t.lanes_per_row, t.chunks);
    out->rows_per_block = rpb;
    out->block_stride = rpb;
    out->step_stride = per_step;
    return true;
}

hipError_t static_sweep_launch(int dt, const StaticPlan &plan, const SweepScratch &s, const void *A, int64_t ldA,
                               int64_t m, int64_t n, const double *b, const double *x, double *r, double *y,
                               int64_t *h, double *max_viol, hipStream_t stream) {
    hipLaunchKernelGGL(ctl_init, dim3(1), dim3(64), 0, stream, s.ctl);
    hipError_t e = aux_row_norms(dt, A, ldA, m, n, s.nu, s.bad, stream);
    if (e != hipSuccess) return e;
    const int sg = (int)std::min<int64_t>(1024, (ldA + 255) / 256);
    if (dt == 0)
        hipLaunchKernelGGL(stage_point<double>, dim3(sg), dim3(256), 0, stream, x, n, ldA, s.work);
    else
        hipLaunchKernelGGL(stage_point<float>, dim3(sg), dim3(256), 0, stream, x, n, ldA, s.work);
    SweepArgs a{};
    a.A = A;
    a.ldA = ldA;
    a.m = m;
    a.n = n;
    a.b_in = b;
    a.b_out = nullptr;
    a.nu = s.nu;
    a.work = s.work;
    a.pd.ctl = s.ctl;
    a.pd.j = 1;          // runs under the fresh state in slot 0
    a.pd.decide = 0;
    a.check_status = 0;
    a.r_out = r;
    a.part = s.part;
    a.ldPart = plan.cov;
    a.h_part = s.h_part;
    a.dmax_part = s.dmax_part;
    a.binf_part = s.binf_part;
    a.rows_per_block = plan.rows_per_block;
    a.block_stride = plan.block_stride;
    a.step_stride = plan.step_stride;
    if ((e = plan.k->launch(a, plan.grid, stream, nullptr, nullptr)) != hipSuccess) return e;
    ReduceArgs ra{};
    ra.part = s.part;
    ra.ldPart = plan.cov;
    ra.G = plan.grid;
    ra.acc_f64 = dt == 0;
    ra.Gs = plan.grid;
    ra.n = n;
    ra.ldA = ldA;
    ra.y = y;
    ra.h_part = s.h_part;
    ra.dmax_part = s.dmax_part;
    ra.binf_part = s.binf_part;
    ra.tot = s.tot;
    ra.ynp = s.ynp;
    if (dt == 0)
        hipLaunchKernelGGL(reduce_y<double>, dim3(plan.R), dim3(kReduceThreads), 0, stream, ra);
    else
        hipLaunchKernelGGL(reduce_y<float>, dim3(plan.R), dim3(kReduceThreads), 0, stream, ra);
    hipLaunchKernelGGL(copy_totals, dim3(1), dim3(64), 0, stream, (const Totals *)s.tot, h, max_viol);
    return hipPeekAtLastError();
}

template <int DT>
static void launch_cert(CertArgs a, hipStream_t s) {
    using Acc = typename Store<DT>::Acc;
    constexpr int VEC = Store<DT>::VEC;
    const int tiles = (int)((a.ldA + 256 * VEC - 1) / (256 * VEC));
    hipLaunchKernelGGL(cert_dot<DT>, dim3(a.Gs), dim3(256), 0, s, a);
    hipLaunchKernelGGL(cert_axpy<DT>, dim3(a.bands, tiles), dim3(256), 0, s, a);
    hipLaunchKernelGGL(cert_reduce, dim3(a.R), dim3(256), 0, s, a);
    hipLaunchKernelGGL(cert_decide<Acc>, dim3(1), dim3(1024), 0, s, a);
}

hipError_t aux_certify(int dt, CertArgs a, hipStream_t s) {
    a.R = (int32_t)((a.n + 63) / 64);
    a.Gs = (int32_t)((a.m + 3) / 4);
    switch (dt) {
        case 0: launch_cert<0>(a, s); break;
        case 1: launch_cert<1>(a, s); break;
        default: launch_cert<2>(a, s); break;
    }
    return hipPeekAtLastError();
}

}  // namespace modap
