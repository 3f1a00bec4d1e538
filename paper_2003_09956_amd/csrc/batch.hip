// Host half of the batched C ABI (modap_batch_* in include/modap.h) and the
// instantiation of the batch kernels.
//
// A batch owns, per system, the same device data as a single-system context
// (rows padded to a 16-byte multiple, b, ||a_i||^2, x, y, the one-shot
// translation, the drift schedule, the working vectors, a control block, the
// totals and the norm parts of y), and for the whole batch the tables the
// kernels read: one descriptor per system, the system of every work item,
// the 64-column blocks of the reduction, the per-item partials and the item
// queue.  The tables are rebuilt at the start of a call after systems were
// added or removed or the tuning changed.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "aux_launch.hpp"
#include "batch_kernels.hpp"
#include "host_common.hpp"
#include "trace.hpp"
#include "batch_plan.hpp"
#include "internal.hpp"
#include "modap.h"

using namespace modap;
using namespace modap_host;

namespace {

struct BSys {
    bool alive = false;
    int64_t m = 0, n = 0, ldA = 0;
    void *A = nullptr;
    double *b = nullptr, *nu = nullptr, *x = nullptr, *y = nullptr, *vpend = nullptr, *V = nullptr;
    double *bref = nullptr, *wsum = nullptr;   // the data are bref + A wsum (see certify.hpp)
    int64_t T = 0;
    void *work = nullptr;
    Ctrl *ctl = nullptr;
    Totals *tot = nullptr;
    double *ynp = nullptr;
    int C = 0;
    bool vpend_maybe = false;
};

constexpr int kBuckets[4] = {1, 2, 4, 8};

}  // namespace

// The untuned tile, near what the autotuner finds on FP32 families with rows
// up to 2048 elements: items of up to 0.5 / 2 / 4 / 8 MiB for the four
// row-length buckets, one workgroup per CU.  On the 512-system family, 8 MiB
// items for the longest rows took the sweep from 2.51 to 2.48 ms (fewer items,
// each with a cost of its own; the largest are handed out first, so they do
// not end the sweep late).
constexpr modap_batch_tile kBuiltinTile{{512, 2048, 4096, 8192}, 0, 0};

struct modap_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    int cu_count = 0;
    int per_cu = 0;         // sweep_batch workgroups resident per CU (0: not asked yet)
    std::string err;
    int dt = 1;
    size_t es = 4;
    std::vector<BSys> sys;
    int64_t jn = 0;
    modap_batch_tile tile = kBuiltinTile;

    // tables of the current membership (rebuilt when dirty)
    bool dirty = true;
    std::vector<int32_t> order;            // alive system ids in table order
    std::vector<BatchSys> h_sys;
    std::vector<int32_t> h_item_sys;
    std::vector<int32_t> h_item_order;     // items by decreasing size (queue order)
    std::vector<BatchCol> h_cols;
    BatchSys *d_sys = nullptr;
    size_t sys_cap = 0;
    int32_t *d_item_sys = nullptr;
    size_t item_cap = 0;
    int32_t *d_item_order = nullptr;
    size_t order_cap = 0;
    BatchCol *d_cols = nullptr;
    size_t cols_cap = 0;
    void *part = nullptr;
    size_t part_bytes = 0;
    int64_t *h_part = nullptr;
    double *dmax_part = nullptr, *binf_part = nullptr;
    int nitems = 0;
    double bytes_per_iter = 0.0;
    int grid = 0;

    int32_t *queue = nullptr;
    int *d_count = nullptr;
    // shared by the systems (their calls are ordered on the batch's stream)
    int *claim = nullptr;                  // row claims of a device-side replacement (zero between calls)
    size_t claim_cap = 0;
    double *rhs = nullptr;                 // exact right-hand side read by modap_batch_query
    size_t rhs_cap = 0;
    int2 *d_states = nullptr;              // statuses gathered for the certificate
    size_t states_cap = 0;
    // FP64 certificate scratch, sized for the largest system certified so far
    double *cert_wt = nullptr, *cert_part = nullptr, *cert_y = nullptr, *cert_ynp = nullptr;
    int64_t *cert_h = nullptr;
    double *cert_dmax = nullptr, *cert_binf = nullptr, *cert_drift = nullptr;
    Totals *cert_tot = nullptr;
    size_t cert_m = 0, cert_part_cap = 0, cert_n = 0;
    int *h_count = nullptr;               // pinned [2]
    unsigned long long *bad = nullptr;
    int *flag = nullptr;
    void *stage = nullptr;
    size_t stage_bytes = 0;
    std::vector<hipEvent_t> events;
    hipEvent_t sync_ev[2] = {nullptr, nullptr};
};

namespace {

modap_status b_to_device(modap_batch *c, void *dst, const void *src, size_t bytes, int on_dev) {
    if (bytes == 0) return MODAP_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    return MODAP_OK;
}

modap_status b_from_device(modap_batch *c, void *dst, const void *src, size_t bytes, int on_dev) {
    if (bytes == 0) return MODAP_OK;
    HIP_TRY(c, hipMemcpyAsync(dst, src, bytes, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    return MODAP_OK;
}

void release_sys(BSys &s) {
    free_dev(s.A);
    free_dev(s.b);
    free_dev(s.nu);
    free_dev(s.x);
    free_dev(s.y);
    free_dev(s.vpend);
    free_dev(s.bref);
    free_dev(s.wsum);
    free_dev(s.V);
    free_dev(s.work);
    free_dev(s.ctl);
    free_dev(s.tot);
    free_dev(s.ynp);
    s.alive = false;
    s.T = 0;
}

BSys *find_sys(modap_batch *c, int64_t id) {
    if (id < 0 || id >= (int64_t)c->sys.size() || !c->sys[(size_t)id].alive) return nullptr;
    return &c->sys[(size_t)id];
}

// The form of the batched sweep for a system: rows of at most 64 VEC
// elements are swept four to a wavefront (16 lanes each, RPW = 4), longer
// ones a wavefront each (RPW = 1); C is the lane's 16-byte chunks of a row.
// MODAP_BATCH_SHORT=0 keeps every row on a wavefront of its own.
void kernel_form(int dt, const BSys &s, int32_t *rpw, int32_t *chunks) {
    const char *e = std::getenv("MODAP_BATCH_SHORT");
    plan_row_form(s.ldA, (int64_t)vec_elems(dt), s.C, !(e && e[0] == '0'), rpw, chunks);
}

// Largest row (padded length) the batched sweep covers.
int64_t max_row(int dt) { return 64 * (int64_t)vec_elems(dt) * kBatchCmax; }

int chunks_for(int dt, int64_t ldA) {
    for (int C : kBuckets)
        if (64 * (int64_t)vec_elems(dt) * C >= ldA) return C;
    return 0;
}

modap_status ensure_stage(modap_batch *c, size_t bytes) {
    if (bytes <= c->stage_bytes) return MODAP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    free_dev(c->stage);
    HIP_TRY(c, hipMalloc(&c->stage, bytes));
    c->stage_bytes = bytes;
    return MODAP_OK;
}

template <typename P>
modap_status ensure_buf(modap_batch *c, P *&p, size_t &cap, size_t count) {
    if (count <= cap) return MODAP_OK;
    free_dev(p);
    const size_t want = std::max(count, cap * 2);
    HIP_TRY(c, hipMalloc(&p, sizeof(P) * want));
    cap = want;
    return MODAP_OK;
}

int64_t rows_per_item(const modap_batch *c, const BSys &s) {
    return plan_rows_per_item(s.m, s.ldA, (int64_t)c->es, c->tile.item_kib[bucket_of(s.C)], c->tile.min_items,
                              kBatchWaves);
}

const void *sweep_fn(int dt);

modap_status rebuild(modap_batch *c) {
    if (!c->dirty) return MODAP_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));  // the previous tables may still be read
    c->order.clear();
    c->h_sys.clear();
    c->h_item_sys.clear();
    std::vector<int64_t> item_bytes;
    c->h_cols.clear();
    int64_t items = 0, part = 0;
    double bytes = 0.0;
    for (size_t id = 0; id < c->sys.size(); ++id) {
        const BSys &s = c->sys[id];
        if (!s.alive) continue;
        BatchSys d{};
        d.A = s.A;
        d.ldA = s.ldA;
        d.m = s.m;
        d.n = s.n;
        d.b = s.b;
        d.nu = s.nu;
        d.x = s.x;
        d.y = s.y;
        d.vpend = s.vpend;
        d.wsum = s.wsum;
        d.V = s.T > 0 ? s.V : nullptr;
        d.work = s.work;
        d.ctl = s.ctl;
        d.tot = s.tot;
        d.ynp = s.ynp;
        d.R = (int32_t)((s.n + 63) / 64);
        kernel_form(c->dt, s, &d.RPW, &d.C);
        d.rows_per_item = rows_per_item(c, s);
        d.item0 = items;
        d.nitems = (s.m + d.rows_per_item - 1) / d.rows_per_item;
        d.part0 = part;
        const int32_t idx = (int32_t)c->h_sys.size();
        for (int64_t q = 0; q < d.nitems; ++q) {
            c->h_item_sys.push_back(idx);
            const int64_t rows = std::min(d.rows_per_item, s.m - q * d.rows_per_item);
            item_bytes.push_back(rows * s.ldA * (int64_t)c->es);
        }
        for (int32_t blk = 0; blk < d.R; ++blk) c->h_cols.push_back(BatchCol{idx, blk});
        items += d.nitems;
        part += d.nitems * s.ldA;
        bytes += (double)s.m * (double)s.n * (double)c->es + 24.0 * (double)s.m;
        c->h_sys.push_back(d);
        c->order.push_back((int32_t)id);
    }
    c->nitems = (int)items;
    c->bytes_per_iter = bytes;
    // hand out the largest items first (ties in item order): the workgroups
    // then end on small items and finish close together
    c->h_item_order.resize((size_t)items);
    for (int64_t q = 0; q < items; ++q) c->h_item_order[(size_t)q] = (int32_t)q;
    std::stable_sort(c->h_item_order.begin(), c->h_item_order.end(),
                     [&](int32_t u, int32_t v) { return item_bytes[(size_t)u] > item_bytes[(size_t)v]; });
    modap_status st;
    if ((st = ensure_buf(c, c->d_sys, c->sys_cap, std::max<size_t>(1, c->h_sys.size())))) return st;
    size_t cap = c->item_cap;
    if ((st = ensure_buf(c, c->d_item_sys, cap, std::max<size_t>(1, (size_t)items)))) return st;
    if (cap != c->item_cap) {
        size_t c2 = 0, c3 = 0, c4 = 0;
        free_dev(c->h_part);
        free_dev(c->dmax_part);
        free_dev(c->binf_part);
        if ((st = ensure_buf(c, c->h_part, c2, cap)) || (st = ensure_buf(c, c->dmax_part, c3, cap)) ||
            (st = ensure_buf(c, c->binf_part, c4, cap)))
            return st;
        c->item_cap = cap;
    }
    if ((st = ensure_buf(c, c->d_item_order, c->order_cap, std::max<size_t>(1, (size_t)items)))) return st;
    if ((st = ensure_buf(c, c->d_cols, c->cols_cap, std::max<size_t>(1, c->h_cols.size())))) return st;
    const size_t pbytes = std::max<size_t>(16, (size_t)part * acc_size(c->dt));
    if (pbytes > c->part_bytes) {
        free_dev(c->part);
        HIP_TRY(c, hipMalloc(&c->part, pbytes));
        c->part_bytes = pbytes;
    }
    if (!c->h_sys.empty()) {
        HIP_TRY(c, hipMemcpyAsync(c->d_sys, c->h_sys.data(), sizeof(BatchSys) * c->h_sys.size(),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_item_sys, c->h_item_sys.data(), sizeof(int32_t) * c->h_item_sys.size(),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_item_order, c->h_item_order.data(),
                                  sizeof(int32_t) * c->h_item_order.size(), hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(c->d_cols, c->h_cols.data(), sizeof(BatchCol) * c->h_cols.size(),
                                  hipMemcpyHostToDevice, c->stream));
    }
    // persistent grid: as many workgroups as are resident at once (two per CU
    // for FP32 and FP64 storage, one for BF16) unless tuned.  Measured on the
    // 512-system FP32 families: the mix 6.40 against 6.28 TB/s at one per CU,
    // the n = 256 family (short rows) 4.95 against 3.87 TB/s.
    if (c->per_cu == 0 &&
        (hipOccupancyMaxActiveBlocksPerMultiprocessor(&c->per_cu, sweep_fn(c->dt), 256, 0) != hipSuccess ||
         c->per_cu < 1))
        c->per_cu = 1;
    c->grid = c->tile.grid > 0 ? c->tile.grid : c->cu_count * c->per_cu;
    c->grid = std::max(1, std::min(c->grid, std::max(1, c->nitems)));
    c->dirty = false;
    return MODAP_OK;
}

BatchArgs batch_args(modap_batch *c) {
    BatchArgs a{};
    a.sys = c->d_sys;
    a.nsys = (int32_t)c->h_sys.size();
    a.nitems = c->nitems;
    a.item_sys = c->d_item_sys;
    a.item_order = c->d_item_order;
    a.part = c->part;
    a.h_part = c->h_part;
    a.dmax_part = c->dmax_part;
    a.binf_part = c->binf_part;
    a.queue = c->queue;
    a.j = c->jn;
    a.check_status = 1;
    a.write_b = 1;
    return a;
}

Decide decide_of(const modap_params *p, int track) {
    Decide d{};
    d.lambda = p->lambda;
    d.eps = p->eps;
    d.eps_relative = p->eps_relative;
    d.rule = p->step == MODAP_STEP_AVG ? 1 : 0;
    d.track = track;
    return d;
}

modap_status check_params(modap_batch *c, const modap_params *p) {
    const char *msg = nullptr;
    const modap_status st = modap_host::check_params(p, &msg);
    return st ? fail(c, st, msg) : MODAP_OK;
}

hipEvent_t event_at(modap_batch *c, size_t i) {
    while (c->events.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->events.push_back(e);
    }
    return c->events[i];
}

modap_status launch(modap_batch *c, const void *f, int grid, int block, BatchArgs a, hipEvent_t e0, hipEvent_t e1,
                    const BatchCol *cols = nullptr, int64_t extra = 0, bool with_cols = false,
                    bool with_i64 = false) {
    void *args3[] = {&a, &cols};
    void *args2[] = {&a, &extra};
    void *args1[] = {&a};
    void **args = with_cols ? args3 : with_i64 ? args2 : args1;
    HIP_TRY(c, hipExtLaunchKernel(f, dim3(grid), dim3(block), args, 0, c->stream, e0, e1, 0));
    return MODAP_OK;
}

const void *sweep_fn(int dt) {
    return dt == 0 ? reinterpret_cast<const void *>(&sweep_batch<0>)
         : dt == 1 ? reinterpret_cast<const void *>(&sweep_batch<1>)
                   : reinterpret_cast<const void *>(&sweep_batch<2>);
}
const void *reduce_fn(int dt) {
    return dt == 0 ? reinterpret_cast<const void *>(&reduce_batch<double>)
                   : reinterpret_cast<const void *>(&reduce_batch<float>);
}
const void *prime_fn(int dt) {
    return dt == 0 ? reinterpret_cast<const void *>(&prime_batch<double>)
                   : reinterpret_cast<const void *>(&prime_batch<float>);
}

// Call start: clear stops of earlier calls, set the step limit, prime the
// working vectors and empty the queue.
modap_status enqueue_begin(modap_batch *c, int64_t max_steps) {
    BatchArgs a = batch_args(c);
    const int nsys = a.nsys;
    modap_status st;
    if ((st = launch(c, reinterpret_cast<const void *>(&begin_batch), (nsys + 255) / 256, 256, a, nullptr, nullptr,
                     nullptr, max_steps, false, true)))
        return st;
    return launch(c, prime_fn(c->dt), nsys, 256, a, nullptr, nullptr);
}

modap_status enqueue_iteration(modap_batch *c, const modap_params *p, int track, int64_t i, size_t *ev_used,
                               double *bytes) {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    if (p->profile > 0 && i % p->profile == 0) {
        for (int k = 0; k < 4; ++k) {
            ev[k] = event_at(c, *ev_used + k);
            if (!ev[k]) return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
        }
        *ev_used += 4;
    }
    BatchArgs a = batch_args(c);
    a.decide = i > 0;
    a.apply_step = i > 0;
    a.dp = decide_of(p, track);
    modap_status st;
    if ((st = launch(c, sweep_fn(c->dt), c->grid, 256, a, ev[0], ev[1]))) return st;
    if ((st = launch(c, reduce_fn(c->dt), (int)c->h_cols.size(), 256, a, ev[2], ev[3], c->d_cols, 0, true)))
        return st;
    c->jn += 1;
    *bytes += c->bytes_per_iter;
    return MODAP_OK;
}

modap_status enqueue_settle(modap_batch *c, const modap_params *p, int track) {
    BatchArgs a = batch_args(c);
    a.j = c->jn - 1;
    a.dp = decide_of(p, track);
    return launch(c, reinterpret_cast<const void *>(&settle_batch), a.nsys, 256, a, nullptr, nullptr);
}

modap_status profile_totals(modap_batch *c, size_t ev_used, modap_batch_stats *o) {
    double sw = 0.0, rd = 0.0;
    int64_t cnt = 0;
    for (size_t i = 0; i + 3 < ev_used; i += 4) {
        float x = 0.f, y = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&x, c->events[i], c->events[i + 1]));
        HIP_TRY(c, hipEventElapsedTime(&y, c->events[i + 2], c->events[i + 3]));
        sw += x;
        rd += y;
        ++cnt;
    }
    o->sweep_ms = sw;
    o->reduce_ms = rd;
    o->profiled = cnt;
    return MODAP_OK;
}

modap_status count_running_now(modap_batch *c, int slot_index, int *out) {
    BatchArgs a = batch_args(c);
    hipLaunchKernelGGL(count_running, dim3(1), dim3(256), 0, c->stream, a, slot_index, c->d_count);
    LAUNCH_TRY(c, "count_running launch");
    HIP_TRY(c, hipMemcpyAsync(out, c->d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return MODAP_OK;
}

int last_slot(const modap_batch *c) { return (int)((c->jn - 1) & 1); }

// Scratch of the FP64 certificate for a system of m rows and padded length
// ldA (row bands of at least 256 rows, at most 128 bands).
modap_status ensure_cert(modap_batch *c, int64_t m, int64_t ldA, int64_t *rpb, int *bands) {
    *rpb = std::max<int64_t>(256, (m + 127) / 128);
    *bands = (int)((m + *rpb - 1) / *rpb);
    const size_t gs = (size_t)((m + 3) / 4);
    if ((size_t)m > c->cert_m) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_dev(c->cert_wt);
        free_dev(c->cert_h);
        free_dev(c->cert_dmax);
        free_dev(c->cert_binf);
        free_dev(c->cert_drift);
        c->cert_m = 0;
        HIP_TRY(c, hipMalloc(&c->cert_wt, sizeof(double) * (size_t)m));
        HIP_TRY(c, hipMalloc(&c->cert_h, sizeof(int64_t) * gs));
        HIP_TRY(c, hipMalloc(&c->cert_dmax, sizeof(double) * gs));
        HIP_TRY(c, hipMalloc(&c->cert_binf, sizeof(double) * gs));
        HIP_TRY(c, hipMalloc(&c->cert_drift, sizeof(double) * gs));
        c->cert_m = (size_t)m;
    }
    if ((size_t)ldA > c->cert_n) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_dev(c->cert_y);
        free_dev(c->cert_ynp);
        c->cert_n = 0;
        HIP_TRY(c, hipMalloc(&c->cert_y, sizeof(double) * (size_t)ldA));
        HIP_TRY(c, hipMalloc(&c->cert_ynp, sizeof(double) * (size_t)((ldA + 63) / 64)));
        c->cert_n = (size_t)ldA;
    }
    const size_t pc = (size_t)*bands * (size_t)ldA;
    if (pc > c->cert_part_cap) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_dev(c->cert_part);
        c->cert_part_cap = 0;
        HIP_TRY(c, hipMalloc(&c->cert_part, sizeof(double) * pc));
        c->cert_part_cap = pc;
    }
    if (!c->cert_tot) HIP_TRY(c, hipMalloc(&c->cert_tot, sizeof(Totals)));
    return MODAP_OK;
}

// Queue the FP64 certificate of system s (a no-op on the device unless its
// committed state is an uncertified stop).
modap_status certify_sys(modap_batch *c, BSys &s, const modap_params *p) {
    int64_t rpb = 0;
    int bands = 0;
    modap_status st;
    if ((st = ensure_cert(c, s.m, s.ldA, &rpb, &bands))) return st;
    CertArgs v{};
    v.A = s.A;
    v.ldA = s.ldA;
    v.m = s.m;
    v.n = s.n;
    v.b = s.b;
    v.bref = s.bref;
    v.nu = s.nu;
    v.x = s.x;
    v.wsum = s.wsum;
    v.V = s.T > 0 ? s.V : nullptr;
    v.ldV = s.ldA;
    v.work = s.work;
    v.ctl = s.ctl;
    v.sl = last_slot(c);
    v.wt = c->cert_wt;
    v.h_part = c->cert_h;
    v.dmax_part = c->cert_dmax;
    v.binf_part = c->cert_binf;
    v.drift_part = c->cert_drift;
    v.bands = bands;
    v.rows_per_band = rpb;
    v.part = c->cert_part;
    v.y = c->cert_y;
    v.ynp = c->cert_ynp;
    v.tot = c->cert_tot;
    v.dp = decide_of(p, 0);
    HIP_TRY(c, aux_certify(c->dt, v, c->stream));
    return MODAP_OK;
}

// The certificate of every system whose committed state is an uncertified
// stop (the states are read first, so only those systems are queued).
// Synchronises.  *count (may be NULL) receives the number certified.
modap_status certify_stopped(modap_batch *c, const modap_params *p, int *count) {
    if (count) *count = 0;
    const int nsys = (int)c->h_sys.size();
    if (nsys == 0) return MODAP_OK;
    modap_status st;
    if ((st = ensure_buf(c, c->d_states, c->states_cap, (size_t)nsys))) return st;
    BatchArgs a = batch_args(c);
    hipLaunchKernelGGL(gather_states, dim3((nsys + 255) / 256), dim3(256), 0, c->stream, a, last_slot(c), c->d_states);
    LAUNCH_TRY(c, "gather_states launch");
    std::vector<int2> hs((size_t)nsys);
    HIP_TRY(c, hipMemcpyAsync(hs.data(), c->d_states, sizeof(int2) * (size_t)nsys, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int cnt = 0;
    for (int i = 0; i < nsys; ++i) {
        if (hs[(size_t)i].x != ST_CONVERGED || hs[(size_t)i].y != 0) continue;
        if ((st = certify_sys(c, c->sys[(size_t)c->order[(size_t)i]], p))) return st;
        ++cnt;
    }
    if (cnt) HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (count) *count = cnt;
    return MODAP_OK;
}

}  // namespace

// Certificate of the stops of the given systems (used by the server, which
// reads each request's state after a round).  Synchronises.
modap_status modap_batch_certify_ids(modap_batch *c, const modap_params *p, const int64_t *ids, int64_t count) {
    TraceRange trace_("modap_batch_certify_ids");
    if (!c) return MODAP_E_INVAL;
    DeviceGuard g(c->device);
    modap_status st;
    for (int64_t q = 0; q < count; ++q) {
        BSys *s = find_sys(c, ids[q]);
        if (!s) return fail(c, MODAP_E_INVAL, "unknown system id");
        if ((st = certify_sys(c, *s, p))) return st;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MODAP_OK;
}

extern "C" {

modap_status modap_batch_create(int device, void *hip_stream, modap_dtype storage, modap_batch **out) {
    if (!out) return MODAP_E_INVAL;
    *out = nullptr;
    if (storage != MODAP_F64 && storage != MODAP_F32 && storage != MODAP_BF16) return MODAP_E_INVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return MODAP_E_INVAL;
    modap_batch *c = new (std::nothrow) modap_batch();
    if (!c) return MODAP_E_NOMEM;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->dt = (int)storage;
    c->es = elem_size(c->dt);
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    bool ok = hipGetDeviceProperties(&prop, device) == hipSuccess;
    if (ok) c->cu_count = prop.multiProcessorCount;
    ok = ok && hipMalloc(&c->queue, sizeof(int32_t)) == hipSuccess && hipMalloc(&c->d_count, sizeof(int)) == hipSuccess &&
         hipMalloc(&c->bad, sizeof(unsigned long long)) == hipSuccess && hipMalloc(&c->flag, sizeof(int)) == hipSuccess &&
         hipHostMalloc(&c->h_count, 2 * sizeof(int)) == hipSuccess &&
         hipEventCreateWithFlags(&c->sync_ev[0], hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&c->sync_ev[1], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        modap_batch_destroy(c);
        return MODAP_E_DEVICE;
    }
    *out = c;
    return MODAP_OK;
}

void modap_batch_destroy(modap_batch *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    for (BSys &s : c->sys) release_sys(s);
    free_dev(c->d_sys);
    free_dev(c->d_item_sys);
    free_dev(c->d_item_order);
    free_dev(c->d_cols);
    free_dev(c->part);
    free_dev(c->h_part);
    free_dev(c->dmax_part);
    free_dev(c->binf_part);
    free_dev(c->queue);
    free_dev(c->d_count);
    free_dev(c->claim);
    free_dev(c->rhs);
    free_dev(c->d_states);
    free_dev(c->cert_wt);
    free_dev(c->cert_part);
    free_dev(c->cert_y);
    free_dev(c->cert_ynp);
    free_dev(c->cert_h);
    free_dev(c->cert_dmax);
    free_dev(c->cert_binf);
    free_dev(c->cert_drift);
    free_dev(c->cert_tot);
    free_dev(c->bad);
    free_dev(c->flag);
    free_dev(c->stage);
    if (c->h_count) (void)hipHostFree(c->h_count);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->sync_ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

modap_status modap_batch_add(modap_batch *c, int64_t m, int64_t n, const void *A, int64_t lda, const double *b,
                             const double *x0, int on_dev, int64_t *id) {
    TraceRange trace_("modap_batch_add");
    if (!c) return MODAP_E_INVAL;
    if (!id) return fail(c, MODAP_E_INVAL, "id is NULL");
    const char *msg = nullptr;
    if (check_system(m, n, lda, A, b, c->dt, &msg)) return fail(c, MODAP_E_INVAL, msg);
    const int64_t v = vec_elems(c->dt);
    const int64_t ldA = (n + v - 1) / v * v;
    if (ldA > max_row(c->dt))
        return fail(c, MODAP_E_INVAL, "rows longer than the batched sweep covers (" + std::to_string(max_row(c->dt)) +
                                          " elements): use a single-system context");
    if (!on_dev) {
        if (!all_finite(b, m)) return fail(c, MODAP_E_INVAL, "b has a non-finite entry");
        if (x0 && !all_finite(x0, n)) return fail(c, MODAP_E_INVAL, "x0 has a non-finite entry");
    }
    DeviceGuard g(c->device);
    BSys s;
    s.m = m;
    s.n = n;
    s.ldA = ldA;
    s.C = chunks_for(c->dt, ldA);
    const size_t abytes = (size_t)m * (size_t)ldA * c->es;
    const size_t vbytes = sizeof(double) * (size_t)ldA;
    const size_t wbytes = 3 * acc_size(c->dt) * (size_t)ldA;
    auto cleanup = [&](modap_status st) {
        release_sys(s);
        return st;
    };
    hipError_t e = hipSuccess;
    if ((e = hipMalloc(&s.A, abytes)) != hipSuccess || (e = hipMalloc(&s.b, sizeof(double) * m)) != hipSuccess ||
        (e = hipMalloc(&s.nu, sizeof(double) * m)) != hipSuccess || (e = hipMalloc(&s.x, vbytes)) != hipSuccess ||
        (e = hipMalloc(&s.y, vbytes)) != hipSuccess || (e = hipMalloc(&s.vpend, vbytes)) != hipSuccess ||
        (e = hipMalloc(&s.wsum, vbytes)) != hipSuccess || (e = hipMalloc(&s.bref, sizeof(double) * m)) != hipSuccess ||
        (e = hipMalloc(&s.work, wbytes)) != hipSuccess || (e = hipMalloc(&s.ctl, sizeof(Ctrl))) != hipSuccess ||
        (e = hipMalloc(&s.tot, sizeof(Totals))) != hipSuccess ||
        (e = hipMalloc(&s.ynp, sizeof(double) * (size_t)((n + 63) / 64))) != hipSuccess)
        return cleanup(hip_fail(c, e, "hipMalloc"));
    modap_status st = MODAP_OK;
    auto q = [&](hipError_t r, const char *what) {
        if (r != hipSuccess && st == MODAP_OK) st = hip_fail(c, r, what);
    };
    if (ldA != n) q(hipMemsetAsync(s.A, 0, abytes, c->stream), "hipMemsetAsync");
    q(hipMemcpy2DAsync(s.A, (size_t)ldA * c->es, A, (size_t)lda * c->es, (size_t)n * c->es, (size_t)m,
                       on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
      "hipMemcpy2DAsync");
    q(hipMemcpyAsync(s.b, b, sizeof(double) * m, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream),
      "copy b");
    q(hipMemsetAsync(s.x, 0, vbytes, c->stream), "hipMemsetAsync");
    if (x0)
        q(hipMemcpyAsync(s.x, x0, sizeof(double) * n, on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         c->stream),
          "copy x0");
    q(hipMemsetAsync(s.y, 0, vbytes, c->stream), "hipMemsetAsync");
    q(hipMemsetAsync(s.vpend, 0, vbytes, c->stream), "hipMemsetAsync");
    q(hipMemsetAsync(s.wsum, 0, vbytes, c->stream), "hipMemsetAsync");
    q(hipMemcpyAsync(s.bref, s.b, sizeof(double) * m, hipMemcpyDeviceToDevice, c->stream), "copy b");
    q(hipMemsetAsync(s.work, 0, wbytes, c->stream), "hipMemsetAsync");
    const unsigned long long none = ULLONG_MAX;
    q(hipMemcpyAsync(c->bad, &none, sizeof none, hipMemcpyHostToDevice, c->stream), "copy");
    q(hipMemsetAsync(c->flag, 0, sizeof(int), c->stream), "hipMemsetAsync");
    q(aux_row_norms(c->dt, s.A, ldA, m, n, s.nu, c->bad, c->stream), "row_norms launch");
    if (on_dev) {
        q(aux_check_finite(s.b, m, c->flag, c->stream), "check_finite launch");
        q(aux_check_finite(s.x, n, c->flag, c->stream), "check_finite launch");
    }
    q(aux_ctl_init(s.ctl, c->stream), "ctl_init launch");
    unsigned long long bad = 0;
    int flag = 0;
    q(hipMemcpyAsync(&bad, c->bad, sizeof bad, hipMemcpyDeviceToHost, c->stream), "copy");
    q(hipMemcpyAsync(&flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream), "copy");
    q(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (st) return cleanup(st);
    if (flag) return cleanup(fail(c, MODAP_E_INVAL, "b or x0 has a non-finite entry"));
    if (bad != ULLONG_MAX) return cleanup(fail(c, MODAP_E_ZERO_ROW, "row " + std::to_string(bad) + " is zero or not finite"));
    s.alive = true;
    // a fresh system's committed state must sit in the batch's slot
    // (jn-1)&1: ctl_init filled both slots
    size_t slot = c->sys.size();
    for (size_t i = 0; i < c->sys.size(); ++i)
        if (!c->sys[i].alive && !c->sys[i].A) {
            slot = i;
            break;
        }
    if (slot == c->sys.size()) c->sys.push_back(s);
    else c->sys[slot] = s;
    *id = (int64_t)slot;
    c->dirty = true;
    c->err.clear();
    return MODAP_OK;
}

modap_status modap_batch_remove(modap_batch *c, int64_t id) {
    TraceRange trace_("modap_batch_remove");
    if (!c) return MODAP_E_INVAL;
    BSys *s = find_sys(c, id);
    if (!s) return fail(c, MODAP_E_INVAL, "unknown system id");
    DeviceGuard g(c->device);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    release_sys(*s);
    c->dirty = true;
    return MODAP_OK;
}

modap_status modap_batch_set_drift(modap_batch *c, int64_t id, int64_t T, const double *V, int64_t ldv, int on_dev) {
    if (!c) return MODAP_E_INVAL;
    BSys *s = find_sys(c, id);
    if (!s) return fail(c, MODAP_E_INVAL, "unknown system id");
    const char *msg = nullptr;
    if (modap_status cs = check_drift(T, V, ldv, s->n, !on_dev, &msg)) return fail(c, cs, msg);
    DeviceGuard g(c->device);
    const int sl = last_slot(c);
    if (s->V) {
        HIP_TRY(c, aux_sched_to_vpend(s->ctl, sl, s->vpend, s->V, s->ldA, s->n, c->stream));
        s->vpend_maybe = true;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        free_dev(s->V);
        s->T = 0;
    }
    if (T > 0 && V) {
        HIP_TRY(c, hipMalloc(&s->V, sizeof(double) * (size_t)T * (size_t)s->ldA));
        HIP_TRY(c, hipMemsetAsync(s->V, 0, sizeof(double) * (size_t)T * (size_t)s->ldA, c->stream));
        HIP_TRY(c, hipMemcpy2DAsync(s->V, sizeof(double) * (size_t)s->ldA, V, sizeof(double) * (size_t)ldv,
                                    sizeof(double) * (size_t)s->n, (size_t)T,
                                    on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
        s->T = T;
    }
    HIP_TRY(c, aux_ctl_set_drift(s->ctl, sl, s->T, c->stream));
    c->dirty = true;
    return MODAP_OK;
}

modap_status modap_batch_update(modap_batch *c, int64_t id, int64_t k, const int64_t *rows, const void *new_rows,
                                const double *new_b, const double *v, int on_dev) {
    TraceRange trace_("modap_batch_update");
    if (!c) return MODAP_E_INVAL;
    BSys *s = find_sys(c, id);
    if (!s) return fail(c, MODAP_E_INVAL, "unknown system id");
    const char *msg = nullptr;
    if (k < 0 || k > s->m) return fail(c, MODAP_E_INVAL, "k out of range");
    if (k > 0 && (!rows || !new_rows || !new_b)) return fail(c, MODAP_E_INVAL, "rows, new_rows and new_b are required");
    const size_t rbytes = (size_t)k * (size_t)s->n * c->es;
    if (k > 0 && !on_dev) {
        if (modap_status cs = check_rows(k, rows, new_rows, new_b, s->m, &msg)) return fail(c, cs, msg);
        if (modap_status cs = check_new_rows(c->dt, new_rows, k, s->n, &msg)) return fail(c, cs, msg);
    }
    if (v && !on_dev && !all_finite(v, s->n)) return fail(c, MODAP_E_INVAL, "translation has a non-finite entry");
    DeviceGuard g(c->device);
    const int64_t *d_rows = rows;
    const void *d_new = new_rows;
    const double *d_b = new_b;
    const double *d_v = v;
    modap_status st;
    if (!on_dev) {
        const size_t o1 = 0, o2 = o1 + (size_t)k * 8, o3 = (o2 + rbytes + 15) / 16 * 16, o4 = o3 + (size_t)k * 8;
        const size_t total = o4 + (v ? (size_t)s->n * 8 : 0);
        if ((st = ensure_stage(c, total + 16))) return st;
        char *p = reinterpret_cast<char *>(c->stage);
        if (k > 0) {
            if ((st = b_to_device(c, p + o1, rows, (size_t)k * 8, 0))) return st;
            if ((st = b_to_device(c, p + o2, new_rows, rbytes, 0))) return st;
            if ((st = b_to_device(c, p + o3, new_b, (size_t)k * 8, 0))) return st;
        }
        if (v && (st = b_to_device(c, p + o4, v, (size_t)s->n * 8, 0))) return st;
        d_rows = reinterpret_cast<const int64_t *>(p + o1);
        d_new = p + o2;
        d_b = reinterpret_cast<const double *>(p + o3);
        d_v = v ? reinterpret_cast<const double *>(p + o4) : nullptr;
    }
    const int sl = last_slot(c);
    if (k > 0 && on_dev) {
        if (c->claim_cap < (size_t)s->m) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            free_dev(c->claim);
            c->claim_cap = 0;
            HIP_TRY(c, hipMalloc(&c->claim, sizeof(int) * (size_t)s->m));
            HIP_TRY(c, hipMemsetAsync(c->claim, 0, sizeof(int) * (size_t)s->m, c->stream));
            c->claim_cap = (size_t)s->m;
        }
        HIP_TRY(c, aux_claim_rows(d_rows, k, s->m, c->claim, s->ctl, sl, c->stream));
    }
    if (k > 0)
        HIP_TRY(c, aux_scatter_rows(c->dt, s->A, s->ldA, s->m, s->n, k, d_rows, d_new, d_b, s->b, s->bref, s->nu,
                                    s->ctl, sl, s->vpend, s->T > 0 ? s->V : nullptr, s->ldA, s->wsum, c->stream));
    if (k > 0 && on_dev) HIP_TRY(c, aux_release_rows(d_rows, k, s->m, c->claim, c->stream));
    if (d_v) {
        HIP_TRY(c, aux_vpend_add(s->ctl, sl, s->vpend, d_v, s->n, c->stream));
        s->vpend_maybe = true;
    }
    // the staging buffer is reused by the next call: wait for the copies out of it
    if (!on_dev) HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MODAP_OK;
}

modap_status modap_batch_iterate(modap_batch *c, const modap_params *p, int64_t k, modap_batch_stats *out) {
    TraceRange trace_("modap_batch_iterate");
    if (!c) return MODAP_E_INVAL;
    modap_status st;
    if ((st = check_params(c, p))) return st;
    if (k < 0) return fail(c, MODAP_E_INVAL, "k < 0");
    DeviceGuard g(c->device);
    if ((st = rebuild(c))) return st;
    if (c->h_sys.empty()) return fail(c, MODAP_E_STATE, "the batch has no systems");
    const auto t0 = std::chrono::steady_clock::now();
    const int track = p->track != 0;
    if (p->profile > 0 && k > 0 && !event_at(c, (size_t)(4 * ((k + p->profile - 1) / p->profile)) - 1))
        return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
    if ((st = enqueue_begin(c, -1))) return st;
    size_t ev = 0;
    double bytes = 0.0;
    for (int64_t i = 0; i < k; ++i)
        if ((st = enqueue_iteration(c, p, track, i, &ev, &bytes))) return st;
    if (k > 0 && (st = enqueue_settle(c, p, track))) return st;
    if (!out) return MODAP_OK;
    if (k > 0 && p->certify && (st = certify_stopped(c, p, nullptr))) return st;
    if ((st = count_running_now(c, last_slot(c), &c->h_count[0]))) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    *out = modap_batch_stats{};
    out->iters = k;
    out->running = c->h_count[0];
    out->systems = (int64_t)c->h_sys.size();
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    out->hbm_bytes = bytes;
    if (p->profile && (st = profile_totals(c, ev, out))) return st;
    return MODAP_OK;
}

modap_status modap_batch_solve(modap_batch *c, const modap_params *p, modap_batch_stats *out) {
    TraceRange trace_("modap_batch_solve");
    if (!c) return MODAP_E_INVAL;
    modap_status st;
    if ((st = check_params(c, p))) return st;
    DeviceGuard g(c->device);
    if ((st = rebuild(c))) return st;
    if (c->h_sys.empty()) return fail(c, MODAP_E_STATE, "the batch has no systems");
    const auto t0 = std::chrono::steady_clock::now();
    if ((st = enqueue_begin(c, p->max_iters))) return st;
    const int64_t total = p->max_iters + 1;
    if (p->profile > 0 && !event_at(c, (size_t)(4 * ((std::min<int64_t>(total, 4096) + p->profile - 1) / p->profile)) - 1))
        return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
    size_t ev = 0;
    double bytes = 0.0;
    int64_t queued_all = 0;
    // Passes of queued iterations until no system runs; stops that the FP64
    // certificate does not confirm have taken a step instead, and the next
    // pass goes on from there (the step limits are the devices').
    for (;;) {
        int64_t queued = 0, chunk = 1;
        int slot = 0, pending = -1;
        bool done = false;
        while (queued < total && !done) {
            const int64_t cnt = std::min(chunk, total - queued);
            for (int64_t i = 0; i < cnt; ++i)
                if ((st = enqueue_iteration(c, p, 0, queued + i, &ev, &bytes))) return st;
            queued += cnt;
            // the newest settled states: the checks before the last queued sweep
            if ((st = count_running_now(c, (int)((c->jn - 2) & 1), &c->h_count[slot]))) return st;
            HIP_TRY(c, hipEventRecord(c->sync_ev[slot], c->stream));
            if (pending >= 0) {
                HIP_TRY(c, hipEventSynchronize(c->sync_ev[pending]));
                if (c->h_count[pending] == 0) done = true;
            }
            pending = slot;
            slot ^= 1;
            chunk = std::min<int64_t>(chunk * 2, 64);
        }
        queued_all += queued;
        if ((st = enqueue_settle(c, p, 0))) return st;
        if (!p->certify) break;
        int certified = 0;
        if ((st = certify_stopped(c, p, &certified))) return st;
        if (certified == 0) break;
        if ((st = count_running_now(c, last_slot(c), &c->h_count[0]))) return st;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->h_count[0] == 0) break;
    }
    if ((st = count_running_now(c, last_slot(c), &c->h_count[0]))) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (out) {
        *out = modap_batch_stats{};
        out->iters = queued_all;
        out->running = c->h_count[0];
        out->systems = (int64_t)c->h_sys.size();
        out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        out->hbm_bytes = bytes;
        if (p->profile && (st = profile_totals(c, ev, out))) return st;
    }
    return MODAP_OK;
}

modap_status modap_batch_query(modap_batch *c, int64_t id, double *x, double *b, modap_stats *out, int on_dev) {
    TraceRange trace_("modap_batch_query");
    if (!c) return MODAP_E_INVAL;
    BSys *s = find_sys(c, id);
    if (!s) return fail(c, MODAP_E_INVAL, "unknown system id");
    DeviceGuard g(c->device);
    modap_status st;
    const int sl = last_slot(c);
    if (x && (st = b_from_device(c, x, s->x, sizeof(double) * s->n, on_dev))) return st;
    if (b) {
        // the data as the caller sees them, in FP64, without committing anything
        if ((st = ensure_buf(c, c->rhs, c->rhs_cap, (size_t)s->m))) return st;
        HIP_TRY(c, aux_rhs_exact(c->dt, s->A, s->ldA, s->m, s->n, s->ctl, sl, s->bref, s->wsum, s->vpend,
                                 s->T > 0 ? s->V : nullptr, s->ldA, c->rhs, c->stream));
        if ((st = b_from_device(c, b, c->rhs, sizeof(double) * s->m, on_dev))) return st;
    }
    State k;
    HIP_TRY(c, hipMemcpyAsync(&k, &s->ctl->st[sl], sizeof(State), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (out) {
        *out = modap_stats{};
        out->iters = k.steps;
        out->sweeps = k.sweeps;
        out->converged = k.feasible;
        out->state = k.status;
        out->max_viol = k.dmax;
        out->h = k.h;
        out->y_norm = k.ynorm;
        out->b_inf = k.binf;
        out->eps_abs = k.eps_abs;
        out->certified = k.certified;
        out->b_drift = k.bdrift;
    }
    return MODAP_OK;
}

modap_status modap_batch_set_tile(modap_batch *c, const modap_batch_tile *t) {
    if (!c) return MODAP_E_INVAL;
    if (!t) {
        c->tile = kBuiltinTile;
    } else {
        for (int q = 0; q < 4; ++q)
            if (t->item_kib[q] < 1) return fail(c, MODAP_E_INVAL, "item_kib must be >= 1");
        if (t->grid < 0) return fail(c, MODAP_E_INVAL, "grid must be >= 0");
        if (t->min_items < 0 || t->min_items > kMaxMinItems)
            return fail(c, MODAP_E_INVAL, "min_items must be in 0 .. 64");
        c->tile = *t;
    }
    c->dirty = true;
    return MODAP_OK;
}

modap_status modap_batch_get_tile(modap_batch *c, modap_batch_tile *t) {
    if (!c) return MODAP_E_INVAL;
    if (!t) return fail(c, MODAP_E_INVAL, "tile is NULL");
    *t = c->tile;
    return MODAP_OK;
}

modap_status modap_batch_autotune(modap_batch *c, int reps, modap_batch_tile *best) {
    TraceRange trace_("modap_batch_autotune");
    if (!c) return MODAP_E_INVAL;
    if (reps < 1) return fail(c, MODAP_E_INVAL, "reps < 1");
    DeviceGuard g(c->device);
    // on any failure the batch keeps the tile it had
    struct Restore {
        modap_batch *c;
        modap_batch_tile t;
        bool armed;
        ~Restore() {
            if (armed) {
                c->tile = t;
                c->dirty = true;
            }
        }
    } restore{c, c->tile, true};
    modap_status st;
    if ((st = rebuild(c))) return st;
    if (c->h_sys.empty()) return fail(c, MODAP_E_STATE, "the batch has no systems");
    bool present[4] = {false, false, false, false};
    for (const BSys &s : c->sys)
        if (s.alive) present[bucket_of(s.C)] = true;
    if (!event_at(c, 2 * (size_t)reps + 1)) return fail(c, MODAP_E_DEVICE, "hipEventCreate failed");
    // one timing: `reps` stateless sweeps (no decision, no b written)
    auto time_sweeps = [&](float *ms) -> modap_status {
        modap_status s2;
        if ((s2 = rebuild(c))) return s2;
        BatchArgs a = batch_args(c);
        if ((s2 = launch(c, prime_fn(c->dt), a.nsys, 256, a, nullptr, nullptr))) return s2;
        a.check_status = 0;
        a.write_b = 0;
        // one untimed sweep, then `reps` timed ones back to back (as the
        // iterations run; a host wait after each would leave the device idle
        // between them), the host waiting once; the shortest counts, the
        // work being the same each time
        for (int r = 0; r <= reps; ++r) {
            HIP_TRY(c, hipMemsetAsync(c->queue, 0, sizeof(int32_t), c->stream));
            hipEvent_t b0 = r ? event_at(c, 2 * (size_t)r) : nullptr, b1 = r ? event_at(c, 2 * (size_t)r + 1) : nullptr;
            if ((s2 = launch(c, sweep_fn(c->dt), c->grid, 256, a, b0, b1))) return s2;
        }
        HIP_TRY(c, hipEventSynchronize(event_at(c, 2 * (size_t)reps + 1)));
        float best = 0.f;
        for (int r = 1; r <= reps; ++r) {
            float x = 0.f;
            HIP_TRY(c, hipEventElapsedTime(&x, event_at(c, 2 * (size_t)r), event_at(c, 2 * (size_t)r + 1)));
            if (r == 1 || x < best) best = x;
        }
        *ms = best;
        return MODAP_OK;
    };
    // Starting from the built-in tile, each bucket's item size and then the
    // grid: the incumbent is timed first and a challenger must beat it by
    // kMargin, so that near-equal choices do not flip with timing noise.
    constexpr float kMargin = 0.98f;
    modap_batch_tile cur = kBuiltinTile;
    auto time_tile = [&](const modap_batch_tile &t, float *ms) -> modap_status {
        c->tile = t;
        c->dirty = true;
        return time_sweeps(ms);
    };
    // the cut of every live system under a tile: a candidate that cuts them
    // all as the incumbent does is the same work, and is not timed (its
    // timing could only differ by noise)
    auto cut_of = [&](const modap_batch_tile &t) {
        std::vector<int64_t> v;
        for (const BSys &s : c->sys)
            if (s.alive) v.push_back(plan_rows_per_item(s.m, s.ldA, (int64_t)c->es, t.item_kib[bucket_of(s.C)],
                                                         t.min_items, kBatchWaves));
        return v;
    };
    // a work item costs a few microseconds beyond its rows (queue, state,
    // staging, partial): large items pay it rarely, small ones balance better
    const int sizes[] = {64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384};
    auto tune_sizes = [&]() -> modap_status {
        for (int q = 0; q < 4; ++q) {
            if (!present[q]) continue;
            float win = 0.f;
            modap_status s2;
            if ((s2 = time_tile(cur, &win))) return s2;
            int pick = cur.item_kib[q];
            std::vector<int64_t> cut = cut_of(cur);
            for (int kib : sizes) {
                if (kib == cur.item_kib[q]) continue;
                modap_batch_tile t = cur;
                t.item_kib[q] = kib;
                if (cut_of(t) == cut) continue;
                float ms = 0.f;
                if ((s2 = time_tile(t, &ms))) return s2;
                if (ms < win * kMargin) {
                    win = ms;
                    pick = kib;
                    cut = cut_of(t);
                }
            }
            cur.item_kib[q] = pick;
        }
        return MODAP_OK;
    };
    if ((st = tune_sizes())) return st;
    // Then the least number of items per system: small systems of a large
    // batch run faster in fewer, larger items.  The counts are compared with
    // every present bucket's item size lifted to the largest, so that the
    // count is what cuts the small systems; if another count wins, the sizes
    // are tuned again under it, and the result is kept only if it beats the
    // tile this stage started from.
    {
        const modap_batch_tile before = cur;
        float t_before = 0.f;
        if ((st = time_tile(before, &t_before))) return st;
        modap_batch_tile lifted = cur;
        for (int q = 0; q < 4; ++q)
            if (present[q]) lifted.item_kib[q] = sizes[sizeof(sizes) / sizeof(sizes[0]) - 1];
        const int inc = cur.min_items > 0 ? cur.min_items : (int)kMinItems;
        float win = 0.f;
        if ((st = time_tile(lifted, &win))) return st;
        int pick = inc;
        std::vector<int64_t> cut = cut_of(lifted);
        for (int mi : {1, 2, 4, 8, 16}) {
            if (mi == inc) continue;
            modap_batch_tile t = lifted;
            t.min_items = mi;
            if (cut_of(t) == cut) continue;
            float ms = 0.f;
            if ((st = time_tile(t, &ms))) return st;
            if (ms < win * kMargin) {
                win = ms;
                pick = mi;
                cut = cut_of(t);
            }
        }
        if (pick != inc) {
            cur = lifted;
            cur.min_items = pick;
            if ((st = tune_sizes())) return st;
            float t_after = 0.f;
            if ((st = time_tile(cur, &t_after))) return st;
            if (!(t_after < t_before * kMargin)) cur = before;
        }
    }
    float win = 0.f;
    if ((st = time_tile(cur, &win))) return st;   // grid 0: every resident workgroup
    int pick = cur.grid;
    for (int mult = 1; mult < c->per_cu; ++mult) {
        modap_batch_tile t = cur;
        t.grid = c->cu_count * mult;
        float ms = 0.f;
        if ((st = time_tile(t, &ms))) return st;
        if (ms < win * kMargin) {
            win = ms;
            pick = t.grid;
        }
    }
    cur.grid = pick;
    c->tile = cur;
    c->dirty = true;
    if ((st = rebuild(c))) return st;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    restore.armed = false;
    if (best) *best = c->tile;
    return MODAP_OK;
}

const char *modap_batch_last_error(modap_batch *c) { return c ? c->err.c_str() : "batch is NULL"; }

}  // extern "C"
