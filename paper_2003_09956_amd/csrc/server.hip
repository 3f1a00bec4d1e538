// Solve server: continuous batching of many requests on one GPU
// (modap_server_* in include/modap.h).
//
// Requests wait in arrival order until their device footprint fits the HBM
// budget.  An admitted request whose rows fit the batched sweep joins the
// server's batch (one persistent launch for all of them); a larger one gets a
// single-system context on a stream of its own, so its kernels overlap with
// the batch's and with the other large requests'.  A round queues the same
// number of iterations for every live request, waits for them, and retires
// the requests that stopped (their x is kept on the host, their device memory
// freed), which lets waiting requests in.  A request's iterations and
// updates depend only on its own rounds, so its result does not depend on the
// other requests it was served with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "host_common.hpp"
#include "trace.hpp"
#include "internal.hpp"
#include "modap.h"

using namespace modap_host;

namespace {

enum ReqState { RQ_QUEUED = 0, RQ_LIVE = 1, RQ_DONE = 2, RQ_FAILED = 3 };

struct Req {
    int state = RQ_QUEUED;
    int64_t m = 0, n = 0, ldA = 0;
    double footprint = 0.0;
    // submission: copies of the caller's inputs, made by modap_server_submit
    // and released at admission -- host inputs in host memory, device inputs
    // in device memory of the server (A row-major with lda = n, V with ldv = n)
    std::vector<char> hA;
    std::vector<double> hb, hx0, hV;
    void *dA = nullptr;
    double *db = nullptr, *dx0 = nullptr, *dV = nullptr;
    bool has_x0 = false;
    int64_t T = 0;
    int on_dev = 0;
    // live
    bool in_batch = false;
    int64_t bid = -1;
    modap_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    int64_t sweeps_seen = 0;
    // outcome
    int32_t status = 0;
    int64_t iters = 0, sweeps = 0;
    double max_viol = 0.0, eps_abs = 0.0;
    double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
    double bytes = 0.0;
    std::string error;
    std::vector<double> x;
    uint64_t trace = 0;   // the request's range on the tracing timeline, open until it ends
    bool released = false;  // the caller released the result (x is freed)
};

void end_trace(Req &r) {
    if (r.trace) trace_stop(r.trace);
    r.trace = 0;
}

// Device memory for the inputs of one update, reusable once the update that
// read it has run (its event has completed).
struct Stage {
    void *p = nullptr;
    size_t size = 0;
    hipEvent_t used = nullptr;
    bool busy = false;
};

}  // namespace

struct modap_server {
    int device = 0;
    int dt = 2;
    size_t es = 2;
    double budget = 0.0, used = 0.0;
    modap_params params{};
    int iters_per_round = 8;
    int64_t max_live = 0;       // 0: no limit besides the budget
    int64_t max_long = 0;       // live requests with contexts of their own at most (0: no limit)
    int64_t long_live = 0;
    int64_t live = 0;
    int64_t max_sweeps = 0;
    modap_batch *batch = nullptr;
    hipStream_t batch_stream = nullptr;
    hipStream_t copy_stream = nullptr;    // staging of device-side update inputs
    std::vector<Stage> stages;
    int batch_live = 0;
    std::vector<Req> reqs;              // every request, indexed by ticket
    std::deque<int64_t> pending;
    std::vector<int64_t> live_ids;      // tickets of the live requests, in admission order
    double bytes = 0.0;
    int64_t rounds = 0;
    std::string err;
};

namespace {

int64_t padded(int dt, int64_t n) {
    const int64_t v = vec_elems(dt);
    return (n + v - 1) / v * v;
}

// Rows the batched sweep covers (64 lanes x 16-byte vectors x 8 chunks).
int64_t batch_row_limit(int dt) { return 64 * (int64_t)vec_elems(dt) * 8; }

// A request whose rows fit the batched sweep joins the batch; a longer one
// gets a context of its own.
bool batched(const modap_server *s, const Req &r) { return r.ldA <= batch_row_limit(s->dt); }

// A staging buffer of at least `bytes` whose last update has run, from the
// server's pool (grown when none is free).
modap_status take_stage(modap_server *s, size_t bytes, Stage **out) {
    for (Stage &t : s->stages) {
        if (t.busy) {
            const hipError_t e = hipEventQuery(t.used);
            if (e == hipSuccess) {
                t.busy = false;
            } else if (e != hipErrorNotReady) {
                s->err = std::string("hipEventQuery: ") + hipGetErrorString(e);
                return MODAP_E_DEVICE;
            }
        }
        if (!t.busy && t.size >= bytes) {
            *out = &t;
            return MODAP_OK;
        }
    }
    Stage t;
    t.size = (bytes + (1u << 20) - 1) / (1u << 20) * (1u << 20);
    if (hipMalloc(&t.p, t.size) != hipSuccess) {
        s->err = "no device memory to stage an update";
        return MODAP_E_NOMEM;
    }
    if (hipEventCreateWithFlags(&t.used, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(t.p);
        s->err = "hipEventCreateWithFlags failed";
        return MODAP_E_DEVICE;
    }
    s->stages.push_back(t);
    *out = &s->stages.back();
    return MODAP_OK;
}

double elapsed_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Release a request's copy of its submitted inputs.
void release_inputs(Req &r) {
    std::vector<char>().swap(r.hA);
    std::vector<double>().swap(r.hb);
    std::vector<double>().swap(r.hx0);
    std::vector<double>().swap(r.hV);
    free_dev(r.dA);
    free_dev(r.db);
    free_dev(r.dx0);
    free_dev(r.dV);
}

// Remove retired tickets from the list of live requests.
void compact_live(modap_server *s) {
    s->live_ids.erase(std::remove_if(s->live_ids.begin(), s->live_ids.end(),
                                     [s](int64_t id) { return s->reqs[(size_t)id].state != RQ_LIVE; }),
                      s->live_ids.end());
}

void drop(modap_server *s, Req &r) {
    if (r.in_batch && r.bid >= 0) {
        (void)modap_batch_remove(s->batch, r.bid);
        --s->batch_live;
    }
    if (r.ctx) {
        modap_destroy(r.ctx);
        --s->long_live;
    }
    if (r.stream) (void)hipStreamDestroy(r.stream);
    r.ctx = nullptr;
    r.stream = nullptr;
    r.bid = -1;
    s->used -= r.footprint;
    --s->live;
}

// Admit request r: copy its data into the batch or a new context.  On
// failure everything created here is released again.
modap_status admit(modap_server *s, Req &r, double now) {
    modap_status st;
    const int od = r.on_dev;
    const void *A = od ? (const void *)r.dA : (const void *)r.hA.data();
    const double *b = od ? r.db : r.hb.data();
    const double *x0 = !r.has_x0 ? nullptr : od ? r.dx0 : r.hx0.data();
    const double *V = r.T == 0 ? nullptr : od ? r.dV : r.hV.data();
    if (batched(s, r)) {
        int64_t id = -1;
        if ((st = modap_batch_add(s->batch, r.m, r.n, A, r.n, b, x0, od, &id))) {
            r.error = modap_batch_last_error(s->batch);
            return st;
        }
        if (r.T > 0 && (st = modap_batch_set_drift(s->batch, id, r.T, V, r.n, od))) {
            r.error = modap_batch_last_error(s->batch);
            (void)modap_batch_remove(s->batch, id);
            return st;
        }
        r.in_batch = true;
        r.bid = id;
        ++s->batch_live;
    } else {
        if (hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking) != hipSuccess) {
            r.stream = nullptr;
            r.error = "hipStreamCreateWithFlags failed";
            return MODAP_E_DEVICE;
        }
        st = modap_create(s->device, r.stream, &r.ctx);
        if (!st) st = modap_set_system(r.ctx, r.m, r.n, (modap_dtype)s->dt, A, r.n, b, x0, od);
        if (!st && r.T > 0) st = modap_set_drift(r.ctx, r.T, V, r.n, od);
        if (st) {
            r.error = r.ctx ? modap_last_error(r.ctx) : "context creation failed";
            if (r.ctx) modap_destroy(r.ctx);
            (void)hipStreamDestroy(r.stream);
            r.ctx = nullptr;
            r.stream = nullptr;
            return st;
        }
    }
    r.state = RQ_LIVE;
    r.t_admit = now;
    s->used += r.footprint;
    ++s->live;
    if (!r.in_batch) ++s->long_live;
    return MODAP_OK;
}

void finish(modap_server *s, Req &r, const modap_stats &q, double now) {
    r.status = q.state;
    r.iters = q.iters;
    r.sweeps = q.sweeps;
    r.max_viol = q.max_viol;
    r.eps_abs = q.eps_abs;
    r.t_done = now;
    r.state = RQ_DONE;
    end_trace(r);
}

}  // namespace

extern "C" {

modap_status modap_server_create(int device, modap_dtype storage, double hbm_budget_bytes, const modap_params *p,
                                 int iters_per_round, modap_server **out) {
    if (!out) return MODAP_E_INVAL;
    *out = nullptr;
    if (!p || !(hbm_budget_bytes > 0.0) || iters_per_round < 1) return MODAP_E_INVAL;
    const char *msg = nullptr;
    if (check_params(p, &msg) || p->max_iters < 1) return MODAP_E_INVAL;
    modap_server *s = new (std::nothrow) modap_server();
    if (!s) return MODAP_E_NOMEM;
    s->device = device;
    s->dt = (int)storage;
    s->es = elem_size(s->dt);
    s->budget = hbm_budget_bytes;
    s->params = *p;
    s->params.profile = 0;
    s->params.track = 0;
    s->iters_per_round = iters_per_round;
    s->max_sweeps = p->max_iters + 1;
    DeviceGuard g(device);
    if (hipStreamCreateWithFlags(&s->batch_stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return MODAP_E_DEVICE;
    }
    if (hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->batch_stream);
        delete s;
        return MODAP_E_DEVICE;
    }
    modap_status st = modap_batch_create(device, s->batch_stream, storage, &s->batch);
    if (st) {
        (void)hipStreamDestroy(s->copy_stream);
        (void)hipStreamDestroy(s->batch_stream);
        delete s;
        return st;
    }
    *out = s;
    return MODAP_OK;
}

void modap_server_destroy(modap_server *s) {
    if (!s) return;
    DeviceGuard g(s->device);
    for (Req &r : s->reqs) {
        if (r.state == RQ_LIVE) drop(s, r);
        release_inputs(r);
        end_trace(r);
    }
    modap_batch_destroy(s->batch);
    for (Stage &t : s->stages) {
        (void)hipEventSynchronize(t.used);
        (void)hipFree(t.p);
        (void)hipEventDestroy(t.used);
    }
    if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
    if (s->batch_stream) (void)hipStreamDestroy(s->batch_stream);
    delete s;
}

modap_status modap_server_submit(modap_server *s, int64_t m, int64_t n, const void *A, const double *b,
                                 const double *x0, int64_t T, const double *V, int64_t ldv, int ptrs_on_device,
                                 double now, int64_t *ticket) {
    TraceRange trace_("modap_server_submit");
    if (!s) return MODAP_E_INVAL;
    if (!ticket) return fail(s, MODAP_E_INVAL, "ticket is NULL");
    const char *msg = nullptr;
    if (modap_status cs = check_request(m, n, A, b, T, V, ldv, &msg)) return fail(s, cs, msg);
    Req r;
    r.m = m;
    r.n = n;
    r.ldA = padded(s->dt, n);
    r.footprint = request_footprint(s->dt, m, n, T);
    if (r.footprint > s->budget) return fail(s, MODAP_E_NOMEM, "the request alone exceeds the HBM budget");
    // Copy the inputs now, so that the caller may release them when this call
    // returns: host inputs into host memory, device inputs into device memory
    // of the server (after the caller's writes to them, which must be done).
    r.T = T;
    r.on_dev = ptrs_on_device;
    r.has_x0 = x0 != nullptr;
    const size_t ab = (size_t)m * (size_t)n * s->es;
    if (!ptrs_on_device) {
        try {
            r.hA.assign(reinterpret_cast<const char *>(A), reinterpret_cast<const char *>(A) + ab);
            r.hb.assign(b, b + m);
            if (x0) r.hx0.assign(x0, x0 + n);
            if (T > 0) {
                r.hV.resize((size_t)T * (size_t)n);
                for (int64_t q = 0; q < T; ++q)
                    std::copy(V + q * ldv, V + q * ldv + n, r.hV.begin() + (ptrdiff_t)(q * n));
            }
        } catch (const std::bad_alloc &) {
            release_inputs(r);
            return fail(s, MODAP_E_NOMEM, "no host memory to copy the request's inputs");
        }
    } else {
        DeviceGuard g(s->device);
        hipError_t e = hipMalloc(&r.dA, ab);
        if (e == hipSuccess) e = hipMalloc(&r.db, sizeof(double) * (size_t)m);
        if (e == hipSuccess && x0) e = hipMalloc(&r.dx0, sizeof(double) * (size_t)n);
        if (e == hipSuccess && T > 0) e = hipMalloc(&r.dV, sizeof(double) * (size_t)T * (size_t)n);
        if (e == hipSuccess) e = hipMemcpyAsync(r.dA, A, ab, hipMemcpyDeviceToDevice, s->copy_stream);
        if (e == hipSuccess) e = hipMemcpyAsync(r.db, b, sizeof(double) * (size_t)m, hipMemcpyDeviceToDevice, s->copy_stream);
        if (e == hipSuccess && x0)
            e = hipMemcpyAsync(r.dx0, x0, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s->copy_stream);
        if (e == hipSuccess && T > 0)
            e = hipMemcpy2DAsync(r.dV, sizeof(double) * (size_t)n, V, sizeof(double) * (size_t)ldv,
                                 sizeof(double) * (size_t)n, (size_t)T, hipMemcpyDeviceToDevice, s->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
        if (e != hipSuccess) {
            release_inputs(r);
            return fail(s, e == hipErrorOutOfMemory ? MODAP_E_NOMEM : MODAP_E_DEVICE,
                        std::string("copying the request's inputs: ") + hipGetErrorString(e));
        }
    }
    r.t_submit = now;
    r.trace = trace_start("modap request");
    *ticket = (int64_t)s->reqs.size();
    s->reqs.push_back(std::move(r));
    s->pending.push_back(*ticket);
    return MODAP_OK;
}

modap_status modap_server_update(modap_server *s, int64_t ticket, int64_t k, const int64_t *rows,
                                 const void *new_rows, const double *new_b, const double *translate_v,
                                 int ptrs_on_device) {
    TraceRange trace_("modap_server_update");
    if (!s) return MODAP_E_INVAL;
    if (ticket < 0 || ticket >= (int64_t)s->reqs.size()) return fail(s, MODAP_E_INVAL, "unknown ticket");
    Req &r = s->reqs[(size_t)ticket];
    if (r.state != RQ_LIVE) return fail(s, MODAP_E_STATE, "the request is not live");
    if (k < 0 || k > r.m) return fail(s, MODAP_E_INVAL, "k out of range");
    if (k > 0 && (!rows || !new_rows || !new_b)) return fail(s, MODAP_E_INVAL, "rows, new_rows and new_b are required");
    DeviceGuard g(s->device);
    // Device inputs are copied into memory of the server's own before the
    // call returns, so that the caller may release or reuse its buffers at
    // once although the update runs later on the request's stream.  The copy
    // is reused only once the update that reads it has run.
    const hipStream_t gs = r.in_batch ? s->batch_stream : r.stream;
    const int64_t *rp = rows;
    const void *np = new_rows;
    const double *bp = new_b, *vp = translate_v;
    Stage *stage = nullptr;
    if (ptrs_on_device && (k > 0 || translate_v)) {
        const size_t rb = (size_t)k * (size_t)r.n * s->es;
        const size_t o2 = (size_t)k * 8, o3 = (o2 + rb + 15) / 16 * 16, o4 = o3 + (size_t)k * 8;
        const size_t total = o4 + (translate_v ? (size_t)r.n * 8 : 0);
        modap_status sst = take_stage(s, total, &stage);
        if (sst) return sst;
        char *p = reinterpret_cast<char *>(stage->p);
        hipError_t e = hipSuccess;
        if (k > 0) {
            if (e == hipSuccess) e = hipMemcpyAsync(p, rows, (size_t)k * 8, hipMemcpyDeviceToDevice, s->copy_stream);
            if (e == hipSuccess) e = hipMemcpyAsync(p + o2, new_rows, rb, hipMemcpyDeviceToDevice, s->copy_stream);
            if (e == hipSuccess) e = hipMemcpyAsync(p + o3, new_b, (size_t)k * 8, hipMemcpyDeviceToDevice, s->copy_stream);
        }
        if (e == hipSuccess && translate_v)
            e = hipMemcpyAsync(p + o4, translate_v, (size_t)r.n * 8, hipMemcpyDeviceToDevice, s->copy_stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy_stream);
        if (e != hipSuccess) return fail(s, MODAP_E_DEVICE, std::string("staging the update: ") + hipGetErrorString(e));
        rp = k > 0 ? reinterpret_cast<const int64_t *>(p) : nullptr;
        np = k > 0 ? p + o2 : nullptr;
        bp = k > 0 ? reinterpret_cast<const double *>(p + o3) : nullptr;
        vp = translate_v ? reinterpret_cast<const double *>(p + o4) : nullptr;
    }
    modap_status st = r.in_batch ? modap_batch_update(s->batch, r.bid, k, rp, np, bp, vp, ptrs_on_device)
                                 : modap_update_coeffs(r.ctx, k, rp, np, bp, vp, ptrs_on_device);
    if (stage) {
        // reusable once whatever the update queued on the request's stream has run
        HIP_TRY(s, hipEventRecord(stage->used, gs));
        stage->busy = true;
    }
    if (st) return fail(s, st, r.in_batch ? modap_batch_last_error(s->batch) : modap_last_error(r.ctx));
    return MODAP_OK;
}

modap_status modap_server_round(modap_server *s, double now, int64_t *outstanding) {
    TraceRange trace_("modap_server_round");
    if (!s) return MODAP_E_INVAL;
    DeviceGuard g(s->device);
    const auto t0 = std::chrono::steady_clock::now();
    modap_status st;
    compact_live(s);
    // admission in arrival order while the footprint fits; a long-row request
    // beyond max_long waits, and the requests behind it may pass it
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        Req &r = s->reqs[(size_t)*it];
        if (!batched(s, r) && s->max_long > 0 && s->long_live >= s->max_long) {
            ++it;
            continue;
        }
        if (!admissible(s->used, r.footprint, s->budget, s->live, s->max_live)) break;
        const int64_t ticket = *it;
        it = s->pending.erase(it);
        st = admit(s, r, now + elapsed_since(t0));
        release_inputs(r);  // the request's data now live in the batch or its context
        if (!st) s->live_ids.push_back(ticket);
        if (st) {
            r.state = RQ_FAILED;
            r.status = -(int32_t)st;
            if (r.error.empty()) r.error = "admission failed";
            end_trace(r);
        }
    }
    // the same number of iterations for every live request
    const int64_t k = s->iters_per_round;
    if (s->batch_live > 0 && (st = modap_batch_iterate(s->batch, &s->params, k, nullptr)))
        return fail(s, st, modap_batch_last_error(s->batch));
    // (the list is compacted at the end of a round; an error return may leave
    // retired tickets in it until then, hence the state checks)
    for (int64_t id : s->live_ids) {
        Req &r = s->reqs[(size_t)id];
        if (r.state == RQ_LIVE && !r.in_batch && (st = modap_iterate(r.ctx, &s->params, k, nullptr)))
            return fail(s, st, modap_last_error(r.ctx));
    }
    // wait, then retire the requests that stopped
    HIP_TRY(s, hipStreamSynchronize(s->batch_stream));
    for (int64_t id : s->live_ids) {
        const Req &r = s->reqs[(size_t)id];
        if (r.state == RQ_LIVE && !r.in_batch) HIP_TRY(s, hipStreamSynchronize(r.stream));
    }
    // Stops of batched requests get their FP64 certificate here (a request
    // with a context of its own had it queued after its iterations).
    if (s->params.certify && s->batch_live > 0) {
        std::vector<int64_t> ids;
        for (int64_t id : s->live_ids) {
            Req &r = s->reqs[(size_t)id];
            if (r.state != RQ_LIVE || !r.in_batch) continue;
            modap_stats q{};
            if ((st = modap_batch_query(s->batch, r.bid, nullptr, nullptr, &q, 0)))
                return fail(s, st, "query of a live request failed");
            if (q.state == 1 && !q.certified) ids.push_back(r.bid);
        }
        if (!ids.empty() && (st = modap_batch_certify_ids(s->batch, &s->params, ids.data(), (int64_t)ids.size())))
            return fail(s, st, modap_batch_last_error(s->batch));
    }
    const double t_end = now + elapsed_since(t0);
    for (int64_t id : s->live_ids) {
        Req &r = s->reqs[(size_t)id];
        if (r.state != RQ_LIVE) continue;
        modap_stats q{};
        st = r.in_batch ? modap_batch_query(s->batch, r.bid, nullptr, nullptr, &q, 0)
                        : modap_query(r.ctx, nullptr, nullptr, &q, 0);
        if (st) return fail(s, st, "query of a live request failed");
        const double per_sweep = (double)r.m * (double)r.n * (double)s->es + 24.0 * (double)r.m;
        r.bytes += (double)(q.sweeps - r.sweeps_seen) * per_sweep;
        s->bytes += (double)(q.sweeps - r.sweeps_seen) * per_sweep;
        r.sweeps_seen = q.sweeps;
        const bool stopped = q.state != 0;
        const bool capped = q.sweeps >= s->max_sweeps;
        if (!stopped && !capped) continue;
        r.x.resize((size_t)r.n);
        st = r.in_batch ? modap_batch_query(s->batch, r.bid, r.x.data(), nullptr, &q, 0)
                        : modap_query(r.ctx, r.x.data(), nullptr, &q, 0);
        if (st) return fail(s, st, "reading a finished request failed");
        finish(s, r, q, t_end);
        if (!stopped) r.status = 4;  // the step limit of the server's parameters
        drop(s, r);
    }
    compact_live(s);
    ++s->rounds;
    if (outstanding) *outstanding = (int64_t)s->pending.size() + (int64_t)s->live_ids.size();
    return MODAP_OK;
}

modap_status modap_server_set_max_long(modap_server *s, int64_t max_long) {
    if (!s) return MODAP_E_INVAL;
    if (max_long < 0) return fail(s, MODAP_E_INVAL, "max_long < 0");
    s->max_long = max_long;
    return MODAP_OK;
}

modap_status modap_server_set_max_live(modap_server *s, int64_t max_live) {
    if (!s) return MODAP_E_INVAL;
    if (max_live < 0) return fail(s, MODAP_E_INVAL, "max_live < 0");
    s->max_live = max_live;
    return MODAP_OK;
}

modap_status modap_server_info(modap_server *s, int64_t ticket, modap_request_info *out) {
    if (!s) return MODAP_E_INVAL;
    if (ticket < 0 || ticket >= (int64_t)s->reqs.size() || !out) return fail(s, MODAP_E_INVAL, "unknown ticket");
    const Req &r = s->reqs[(size_t)ticket];
    *out = modap_request_info{};
    out->state = r.state;
    out->status = r.status;
    out->batched = r.in_batch || (r.state != RQ_QUEUED && r.ldA <= batch_row_limit(s->dt));
    out->iters = r.iters;
    out->sweeps = r.state == RQ_DONE ? r.sweeps : r.sweeps_seen;
    out->max_viol = r.max_viol;
    out->eps_abs = r.eps_abs;
    out->t_submit = r.t_submit;
    out->t_admit = r.t_admit;
    out->t_done = r.t_done;
    out->hbm_bytes = r.bytes;
    out->footprint = r.footprint;
    return MODAP_OK;
}

modap_status modap_server_result(modap_server *s, int64_t ticket, double *x) {
    TraceRange trace_("modap_server_result");
    if (!s) return MODAP_E_INVAL;
    if (ticket < 0 || ticket >= (int64_t)s->reqs.size() || !x) return fail(s, MODAP_E_INVAL, "unknown ticket");
    const Req &r = s->reqs[(size_t)ticket];
    if (r.state != RQ_DONE) return fail(s, MODAP_E_STATE, "the request has not finished");
    if (r.released) return fail(s, MODAP_E_STATE, "the request's result was released");
    for (size_t i = 0; i < r.x.size(); ++i) x[i] = r.x[i];
    return MODAP_OK;
}

modap_status modap_server_release(modap_server *s, int64_t ticket) {
    if (!s) return MODAP_E_INVAL;
    if (ticket < 0 || ticket >= (int64_t)s->reqs.size()) return fail(s, MODAP_E_INVAL, "unknown ticket");
    Req &r = s->reqs[(size_t)ticket];
    if (r.state != RQ_DONE && r.state != RQ_FAILED) return fail(s, MODAP_E_STATE, "the request has not finished");
    std::vector<double>().swap(r.x);
    r.released = true;
    return MODAP_OK;
}

modap_status modap_server_totals(modap_server *s, double *hbm_bytes, int64_t *rounds, double *memory_in_use) {
    if (!s) return MODAP_E_INVAL;
    if (hbm_bytes) *hbm_bytes = s->bytes;
    if (rounds) *rounds = s->rounds;
    if (memory_in_use) *memory_in_use = s->used;
    return MODAP_OK;
}

const char *modap_server_last_error(modap_server *s) { return s ? s->err.c_str() : "server is NULL"; }

}  // extern "C"
