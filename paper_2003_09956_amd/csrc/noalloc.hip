// modap_eval_sweep_static: one sweep that allocates nothing.
//
// The same pure sweep as modap_eval_sweep (section 3: Map of the positive
// slices, eq. 7, and Reduce(+); the measures of eq. 10), for callers that
// cannot allocate device memory -- code under HIP graph capture, tight
// serving loops, harnesses that forbid it.  It needs no context: the caller
// passes the system, the point and the outputs in device memory, and every
// intermediate (row norms, working vectors, partial sums, totals) lives in
// `scratch`, a file-scope device array of kScratchBytes held by each GPU the
// library runs on until the process ends.  Host code never uses the array's
// name as an address: its device address is taken once per device with
// hipGetSymbolAddress and kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_common.hpp"
#include "internal.hpp"
#include "modap.h"

namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per device
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};
int g_cus[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), taken on
// the first call on that device.
modap_status scratch_of(int device, unsigned char **p, int *cus) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MODAP_E_DEVICE;
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c < 1)
            return MODAP_E_DEVICE;
        g_scratch[device] = ptr;
        g_cus[device] = c;
    }
    *p = static_cast<unsigned char *>(g_scratch[device]);
    *cus = g_cus[device];
    return MODAP_OK;
}

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

extern "C" modap_status modap_eval_sweep_static(int device, void *hip_stream, int64_t m, int64_t n, modap_dtype storage,
                                                const void *A, int64_t lda, const double *b, const double *x,
                                                double *r, double *y, int64_t *h, double *max_viol) {
    using namespace modap;
    const char *msg = nullptr;
    if (modap_host::check_system(m, n, lda, A, b, (int)storage, &msg) != MODAP_OK) return MODAP_E_INVAL;
    if (!x || !y) return MODAP_E_INVAL;
    const int dt = (int)storage;
    const int64_t vec = 16 / (int64_t)modap_host::storage_bytes(dt);
    if (lda % vec != 0) return MODAP_E_INVAL;   // rows start on 16-byte boundaries
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return MODAP_E_DEVICE;
    if (device < 0 || device >= count || device >= kMaxDevices) return MODAP_E_INVAL;
    modap_host::DeviceGuard g(device);
    unsigned char *base = nullptr;
    int cus = 0;
    if (modap_status st = scratch_of(device, &base, &cus)) return st;
    StaticPlan plan{};
    if (!static_sweep_plan(dt, lda, m, n, cus, &plan)) return MODAP_E_INVAL;   // rows too long for one pass
    // the layout of this call inside the scratch array
    const size_t acc = dt == 0 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += up256(bytes);
        return p;
    };
    SweepScratch s{};
    s.ctl = reinterpret_cast<Ctrl *>(take(sizeof(Ctrl)));
    s.tot = reinterpret_cast<Totals *>(take(sizeof(Totals)));
    s.bad = reinterpret_cast<unsigned long long *>(take(sizeof(unsigned long long)));
    s.h_part = reinterpret_cast<int64_t *>(take(sizeof(int64_t) * (size_t)plan.grid));
    s.dmax_part = reinterpret_cast<double *>(take(sizeof(double) * (size_t)plan.grid));
    s.binf_part = reinterpret_cast<double *>(take(sizeof(double) * (size_t)plan.grid));
    s.ynp = reinterpret_cast<double *>(take(sizeof(double) * (size_t)plan.R));
    s.nu = reinterpret_cast<double *>(take(sizeof(double) * (size_t)m));
    s.work = take(3 * acc * (size_t)lda);
    s.part = take(acc * (size_t)plan.grid * (size_t)plan.cov);
    if (off > kScratchBytes) return MODAP_E_INVAL;      // beyond the static scratch
    const hipError_t e = static_sweep_launch(dt, plan, s, A, lda, m, n, b, x, r, y, h, max_viol,
                                             reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? MODAP_E_NOMEM : MODAP_E_DEVICE;
    }
    return MODAP_OK;
}
