// Host-side helpers shared by the single-system and the batched halves of the
// library: device selection, error reporting into a context's message, and
// storage-type sizes.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "modap.h"
#include "validate.hpp"

namespace modap_host {

// Make `d` the current device for the guard's lifetime.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Record `msg` as the context's last error and return `st` (any context type
// with a std::string member `err`).
template <typename Ctx>
modap_status fail(Ctx *c, modap_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

template <typename Ctx>
modap_status hip_fail(Ctx *c, hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory) return fail(c, MODAP_E_NOMEM, std::string(what) + ": out of device memory");
    return fail(c, MODAP_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

inline size_t elem_size(int dt) { return dt == 0 ? 8 : dt == 1 ? 4 : 2; }
inline size_t acc_size(int dt) { return dt == 0 ? 8 : 4; }
inline int vec_elems(int dt) { return 16 / (int)elem_size(dt); }

template <typename P>
void free_dev(P *&p) {
    if (p) (void)hipFree((void *)p);
    p = nullptr;
}

}  // namespace modap_host

#define HIP_TRY(c, expr)                                                \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return ::modap_host::hip_fail((c), e_, #expr); \
    } while (0)

#define LAUNCH_TRY(c, what)                                             \
    do {                                                                \
        hipError_t e_ = hipPeekAtLastError();                           \
        if (e_ != hipSuccess) {                                         \
            (void)hipGetLastError();                                    \
            return ::modap_host::hip_fail((c), e_, what);               \
        }                                                               \
    } while (0)
