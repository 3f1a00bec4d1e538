// Launchers of the auxiliary kernels (defined once, in host.hip) for the
// other translation units of the library.  Each queues its kernel(s) on
// `s` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modap_device.hpp"

namespace modap {

// ||a_i||^2 of rows [0, m) in FP64; *bad <- min index of a zero or non-finite row.
hipError_t aux_row_norms(int dt, const void *A, int64_t ldA, int64_t m, int64_t n, double *nu,
                         unsigned long long *bad, hipStream_t s);
// *flag <- 1 when p[0..count) holds a NaN or infinity.
hipError_t aux_check_finite(const double *p, int64_t count, int *flag, hipStream_t s);
// Both state slots fresh (running, no translation pending, no drift).
hipError_t aux_ctl_init(Ctrl *c, hipStream_t s);
// Replace k rows in place (see scatter_rows).
hipError_t aux_scatter_rows(int dt, void *A, int64_t ldA, int64_t m, int64_t n, int64_t k, const int64_t *rows,
                            const void *new_rows, const double *new_b, double *b, double *nu, Ctrl *ctl, int sl,
                            const double *vpend, hipStream_t s);
// Add v to the one-shot translation of the state in slot sl.
hipError_t aux_vpend_add(Ctrl *c, int sl, double *vpend, const double *v, int64_t n, hipStream_t s);
// Move a scheduled translation that is due into the one-shot slot.
hipError_t aux_sched_to_vpend(Ctrl *c, int sl, double *vpend, const double *V, int64_t ldV, int64_t n, hipStream_t s);
// Install a drift schedule of T rows (the state restarts at its first row).
hipError_t aux_ctl_set_drift(Ctrl *c, int sl, int64_t T, hipStream_t s);
// Apply every translation still pending in slot sl to b with a pass of its own.
hipError_t aux_flush(int dt, const void *A, int64_t ldA, int64_t m, int64_t n, Ctrl *ctl, int sl, double *vpend,
                     const double *V, double *b, hipStream_t s);

}  // namespace modap
