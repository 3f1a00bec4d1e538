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
                            const void *new_rows, const double *new_b, double *b, double *bref, double *nu, Ctrl *ctl,
                            int sl, const double *vpend, const double *V, int64_t ldV, const double *wsum,
                            hipStream_t s);
// Claim the rows of a device-side replacement before it (ST_BAD_ROW on an
// index out of range or repeated), and release the claims after it.
hipError_t aux_claim_rows(const int64_t *rows, int64_t k, int64_t m, int *claim, Ctrl *ctl, int sl, hipStream_t s);
hipError_t aux_release_rows(const int64_t *rows, int64_t k, int64_t m, int *claim, hipStream_t s);
// Add v to the one-shot translation of the state in slot sl.
hipError_t aux_vpend_add(Ctrl *c, int sl, double *vpend, const double *v, int64_t n, hipStream_t s);
// Move a scheduled translation that is due into the one-shot slot.
hipError_t aux_sched_to_vpend(Ctrl *c, int sl, double *vpend, const double *V, int64_t ldV, int64_t n, hipStream_t s);
// Install a drift schedule of T rows (the state restarts at its first row).
hipError_t aux_ctl_set_drift(Ctrl *c, int sl, int64_t T, hipStream_t s);
// out <- bref + A (wsum + pending translation of slot sl), FP64; changes no state.
hipError_t aux_rhs_exact(int dt, const void *A, int64_t ldA, int64_t m, int64_t n, const Ctrl *ctl, int sl,
                         const double *bref, const double *wsum, const double *vpend, const double *V, int64_t ldV,
                         double *out, hipStream_t s);
struct ResidentArgs;
// Cooperative launch of the resident iteration (resident.hpp) with `grid`
// workgroups and `lds` bytes of dynamic LDS each.
hipError_t aux_resident_launch(int dt, const ResidentArgs &a, int grid, size_t lds, hipStream_t s);
// Dynamic LDS of a resident workgroup holding `rows` rows of ldR elements.
size_t resident_lds_bytes(int dt, int rows, int ldR);
// Queue the FP64 certificate of the stop in slot a.sl (see certify.hpp); R and Gs are filled in.
hipError_t aux_certify(int dt, CertArgs a, hipStream_t s);

}  // namespace modap
