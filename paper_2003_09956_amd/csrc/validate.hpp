// Host-side argument checks and admission accounting of the library.  Plain
// C++ with no device code and no HIP dependency, so that it can be built and
// tested on a machine without a GPU (under AddressSanitizer and
// UndefinedBehaviorSanitizer).  Every check returns MODAP_OK or an error code
// and sets *msg to a static description of the failure.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "modap.h"

namespace modap_host {

// Bytes of one stored element and elements per 16-byte vector.
size_t storage_bytes(int dt);
int64_t padded_length(int dt, int64_t n);   // n rounded up to a whole number of 16-byte vectors

// lambda > 0 finite, eps > 0 finite, a known step rule, max_iters >= 0, profile >= 0.
modap_status check_params(const modap_params *p, const char **msg);

// m, n >= 1, lda >= n, A and b given, a known storage type.
modap_status check_system(int64_t m, int64_t n, int64_t lda, const void *A, const double *b, int dt,
                          const char **msg);

// Every entry of p[0..count) finite.
bool all_finite(const double *p, int64_t count);

// A row replacement from host memory: 0 <= k <= m; rows, new_rows and new_b
// given when k > 0; every index in [0, m) and distinct; every new_b finite.
modap_status check_rows(int64_t k, const int64_t *rows, const void *new_rows, const double *new_b, int64_t m,
                        const char **msg);

// Each of the k replacement rows (n elements of storage type dt, row-major)
// finite and non-zero (section 2 assumes a_i != 0): E_ZERO_ROW otherwise.
modap_status check_new_rows(int dt, const void *new_rows, int64_t k, int64_t n, const char **msg);

// A drift schedule V [T x ldv] from host memory: T >= 0, ldv >= n, finite.
modap_status check_drift(int64_t T, const double *V, int64_t ldv, int64_t n, bool host, const char **msg);

// Device bytes a served request holds while live: A, b, ||a||^2, the exact
// right-hand side, r, the FP64 vectors (x, y, translation, its running sum,
// two evaluation vectors), the working vectors, the y partials of one sweep
// (about one row of the accumulation type per 64 rows) and the drift schedule.
double request_footprint(int dt, int64_t m, int64_t n, int64_t T);

// Admission: the request at the head of the queue is admitted when its
// footprint fits the budget beside the live ones and the live count is below
// max_live (0: no such cap).
bool admissible(double used, double footprint, double budget, int64_t live, int64_t max_live);

// A submitted request: sizes, data and drift schedule.
modap_status check_request(int64_t m, int64_t n, const void *A, const double *b, int64_t T, const double *V,
                           int64_t ldv, const char **msg);

}  // namespace modap_host
