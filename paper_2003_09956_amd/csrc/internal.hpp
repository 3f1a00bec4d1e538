// Entry points shared between the translation units of the library that are
// not part of the C ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "modap.h"
#include "modap_device.hpp"
#include "sweep_table.hpp"

// The FP64 certificate of the stops of the given batch systems (each a no-op
// unless the system's committed state is an uncertified stop).  Synchronises.
modap_status modap_batch_certify_ids(modap_batch *batch, const modap_params *p, const int64_t *ids, int64_t count);

namespace modap {

// A stateless one-pass sweep in the library's built-in launch shape (the shape
// and row mapping a context would choose for the same storage type, padded
// row length and m), without the translation.
struct StaticPlan {
    const SweepKernel *k;   // the sweep kernel (no translation)
    int grid;               // workgroups
    int R;                  // reduction workgroups: ceil(n / 64)
    int64_t cov;            // columns of one partial y (the shape's row coverage)
    int64_t rows_per_block, block_stride, step_stride;
};

// false when no one-pass shape covers rows of padded length ldA.
bool static_sweep_plan(int dt, int64_t ldA, int64_t m, int64_t n, int cu_count, StaticPlan *out);

// Device memory the stateless sweep works in (caller-provided, see noalloc.hip).
struct SweepScratch {
    double *nu;                 // [m]
    void *work;                 // [3 x ldA] accumulation type
    void *part;                 // [grid x cov] accumulation type
    int64_t *h_part;            // [grid]
    double *dmax_part;          // [grid]
    double *binf_part;          // [grid]
    Totals *tot;
    double *ynp;                // [R]
    Ctrl *ctl;
    unsigned long long *bad;
};

// Queue the stateless sweep on `stream`: row norms, the working vectors of x,
// the sweep, the fixed-order reduction to y, and the totals to *h and
// *max_viol.  Every pointer is device memory.
hipError_t static_sweep_launch(int dt, const StaticPlan &plan, const SweepScratch &s, const void *A, int64_t ldA,
                               int64_t m, int64_t n, const double *b, const double *x, double *r, double *y,
                               int64_t *h, double *max_viol, hipStream_t stream);

}  // namespace modap
