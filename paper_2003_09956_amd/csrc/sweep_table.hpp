// Registry of the compiled sweep kernel shapes.
#pragma once

#include "modap_device.hpp"

namespace modap {

// Launch on `stream`; when e0/e1 are given, they record the kernel's start
// and end as part of its dispatch (no separate event packets).
using SweepLaunch = hipError_t (*)(const SweepArgs &, int grid, hipStream_t stream, hipEvent_t e0, hipEvent_t e1);

struct SweepKernel {
    int dt;
    int block;
    int lpr;
    int chunks;
    int rs;
    int pd;          // steps of rows in flight + 1
    bool has_v;
    SweepLaunch launch;
    const void *func;
};

// Defined once per storage type (sweep_f64.hip, sweep_f32.hip, sweep_bf16.hip).
const SweepKernel *sweep_kernels_0(int *count);
const SweepKernel *sweep_kernels_1(int *count);
const SweepKernel *sweep_kernels_2(int *count);

struct SplitArgs;
// Split-row two-phase kernels of one storage type (workgroup of 256, C chunks
// per column tile).
struct SplitKernels {
    int dt;
    int block;
    int chunks;
    hipError_t (*dot)(const SplitArgs &, int bands, int tiles, bool has_v, hipStream_t);
    hipError_t (*finish)(const SplitArgs &, int blocks, bool has_v, hipStream_t);
    hipError_t (*axpy)(const SplitArgs &, int bands, int tiles, hipStream_t);
};
const SplitKernels *split_kernels_0();
const SplitKernels *split_kernels_1();
const SplitKernels *split_kernels_2();

}  // namespace modap
