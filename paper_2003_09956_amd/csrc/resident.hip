// Instantiation and cooperative launch of the resident iteration (resident.hpp).
#include <hip/hip_runtime.h>

#include "aux_launch.hpp"
#include "resident.hpp"

namespace modap {

namespace {

template <int DT, int CPL>
hipError_t launch_resident_cpl(const ResidentArgs &a, int grid, size_t lds, hipStream_t s) {
    const void *f = reinterpret_cast<const void *>(&resident_iterate<DT, CPL>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    ResidentArgs copy = a;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kResidentThreads), args, (unsigned)lds, s);
}

template <int DT>
hipError_t launch_resident_dt(const ResidentArgs &a, int grid, size_t lds, hipStream_t s) {
    switch (a.ldR / 64) {
        case 1: return launch_resident_cpl<DT, 1>(a, grid, lds, s);
        case 2: return launch_resident_cpl<DT, 2>(a, grid, lds, s);
        case 3: return launch_resident_cpl<DT, 3>(a, grid, lds, s);
        case 4: return launch_resident_cpl<DT, 4>(a, grid, lds, s);
        case 5: return launch_resident_cpl<DT, 5>(a, grid, lds, s);
        case 6: return launch_resident_cpl<DT, 6>(a, grid, lds, s);
        case 7: return launch_resident_cpl<DT, 7>(a, grid, lds, s);
        case 8: return launch_resident_cpl<DT, 8>(a, grid, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t aux_resident_launch(int dt, const ResidentArgs &a, int grid, size_t lds, hipStream_t s) {
    switch (dt) {
        case 0: return launch_resident_dt<0>(a, grid, lds, s);
        case 1: return launch_resident_dt<1>(a, grid, lds, s);
        default: return launch_resident_dt<2>(a, grid, lds, s);
    }
}

size_t resident_lds_bytes(int dt, int rows, int ldR) {
    auto up16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    const size_t es = dt == 0 ? 8 : dt == 1 ? 4 : 2, acc = dt == 0 ? 8 : 4;
    return up16((size_t)rows * ldR * es) + 3 * up16((size_t)rows * 8) + 3 * (size_t)ldR * 8 + 2 * up16((size_t)ldR * acc) +
           (size_t)kResidentWaves * ldR * acc;
}

}  // namespace modap
