// Launch entry points of the sweep kernel (instantiated in sweep.hip for 7
// and 8 waves per SIMD).
#pragma once
#include <hip/hip_runtime.h>

#include "sweep_kernel.h"

namespace wpm {
hipError_t launch_sweep(int waves, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        const uint32_t *tables, const int64_t *offsets, const wpm_item *items,
                        const KArgs &a);
hipError_t occupancy_sweep(int waves, int *nb, int block, size_t lds);
}  // namespace wpm
