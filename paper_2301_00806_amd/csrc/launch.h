// Launch entry points of the kernel instantiations (one translation unit per
// maximum group count GM in {2, 4, 8, 16}; slot stride QS in {4, 8}; facet
// words WM in {4, 10, 16, 32}).
#pragma once
#include <hip/hip_runtime.h>

#include "sweep_kernel.h"

namespace wpm {
hipError_t launch_sweep_g2(int qs, int wm, dim3 grid, dim3 block, size_t lds, hipStream_t st, const uint32_t *tables, const int64_t *offsets, const wpm_item *items, const KArgs &a);
hipError_t launch_sweep_g4(int qs, int wm, dim3 grid, dim3 block, size_t lds, hipStream_t st, const uint32_t *tables, const int64_t *offsets, const wpm_item *items, const KArgs &a);
hipError_t launch_sweep_g8(int qs, int wm, dim3 grid, dim3 block, size_t lds, hipStream_t st, const uint32_t *tables, const int64_t *offsets, const wpm_item *items, const KArgs &a);
hipError_t launch_sweep_g16(int qs, int wm, dim3 grid, dim3 block, size_t lds, hipStream_t st, const uint32_t *tables, const int64_t *offsets, const wpm_item *items, const KArgs &a);
hipError_t occupancy_sweep_g2(int qs, int wm, int *nb, int block, size_t lds);
hipError_t occupancy_sweep_g4(int qs, int wm, int *nb, int block, size_t lds);
hipError_t occupancy_sweep_g8(int qs, int wm, int *nb, int block, size_t lds);
hipError_t occupancy_sweep_g16(int qs, int wm, int *nb, int block, size_t lds);
}  // namespace wpm
