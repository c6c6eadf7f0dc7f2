// Instantiations of the sweep kernel: one for 7 and one for 8 waves per SIMD
// (the register budget the compiler works to; the tuner picks between them).
#include "sweep_kernel.h"
#include "launch.h"

namespace wpm {

hipError_t launch_sweep(int waves, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                        const uint32_t *tables, const int64_t *offsets, const wpm_item *items,
                        const KArgs &a) {
    if (waves == 7)
        hipLaunchKernelGGL(sweep_kernel<7>, grid, block, lds, st, tables, offsets, items, a);
    else
        hipLaunchKernelGGL(sweep_kernel<8>, grid, block, lds, st, tables, offsets, items, a);
    return hipGetLastError();
}

hipError_t occupancy_sweep(int waves, int *nb, int block, size_t lds) {
    if (waves == 7) return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, sweep_kernel<7>, block, lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, sweep_kernel<8>, block, lds);
}

}  // namespace wpm
