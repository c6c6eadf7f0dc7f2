// Instantiations of the sweep kernel for up to 16 ridge groups.
#include "sweep_kernel.h"
#include "launch.h"

namespace wpm {

#define WPM_GM 16
template <int QS, int WM>
static hipError_t launch_one(dim3 grid, dim3 block, size_t lds, hipStream_t st, const uint32_t *tables,
                             const int64_t *offsets, const wpm_item *items, const KArgs &a) {
    hipLaunchKernelGGL((sweep_kernel<WPM_GM, QS, WM>), grid, block, lds, st, tables, offsets, items, a);
    return hipGetLastError();
}
template <int QS, int WM>
static hipError_t occ_one(int *nb, int block, size_t lds) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(nb, sweep_kernel<WPM_GM, QS, WM>, block, lds);
}

hipError_t launch_sweep_g16(int qs, int wm, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                            const uint32_t *tables, const int64_t *offsets, const wpm_item *items,
                            const KArgs &a) {
    if (qs == 4) {
        if (wm == 4) return launch_one<4, 4>(grid, block, lds, st, tables, offsets, items, a);
        if (wm == 10) return launch_one<4, 10>(grid, block, lds, st, tables, offsets, items, a);
        if (wm == 16) return launch_one<4, 16>(grid, block, lds, st, tables, offsets, items, a);
        return launch_one<4, 32>(grid, block, lds, st, tables, offsets, items, a);
    }
    if (wm == 4) return launch_one<8, 4>(grid, block, lds, st, tables, offsets, items, a);
    if (wm == 10) return launch_one<8, 10>(grid, block, lds, st, tables, offsets, items, a);
    if (wm == 16) return launch_one<8, 16>(grid, block, lds, st, tables, offsets, items, a);
    return launch_one<8, 32>(grid, block, lds, st, tables, offsets, items, a);
}

hipError_t occupancy_sweep_g16(int qs, int wm, int *nb, int block, size_t lds) {
    if (qs == 4) {
        if (wm == 4) return occ_one<4, 4>(nb, block, lds);
        if (wm == 10) return occ_one<4, 10>(nb, block, lds);
        if (wm == 16) return occ_one<4, 16>(nb, block, lds);
        return occ_one<4, 32>(nb, block, lds);
    }
    if (wm == 4) return occ_one<8, 4>(nb, block, lds);
    if (wm == 10) return occ_one<8, 10>(nb, block, lds);
    if (wm == 16) return occ_one<8, 16>(nb, block, lds);
    return occ_one<8, 32>(nb, block, lds);
}

}  // namespace wpm
