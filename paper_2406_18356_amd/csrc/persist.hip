// persist.hip -- instantiates the persistent kernel (persist_kernels.hpp)
// for single precision: one kernel for sizes 512..2048 (about 37 KB of LDS per
// block, four blocks per CU) and one that also runs 4096 (about 70 KB).
#include "persist_kernels.hpp"

namespace msr {

// Launches `grid` persistent blocks after resetting the counters, on stream s.
hipError_t persist_launch_f32(const PersistArgs<float>& pa, bool with_4096, int grid, hipStream_t s) {
    const int n = pa.C * pa.npass;
    hipLaunchKernelGGL(persist_reset, dim3((n + 255) / 256 + 1), dim3(256), 0, s, pa.ctl, pa.done, n);
    if (with_4096) hipLaunchKernelGGL((persist_kernel<float, 4>), dim3(grid), dim3(256), 0, s, pa);
    else hipLaunchKernelGGL((persist_kernel<float, 3>), dim3(grid), dim3(256), 0, s, pa);
    return hipGetLastError();
}

// Blocks of the persistent kernel a CU holds at once (for the grid size).
int persist_occupancy_f32(bool with_4096) {
    int n = 0;
    const hipError_t e = with_4096
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_kernel<float, 4>, 256, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persist_kernel<float, 3>, 256, 0);
    return e == hipSuccess && n > 0 ? n : 1;
}

}  // namespace msr
