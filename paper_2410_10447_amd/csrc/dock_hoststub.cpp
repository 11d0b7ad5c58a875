// Host-only stand-ins for the kernel launchers (dock_kernels.hip,
// dock_ga.hip, dock_static.hip), linked instead of them into the sanitizer
// build of the host code (build_lib.build_sanitized): the preparation and
// the C ABI's validation run under AddressSanitizer and UBSan on a machine
// without a GPU, and any call that would reach a kernel fails with
// hipErrorNoDevice. Not part of the product library.
#include <hip/hip_runtime.h>

#include "dock_launch.h"

namespace docklaunch {

hipError_t launch_score(const GridParams&, const uint8_t*, int, int, const float*, float*, float*, float*, int, int,
                        hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_score_two(const GridParams&, const uint8_t*, int, const float*, float*, float*, float*, int,
                            hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_ls(const LsParams&, int, int, int, hipStream_t) { return hipErrorNoDevice; }
int ls_blocks_per_cu(int, int) { return 0; }
hipError_t launch_block_sum4(const float*, float*, int, int, int, int, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_expand_corners(const GridParams&, float*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_sw(const GridParams&, const uint8_t*, int, int, const SwParams&, hipStream_t) {
    return hipErrorNoDevice;
}
hipError_t launch_ga_step(const GaParams&, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_select_rows(const float*, int, float, int32_t*, int32_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_move_rows(bool, const float*, float*, const int32_t*, int, int, int, hipStream_t) {
    return hipErrorNoDevice;
}
int64_t static_workspace_capacity() { return kWorkspaceHeader; }
hipError_t static_workspace(void**) { return hipErrorNoDevice; }
hipError_t launch_table_fill(void*, const void*, int64_t, hipStream_t) { return hipErrorNoDevice; }

}  // namespace docklaunch
