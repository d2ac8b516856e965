// Host-only stand-ins for the GPU library's device-side symbols, so that the
// C-ABI host code (api.cpp, tsdf_api.cpp) links into a sanitizer build that
// runs on a machine without a GPU: no kernels, empty kernel tables.  Test
// infrastructure only; never part of libpsweep.so.
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace psw {
struct KernelEntry;
}

extern "C" {
int psw_kernels_grid(const psw::KernelEntry **out) { *out = nullptr; return 0; }
int psw_kernels_extra(const psw::KernelEntry **out) { *out = nullptr; return 0; }
int psw_kernels_small(const psw::KernelEntry **out) { *out = nullptr; return 0; }
int psw_kernels_grid8(const psw::KernelEntry **out) { *out = nullptr; return 0; }
int psw_kernels_f32img(const psw::KernelEntry **out) { *out = nullptr; return 0; }
int psw_kernels_persistent(const psw::KernelEntry **out) { *out = nullptr; return 0; }
const void *psw_setup_kernel() { return nullptr; }
const void *psw_prep_kernel() { return nullptr; }
const void *psw_reset_kernel() { return nullptr; }
const void *psw_merge_kernel() { return nullptr; }
const void *psw_chunk_merge_kernel() { return nullptr; }
const void *psw_filter_kernel() { return nullptr; }
const void *psw_mask_kernel() { return nullptr; }
const void *psw_backward_kernel(int, int, int, int, int) { return nullptr; }
size_t psw_backward_lds(int, int, int) { return 0; }
int psw_backward_tile_rows() { return 4; }
int psw_backward_threads(int) { return 512; }
const void *psw_zero_kernel() { return nullptr; }
const void *psw_pose_reduce_kernel() { return nullptr; }
const void *psw_tsdf_kernel(int) { return nullptr; }
hipError_t psw_static_scratch(void **ptr, size_t *bytes) { *ptr = nullptr; *bytes = 0; return hipErrorNoDevice; }
}
