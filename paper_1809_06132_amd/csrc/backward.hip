// Soft-argmin backward pass (the kernels themselves are in backward_impl.h):
// the forms for levels of fronto planes only, the zero and pose-reduce
// kernels, and the lookup of a form by window, source count, image format,
// image-gradient request and plane families.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "backward_impl.h"

namespace psw {

__global__ void zero_kernel(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

// Sum of the workgroups' pose partial rows: workgroup c adds column c, each
// of its 256 threads a strided share of the rows, then a fixed tree (the
// same order every time).
__global__ __launch_bounds__(256) void pose_reduce_kernel(const double *__restrict__ gpart, int n_rows, int n,
                                                          double *__restrict__ gpose) {
    __shared__ double part[256];
    const int c = blockIdx.x, t = threadIdx.x;
    double acc = 0.0;
    for (int r = t; r < n_rows; r += 256) acc += gpart[(int64_t)r * n + c];
    part[t] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) gpose[c] = part[0];
}

}  // namespace psw

extern "C" {
const void *psw_backward_ground_kernel(int win, int n_src, int img, int image_grads);   // backward_ground.hip

const void *psw_zero_kernel() { return (const void *)&psw::zero_kernel; }
const void *psw_pose_reduce_kernel() { return (const void *)&psw::pose_reduce_kernel; }

const void *psw_backward_kernel(int win, int n_src, int img, int image_grads, int ground) {
    if (ground) return psw_backward_ground_kernel(win, n_src, img, image_grads);
#define PSW_B(W, I, G)                                                                      \
    if (win == W && img == I && (image_grads != 0) == G) {                                  \
        if (n_src == 1) return (const void *)&psw::backward_kernel<W, 1, I, G, false>;     \
        if (n_src == 2) return (const void *)&psw::backward_kernel<W, 2, I, G, false>;     \
        if (n_src == 3) return (const void *)&psw::backward_kernel<W, 3, I, G, false>;     \
        if (n_src == 4) return (const void *)&psw::backward_kernel<W, 4, I, G, false>;     \
    }
    PSW_B(5, 0, true) PSW_B(7, 0, true) PSW_B(9, 0, true) PSW_B(5, 1, true) PSW_B(7, 1, true) PSW_B(9, 1, true)
    PSW_B(5, 0, false) PSW_B(7, 0, false) PSW_B(9, 0, false) PSW_B(5, 1, false) PSW_B(7, 1, false)
    PSW_B(9, 1, false)
#undef PSW_B
    return nullptr;
}

int psw_backward_tile_rows() { return psw::Backward<5, 1, 0, true, false>::TYO; }
int psw_backward_threads(int image_grads) {
    return image_grads ? psw::Backward<5, 1, 0, true, false>::NW * psw::kWave : psw::Backward<5, 1, 0, false, false>::NW * psw::kWave;
}

size_t psw_backward_lds(int win, int n_src, int image_grads) {
#define PSW_L(W, G)                                                          \
    if (win == W && (image_grads != 0) == G) {                               \
        if (n_src == 1) return psw::Backward<W, 1, 0, G, false>::lds_bytes();       \
        if (n_src == 2) return psw::Backward<W, 2, 0, G, false>::lds_bytes();       \
        if (n_src == 3) return psw::Backward<W, 3, 0, G, false>::lds_bytes();       \
        if (n_src == 4) return psw::Backward<W, 4, 0, G, false>::lds_bytes();       \
    }
    PSW_L(5, true) PSW_L(7, true) PSW_L(9, true) PSW_L(5, false) PSW_L(7, false) PSW_L(9, false)
#undef PSW_L
    return 0;
}
}
